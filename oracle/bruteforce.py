"""ctypes wrapper around the brute-force C oracle (``orc.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows sec. "Symmetry adapted basis states" (orbits, representative as the
orbit minimum, matrix element between representatives) with the first,
memory-free representative search of sec. "Sublattice coding algorithm", and
the scatter order of the parallel matrix-vector algorithm (Alg. "Parallel
matrix-vector multiply", with received coefficients *added* to the target).

Pins (tests/test_oracle.py): the two worked chain examples (exact integers),
the definition-level sector matrix of ``definition.py``, closed-form ground
energies, character-formula dimensions, Hermiticity, and the union of all
momentum-sector spectra against the full fixed-Sz spectrum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force=False):
    """Compile orc.c with gcc (OpenMP) into oracle/liborc.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.orc_act.argtypes = [ctypes.c_int, P, ctypes.c_int, u64]
        L.orc_act.restype = u64
        L.orc_rep.argtypes = [ctypes.c_int, ctypes.c_int, P, P, u64, P]
        L.orc_rep.restype = u64
        L.orc_rep_many.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, i64, P, P, P, P, P]
        L.orc_rep_many.restype = None
        L.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P, i64]
        L.orc_basis.restype = i64
        L.orc_basis_range.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, u64, u64, P, P, i64]
        L.orc_basis_range.restype = i64
        L.orc_unrank.argtypes = [ctypes.c_int, ctypes.c_int, u64]
        L.orc_unrank.restype = u64
        L.orc_apply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, i64, P, P,
                                P, P, ctypes.c_int, P, P]
        L.orc_apply.restype = None
        L.orc_row_terms.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, i64,
                                    P, P, P, P, P, P, P, P]
        L.orc_row_terms.restype = None
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_fsign.argtypes = [ctypes.c_int, P, u64]
        L.orc_fsign.restype = ctypes.c_int
        L.orc_frep_many.argtypes = [ctypes.c_int, ctypes.c_int, P, P, i64, P, P, P, P, P, P]
        L.orc_frep_many.restype = None
        L.orc_fbasis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, i64]
        L.orc_fbasis.restype = i64
        L.orc_fapply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, P, P, i64, P, P, P, P, P, P]
        L.orc_fapply.restype = None
        L.orc_frow_terms.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, P, P, i64, P, P, P, P,
                                     P, P, P, P]
        L.orc_frow_terms.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pz(model):
    return None if model.Jz is None else _p(model.Jz)


class Model:
    """Group, irrep and bonds in the flat layout the C oracle reads."""

    def __init__(self, n_sites, perm, flip, chi, bonds=None, J=None, Jz=None):
        self.n = int(n_sites)
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)
        self.ng = int(self.perm.shape[0])
        self.flip = np.ascontiguousarray(flip, dtype=np.uint8)
        chi = np.asarray(chi, dtype=np.complex128)
        self.chi_c = chi
        self.chi = np.ascontiguousarray(np.stack([chi.real, chi.imag], 1))
        self.bonds = None if bonds is None else np.ascontiguousarray(bonds, dtype=np.int32)
        self.J = None if J is None else np.ascontiguousarray(J, dtype=np.float64)
        # Ising couplings of the XXZ model; None means Jz = J (Heisenberg)
        self.Jz = None if Jz is None else np.ascontiguousarray(Jz, dtype=np.float64)

    @classmethod
    def from_workload(cls, w, J=None, Jz=None):
        c = w.cluster
        return cls(c.n_sites, c.perm, c.flip, w.chi, c.bonds, w.J if J is None else J, Jz)

    @property
    def nb(self):
        return 0 if self.bonds is None else int(self.bonds.shape[0])


def act(model, g, state):
    return int(lib().orc_act(model.n, _p(model.perm[g]), int(model.flip[g]), int(state)))


def rep(model, state):
    """(representative, first minimising group element) of one configuration."""
    g = np.zeros(1, dtype=np.int32)
    r = lib().orc_rep(model.n, model.ng, _p(model.perm), _p(model.flip), int(state), _p(g))
    return int(r), int(g[0])


def rep_many(model, states):
    """Representatives, minimisers, stabiliser sizes and sector compatibility."""
    s = np.ascontiguousarray(states, dtype=np.uint64)
    m = s.shape[0]
    r = np.empty(m, np.uint64)
    g = np.empty(m, np.int32)
    st = np.empty(m, np.int32)
    cp = np.empty(m, np.uint8)
    lib().orc_rep_many(model.n, model.ng, _p(model.perm), _p(model.flip), _p(model.chi), m,
                       _p(s), _p(r), _p(g), _p(st), _p(cp))
    return r, g, st, cp.astype(bool)


def basis(model, n_up, count_only=False):
    """Ascending sector representatives and stabiliser sizes (brute force)."""
    L = lib()
    d = L.orc_basis(model.n, n_up, model.ng, _p(model.perm), _p(model.flip), _p(model.chi),
                    None, None, 0)
    if count_only:
        return int(d)
    states = np.empty(d, np.uint64)
    stab = np.empty(d, np.int32)
    d2 = L.orc_basis(model.n, n_up, model.ng, _p(model.perm), _p(model.flip), _p(model.chi),
                     _p(states), _p(stab), d)
    assert d2 == d
    return states, stab


def basis_range(model, n_up, rank_lo, rank_hi):
    """Sector representatives (and stabiliser sizes) among the configurations
    of ranks [rank_lo, rank_hi) in the ascending popcount-n_up enumeration."""
    L = lib()
    args = (model.n, n_up, model.ng, _p(model.perm), _p(model.flip), _p(model.chi), int(rank_lo), int(rank_hi))
    d = L.orc_basis_range(*args, None, None, 0)
    states = np.empty(d, np.uint64)
    stab = np.empty(d, np.int32)
    d2 = L.orc_basis_range(*args, _p(states), _p(stab), d)
    assert d2 == d
    return states, stab


def unrank(n, n_up, r):
    """The r-th (0-based) n-bit configuration with n_up set bits, ascending."""
    return int(lib().orc_unrank(int(n), int(n_up), int(r)))


def apply(model, states, stab, x, nthreads=None):
    """y = H x in the sector, scatter order; returns (y, kept, dropped)."""
    L = lib()
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    xc = np.ascontiguousarray(np.stack([x.real, x.imag if cplx else np.zeros_like(x)], 1),
                              dtype=np.float64)
    d = int(states.shape[0])
    y = np.empty((d, 2), np.float64)
    kept = np.zeros(1, np.int64)
    dropped = np.zeros(1, np.int64)
    if nthreads is None:
        nthreads = 1 if d < 20000 else min(8, L.orc_max_threads())
    L.orc_apply(model.n, model.ng, _p(model.perm), _p(model.flip), _p(model.chi), model.nb,
                _p(model.bonds), _p(model.J), _pz(model), d, _p(np.ascontiguousarray(states, np.uint64)),
                _p(np.ascontiguousarray(stab, np.int32)), _p(xc), _p(y), int(nthreads),
                _p(kept), _p(dropped))
    yc = y[:, 0] + 1j * y[:, 1]
    return (yc if cplx else yc.real.copy()), int(kept[0]), int(dropped[0])


def row_terms(model, rows):
    """Per-row matrix elements of the Hermitian sector matrix (see orc.c)."""
    L = lib()
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    m = rows.shape[0]
    nb = model.nb
    out = dict(
        row_stab=np.empty(m, np.int32), row_compat=np.empty(m, np.uint8),
        row_diag=np.empty(m, np.float64), tgt=np.empty((m, nb), np.uint64),
        tgt_stab=np.empty((m, nb), np.int32), tgt_flag=np.empty((m, nb), np.uint8),
        coef=np.empty((m, nb, 2), np.float64))
    L.orc_row_terms(model.n, model.ng, _p(model.perm), _p(model.flip), _p(model.chi), nb,
                    _p(model.bonds), _p(model.J), _pz(model), m, _p(rows), _p(out["row_stab"]),
                    _p(out["row_compat"]), _p(out["row_diag"]), _p(out["tgt"]),
                    _p(out["tgt_stab"]), _p(out["tgt_flag"]), _p(out["coef"]))
    out["coef"] = out["coef"][..., 0] + 1j * out["coef"][..., 1]
    out["row_compat"] = out["row_compat"].astype(bool)
    return out


def dense_matrix(model, states):
    """The Hermitian sector matrix on the ascending basis ``states``, row by
    row from row_terms (one brute-force pass instead of one H.v per column)."""
    t = row_terms(model, states)
    return _dense_from_rows(states, t["row_diag"], t["tgt"], t["tgt_flag"], t["coef"])


def _dense_from_rows(states, diag, tgt, flag, coef):
    states = np.asarray(states, np.uint64)
    d = states.shape[0]
    H = np.zeros((d, d), np.complex128)
    H[np.arange(d), np.arange(d)] = diag
    r, b = np.nonzero(flag == 1)
    cols = np.searchsorted(states, tgt[r, b])
    assert np.array_equal(states[cols], tgt[r, b])
    np.add.at(H, (r, cols), coef[r, b])
    return H


def rows_apply(model, rows, amplitude):
    """(H x)_row for sampled representative rows, with x given as a function.

    ``amplitude(states) -> values`` returns x for arbitrary representatives
    (a state-hashed input vector), so no index into any basis is needed.
    Returns (y_rows, n_kept_terms, n_dropped_terms, row_compat).
    """
    t = row_terms(model, rows)
    xr = amplitude(np.asarray(rows, np.uint64))
    y = t["row_diag"] * xr
    kept = t["tgt_flag"] == 1
    if kept.any():
        xt = np.zeros(t["tgt"].shape, dtype=np.result_type(xr, np.complex128))
        xt[kept] = amplitude(t["tgt"][kept])
        contrib = np.where(kept, t["coef"] * xt, 0)
        y = y + contrib.sum(axis=1)
    if not np.iscomplexobj(xr) and np.all(np.abs(np.imag(y)) < 1e-300):
        y = np.real(y)
    return y, int(kept.sum()), int((t["tgt_flag"] == 2).sum()), t["row_compat"]


def random_representatives(model, n_up, count, seed):
    """Distinct sector representatives drawn from seeded random configurations."""
    rng = np.random.default_rng(seed)
    n = model.n
    reps = []
    seen = set()
    tries = 0
    while len(reps) < count and tries < 50:
        tries += 1
        m = max(64, 2 * (count - len(reps)))
        # random configurations with n_up set bits among n sites
        keys = rng.random((m, n)).argsort(axis=1)[:, :n_up]
        s = np.zeros(m, np.uint64)
        for c in range(n_up):
            s |= np.left_shift(np.uint64(1), (n - 1 - keys[:, c]).astype(np.uint64))
        r, _, _, comp = rep_many(model, s)
        for v, ok in zip(r.tolist(), comp.tolist()):
            if ok and v not in seen:
                seen.add(v)
                reps.append(v)
                if len(reps) == count:
                    break
    return np.array(sorted(reps), dtype=np.uint64)


# ---- fermions in the occupation-number basis (see orc.c) -------------------

class FermionModel:
    """Orbitals, group (site permutations, no spin flip), irrep and bonds with
    hopping t_b and density interaction V_b, in the layout orc.c reads."""

    def __init__(self, n_orb, perm, chi, bonds, t, V=None):
        self.n = int(n_orb)
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)
        self.ng = int(self.perm.shape[0])
        chi = np.asarray(chi, dtype=np.complex128)
        self.chi = np.ascontiguousarray(np.stack([chi.real, chi.imag], 1))
        self.bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
        self.t = np.ascontiguousarray(t, dtype=np.float64)
        self.V = None if V is None else np.ascontiguousarray(V, dtype=np.float64)

    @property
    def nb(self):
        return int(self.bonds.shape[0])


def fsign(n, perm_row, state):
    """Parity of the Fermi sign of one group element on one configuration."""
    return int(lib().orc_fsign(int(n), _p(np.ascontiguousarray(perm_row, np.int32)), int(state)))


def frep_many(model, states):
    """Representatives, minimisers, Fermi-sign parities of the minimiser on the
    input, stabiliser sizes and sector compatibility."""
    s = np.ascontiguousarray(states, dtype=np.uint64)
    m = s.shape[0]
    r = np.empty(m, np.uint64)
    g = np.empty(m, np.int32)
    sg = np.empty(m, np.int32)
    st = np.empty(m, np.int32)
    cp = np.empty(m, np.uint8)
    lib().orc_frep_many(model.n, model.ng, _p(model.perm), _p(model.chi), m, _p(s), _p(r), _p(g), _p(sg), _p(st),
                        _p(cp))
    return r, g, sg, st, cp.astype(bool)


def fbasis(model, n_part):
    """Ascending fermionic sector representatives and stabiliser sizes."""
    L = lib()
    d = L.orc_fbasis(model.n, n_part, model.ng, _p(model.perm), _p(model.chi), None, None, 0)
    states = np.empty(d, np.uint64)
    stab = np.empty(d, np.int32)
    d2 = L.orc_fbasis(model.n, n_part, model.ng, _p(model.perm), _p(model.chi), _p(states), _p(stab), d)
    assert d2 == d
    return states, stab


def fapply(model, states, stab, x):
    """y = H x in the fermionic sector, scatter order; returns (y, kept, dropped)."""
    L = lib()
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    xc = np.ascontiguousarray(np.stack([x.real, x.imag if cplx else np.zeros_like(x)], 1), dtype=np.float64)
    d = int(states.shape[0])
    y = np.empty((d, 2), np.float64)
    kept = np.zeros(1, np.int64)
    dropped = np.zeros(1, np.int64)
    L.orc_fapply(model.n, model.ng, _p(model.perm), _p(model.chi), model.nb, _p(model.bonds), _p(model.t),
                 None if model.V is None else _p(model.V), d, _p(np.ascontiguousarray(states, np.uint64)),
                 _p(np.ascontiguousarray(stab, np.int32)), _p(xc), _p(y), _p(kept), _p(dropped))
    yc = y[:, 0] + 1j * y[:, 1]
    return (yc if cplx else yc.real.copy()), int(kept[0]), int(dropped[0])


def frow_terms(model, rows):
    """Per-row elements of the Hermitian fermionic sector matrix (orc.c)."""
    L = lib()
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    m, nb = rows.shape[0], model.nb
    out = dict(row_stab=np.empty(m, np.int32), row_compat=np.empty(m, np.uint8), row_diag=np.empty(m, np.float64),
               tgt=np.empty((m, nb), np.uint64), tgt_stab=np.empty((m, nb), np.int32),
               tgt_flag=np.empty((m, nb), np.uint8), coef=np.empty((m, nb, 2), np.float64))
    L.orc_frow_terms(model.n, model.ng, _p(model.perm), _p(model.chi), nb, _p(model.bonds), _p(model.t),
                     None if model.V is None else _p(model.V), m, _p(rows), _p(out["row_stab"]),
                     _p(out["row_compat"]), _p(out["row_diag"]), _p(out["tgt"]), _p(out["tgt_stab"]),
                     _p(out["tgt_flag"]), _p(out["coef"]))
    out["coef"] = out["coef"][..., 0] + 1j * out["coef"][..., 1]
    out["row_compat"] = out["row_compat"].astype(bool)
    return out


def fdense_matrix(model, states):
    """The Hermitian fermionic sector matrix on the ascending basis ``states``."""
    t = frow_terms(model, states)
    return _dense_from_rows(states, t["row_diag"], t["tgt"], t["tgt_flag"], t["coef"])


def frows_apply(model, rows, amplitude):
    """(H x)_row of the fermionic sector matrix for sampled representatives,
    with x given as a function of the state (as rows_apply)."""
    L = lib()
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    m, nb = rows.shape[0], model.nb
    row_stab, row_compat = np.empty(m, np.int32), np.empty(m, np.uint8)
    row_diag = np.empty(m, np.float64)
    tgt, tgt_stab = np.empty((m, nb), np.uint64), np.empty((m, nb), np.int32)
    tgt_flag, coef = np.empty((m, nb), np.uint8), np.empty((m, nb, 2), np.float64)
    L.orc_frow_terms(model.n, model.ng, _p(model.perm), _p(model.chi), nb, _p(model.bonds), _p(model.t),
                     None if model.V is None else _p(model.V), m, _p(rows), _p(row_stab), _p(row_compat),
                     _p(row_diag), _p(tgt), _p(tgt_stab), _p(tgt_flag), _p(coef))
    coef = coef[..., 0] + 1j * coef[..., 1]
    xr = amplitude(rows)
    y = row_diag * xr
    kept = tgt_flag == 1
    if kept.any():
        xt = np.zeros(tgt.shape, dtype=np.result_type(xr, np.complex128))
        xt[kept] = amplitude(tgt[kept])
        y = y + np.where(kept, coef * xt, 0).sum(axis=1)
    if not np.iscomplexobj(xr) and np.all(np.abs(np.imag(y)) < 1e-300):
        y = np.real(y)
    return y, int(kept.sum()), int((tgt_flag == 2).sum()), row_compat.astype(bool)
