"""ctypes binding of libed.so with the same names as the C ABI (include/ed.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Importing this module fails loudly when libed.so has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libed.so")

ED_OK = 0
ERRORS = {
    -1: "ED_ERR_ARG", -2: "ED_ERR_NOT_GROUP", -3: "ED_ERR_BAD_IRREP", -4: "ED_ERR_NOT_SUBLATTICE_STABLE",
    -5: "ED_ERR_FLIP_NEEDS_SZ0", -6: "ED_ERR_NONINVARIANT_H", -7: "ED_ERR_OOM", -8: "ED_ERR_HIP",
    -9: "ED_ERR_UNSUPPORTED",
}


class EDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class ed_lattice_t(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32),
                ("bonds", ctypes.c_void_p), ("n_sublat", ctypes.c_int32)]


class ed_group_t(ctypes.Structure):
    _fields_ = [("n_elems", ctypes.c_int32), ("perm", ctypes.c_void_p), ("flip", ctypes.c_void_p)]


class ed_irrep_t(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_void_p)]


class ed_tuning_t(ctypes.Structure):
    _fields_ = [("limits_bits", ctypes.c_int32), ("index_mode", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("chunk_bits", ctypes.c_int32), ("hash_load_pct", ctypes.c_int32),
                ("table_entry_bytes", ctypes.c_int32), ("search_mode", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32), ("lanczos_direct", ctypes.c_int32)]


ED_SEARCH_ONE_STAGE = 1
ED_SEARCH_TWO_STAGE = 2


class ed_tables_info_t(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_sublat", ctypes.c_int32), ("sub_bits", ctypes.c_int32),
                ("n_elems", ctypes.c_int32), ("n_perms", ctypes.c_int32), ("rep_entries", ctypes.c_int64),
                ("sym_entries", ctypes.c_int64), ("action_bytes", ctypes.c_int64),
                ("max_sym_len", ctypes.c_int32), ("n_top", ctypes.c_int32)]


class ed_basis_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("is_complex", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("n_up", ctypes.c_int32), ("n_sublat", ctypes.c_int32), ("sub_bits", ctypes.c_int32),
                ("n_elems", ctypes.c_int32), ("n_bonds", ctypes.c_int32), ("index_mode", ctypes.c_int32),
                ("limits_bits", ctypes.c_int32), ("n_keys", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("chunk_bits", ctypes.c_int32), ("table_entry_bytes", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double), ("search_mode", ctypes.c_int32),
                ("mean_candidates", ctypes.c_double), ("is_fermion", ctypes.c_int32)]


class ed_multi_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("n_sectors", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("n_up", ctypes.c_int32), ("n_sublat", ctypes.c_int32), ("n_elems", ctypes.c_int32),
                ("n_bonds", ctypes.c_int32), ("chunk_bits", ctypes.c_int32),
                ("table_entry_bytes", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("n_slots", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("lanes_per_row", ctypes.c_int32), ("chi_in_lds", ctypes.c_int32), ("chi_signs", ctypes.c_int32)]


ED_LANCZOS_NO_GRAPH = 1


def _struct_dict(s):
    return {name: getattr(s, name) for name, _ in s._fields_}


P = ctypes.c_void_p
I32, I64, U32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
PROTOTYPES = {
    "ed_version": (ctypes.c_char_p, []),
    "ed_last_error": (ctypes.c_char_p, []),
    "ed_validate": (ctypes.c_int, [P, P, P, I32]),
    "ed_tables_create": (ctypes.c_int, [P, P, P]),
    "ed_tables_free": (None, [P]),
    "ed_tables_info": (ctypes.c_int, [P, P]),
    "ed_tables_sublattice": (ctypes.c_int, [P, I32, U32, P, P, I32, P]),
    "ed_tables_find_rep": (ctypes.c_int, [P, I64, P, P, P, P]),
    "ed_build_basis": (ctypes.c_int, [P, P, P, I32, P, P, P]),
    "ed_free_basis": (None, [P]),
    "ed_basis_dim": (I64, [P]),
    "ed_basis_is_complex": (ctypes.c_int, [P]),
    "ed_basis_info": (ctypes.c_int, [P, P]),
    "ed_basis_copy_states": (ctypes.c_int, [P, P, P]),
    "ed_basis_copy_states_device": (ctypes.c_int, [P, P, P]),
    "ed_basis_copy_norms": (ctypes.c_int, [P, P, P]),
    "ed_apply_H": (ctypes.c_int, [P, P, P, P, P]),
    "ed_apply_H_stats": (ctypes.c_int, [P, P, P, P, P]),
    "ed_apply_H_timed": (ctypes.c_int, [P, P, P, P, P, I32, P, P, P]),
    "ed_probe_random_reads": (ctypes.c_int, [P, ctypes.c_int64, I32, I32, I32, P, P]),
    "ed_build_basis_fermions": (ctypes.c_int, [P, P, P, I32, P, P, P]),
    "ed_apply_H_fermions": (ctypes.c_int, [P, P, P, P, P, P]),
    "ed_lanczos_fermions": (ctypes.c_int, [P, P, P, P, I32, P, P, P, P, P]),
    "ed_lanczos": (ctypes.c_int, [P, P, P, I32, P, P, P, P, P]),
    "ed_apply_H_backward": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "ed_apply_H_backward_noalloc": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "ed_tridiag_eigh": (ctypes.c_int, [I32, P, P, P, P]),
    "ed_apply_H_xxz": (ctypes.c_int, [P, P, P, P, P, P]),
    "ed_lanczos_xxz": (ctypes.c_int, [P, P, P, P, I32, P, P, P, P, P]),
    "ed_build_multi": (ctypes.c_int, [P, P, I32, P, I32, P, P, P]),
    "ed_free_multi": (None, [P]),
    "ed_multi_info": (ctypes.c_int, [P, P]),
    "ed_multi_sector_dims": (ctypes.c_int, [P, P]),
    "ed_multi_copy_states": (ctypes.c_int, [P, P, P]),
    "ed_multi_copy_masks": (ctypes.c_int, [P, P, P]),
    "ed_apply_H_batched": (ctypes.c_int, [P, P, P, P, P]),
    "ed_apply_H_batched_stats": (ctypes.c_int, [P, P, P, P]),
    "ed_lanczos_batched": (ctypes.c_int, [P, P, P, I32, P, P, P, I32, P]),
}

_lib = None


def lib():
    """Load libed.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1804_05028_amd.build` "
                              "(the H.v path has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(PROTOTYPES)


def check(rc):
    if rc != ED_OK:
        msg = lib().ed_last_error().decode(errors="replace")
        raise EDError(rc, msg)
    return rc


def ptr(a):
    """Address of a numpy array, a torch tensor, or an int; None -> NULL."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    raise TypeError(type(a))


class ModelArrays:
    """Keeps the host arrays of one model alive while structs point at them."""

    def __init__(self, n_sites, bonds, n_sublat, perm, flip, chi=None):
        self.bonds = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
        self.perm = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
        self.flip = np.ascontiguousarray(np.asarray(flip, dtype=np.uint8))
        self.lat = ed_lattice_t(int(n_sites), int(self.bonds.shape[0]), self.bonds.ctypes.data, int(n_sublat))
        self.grp = ed_group_t(int(self.perm.shape[0]), self.perm.ctypes.data, self.flip.ctypes.data)
        self.chi = None
        self.irrep = None
        if chi is not None:
            chi = np.asarray(chi)
            if np.iscomplexobj(chi) or chi.ndim == 1:
                chi = np.stack([np.real(chi), np.imag(chi)], 1)
            self.chi = np.ascontiguousarray(chi, dtype=np.float64)
            self.irrep = ed_irrep_t(self.chi.ctypes.data)

    def refs(self):
        return (ctypes.byref(self.lat), ctypes.byref(self.grp),
                ctypes.byref(self.irrep) if self.irrep is not None else None)


# ---- thin wrappers with the ABI's names --------------------------------------

def ed_version():
    return lib().ed_version().decode()


def ed_last_error():
    return lib().ed_last_error().decode()


def ed_validate(arrays: ModelArrays, n_up):
    lat, grp, irr = arrays.refs()
    return check(lib().ed_validate(lat, grp, irr, int(n_up)))


def ed_tables_create(arrays: ModelArrays):
    lat, grp, _ = arrays.refs()
    h = ctypes.c_void_p()
    check(lib().ed_tables_create(lat, grp, ctypes.byref(h)))
    return h


def ed_tables_free(h):
    lib().ed_tables_free(h)


def ed_tables_info(h):
    info = ed_tables_info_t()
    check(lib().ed_tables_info(h, ctypes.byref(info)))
    return _struct_dict(info)


def ed_tables_sublattice(h, X, substate, cap=4096):
    rep = ctypes.c_uint32()
    n = ctypes.c_int32()
    out = np.zeros(cap, np.int32)
    check(lib().ed_tables_sublattice(h, int(X), int(substate), ctypes.byref(rep), out.ctypes.data, cap,
                                     ctypes.byref(n)))
    return int(rep.value), out[: min(n.value, cap)].tolist()


def ed_tables_find_rep(h, states):
    s = np.ascontiguousarray(states, dtype=np.uint64)
    r = np.empty_like(s)
    g = np.empty(s.shape[0], np.int32)
    c = np.empty(s.shape[0], np.int32)
    check(lib().ed_tables_find_rep(h, s.shape[0], s.ctypes.data, r.ctypes.data, g.ctypes.data, c.ctypes.data))
    return r, g, c


def _tuning(tuning):
    if tuning is None:
        return None
    return ed_tuning_t(int(tuning.get("limits_bits", 0)), int(tuning.get("index_mode", 0)),
                       int(tuning.get("block_threads", 0)), int(tuning.get("blocks_per_cu", 0)),
                       int(tuning.get("chunk_bits", 0)), int(tuning.get("hash_load_pct", 0)),
                       int(tuning.get("table_entry_bytes", 0)), int(tuning.get("search_mode", 0)),
                       int(tuning.get("lanes_per_row", 0)), int(tuning.get("lanczos_direct", 0)))


def ed_build_basis(arrays: ModelArrays, n_up, tuning=None, stream=None):
    lat, grp, irr = arrays.refs()
    h = ctypes.c_void_p()
    tn = _tuning(tuning)
    check(lib().ed_build_basis(lat, grp, irr, int(n_up), ctypes.byref(tn) if tn is not None else None,
                               stream, ctypes.byref(h)))
    return h


def ed_build_basis_fermions(arrays: ModelArrays, n_particles, tuning=None, stream=None):
    lat, grp, irr = arrays.refs()
    h = ctypes.c_void_p()
    tn = _tuning(tuning)
    check(lib().ed_build_basis_fermions(lat, grp, irr, int(n_particles),
                                        ctypes.byref(tn) if tn is not None else None, stream, ctypes.byref(h)))
    return h


def ed_free_basis(h):
    lib().ed_free_basis(h)


def ed_basis_dim(h):
    return int(lib().ed_basis_dim(h))


def ed_basis_is_complex(h):
    return bool(lib().ed_basis_is_complex(h))


def ed_basis_info(h):
    info = ed_basis_info_t()
    check(lib().ed_basis_info(h, ctypes.byref(info)))
    return _struct_dict(info)


def ed_basis_copy_states(h, out, stream=None):
    return check(lib().ed_basis_copy_states(h, ptr(out), stream))


def ed_basis_copy_states_device(h, out_dev, stream=None):
    return check(lib().ed_basis_copy_states_device(h, ptr(out_dev), stream))


def ed_basis_copy_norms(h, out, stream=None):
    return check(lib().ed_basis_copy_norms(h, ptr(out), stream))


def ed_apply_H(h, J, x_dev, y_dev, stream=None):
    J = np.ascontiguousarray(J, dtype=np.float64)
    return check(lib().ed_apply_H(h, J.ctypes.data, ptr(x_dev), ptr(y_dev), stream))


def ed_apply_H_xxz(h, Jxy, Jz, x_dev, y_dev, stream=None):
    Jxy = np.ascontiguousarray(Jxy, dtype=np.float64)
    Jz = None if Jz is None else np.ascontiguousarray(Jz, dtype=np.float64)
    return check(lib().ed_apply_H_xxz(h, Jxy.ctypes.data, None if Jz is None else Jz.ctypes.data, ptr(x_dev),
                                      ptr(y_dev), stream))


def ed_lanczos_xxz(h, Jxy, Jz, v0_dev, n_steps, psi0_dev=None, stream=None):
    Jxy = np.ascontiguousarray(Jxy, dtype=np.float64)
    Jz = None if Jz is None else np.ascontiguousarray(Jz, dtype=np.float64)
    alpha = np.zeros(max(n_steps, 1), np.float64)
    beta = np.zeros(max(n_steps, 1), np.float64)
    nd = ctypes.c_int32()
    check(lib().ed_lanczos_xxz(h, Jxy.ctypes.data, None if Jz is None else Jz.ctypes.data, ptr(v0_dev),
                               int(n_steps), alpha.ctypes.data, beta.ctypes.data, ctypes.byref(nd),
                               ptr(psi0_dev), stream))
    n = nd.value
    return alpha[:n].copy(), beta[:n].copy(), n


def ed_apply_H_timed(h, J, Jz, x_dev, y_dev, reps, stream=None):
    """reps launches of y = H x; returns the mean (scatter ms, H.v kernel ms)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    Jz = None if Jz is None else np.ascontiguousarray(Jz, dtype=np.float64)
    pack = ctypes.c_double()
    kern = ctypes.c_double()
    check(lib().ed_apply_H_timed(h, J.ctypes.data, None if Jz is None else Jz.ctypes.data, ptr(x_dev), ptr(y_dev),
                                 int(reps), ctypes.byref(pack), ctypes.byref(kern), stream))
    return pack.value, kern.value


def ed_probe_random_reads(buf_dev, nbytes, iters=512, reps=3, stream=None, slot_bytes=16):
    """Independent random slot reads (16 or 32 bytes each) per second over a
    device buffer."""
    rate = ctypes.c_double()
    check(lib().ed_probe_random_reads(ptr(buf_dev), int(nbytes), int(slot_bytes), int(iters), int(reps),
                                      ctypes.byref(rate), stream))
    return rate.value


def ed_apply_H_fermions(h, t, V, x_dev, y_dev, stream=None):
    t = np.ascontiguousarray(t, dtype=np.float64)
    V = None if V is None else np.ascontiguousarray(V, dtype=np.float64)
    return check(lib().ed_apply_H_fermions(h, t.ctypes.data, None if V is None else V.ctypes.data, ptr(x_dev),
                                           ptr(y_dev), stream))


def ed_lanczos_fermions(h, t, V, v0_dev, n_steps, psi0_dev=None, stream=None):
    t = np.ascontiguousarray(t, dtype=np.float64)
    V = None if V is None else np.ascontiguousarray(V, dtype=np.float64)
    a = np.zeros(max(n_steps, 1), np.float64)
    b = np.zeros(max(n_steps, 1), np.float64)
    n = ctypes.c_int32(0)
    check(lib().ed_lanczos_fermions(h, t.ctypes.data, None if V is None else V.ctypes.data, ptr(v0_dev),
                                    int(n_steps), a.ctypes.data, b.ctypes.data, ctypes.byref(n), ptr(psi0_dev),
                                    stream))
    return a[: n.value].copy(), b[: n.value].copy(), n.value


def ed_apply_H_stats(h, stream=None):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().ed_apply_H_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), stream))
    return int(a.value), int(b.value), int(c.value)


def ed_lanczos(h, J, v0_dev, n_steps, psi0_dev=None, stream=None):
    J = np.ascontiguousarray(J, dtype=np.float64)
    alpha = np.zeros(max(n_steps, 1), np.float64)
    beta = np.zeros(max(n_steps, 1), np.float64)
    nd = ctypes.c_int32()
    check(lib().ed_lanczos(h, J.ctypes.data, ptr(v0_dev), int(n_steps), alpha.ctypes.data, beta.ctypes.data,
                           ctypes.byref(nd), ptr(psi0_dev), stream))
    n = nd.value
    return alpha[:n].copy(), beta[:n].copy(), n


def ed_apply_H_backward(h, J, x_dev, gy_dev, gx_dev=None, want_gJ=True, stream=None):
    J = np.ascontiguousarray(J, dtype=np.float64)
    gJ = np.zeros(J.shape[0], np.float64) if want_gJ else None
    check(lib().ed_apply_H_backward(h, J.ctypes.data, ptr(x_dev), ptr(gy_dev), ptr(gx_dev),
                                    gJ.ctypes.data if gJ is not None else None, stream))
    return gJ


def ed_apply_H_backward_noalloc(h, J, x_dev, gy_dev, gx_dev=None, want_gJ=True, stream=None):
    """ed_apply_H_backward with its partial sums in the library's static device array."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    gJ = np.zeros(J.shape[0], np.float64) if want_gJ else None
    check(lib().ed_apply_H_backward_noalloc(h, J.ctypes.data, ptr(x_dev), ptr(gy_dev), ptr(gx_dev),
                                            gJ.ctypes.data if gJ is not None else None, stream))
    return gJ


def ed_tridiag_eigh(alpha, beta, want_vec=True):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    m = a.shape[0]
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64)[: max(m - 1, 0)])
    if b.shape[0] == 0:
        b = np.zeros(1)
    ev = np.empty(max(m, 1), np.float64)
    vec = np.empty(max(m, 1), np.float64) if want_vec else None
    check(lib().ed_tridiag_eigh(m, a.ctypes.data, b.ctypes.data, ev.ctypes.data,
                                vec.ctypes.data if vec is not None else None))
    return ev[:m], (vec[:m] if vec is not None else None)


# ---- batched sectors -----------------------------------------------------------

def ed_build_multi(arrays: ModelArrays, chis, n_up, tuning=None, stream=None):
    """chis: K character tables (complex [n_elems] or [n_elems][2] each)."""
    lat, grp, _ = arrays.refs()
    tabs = []
    for c in chis:
        c = np.asarray(c)
        if np.iscomplexobj(c) or c.ndim == 1:
            c = np.stack([np.real(c), np.imag(c)], 1)
        tabs.append(np.ascontiguousarray(c, dtype=np.float64))
    irreps = (ed_irrep_t * len(tabs))(*[ed_irrep_t(t.ctypes.data) for t in tabs])
    tn = _tuning(tuning)
    h = ctypes.c_void_p()
    check(lib().ed_build_multi(lat, grp, len(tabs), irreps, int(n_up), ctypes.byref(tn) if tn is not None else None,
                               stream, ctypes.byref(h)))
    return h


def ed_free_multi(h):
    lib().ed_free_multi(h)


def ed_multi_info(h):
    info = ed_multi_info_t()
    check(lib().ed_multi_info(h, ctypes.byref(info)))
    return _struct_dict(info)


def ed_multi_sector_dims(h, n_sectors):
    d = np.zeros(n_sectors, np.int64)
    check(lib().ed_multi_sector_dims(h, d.ctypes.data))
    return d


def ed_multi_copy_states(h, out, stream=None):
    return check(lib().ed_multi_copy_states(h, ptr(out), stream))


def ed_multi_copy_masks(h, out, stream=None):
    return check(lib().ed_multi_copy_masks(h, ptr(out), stream))


def ed_apply_H_batched(h, J, x_dev, y_dev, stream=None):
    J = np.ascontiguousarray(J, dtype=np.float64)
    return check(lib().ed_apply_H_batched(h, J.ctypes.data, ptr(x_dev), ptr(y_dev), stream))


def ed_apply_H_batched_stats(h, n_sectors, stream=None):
    t = np.zeros(n_sectors, np.int64)
    sh = ctypes.c_int64()
    check(lib().ed_apply_H_batched_stats(h, t.ctypes.data, ctypes.byref(sh), stream))
    return t, int(sh.value)


def ed_lanczos_batched(h, J, v0_dev, n_steps, n_sectors, flags=0, stream=None):
    J = np.ascontiguousarray(J, dtype=np.float64)
    alpha = np.zeros((n_sectors, max(n_steps, 1)), np.float64)
    beta = np.zeros((n_sectors, max(n_steps, 1)), np.float64)
    nd = np.zeros(n_sectors, np.int32)
    check(lib().ed_lanczos_batched(h, J.ctypes.data, ptr(v0_dev), int(n_steps), alpha.ctypes.data,
                                   beta.ctypes.data, nd.ctypes.data, int(flags), stream))
    return alpha[:, :n_steps], beta[:, :n_steps], nd
