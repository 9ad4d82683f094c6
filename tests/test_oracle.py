"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

Each pin is chosen so that a plausible mistake in the oracle fails it:
bit order or the direction of the group action (worked examples), a missing
conjugate or an inverted norm ratio (definition-level matrix with complex
characters), a dropped term (closed-form energies, full spectrum), a wrong
compatibility rule (character-formula dimensions).  test_oracle_mutants.py
plants such mistakes in a copy of the oracle and checks these pins catch them.
"""
import json
import math
import os

import numpy as np
import pytest

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import definition as de
from oracle import dimension as dm
from oracle import lanczos as lz

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _spins_to_int(s):
    s = s.replace(" ", "")
    v = 0
    for ch in s:
        v = 2 * v + (1 if ch == "u" else 0)
    return v


# ---------------------------------------------------------------- worked examples

@pytest.mark.parametrize("key", ["two_sublattice", "three_sublattice"])
def test_worked_example_representative(key):
    ex = _gold("worked_examples.json")[key]
    c = lat.chain(ex["n_sites"], superlattice_period=ex["sublattice_period"])
    m = bf.Model(c.n_sites, c.perm, c.flip, np.ones(c.n_elems))
    s = _spins_to_int(ex["state"])
    assert s == ex["state_int"]
    r, g = bf.rep(m, s)
    assert r == ex["representative"]["int"] == _spins_to_int(ex["representative"]["spins"])
    assert g == ex["representative"]["g"]
    if key == "three_sublattice":
        assert bf.act(m, 2, s) == ex["T2_image"]["int"]
        assert bf.act(m, 5, s) == ex["T5_image"]["int"]


def test_two_sublattice_images_order():
    # all six translates of the example state (two-sublattice labelling): the
    # representative is the unique minimum, reached only by T_1
    c = lat.chain(6, superlattice_period=2)
    m = bf.Model(6, c.perm, c.flip, np.ones(6))
    imgs = [bf.act(m, g, 50) for g in range(6)]
    assert min(imgs) == 14 and imgs.index(14) == 1 and imgs.count(14) == 1


# ---------------------------------------------------------------- closed forms

def _ring(n):
    c = lat.chain(n)
    return c


def _lowest_sector_energy(perm, flip, chi, bonds, J, n, n_up):
    m = bf.Model(n, perm, flip, chi, bonds, J)
    st, stab = bf.basis(m, n_up)
    if len(st) == 0:
        return None
    H = np.stack([bf.apply(m, st, stab, e)[0] for e in np.eye(len(st))], 1)
    return np.linalg.eigvalsh(H)[0]


def test_dimer_energy():
    e = _gold("closed_form_energies.json")["dimer"]
    perm = np.array([[0, 1]], np.int32)
    E = _lowest_sector_energy(perm, [0], [1.0], np.array([[0, 1]]), [1.0], 2, 1)
    assert abs(E - e) < 1e-14


@pytest.mark.parametrize("n,key", [(4, "ring4"), (6, "ring6")])
def test_ring_energies_all_sectors(n, key):
    e = _gold("closed_form_energies.json")[key]
    assert abs(e - {4: -2.0, 6: -1 - math.sqrt(13) / 2}[n]) < 1e-15
    c = _ring(n)
    best = min(_lowest_sector_energy(c.perm, c.flip, lat.characters(c, k), c.bonds, np.ones(n), n, n // 2)
               for k in range(n))
    assert abs(best - e) < 1e-12


def test_square16_ground_energy_two_ways():
    # oracle sector Lanczos (k=0 translations) against the full fixed-Sz
    # space solved by sparse eigsh with no symmetry at all
    w = wl.square_4x4()
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, 8)
    assert len(st) == 822
    v0 = vec.normal_vector(len(st))
    res = lz.lanczos(lambda v: bf.apply(m, st, stab, v)[0], v0, 200)
    e_sector = res["eigenvalues"][0]
    e_full = de.full_ground_energy(16, 8, w.cluster.bonds, w.J)[0]
    assert abs(e_sector - e_full) < 1e-10
    assert abs(e_sector / 16 - (-0.701780)) < 5e-7
    _, kept, dropped = bf.apply(m, st, stab, v0)
    assert kept == 14048 and dropped == 0


# ---------------------------------------------------------------- definition level

def _models_small():
    out = []
    # 8-site ring: all momenta (complex characters), with reflection-free group
    c = lat.chain(8)
    for k in range(8):
        out.append((f"ring8_k{k}", c, lat.characters(c, k), 4))
    # 10-site ring with flip, odd flip parity
    c = lat.chain(10, spin_flip=True)
    out.append(("ring10_flip_odd_k3", c, lat.characters(c, 3, flip_parity=-1), 5))
    # 12-site triangular, full group + flip, several 1-D irreps
    c = lat.triangular((2, 2), (-2, 4), spin_flip=True, superlattice=wl.TRI_3)
    chars = lat.point_group_chars_1d(c.point_group)
    out.append(("tri12_A1_even", c, lat.characters(c, 0, chars[0], +1), 6))
    out.append(("tri12_last_odd", c, lat.characters(c, 0, chars[-1], -1), 6))
    # 3x4 square... use 10-site tilted square with C4 and a complex C4 irrep
    c = lat.square((3, 1), (-1, 3), rotations=True)
    pc = lat.point_group_chars_1d(c.point_group)
    cplx = [p for p in pc if np.abs(p.imag).max() > 0.5][0]
    out.append(("sq10_C4_complex", c, lat.characters(c, 0, cplx), 5))
    out.append(("sq10_C4_complex_nup4", c, lat.characters(c, 0, cplx), 4))
    return out


@pytest.mark.parametrize("name,cl,chi,n_up", _models_small(), ids=[m[0] for m in _models_small()])
def test_formula_matches_definition(name, cl, chi, n_up):
    rng = np.random.default_rng(7)
    J = np.ones(cl.n_bonds) if "tri" in name or "ring" in name else np.ones(cl.n_bonds)
    reps_def, Mdef = de.sector_matrix(cl.n_sites, n_up, cl.perm, cl.flip, chi, cl.bonds, J)
    m = bf.Model(cl.n_sites, cl.perm, cl.flip, chi, cl.bonds, J)
    st, stab = bf.basis(m, n_up)
    assert np.array_equal(st, reps_def)
    assert len(st) == dm.sector_dimension(cl.perm, cl.flip, chi, n_up)
    if len(st) == 0:
        return
    cols = [bf.apply(m, st, stab, e.astype(np.complex128))[0] for e in np.eye(len(st))]
    Mf = np.stack(cols, 1)
    assert np.abs(Mf - Mdef).max() < 1e-12
    assert np.abs(Mf - Mf.conj().T).max() < 1e-13
    # gather rows (row_terms) reproduce the scatter product for a hashed x
    x = vec.hashed_amplitudes(st, salt=5, complex_=True)
    y, _, _ = bf.apply(m, st, stab, x)
    amp = lambda s: vec.hashed_amplitudes(s, salt=5, complex_=True)
    yr, _, _, comp = bf.rows_apply(m, st, amp)
    assert comp.all()
    assert np.abs(yr - y).max() < 1e-12
    _ = rng


def test_spectrum_union_equals_full_translations_and_flip():
    # abelian group (translations x flip) at Sz=0: the sector spectra together
    # are exactly the full fixed-Sz spectrum
    c = lat.triangular((2, 2), (-2, 4), rotations=False, mirrors=False, spin_flip=True)
    n, n_up = 12, 6
    J = np.ones(c.n_bonds)
    full = de.full_spectrum(n, n_up, c.bonds, J)
    parts = []
    total_dim = 0
    for k in range(12):
        for par in (+1, -1):
            chi = lat.characters(c, k, flip_parity=par)
            m = bf.Model(n, c.perm, c.flip, chi, c.bonds, J)
            st, stab = bf.basis(m, n_up)
            total_dim += len(st)
            if len(st):
                H = np.stack([bf.apply(m, st, stab, e.astype(np.complex128))[0] for e in np.eye(len(st))], 1)
                parts.append(np.linalg.eigvalsh(H))
    assert total_dim == math.comb(12, 6)
    union = np.sort(np.concatenate(parts))
    assert np.abs(union - full).max() < 1e-11


def test_su2_multiplets():
    # every level at Sz=-1 (n_up = N/2 - 1) also appears at Sz=0
    c = lat.chain(10)
    J = np.ones(10)
    lo = de.full_spectrum(10, 4, c.bonds, J)
    hi = de.full_spectrum(10, 5, c.bonds, J)
    for e in lo:
        assert np.abs(hi - e).min() < 1e-10


# ---------------------------------------------------------------- dimensions

@pytest.mark.parametrize("wlname", ["square16", "tri12", "sq20"])
def test_character_formula_vs_bruteforce(wlname):
    if wlname == "square16":
        w = wl.square_4x4(group="full")
    elif wlname == "tri12":
        w = wl.triangular_12()
    else:
        w = wl.square_20_j1j2()
    c = w.cluster
    m = bf.Model(c.n_sites, c.perm, c.flip, w.chi)
    assert bf.basis(m, w.n_up, count_only=True) == dm.sector_dimension(c.perm, c.flip, w.chi, w.n_up)


def test_momentum_dims_sum_to_binomial():
    c = lat.square((4, 0), (0, 4), rotations=False)
    dims = [dm.sector_dimension(c.perm, c.flip, lat.characters(c, k), 8) for k in range(16)]
    assert sum(dims) == math.comb(16, 8) == 12870
    assert dims[0] == 822


def test_paper_shaped_dimensions():
    # dimensions of the large sectors by the character formula (exact integers)
    assert dm.sector_dimension(*_pfc(wl.triangular_36())) == 10_524_036
    assert dm.sector_dimension(*_pfc(wl.square_40_j1j2())) == 430_909_650
    assert dm.sector_dimension(*_pfc(wl.square_32_disorder())) == 18_784_998


def _pfc(w):
    return w.cluster.perm, w.cluster.flip, w.chi, w.n_up


def test_hashed_vector_and_row_sampling_consistency():
    # sampled representatives are representatives, and row-sampled products at
    # the 20-site cluster agree with the full scatter product
    w = wl.square_20_j1j2()
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    rows = bf.random_representatives(m, w.n_up, 200, vec.SEED_ROWS)
    assert np.all(np.isin(rows, st))
    x = vec.hashed_amplitudes(st, salt=1)
    y, kept, dropped = bf.apply(m, st, stab, x)
    assert dropped == 0
    yr, _, _, _ = bf.rows_apply(m, rows, lambda s: vec.hashed_amplitudes(s, salt=1))
    idx = np.searchsorted(st, rows)
    assert np.abs(yr - y[idx]).max() < 1e-12


def test_dense_row_matrix_equals_scatter_columns():
    """dense_matrix (row form, one pass) equals the matrix whose columns are
    the scatter H.v of unit vectors, for real and complex sectors, spins and
    fermions."""
    c = lat.chain(8)
    for k in (0, 1, 4):
        m = bf.Model(8, c.perm, c.flip, lat.characters(c, k), c.bonds, np.ones(8))
        st, stab = bf.basis(m, 4)
        cols = np.stack([bf.apply(m, st, stab, e.astype(np.complex128))[0] for e in np.eye(len(st))], 1)
        assert np.abs(bf.dense_matrix(m, st) - cols).max() < 1e-13
        fm = bf.FermionModel(8, c.perm, lat.characters(c, k), c.bonds, np.ones(8), np.full(8, 0.6))
        fst, fstab = bf.fbasis(fm, 3)
        fcols = np.stack([bf.fapply(fm, fst, fstab, e.astype(np.complex128))[0] for e in np.eye(len(fst))], 1)
        assert np.abs(bf.fdense_matrix(fm, fst) - fcols).max() < 1e-13
