"""Pins of the fermionic oracle (CPU only).

The formula-level oracle (orc.c: Fermi sign of a group element as the parity
of its inversions on occupied orbitals, hop sign from the occupied orbitals
between the two sites) and the definition-level oracle (oracle/fermions.py:
creation and annihilation operators applied one at a time) are pinned by:
  * free fermions (V = 0): over all momentum sectors of an abelian
    translation group, the sector spectra together are exactly the sums of
    n_part distinct single-particle energies of the hopping matrix, and the
    sector dimensions add up to the Fock dimension;
  * the two-site Hubbard model at two electrons: {0, 0, 0, U,
    (U +- sqrt(U^2 + 16 t^2)) / 2};
  * agreement of the two levels, element by element, on sectors with real
    and complex characters, point groups and interactions.
Planted sign mistakes in a copy of orc.c must fail a pin.
"""
import math
import os
import subprocess

import numpy as np
import pytest

from ed_inputs import lattice as lat
from oracle import bruteforce as bf
from oracle import dimension as dm
from oracle import fermions as fe

SRC = os.path.join(os.path.dirname(bf.__file__), "orc.c")


def _formula_matrix(model, n_part):
    st, stab = bf.fbasis(model, n_part)
    if len(st) == 0:
        return st, np.zeros((0, 0))
    M = np.stack([bf.fapply(model, st, stab, e.astype(complex))[0] for e in np.eye(len(st))], 1)
    return st, M


def _single_particle(n, bonds, t):
    h = np.zeros((n, n))
    for (p, q), tb in zip(bonds, t):
        h[p, q] -= tb
        h[q, p] -= tb
    return np.linalg.eigvalsh(h)


def _free_sums(eps, n_part):
    return np.sort([sum(c) for c in __import__("itertools").combinations(eps, n_part)])


def hubbard_ring(L, t=1.0, U=4.0):
    """L-site Hubbard ring as 2L orbitals (spin up 0..L-1, spin down L..2L-1):
    translations act on both species; hopping bonds within each species and
    on-site interaction bonds (i up, i down) with t = 0, V = U."""
    perm = np.array([[(i + s) % L for i in range(L)] + [L + (i + s) % L for i in range(L)] for s in range(L)])
    hop = [(i, (i + 1) % L) for i in range(L)] if L > 2 else [(0, 1)]
    bonds = hop + [(L + p, L + q) for p, q in hop] + [(i, L + i) for i in range(L)]
    tt = [t] * (2 * len(hop)) + [0.0] * L
    V = [0.0] * (2 * len(hop)) + [U] * L
    return perm, np.array(bonds), np.array(tt), np.array(V)


def _free_cases():
    out = []
    c = lat.chain(8)
    out += [("ring8", c, 3), ("ring8", c, 4)]
    c = lat.triangular((2, 2), (-2, 4), rotations=False, mirrors=False, name="tri12T")
    out += [("tri12T", c, 4), ("tri12T", c, 5)]
    c = lat.square((4, 0), (0, 4), rotations=False, name="sq16T")
    out += [("sq16T", c, 3)]
    return out


def _free_pin(cluster, n_part, level):
    n = cluster.n_sites
    t = np.ones(cluster.n_bonds)
    evs, dim = [], 0
    for k in range(cluster.n_elems):
        chi = lat.characters(cluster, k)
        if level == "formula":
            m = bf.FermionModel(n, cluster.perm, chi, cluster.bonds, t)
            st, M = _formula_matrix(m, n_part)
        else:
            st, M = fe.sector_matrix(n, n_part, cluster.perm, chi, cluster.bonds, t)
        dim += len(st)
        if len(st):
            evs.extend(np.linalg.eigvalsh((M + M.conj().T) / 2))
    want = _free_sums(_single_particle(n, np.asarray(cluster.bonds), t), n_part)
    return dim == math.comb(n, n_part) and np.allclose(np.sort(evs), want, atol=1e-10)


# the dense definition level is kept to the clusters of at most 12 orbitals
FREE = [(lvl, c) for c in _free_cases() for lvl in ("formula", "definition")
        if lvl == "formula" or c[1].n_sites <= 12]


@pytest.mark.parametrize("level,case", FREE, ids=[f"{c[0]}_N{c[2]}-{lvl}" for lvl, c in FREE])
def test_free_fermion_spectra(level, case):
    name, cluster, n_part = case
    assert _free_pin(cluster, n_part, level)


def _hubbard2_pin(level, U=3.0, t=1.0):
    perm, bonds, tt, V = hubbard_ring(2, t, U)
    evs = []
    for chi in (np.ones(2), np.array([1.0, -1.0])):
        if level == "formula":
            st, M = _formula_matrix(bf.FermionModel(4, perm, chi, bonds, tt, V), 2)
        else:
            st, M = fe.sector_matrix(4, 2, perm, chi, bonds, tt, V)
        if len(st):
            evs.extend(np.linalg.eigvalsh((M + M.conj().T) / 2))
    r = math.sqrt(U * U + 16 * t * t)
    want = np.sort([0.0, 0.0, 0.0, U, (U - r) / 2, (U + r) / 2])
    return len(evs) == 6 and np.allclose(np.sort(evs), want, atol=1e-12)


@pytest.mark.parametrize("level", ["formula", "definition"])
def test_two_site_hubbard_closed_form(level):
    assert _hubbard2_pin(level)


def _level_cases():
    out = []
    c = lat.chain(8)
    out += [("ring8_k1_V", c.n_sites, c.perm, lat.characters(c, 1), c.bonds, 3, 0.7),
            ("ring8_k4_V", c.n_sites, c.perm, lat.characters(c, 4), c.bonds, 4, -0.3)]
    c = lat.triangular((2, 2), (-2, 4), name="tri12full")
    for p, pc in enumerate(lat.point_group_chars_1d(c.point_group)):
        out.append((f"tri12full_G{p}", c.n_sites, c.perm, lat.characters(c, 0, pc), c.bonds, 5, 0.5))
    perm, bonds, tt, V = hubbard_ring(4, 1.0, 2.5)
    for k in range(4):
        chi = np.exp(2j * np.pi * k * np.arange(4) / 4)
        out.append((f"hubbard4_k{k}", 8, perm, chi, bonds, 4, (tt, V)))
    return out


@pytest.mark.parametrize("case", _level_cases(), ids=[c[0] for c in _level_cases()])
def test_definition_level_equals_formula_level(case):
    name, n, perm, chi, bonds, n_part, inter = case
    if isinstance(inter, tuple):
        t, V = inter
    else:
        t, V = np.ones(len(bonds)), np.full(len(bonds), inter)
    reps, Md = fe.sector_matrix(n, n_part, perm, chi, bonds, t, V)
    st, Mf = _formula_matrix(bf.FermionModel(n, perm, chi, bonds, t, V), n_part)
    assert np.array_equal(st, reps)
    assert len(st) > 0
    assert np.abs(Md - Mf).max() < 1e-12
    assert np.abs(Mf - Mf.conj().T).max() < 1e-12


def test_fsign_examples():
    # a transposition of two occupied orbitals is odd; of one occupied, even
    perm = np.array([1, 0, 2, 3])
    assert bf.fsign(4, perm, 0b1100) == 1
    assert bf.fsign(4, perm, 0b1010) == 0
    # a 3-cycle is even on three particles
    assert bf.fsign(4, np.array([1, 2, 0, 3]), 0b1110) == 0
    # the cyclic shift of 4 orbitals on 4 particles is odd
    assert bf.fsign(4, np.array([1, 2, 3, 0]), 0b1111) == 1


MUTANTS = {
    "no_group_sign": ("int par = hop_parity(s, n, p, q) ^ orc_fsign(n, perm + (size_t)h * n, sp);",
                      "int par = hop_parity(s, n, p, q);"),
    "no_hop_sign": ("int par = hop_parity(s, n, p, q) ^ orc_fsign(n, perm + (size_t)h * n, sp);",
                    "int par = orc_fsign(n, perm + (size_t)h * n, sp);"),
    "hop_sign_inclusive": ("for (int i = lo + 1; i < hi; ++i) c += get_bit(s, n, i);",
                           "for (int i = lo; i <= hi; ++i) c += get_bit(s, n, i);"),
    "compat_without_sign": ("const double sg = orc_fsign(n, pg, s) ? -1.0 : 1.0;", "const double sg = 1.0;"),
}


def _formula_pins_pass():
    ok = _hubbard2_pin("formula")
    for name, cluster, n_part in _free_cases()[:4]:
        ok = ok and _free_pin(cluster, n_part, "formula")
    for case in _level_cases()[:4]:
        name, n, perm, chi, bonds, n_part, v = case
        t, V = np.ones(len(bonds)), np.full(len(bonds), v)
        reps, Md = fe.sector_matrix(n, n_part, perm, chi, bonds, t, V)
        st, Mf = _formula_matrix(bf.FermionModel(n, perm, chi, bonds, t, V), n_part)
        ok = ok and np.array_equal(st, reps) and Md.shape == Mf.shape and np.abs(Md - Mf).max() < 1e-12
    return bool(ok)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_fermion_mutant_is_caught(tmp_path, name, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new)
    csrc = os.path.join(str(tmp_path), f"orc_{name}.c")
    path = os.path.join(str(tmp_path), f"liborc_{name}.so")
    with open(csrc, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", path, csrc])
    saved = bf._lib
    try:
        bf._lib = None
        monkeypatch.setattr(bf, "_LIB", path)
        monkeypatch.setattr(bf, "build", lambda force=False: path)
        assert not _formula_pins_pass(), f"planted mistake '{name}' passed every pin"
    finally:
        bf._lib = saved


def _dim_cases():
    out = []
    c = lat.chain(8)
    out += [(c, lat.characters(c, k), n) for k in range(8) for n in (2, 3, 4)]
    c = lat.triangular((2, 2), (-2, 4), name="tri12full")
    out += [(c, lat.characters(c, 0, pc), n) for pc in lat.point_group_chars_1d(c.point_group) for n in (4, 5, 6)]
    c = lat.square((4, 0), (0, 4), name="sq16C4")
    U, det = lat.momenta(c)
    out += [(c, lat.characters(c, k, pc), 5) for k in (0, U.index((det // 2, det // 2)))
            for pc in lat.point_group_chars_1d(c.point_group)]
    return out


def test_fermion_character_formula_matches_enumeration():
    """Sector dimensions from the fermionic character formula equal the
    brute-force counts of surviving orbit minima, real and complex irreps."""
    for c, chi, n in _dim_cases():
        m = bf.FermionModel(c.n_sites, c.perm, chi, c.bonds, np.ones(c.n_bonds))
        st, _ = bf.fbasis(m, n)
        assert len(st) == dm.fermion_sector_dimension(c.perm, chi, n), (c.name, n)
