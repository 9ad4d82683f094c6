"""Oracle pins for the XXZ and J1-J2-J3 extensions of the bond Hamiltonian.

Each bond carries an exchange J_b/2 (S+S- + S-S+) and an Ising term
Jz_b Sz Sz (non-branching two-site terms, sec. "Parallel matrix-vector
multiply").  Pins: the free-fermion XX ring (Jordan-Wigner), the Ising limit,
the XXZ dimer, and the formula-level sector matrices against the
definition-level projection B^dagger H B.
"""
import math

import numpy as np
import pytest

from ed_inputs import lattice as lat
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import definition as de
from oracle import dimension as dm

from test_oracle_mutants import xx_ring_ground_energy


def _sector_dense(m, n_up):
    st, stab = bf.basis(m, n_up)
    if len(st) == 0:
        return st, np.zeros((0, 0))
    H = np.stack([bf.apply(m, st, stab, e.astype(complex))[0] for e in np.eye(len(st))], 1)
    return st, H


@pytest.mark.parametrize("n", [6, 8, 10])
def test_xx_ring_free_fermions_definition_level(n):
    c = lat.chain(n)
    for n_up in (n // 2, n // 2 - 1, 1):
        e = de.full_spectrum(n, n_up, c.bonds, np.ones(n), np.zeros(n))[0]
        assert abs(e - xx_ring_ground_energy(n, n_up)) < 1e-10


@pytest.mark.parametrize("n,n_up", [(8, 4), (10, 5), (10, 4), (12, 6)])
def test_xx_ring_free_fermions_formula_level(n, n_up):
    c = lat.chain(n)
    best = math.inf
    for k in range(n):
        m = bf.Model(n, c.perm, c.flip, lat.characters(c, k), c.bonds, np.ones(n), np.zeros(n))
        st, H = _sector_dense(m, n_up)
        if len(st):
            assert np.abs(H - H.conj().T).max() < 1e-13
            best = min(best, np.linalg.eigvalsh(H)[0])
    assert abs(best - xx_ring_ground_energy(n, n_up)) < 1e-10


def test_ising_limit_and_xxz_dimer():
    # Ising ring: Jxy = 0, the Neel states give -N Jz / 4
    c = lat.chain(10)
    best = min(np.linalg.eigvalsh(_sector_dense(
        bf.Model(10, c.perm, c.flip, lat.characters(c, k), c.bonds, np.zeros(10), 2.0 * np.ones(10)), 5)[1])[0]
        for k in range(10))
    assert abs(best - (-10 * 2.0 / 4)) < 1e-12
    # dimer, Sz = 0: -Jz/4 +- Jxy/2
    m = bf.Model(2, np.array([[0, 1]]), np.zeros(1, np.uint8), np.ones(1), np.array([[0, 1]]),
                 np.array([0.7]), np.array([1.9]))
    _, H = _sector_dense(m, 1)
    ev = np.linalg.eigvalsh(H)
    assert np.allclose(ev, [-1.9 / 4 - 0.7 / 2, -1.9 / 4 + 0.7 / 2], atol=1e-14)


def _xxz_cases():
    out = []
    c8 = lat.chain(8)
    out.append(("ring8_k1", c8, lat.characters(c8, 1), 4, np.ones(8), 0.5 * np.ones(8)))
    ct = lat.triangular((2, 2), (-2, 4), spin_flip=True)
    out.append(("tri12_A1", ct, lat.characters(ct, 0), 6, np.ones(ct.n_bonds), 2.0 * np.ones(ct.n_bonds)))
    c = lat.square((4, 0), (0, 4), j2=True, j3=True, rotations=False, superlattice=wl.SQ_2X2, name="sq16j3")
    J = np.array([1.0, 0.5, 0.25])[c.bond_kind]
    out.append(("sq16_j1j2j3_k3", c, lat.characters(c, 3), 8, J, J))
    out.append(("sq16_j1j2j3_xxz", c, lat.characters(c, 0), 7, J, 1.5 * J))
    return out


@pytest.mark.parametrize("case", _xxz_cases(), ids=lambda c: c[0])
def test_formula_level_matches_definition_level(case):
    name, cl, chi, n_up, J, Jz = case
    reps, Md = de.sector_matrix(cl.n_sites, n_up, cl.perm, cl.flip, chi, cl.bonds, J, Jz)
    m = bf.Model(cl.n_sites, cl.perm, cl.flip, chi, cl.bonds, J, Jz)
    st, Mf = _sector_dense(m, n_up)
    assert len(st) == dm.sector_dimension(cl.perm, cl.flip, chi, n_up)
    assert np.array_equal(st, reps)
    assert np.abs(Mf - Md).max() < 1e-12
