"""Named model configurations shaped like the paper's benchmark clusters.

The paper benchmarks the nearest-neighbour Heisenberg antiferromagnet on
triangular, square and kagome clusters with translations, a (sublattice
stable) point group and spin flip, each with a multi-sublattice decomposition
(sec. "Benchmarks", Table of benchmarks, Fig. of benchmark geometries).  Those
48/50-site sectors do not fit one GPU, so the workloads here are the same
families at 16-40 sites.  Each workload returns the cluster (with its
sublattice renumbering), the irrep characters, n_up and the couplings.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lattice as lat
from .vectors import couplings_by_kind, random_couplings


@dataclass
class Workload:
    name: str
    cluster: lat.Cluster
    chi: np.ndarray          # complex128 [n_elems]
    n_up: int
    J: np.ndarray            # float64 [n_bonds]
    description: str = ""

    @property
    def is_complex(self):
        return bool(np.any(np.abs(self.chi.imag) > 1e-14))


# sublattice superlattices (generators in lattice coordinates)
SQ_CHECKER = ((1, 1), (1, -1))        # 2 sublattices
SQ_2X2 = ((2, 0), (0, 2))             # 4 sublattices
SQ_5 = ((1, 2), (-2, 1))              # 5 sublattices, label (x + 2y) mod 5
SQ_8 = ((2, 2), (-2, 2))              # 8 sublattices
SQ_10 = ((3, 1), (-1, 3))             # 10 sublattices
TRI_3 = ((1, 1), (3, 0))              # 3 sublattices, label (a - b) mod 3
TRI_4 = ((2, 0), (0, 2))              # 4 sublattices
TRI_9 = ((3, 0), (0, 3))              # 9 sublattices


def _trivial(cl):
    return lat.characters(cl, 0)


def square_4x4(n_sub=4, group="translations", momentum_index=0):
    """4x4 periodic square, J=1, Sz=0; translation group, k=(0,0) by default."""
    sup = {1: None, 2: SQ_CHECKER, 4: SQ_2X2}[n_sub]
    if group == "translations":
        cl = lat.square((4, 0), (0, 4), rotations=False, superlattice=sup, name="square16")
    elif group == "full":
        cl = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True,
                        superlattice=sup, name="square16full")
    else:
        raise ValueError(group)
    chi = lat.characters(cl, momentum_index)
    return Workload("square16", cl, chi, 8, np.ones(cl.n_bonds),
                    "Heisenberg J=1, 4x4 periodic square, Sz=0, translations, k=(0,0)")


def triangular_36(n_sub=4):
    """36-site triangular, full space group (36 T x C6v) x spin flip, Gamma.A1.even."""
    sup = {3: TRI_3, 4: TRI_4, 9: TRI_9}[n_sub]
    cl = lat.triangular((6, 0), (0, 6), spin_flip=True, superlattice=sup, name="triangular36")
    return Workload("triangular36", cl, _trivial(cl), 18, np.ones(cl.n_bonds),
                    "Heisenberg J=1, 36-site triangular, Sz=0, 36 T x C6v x flip, Gamma.A1.even")


def square_40_j1j2(n_sub=5, j2=0.5):
    """40-site tilted square (L1=(6,2), L2=(-2,6)), J1-J2, 40 T x C4 x flip, Gamma."""
    sup = {2: SQ_CHECKER, 4: SQ_2X2, 5: SQ_5, 8: SQ_8, 10: SQ_10}[n_sub]
    cl = lat.square((6, 2), (-2, 6), j2=True, spin_flip=True, superlattice=sup, name="square40")
    J = couplings_by_kind(cl.bond_kind, [1.0, j2])
    return Workload("square40_j1j2", cl, _trivial(cl), 20, J,
                    f"J1-J2 (J2/J1={j2}), 40-site tilted square, Sz=0, 40 T x C4 x flip, Gamma.A.even")


def square_40_j1j2j3(n_sub=4, j2=0.5, j3=0.25):
    """40-site tilted square, J1-J2-J3 (the model of the paper's strong-scaling
    benchmark), 40 T x C4 x flip, Gamma.A.even, Sz=0."""
    sup = {2: SQ_CHECKER, 4: SQ_2X2, 5: SQ_5, 8: SQ_8, 10: SQ_10}[n_sub]
    cl = lat.square((6, 2), (-2, 6), j2=True, j3=True, spin_flip=True, superlattice=sup, name="square40j3")
    J = couplings_by_kind(cl.bond_kind, [1.0, j2, j3])
    return Workload("square40_j1j2j3", cl, _trivial(cl), 20, J,
                    f"J1-J2-J3 (J2={j2}, J3={j3}), 40-site tilted square, Sz=0, 40 T x C4 x flip, Gamma.A.even")


def square_20_j1j2j3(n_sub=5, j2=0.5, j3=0.25, spin_flip=True):
    """20-site tilted square (L1=(4,2), L2=(-2,4)), J1-J2-J3; small analogue of the 40-site model."""
    sup = {1: None, 2: SQ_CHECKER, 4: SQ_2X2, 5: ((2, 1), (-1, 2)), 10: ((1, 3), (-3, 1))}[n_sub]
    cl = lat.square((4, 2), (-2, 4), j2=True, j3=True, spin_flip=spin_flip, superlattice=sup, name="square20j3")
    J = couplings_by_kind(cl.bond_kind, [1.0, j2, j3])
    return Workload("square20_j1j2j3", cl, _trivial(cl), 10, J, "J1-J2-J3, 20-site tilted square")


def triangular_36_momentum(momentum_index, n_sub=4):
    """36-site triangular, translations only, momentum sector k (complex if k != -k)."""
    sup = {3: TRI_3, 4: TRI_4, 9: TRI_9}[n_sub]
    cl = lat.triangular((6, 0), (0, 6), rotations=False, mirrors=False, superlattice=sup,
                        name="triangular36T")
    return Workload(f"triangular36_k{momentum_index}", cl, lat.characters(cl, momentum_index), 18,
                    np.ones(cl.n_bonds), "Heisenberg J=1, 36-site triangular, translations, one momentum")


def square_32_disorder(n_sub=8, seed=1):
    """32-site tilted square (L1=(4,4), L2=(-4,4)), translations, k=0, J_b ~ U(0.8,1.2)."""
    sup = {2: SQ_CHECKER, 4: SQ_2X2, 8: SQ_8}[n_sub]
    cl = lat.square((4, 4), (-4, 4), rotations=False, superlattice=sup, name="square32")
    return Workload("square32_disorder", cl, _trivial(cl), 16, random_couplings(cl.n_bonds, seed),
                    "Heisenberg, 32-site tilted square, Sz=0, translations, k=0, J_b~U(0.8,1.2)")


def square_20_j1j2(n_sub=5, j2=0.5, spin_flip=True):
    """20-site tilted square (L1=(4,2), L2=(-2,4)), J1-J2, T x C4 (x flip); small C3 analogue."""
    sup = {1: None, 2: SQ_CHECKER, 4: SQ_2X2, 5: ((2, 1), (-1, 2)), 10: ((1, 3), (-3, 1))}[n_sub]
    cl = lat.square((4, 2), (-2, 4), j2=True, spin_flip=spin_flip, superlattice=sup, name="square20")
    J = couplings_by_kind(cl.bond_kind, [1.0, j2])
    return Workload("square20_j1j2", cl, _trivial(cl), 10, J, "J1-J2, 20-site tilted square")


def triangular_12(n_sub=3, spin_flip=True, momentum_index=0, rotations=True, mirrors=True):
    """12-site triangular (L1=(4,-2)... via (2,2),(-2,4)), small C2 analogue."""
    sup = {1: None, 3: TRI_3}[n_sub]
    cl = lat.triangular((2, 2), (-2, 4), rotations=rotations, mirrors=mirrors, spin_flip=spin_flip,
                        superlattice=sup, name="triangular12")
    return Workload("triangular12", cl, lat.characters(cl, momentum_index), 6, np.ones(cl.n_bonds),
                    "Heisenberg, 12-site triangular")


def triangular_36_all_momenta(n_sub=4, which="all"):
    """Momentum sectors of the 36-site triangular cluster with translations
    only: all 36, or the 20 inequivalent ones (Gamma, the three M points and
    one momentum of every +-k pair; for real H the sector -k is the complex
    conjugate of sector k)."""
    w0 = triangular_36_momentum(0, n_sub=n_sub)
    ks = range(w0.cluster.n_elems)
    if which == "inequivalent":
        ks = [k for k in ks if k <= lat.conjugate_momentum_index(w0.cluster, k)]
    return [triangular_36_momentum(k, n_sub=n_sub) for k in ks]


def gamma_irreps(w0):
    """The one-dimensional irreps at Gamma of a cluster's full group: every
    1-D point-group irrep, each with even and odd spin-flip parity."""
    c = w0.cluster
    return [Workload(f"{w0.name}_G{p}{'e' if f > 0 else 'o'}", c, lat.characters(c, 0, pc, f), w0.n_up, w0.J)
            for p, pc in enumerate(lat.point_group_chars_1d(c.point_group)) for f in (1, -1)]


def triangular_36_gamma(n_sub=4):
    """The eight one-dimensional irreps at Gamma of the 36-site triangular
    cluster's full group 36 T x C6v x spin flip: A1, A2, B1, B2 of C6v, each
    with even and odd spin-flip parity."""
    return gamma_irreps(triangular_36(n_sub=n_sub))


@dataclass
class FermionWorkload:
    """Fermions in the occupation-number basis: orbitals are the cluster's
    sites, n_part particles, H = sum_b [-t_b (c+_p c_q + h.c.) + V_b n_p n_q]."""
    name: str
    cluster: lat.Cluster
    chi: np.ndarray          # complex128 [n_elems]
    n_part: int
    t: np.ndarray            # float64 [n_bonds]
    V: np.ndarray            # float64 [n_bonds]
    description: str = ""

    @property
    def n_up(self):
        return self.n_part

    @property
    def is_complex(self):
        return bool(np.any(np.abs(self.chi.imag) > 1e-14))


def triangular_36_tV(n_sub=4, V=1.0, n_part=18, pg_irrep=0):
    """Spinless fermions on the 36-site triangular cluster, t = 1 and
    nearest-neighbour V, 36 T x C6 (216 elements; with the mirrors the
    fermionic tables, whose 4-byte entries carry sign parities, exceed the
    LDS), Gamma, 1-D point-group irrep pg_irrep (0 = trivial)."""
    sup = {3: TRI_3, 4: TRI_4, 9: TRI_9}[n_sub]
    cl = lat.triangular((6, 0), (0, 6), mirrors=False, superlattice=sup, name="triangular36f")
    pc = lat.point_group_chars_1d(cl.point_group)[pg_irrep]
    return FermionWorkload(f"triangular36_tV_G{pg_irrep}", cl, lat.characters(cl, 0, pc), n_part,
                           np.ones(cl.n_bonds), np.full(cl.n_bonds, float(V)),
                           f"spinless t-V (t=1, V={V}), 36-site triangular, {n_part} fermions, 36 T x C6, Gamma")


def hubbard_ring(L, t=1.0, U=4.0, n_part=None, momentum_index=0, n_sub=2):
    """L-site Hubbard ring as 2L orbitals (spin up 0..L-1, spin down
    L..2L-1), translations acting on both species; hopping bonds within each
    species and on-site bonds (i up, i down) with t = 0 and V = U.  The two
    species form the sublattice blocks (n_sub = 2), or each species splits
    into even and odd sites (n_sub = 4, L even)."""
    n = 2 * L
    if n_sub == 2:
        order = list(range(n))
    else:
        order = [i for i in range(L) if i % 2 == 0] + [i for i in range(L) if i % 2 == 1]
        order = order + [L + i for i in order]
    pos = {o: k for k, o in enumerate(order)}          # orbital -> renumbered site
    perm = np.zeros((L, n), np.int32)
    for s in range(L):
        for i in range(L):
            perm[s, pos[i]] = pos[(i + s) % L]
            perm[s, pos[L + i]] = pos[L + (i + s) % L]
    hop = [(i, (i + 1) % L) for i in range(L)]
    bonds = [(pos[p], pos[q]) for p, q in hop] + [(pos[L + p], pos[L + q]) for p, q in hop] + \
            [(pos[i], pos[L + i]) for i in range(L)]
    tt = np.array([t] * (2 * L) + [0.0] * L)
    V = np.array([0.0] * (2 * L) + [U] * L)
    chi = np.exp(2j * np.pi * momentum_index * np.arange(L) / L)
    cl = lat.Cluster(name=f"hubbard{L}", n_sites=n, coords=list(range(n)), bonds=np.array(bonds, np.int32),
                     bond_kind=np.zeros(len(bonds), np.int32), perm=perm, flip=np.zeros(L, np.uint8),
                     trans=np.stack([np.arange(L), np.zeros(L, int)], 1).astype(np.int32),
                     rot_index=np.zeros(L, np.int32), point_group=[((1, 0), (0, 1))], n_sublat=n_sub, periods=(L,))
    return FermionWorkload(f"hubbard{L}_k{momentum_index}", cl, chi, L if n_part is None else n_part, tt, V,
                           f"Hubbard ring L={L}, t={t}, U={U}")


WORKLOADS = {
    "square16": square_4x4,
    "triangular36": triangular_36,
    "square40_j1j2": square_40_j1j2,
    "square32_disorder": square_32_disorder,
}
