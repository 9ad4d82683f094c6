"""Finite periodic clusters, their symmetry groups and 1-D characters.

This module only *describes models*: sites, bonds, the site permutations of
the space group (optionally times global spin flip), the characters of 1-D
irreducible representations, and a site numbering that puts each sublattice
on a contiguous block of sites.  It contains none of the exact-diagonalisation
arithmetic (no representatives, no basis, no matrix elements); both the
product library and the independent CPU oracle consume its output.

Conventions (Wietek & Laeuchli, sec. "Symmetry adapted basis states" and
sec. "Generic sublattice coding algorithm"):

* A group element is ``g = (t, R, f)``: the spin on site ``p`` moves to site
  ``R p + t`` (coordinates reduced modulo the cluster periods) and, if
  ``f == 1``, every spin is inverted afterwards.  ``perm[g, s]`` is the new
  site of the spin that sat on site ``s``.
* Site ``s`` is bit ``N-1-s`` of the integer code (site 0 is the most
  significant bit), up = 1.
* A sublattice decomposition is given by a superlattice ``M`` that contains
  the cluster's period lattice; the cosets of ``M`` are the sublattices.  Sites
  are renumbered so that sublattice ``X`` occupies sites
  ``[X*N/n_sub, (X+1)*N/n_sub)``, which puts sublattice 0 on the most
  significant bits, as the sublattice-coding definition requires.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

# --------------------------------------------------------------------------
# integer lattice helpers (2-D, coordinates in units of the Bravais vectors)
# --------------------------------------------------------------------------


def _det(a, b):
    return a[0] * b[1] - a[1] * b[0]


class _PeriodLattice:
    """The integer lattice spanned by two period vectors, with reduction."""

    def __init__(self, L1, L2):
        L1 = (int(L1[0]), int(L1[1]))
        L2 = (int(L2[0]), int(L2[1]))
        d = _det(L1, L2)
        if d == 0:
            raise ValueError("degenerate period vectors")
        if d < 0:
            L1, L2, d = L2, L1, -d
        self.L1, self.L2, self.det = L1, L2, d

    def coeffs(self, p):
        """Integer floor of the coordinates of p in the (L1, L2) basis."""
        a_num = p[0] * self.L2[1] - p[1] * self.L2[0]
        b_num = self.L1[0] * p[1] - self.L1[1] * p[0]
        return a_num // self.det, b_num // self.det, a_num % self.det == 0 and b_num % self.det == 0

    def reduce(self, p):
        a, b, _ = self.coeffs(p)
        return (p[0] - a * self.L1[0] - b * self.L2[0], p[1] - a * self.L1[1] - b * self.L2[1])

    def contains(self, p):
        return self.coeffs(p)[2]


def _mat_apply(R, p):
    return (R[0][0] * p[0] + R[0][1] * p[1], R[1][0] * p[0] + R[1][1] * p[1])


def _mat_mul(A, B):
    return tuple(tuple(sum(A[i][k] * B[k][j] for k in range(2)) for j in range(2)) for i in range(2))


IDENTITY = ((1, 0), (0, 1))

# point-group generators in lattice coordinates
SQUARE_R90 = ((0, -1), (1, 0))          # (x, y) -> (-y, x)
SQUARE_MX = ((1, 0), (0, -1))           # (x, y) -> (x, -y)
TRI_R60 = ((0, -1), (1, 1))             # a1 -> a2, a2 -> a2 - a1
TRI_M = ((1, 1), (0, -1))               # a1 -> a1, a2 -> a1 - a2
CHAIN_M = ((-1, 0), (0, 1))             # x -> -x


def generate_group(gens):
    """Closure of a set of 2x2 integer matrices, identity first, in BFS order."""
    elems = [IDENTITY]
    seen = {IDENTITY}
    frontier = [IDENTITY]
    while frontier:
        nxt = []
        for A in frontier:
            for G in gens:
                C = _mat_mul(G, A)
                if C not in seen:
                    seen.add(C)
                    elems.append(C)
                    nxt.append(C)
        frontier = nxt
    return elems


# --------------------------------------------------------------------------
# cluster
# --------------------------------------------------------------------------


@dataclass
class Cluster:
    """A periodic cluster with its bonds, symmetry group and site numbering.

    Arrays use the *final* site numbering (sublattice blocks contiguous).
    """

    name: str
    n_sites: int
    coords: list                 # final site s -> lattice coordinates
    bonds: np.ndarray            # [n_bonds, 2] int32
    bond_kind: np.ndarray        # [n_bonds] int32 (0 = nearest, 1 = next-nearest, ...)
    perm: np.ndarray             # [n_elems, n_sites] int32
    flip: np.ndarray             # [n_elems] uint8
    trans: np.ndarray            # [n_elems, 2] translation part t (lattice coords)
    rot_index: np.ndarray        # [n_elems] index into point_group
    point_group: list            # list of 2x2 integer matrices
    n_sublat: int
    periods: tuple
    superlattice: tuple | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_elems(self):
        return int(self.perm.shape[0])

    @property
    def n_bonds(self):
        return int(self.bonds.shape[0])


def build_cluster(name, L1, L2, bond_vectors, point_group_gens=(), spin_flip=False,
                  superlattice=None, bond_kinds=None, keep_point_group=None):
    """Build a cluster from its period vectors.

    bond_vectors: list of lattice vectors d; every site p gets a bond (p, p+d).
    point_group_gens: generator matrices; the generated group is intersected
      with the cluster's symmetries (R must map the period lattice onto itself).
    superlattice: (M1, M2) generating the sublattice superlattice, or None for a
      single sublattice.
    bond_kinds: kind label per bond vector (defaults to 0).
    keep_point_group: optional predicate on matrices to restrict the point group.
    """
    per = _PeriodLattice(L1, L2)
    n = per.det
    # enumerate canonical sites in a bounding box of the fundamental cell
    corners = [(0, 0), per.L1, per.L2, (per.L1[0] + per.L2[0], per.L1[1] + per.L2[1])]
    xs = [c[0] for c in corners]
    ys = [c[1] for c in corners]
    sites = set()
    for x in range(min(xs) - 1, max(xs) + 2):
        for y in range(min(ys) - 1, max(ys) + 2):
            sites.add(per.reduce((x, y)))
    sites = sorted(sites, key=lambda p: (p != (0, 0), p[1], p[0]))
    if len(sites) != n:
        raise RuntimeError("site enumeration failed")

    # sublattice labels and the final numbering
    if superlattice is None:
        labels = [(0, 0)] * n
        n_sub = 1
    else:
        sup = _PeriodLattice(*superlattice)
        if not (sup.contains(per.L1) and sup.contains(per.L2)):
            raise ValueError("superlattice must contain the cluster periods")
        labels = [sup.reduce(p) for p in sites]
        distinct = sorted(set(labels), key=lambda p: (p[1], p[0]))
        n_sub = len(distinct)
        rank = {lab: i for i, lab in enumerate(distinct)}
        labels = [rank[lab] for lab in labels]
    order = sorted(range(n), key=lambda i: (labels[i] if superlattice is not None else 0, i))
    coords = [sites[i] for i in order]
    index = {p: s for s, p in enumerate(coords)}

    # point group restricted to cluster symmetries
    pg_all = generate_group(list(point_group_gens)) if point_group_gens else [IDENTITY]
    pg = []
    for R in pg_all:
        if per.contains(_mat_apply(R, per.L1)) and per.contains(_mat_apply(R, per.L2)):
            if keep_point_group is None or keep_point_group(R):
                pg.append(R)

    # group elements: flip-major, then rotation, then translation
    translations = list(sites)          # translation by each site vector, identity first
    perms, flips, trans, rots = [], [], [], []
    for f in ([0, 1] if spin_flip else [0]):
        for ri, R in enumerate(pg):
            for t in translations:
                row = []
                for p in coords:
                    q = _mat_apply(R, p)
                    q = per.reduce((q[0] + t[0], q[1] + t[1]))
                    row.append(index[q])
                perms.append(row)
                flips.append(f)
                trans.append(t)
                rots.append(ri)
    perm = np.asarray(perms, dtype=np.int32)
    # bonds
    if bond_kinds is None:
        bond_kinds = [0] * len(bond_vectors)
    bl, bk = [], []
    for d, kind in zip(bond_vectors, bond_kinds):
        for s, p in enumerate(coords):
            q = per.reduce((p[0] + d[0], p[1] + d[1]))
            bl.append((s, index[q]))
            bk.append(kind)
    bonds = np.asarray(bl, dtype=np.int32).reshape(-1, 2)
    if np.any(bonds[:, 0] == bonds[:, 1]):
        raise ValueError("a bond vector closes on itself in this cluster")
    return Cluster(name=name, n_sites=n, coords=coords, bonds=bonds,
                   bond_kind=np.asarray(bk, dtype=np.int32), perm=perm,
                   flip=np.asarray(flips, dtype=np.uint8),
                   trans=np.asarray(trans, dtype=np.int64).reshape(-1, 2),
                   rot_index=np.asarray(rots, dtype=np.int32), point_group=pg,
                   n_sublat=n_sub, periods=(per.L1, per.L2),
                   superlattice=superlattice)


# --------------------------------------------------------------------------
# sublattice decompositions
# --------------------------------------------------------------------------


def _hnf(M1, M2):
    """Hermite normal form ((a, 0), (b, d)), a, d > 0, 0 <= b < a, of the
    lattice spanned by M1, M2 (the unique basis of that shape)."""
    # column operations on [M1 M2] (2x2 integer) to lower-triangular form
    (x1, y1), (x2, y2) = M1, M2
    # make the second coordinate of the first vector 0 by the Euclidean algorithm on y
    while y1 != 0:
        q = y2 // y1
        x2, y2 = x2 - q * x1, y2 - q * y1
        x1, y1, x2, y2 = x2, y2, x1, y1
    a, b, d = x1, x2, y2
    if a < 0:
        a = -a
    if d < 0:
        b, d = -b, -d
    b %= a
    return ((a, 0), (b, d))


def _in_lattice(p, a, b, d):
    if p[1] % d:
        return False
    v = p[1] // d
    return (p[0] - v * b) % a == 0


def stable_superlattices(L1, L2, point_group, n_sub):
    """Every superlattice M of index n_sub in Z^2 that contains the cluster's
    period lattice and is mapped onto itself by every point-group matrix.

    Its cosets are sublattices that every group element maps onto
    sublattices: a translation permutes the cosets, and R (p + M) = Rp + M
    when RM = M, which is the sublattice stability of sec. "Generic
    sublattice coding algorithm".  Returned as Hermite-normal-form bases
    ((a, 0), (b, d)) with a * d = n_sub, 0 <= b < a, in a fixed order.
    """
    out = []
    for a in range(1, n_sub + 1):
        if n_sub % a:
            continue
        d = n_sub // a
        for b in range(a):
            if not (_in_lattice(L1, a, b, d) and _in_lattice(L2, a, b, d)):
                continue
            ok = True
            for R in point_group:
                for v in ((a, 0), (b, d)):
                    if not _in_lattice(_mat_apply(R, v), a, b, d):
                        ok = False
            if ok:
                out.append(((a, 0), (b, d)))
    return out


def sublattice_decompositions(L1, L2, point_group, n_sites, max_sub_sites=16):
    """(n_sub, superlattice) for every sublattice-stable superlattice with at
    most max_sub_sites sites per sublattice, fewest sublattices first."""
    out = []
    for n_sub in range(1, n_sites + 1):
        if n_sites % n_sub or n_sites // n_sub > max_sub_sites:
            continue
        for M in stable_superlattices(L1, L2, point_group, n_sub):
            out.append((n_sub, M))
    return out


# --------------------------------------------------------------------------
# named lattice families
# --------------------------------------------------------------------------


def chain(n, superlattice_period=None, reflection=False, spin_flip=False, translations=True):
    """Periodic chain of n sites, nearest-neighbour bonds.

    superlattice_period=k puts sites with equal position mod k on one sublattice
    (the two- and three-sublattice chains of the worked examples use k=2, 3).
    """
    sup = None if superlattice_period is None else ((superlattice_period, 0), (0, 1))
    gens = [CHAIN_M] if reflection else []
    return build_cluster(f"chain{n}", (n, 0), (0, 1), [(1, 0)], gens, spin_flip, sup)


def square(L1, L2, j2=False, rotations=True, mirrors=False, spin_flip=False, superlattice=None, name=None,
           j3=False):
    """Square lattice cluster; nearest (kind 0), optional diagonal (kind 1) and
    optional third-neighbour (distance 2 along the axes, kind 2) bonds."""
    bv = [(1, 0), (0, 1)]
    kinds = [0, 0]
    if j2:
        bv += [(1, 1), (1, -1)]
        kinds += [1, 1]
    if j3:
        bv += [(2, 0), (0, 2)]
        kinds += [2, 2]
    gens = []
    if rotations:
        gens.append(SQUARE_R90)
    if mirrors:
        gens.append(SQUARE_MX)
    return build_cluster(name or f"square{L1}{L2}", L1, L2, bv, gens, spin_flip, superlattice, kinds)


def triangular(L1, L2, rotations=True, mirrors=True, spin_flip=False, superlattice=None, name=None):
    """Triangular lattice cluster (a1=(1,0), a2=(1/2, sqrt3/2)), nearest bonds."""
    gens = []
    if rotations:
        gens.append(TRI_R60)
    if mirrors:
        gens.append(TRI_M)
    return build_cluster(name or f"tri{L1}{L2}", L1, L2, [(1, 0), (0, 1), (-1, 1)], gens, spin_flip, superlattice)


# --------------------------------------------------------------------------
# 1-D characters
# --------------------------------------------------------------------------


def momenta(cluster):
    """Allowed momenta as integer vectors U with k.t = 2*pi*(U.t)/det.

    They are the characters of the translation group Z^2 / span(L1, L2).
    Returned in a deterministic order, Gamma first.
    """
    (L1, L2) = cluster.periods
    det = _det(L1, L2)
    # u = P^{-T} n  with P = [L1 L2] as columns; adj(P)^T n / det
    adjT = ((L2[1], -L1[1]), (-L2[0], L1[0]))
    out = set()
    for a in range(det):
        for b in range(det):
            U = (adjT[0][0] * a + adjT[0][1] * b, adjT[1][0] * a + adjT[1][1] * b)
            out.add((U[0] % det, U[1] % det))
            if len(out) == det:
                break
        if len(out) == det:
            break
    out = sorted(out)
    if len(out) != det:
        raise RuntimeError("momentum enumeration failed")
    return out, det


def _fixes_momentum(R, U, det, cluster):
    # R^T U == U modulo the dual lattice: check the character on translations
    RtU = (R[0][0] * U[0] + R[1][0] * U[1], R[0][1] * U[0] + R[1][1] * U[1])
    for t in cluster.coords:
        if ((RtU[0] - U[0]) * t[0] + (RtU[1] - U[1]) * t[1]) % det:
            return False
    return True


def point_group_chars_1d(point_group):
    """All 1-D characters of a finite matrix group (brute force over generators)."""
    elems = list(point_group)
    idx = {R: i for i, R in enumerate(elems)}
    n = len(elems)
    table = [[idx[_mat_mul(A, B)] for B in elems] for A in elems]
    # greedy generating set
    gens = []
    span = {0}

    def closure(gs):
        s = {0}
        frontier = [0]
        while frontier:
            nxt = []
            for a in frontier:
                for g in gs:
                    c = table[g][a]
                    if c not in s:
                        s.add(c)
                        nxt.append(c)
            frontier = nxt
        return s

    for i in range(n):
        if i not in span:
            gens.append(i)
            span = closure(gens)
    chars = []
    roots = [np.exp(2j * np.pi * k / n) for k in range(n)]
    for vals in itertools.product(range(n), repeat=len(gens)):
        chi = {0: 1.0 + 0j}
        frontier = [0]
        ok = True
        while frontier and ok:
            nxt = []
            for a in frontier:
                for g, v in zip(gens, vals):
                    c = table[g][a]
                    val = roots[v] * chi[a]
                    if c in chi:
                        if abs(chi[c] - val) > 1e-9:
                            ok = False
                            break
                    else:
                        chi[c] = val
                        nxt.append(c)
                if not ok:
                    break
            frontier = nxt
        if not ok:
            continue
        vec = np.array([chi[i] for i in range(n)])
        good = all(abs(vec[table[a][b]] - vec[a] * vec[b]) < 1e-9 for a in range(n) for b in range(n))
        if good and not any(np.allclose(vec, c) for c in chars):
            chars.append(vec)
    chars.sort(key=lambda c: (0 if np.allclose(c, 1) else 1, tuple(np.round(np.angle(c), 6))))
    return chars


def characters(cluster, momentum_index=0, pg_char=None, flip_parity=+1):
    """Character chi(g) of a 1-D irrep, as complex128 [n_elems].

    chi(t, R, f) = exp(i k.t) * pg_char[R] * flip_parity**f.  The momentum
    must be invariant under every point-group element present (the caller
    restricts the point group to the little group of k); this is not checked
    here -- the library and the oracle both validate the homomorphism.
    """
    U_list, det = momenta(cluster)
    U = U_list[momentum_index]
    phase = (cluster.trans[:, 0] * U[0] + cluster.trans[:, 1] * U[1]) % det
    chi = np.exp(2j * np.pi * phase / det)
    if pg_char is not None:
        chi = chi * np.asarray(pg_char)[cluster.rot_index]
    chi = chi * np.where(cluster.flip.astype(bool), float(flip_parity), 1.0)
    # snap exact values
    chi = np.where(np.abs(chi.real) < 1e-15, 1j * chi.imag, chi)
    chi = np.where(np.abs(chi.imag) < 1e-15, chi.real + 0j, chi)
    return chi.astype(np.complex128)


def conjugate_momentum_index(cluster, momentum_index):
    U_list, det = momenta(cluster)
    U = U_list[momentum_index]
    return U_list.index(((-U[0]) % det, (-U[1]) % det))


def chi_to_interleaved(chi):
    """complex128[n] -> float64[n, 2] (re, im), the layout the C-ABI takes."""
    chi = np.asarray(chi, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([chi.real, chi.imag], axis=1))


def bond_orbits(cluster):
    """Orbit id of every bond under the group (bonds as unordered pairs)."""
    key = {}
    for b, (p, q) in enumerate(cluster.bonds):
        key.setdefault((min(p, q), max(p, q)), []).append(b)
    orbit = -np.ones(cluster.n_bonds, dtype=np.int64)
    nxt = 0
    for b in range(cluster.n_bonds):
        if orbit[b] >= 0:
            continue
        p, q = cluster.bonds[b]
        members = set()
        for g in range(cluster.n_elems):
            a, c = cluster.perm[g, p], cluster.perm[g, q]
            members.update(key.get((min(a, c), max(a, c)), []))
        for m in members:
            orbit[m] = nxt
        nxt += 1
    return orbit


def orbit_mean(values, orbit):
    values = np.asarray(values, dtype=np.float64)
    out = np.empty_like(values)
    for o in np.unique(orbit):
        sel = orbit == o
        out[sel] = values[sel].mean()
    return out


def frac(x):
    return Fraction(x).limit_denominator(10 ** 6)
