"""Definition-level fermionic sector matrix, B^dagger H B, for small systems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the remark of sec. "Discussion" that the method applies to fermions
in the occupation-number basis, with a Fermi sign joining the
representative and its symmetry.  Nothing here uses a sign formula: states
are ordered products of creation operators, c+_{i1} ... c+_{ik} |0> with
i1 < ... < ik (orbital i <-> bit N-1-i, as for spins), and every operator is
applied by the canonical anticommutation rules, one creation or annihilation
operator at a time:
  * c+_p on a product with p absent inserts p and gives (-1)^(number of
    occupied orbitals before p); c_q removes q with (-1)^(number before q);
  * a site permutation g acts as c+_i -> c+_{g(i)}: the image of a state is
    the product of the permuted creation operators, applied right to left to
    the vacuum;
  * the Hamiltonian is sum_b [ -t_b (c+_p c_q + c+_q c_p) + V_b n_p n_q ].
The sector of a 1-D irrep chi holds the normalised columns
sum_g conj(chi(g)) U_g |sigma> of the orbit minima sigma whose column does
not vanish (sec. "Symmetry adapted basis states", with operators in place of
spin flips).

Pins (tests/test_oracle_fermions.py): free-fermion spectra (every sum of
n_part distinct single-particle energies, over all momentum sectors), the
two-site Hubbard closed form, sector dimensions adding up to the Fock
dimension, and agreement with the formula-level oracle in orc.c.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def fock_states(n, n_part):
    """All n-orbital occupations with n_part particles as sorted tuples of
    orbitals, ordered by their integer code (orbital i <-> bit n-1-i)."""
    occs = list(itertools.combinations(range(n), n_part))
    return sorted(occs, key=lambda o: code(n, o))


def code(n, occ):
    v = 0
    for i in occ:
        v |= 1 << (n - 1 - i)
    return v


def create(occ, p):
    """c+_p |occ> as (sign, occ') or None."""
    if p in occ:
        return None
    before = sum(1 for i in occ if i < p)
    return (-1) ** before, tuple(sorted(occ + (p,)))


def annihilate(occ, q):
    """c_q |occ> as (sign, occ') or None."""
    if q not in occ:
        return None
    before = sum(1 for i in occ if i < q)
    return (-1) ** before, tuple(i for i in occ if i != q)


def hop(occ, p, q):
    """c+_p c_q |occ> as (sign, occ') or None."""
    a = annihilate(occ, q)
    if a is None:
        return None
    b = create(a[1], p)
    if b is None:
        return None
    return a[0] * b[0], b[1]


def group_image(occ, perm_row):
    """U_g |occ>: the product of c+_{g(i)} over the occupied i (in ascending
    i), applied right to left to the vacuum; returns (sign, occ')."""
    sign, state = 1, ()
    for i in reversed(occ):
        r = create(state, int(perm_row[i]))
        sign *= r[0]
        state = r[1]
    return sign, state


def hamiltonian(n, states, bonds, t, V=None):
    index = {o: k for k, o in enumerate(states)}
    m = len(states)
    rows, cols, vals = [], [], []
    diag = np.zeros(m)
    for k, occ in enumerate(states):
        for b, (p, q) in enumerate(bonds):
            p, q = int(p), int(q)
            if V is not None and p in occ and q in occ:
                diag[k] += V[b]
            for a, c in ((p, q), (q, p)):
                r = hop(occ, a, c)
                if r is not None:
                    rows.append(index[r[1]])
                    cols.append(k)
                    vals.append(-t[b] * r[0])
    H = sp.coo_matrix((vals, (rows, cols)), shape=(m, m)).tocsr()
    return H + sp.diags(diag)


def symmetrised_columns(n, n_part, perm, chi):
    """(representatives ascending, B, Fock states) of the sector of chi."""
    states = fock_states(n, n_part)
    index = {o: k for k, o in enumerate(states)}
    ng = perm.shape[0]
    reps, cols = [], []
    for occ in states:
        imgs = [group_image(occ, perm[g]) for g in range(ng)]
        c0 = code(n, occ)
        if min(code(n, o) for _, o in imgs) != c0:
            continue                       # not the orbit minimum
        v = {}
        for g, (s, o) in enumerate(imgs):
            k = index[o]
            v[k] = v.get(k, 0) + np.conj(chi[g]) * s
        norm2 = sum(abs(c) ** 2 for c in v.values())
        if norm2 > 1e-9:
            reps.append(c0)
            cols.append({k: c / np.sqrt(norm2) for k, c in v.items()})
    data, ri, ci = [], [], []
    for c, col in enumerate(cols):
        for k, val in col.items():
            ri.append(k)
            ci.append(c)
            data.append(val)
    B = sp.coo_matrix((np.array(data, dtype=np.complex128), (ri, ci)), shape=(len(states), len(cols))).tocsc()
    return np.array(reps, dtype=np.uint64), B, states


def sector_matrix(n, n_part, perm, chi, bonds, t, V=None):
    """(representatives, dense B^dagger H B) of one fermionic sector."""
    reps, B, states = symmetrised_columns(n, n_part, np.asarray(perm), np.asarray(chi, dtype=np.complex128))
    H = hamiltonian(n, states, np.asarray(bonds), np.asarray(t, dtype=np.float64),
                    None if V is None else np.asarray(V, dtype=np.float64))
    return reps, (B.conj().T @ (H @ B)).toarray()


def full_spectrum(n, n_part, bonds, t, V=None):
    states = fock_states(n, n_part)
    H = hamiltonian(n, states, np.asarray(bonds), np.asarray(t, dtype=np.float64),
                    None if V is None else np.asarray(V, dtype=np.float64))
    return np.linalg.eigvalsh(H.toarray())
