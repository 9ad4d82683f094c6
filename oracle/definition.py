"""Definition-level sector matrix, B^dagger H B, for small clusters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows sec. "Symmetry adapted basis states" literally: the symmetry-adapted
state of a representative sigma is sum_g conj(chi(g)) g|sigma>, normalised
(Eq. for symmetry-adapted basis states); the representatives are the orbit
minima of the integer code (Eq. for the representative condition); the
Hamiltonian is the Heisenberg model J sum S_i.S_j of sec. "Benchmarks" with
one coupling per bond.  No matrix-element formula is used: the sector matrix
is the plain projection of the full fixed-Sz Hamiltonian onto the
orthonormal symmetry-adapted columns.  Everything is NumPy/SciPy; the group
action is re-implemented here independently of ``orc.c``.

Pins: closed-form energies (2-, 4-, 6-site rings), the full-space spectrum
(union over momentum sectors), Hermiticity by construction.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def fixed_sz_states(n, n_up):
    """All n-bit integers with n_up set bits, ascending (site s <-> bit n-1-s)."""
    out = []
    for ups in itertools.combinations(range(n), n_up):
        v = 0
        for s in ups:
            v |= 1 << (n - 1 - s)
        out.append(v)
    return np.array(sorted(out), dtype=np.uint64)


def act_all(states, perm_row, flip, n):
    """Image of every state under one group element (vectorised)."""
    out = np.zeros_like(states)
    one = np.uint64(1)
    for i in range(n):
        bit = (states >> np.uint64(n - 1 - i)) & one
        out |= bit << np.uint64(n - 1 - int(perm_row[i]))
    if flip:
        out ^= np.uint64((1 << n) - 1)
    return out


def full_hamiltonian(n, states, bonds, J, Jz=None):
    """H = sum_b [J_b/2 (S+_p S-_q + S-_p S+_q) + Jz_b Sz_p Sz_q] on the fixed-Sz
    basis, sparse CSR; Jz = J (None) is the Heisenberg model S_p.S_q."""
    Jz = J if Jz is None else Jz
    m = states.shape[0]
    index = {int(v): k for k, v in enumerate(states.tolist())}
    rows, cols, vals = [], [], []
    diag = np.zeros(m)
    one = np.uint64(1)
    for (p, q), j, jz in zip(bonds, J, Jz):
        bp = (states >> np.uint64(n - 1 - p)) & one
        bq = (states >> np.uint64(n - 1 - q)) & one
        same = bp == bq
        diag += np.where(same, 0.25 * jz, -0.25 * jz)
        flipped = states ^ (one << np.uint64(n - 1 - p)) ^ (one << np.uint64(n - 1 - q))
        for k in np.nonzero(~same)[0]:
            rows.append(index[int(flipped[k])])
            cols.append(k)
            vals.append(0.5 * j)
    H = sp.coo_matrix((vals, (rows, cols)), shape=(m, m)).tocsr()
    return H + sp.diags(diag)


def symmetrised_columns(n, n_up, perm, flip, chi):
    """Representatives (ascending) kept in the sector and the matrix B.

    Column k of B is the normalised sum_g conj(chi(g)) g|sigma_k>; a
    representative whose sum vanishes is not part of the sector.
    """
    states = fixed_sz_states(n, n_up)
    index = {int(v): k for k, v in enumerate(states.tolist())}
    ng = perm.shape[0]
    images = np.stack([act_all(states, perm[g], flip[g], n) for g in range(ng)])
    is_rep = images.min(axis=0) == states
    reps = states[is_rep]
    rep_pos = np.nonzero(is_rep)[0]
    cols, kept = [], []
    for r, pos in zip(reps.tolist(), rep_pos.tolist()):
        v = {}
        for g in range(ng):
            k = index[int(images[g, pos])]
            v[k] = v.get(k, 0) + np.conj(chi[g])
        norm2 = sum(abs(c) ** 2 for c in v.values())
        if norm2 > 1e-9:
            kept.append(r)
            cols.append({k: c / np.sqrt(norm2) for k, c in v.items()})
    data, ri, ci = [], [], []
    for c, col in enumerate(cols):
        for k, val in col.items():
            ri.append(k)
            ci.append(c)
            data.append(val)
    B = sp.coo_matrix((np.array(data, dtype=np.complex128), (ri, ci)),
                      shape=(states.shape[0], len(cols))).tocsc()
    return np.array(kept, dtype=np.uint64), B, states


def sector_matrix(n, n_up, perm, flip, chi, bonds, J, Jz=None):
    """(representatives, dense B^dagger H B) for one 1-D irrep sector."""
    reps, B, states = symmetrised_columns(n, n_up, np.asarray(perm), np.asarray(flip),
                                          np.asarray(chi, dtype=np.complex128))
    H = full_hamiltonian(n, states, np.asarray(bonds), np.asarray(J, dtype=np.float64),
                         None if Jz is None else np.asarray(Jz, dtype=np.float64))
    M = (B.conj().T @ (H @ B)).toarray()
    return reps, M


def full_spectrum(n, n_up, bonds, J, Jz=None):
    states = fixed_sz_states(n, n_up)
    H = full_hamiltonian(n, states, np.asarray(bonds), np.asarray(J, dtype=np.float64),
                         None if Jz is None else np.asarray(Jz, dtype=np.float64))
    return np.linalg.eigvalsh(H.toarray())


def full_ground_energy(n, n_up, bonds, J, k=1):
    """Lowest eigenvalue(s) of the full fixed-Sz Hamiltonian (sparse eigsh)."""
    import scipy.sparse.linalg as sla
    states = fixed_sz_states(n, n_up)
    H = full_hamiltonian(n, states, np.asarray(bonds), np.asarray(J, dtype=np.float64))
    if states.shape[0] < 500:
        return np.linalg.eigvalsh(H.toarray())[:k]
    vals = sla.eigsh(H, k=k, which="SA", tol=1e-13, maxiter=100000)[0]
    return np.sort(vals)
