"""Sector dimensions from the character formula.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The sector of a 1-D irrep chi is the image of the projector
P = |G|^-1 sum_g conj(chi(g)) g (sec. "Symmetry adapted basis states"), so its
dimension is |G|^-1 sum_g conj(chi(g)) Tr(g) over the fixed-Sz space.  For a
pure site permutation Tr(g) counts the configurations it fixes: unions of its
cycles holding n_up up spins, the x^n_up coefficient of prod_c (1 + x^len(c)).
With spin flip, a fixed configuration alternates along every cycle, so every
cycle must have even length, Sz must be 0, and Tr(g) = 2^#cycles.

For fermions in the occupation-number basis (sec. "Discussion") the group
acts with a Fermi sign, so Tr(g) sums that sign over the fixed
configurations.  A fixed configuration occupies whole cycles, and on an
occupied cycle of length L the element is a cyclic shift of L creation
operators, of sign (-1)^(L-1); Tr(g) is the x^n coefficient of
prod_c (1 + (-1)^(len(c)-1) x^len(c)).

Pins: brute-force counts of compatible representatives (orc.c) at small N,
and the sum over all momentum sectors equal to the binomial coefficient.
"""
from __future__ import annotations

import numpy as np


def cycle_lengths(perm_row):
    n = len(perm_row)
    seen = [False] * n
    out = []
    for i in range(n):
        if seen[i]:
            continue
        length = 0
        j = i
        while not seen[j]:
            seen[j] = True
            j = int(perm_row[j])
            length += 1
        out.append(length)
    return out


def trace(perm_row, flip, n_up):
    lens = cycle_lengths(perm_row)
    n = len(perm_row)
    if flip:
        if 2 * n_up != n or any(L % 2 for L in lens):
            return 0
        return 2 ** len(lens)
    poly = [1] + [0] * n_up
    for L in lens:
        new = poly[:]
        for k in range(n_up + 1 - L):
            new[k + L] += poly[k]
        poly = new
    return poly[n_up]


def sector_dimension(perm, flip, chi, n_up):
    """Exact integer dimension of the chi sector at fixed n_up."""
    perm = np.asarray(perm)
    chi = np.asarray(chi, dtype=np.complex128)
    total = 0j
    for g in range(perm.shape[0]):
        t = trace(perm[g], int(flip[g]), n_up)
        if t:
            total += np.conj(chi[g]) * t
    d = total / perm.shape[0]
    r = int(round(d.real))
    if abs(d.real - r) > 1e-6 * max(1, abs(r)) or abs(d.imag) > 1e-6 * max(1, abs(r)):
        raise ValueError(f"character formula not integral: {d}")
    return r


def fermion_trace(perm_row, n_part):
    poly = [1] + [0] * n_part
    for L in cycle_lengths(perm_row):
        sgn = -1 if L % 2 == 0 else 1
        new = poly[:]
        for k in range(n_part + 1 - L):
            new[k + L] += sgn * poly[k]
        poly = new
    return poly[n_part]


def fermion_sector_dimension(perm, chi, n_part):
    """Exact dimension of the chi sector of n_part fermions (no spin flip)."""
    perm = np.asarray(perm)
    chi = np.asarray(chi, dtype=np.complex128)
    total = 0j
    for g in range(perm.shape[0]):
        t = fermion_trace(perm[g], n_part)
        if t:
            total += np.conj(chi[g]) * t
    d = total / perm.shape[0]
    r = int(round(d.real))
    if abs(d.real - r) > 1e-6 * max(1, abs(r)) or abs(d.imag) > 1e-6 * max(1, abs(r)):
        raise ValueError(f"character formula not integral: {d}")
    return r
