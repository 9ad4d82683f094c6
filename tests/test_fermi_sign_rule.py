"""The chunked Fermi-sign rule of the HIP kernels, restated on the CPU.

A group element's Fermi sign on an occupation pattern is (-1) to the number
of occupied orbital pairs whose order it reverses (orc.c counts them pair by
pair).  The kernels count them from the sublattice-coding tables instead:
  * pairs in two different source blocks are reversed iff the two target
    blocks are, so they contribute occ(X1) occ(X2) for each reversed block
    pair;
  * pairs inside one table chunk come from a parity bit stored with the
    chunk's image;
  * pairs in two chunks of one block are counted from the chunk images: for
    the chunks in source order, each image bit pairs with every image bit of
    the earlier chunks that lies below it.
This file writes that rule out in Python, with block images taken from the
permutations themselves, and compares it with the oracle's pair count on
random configurations of the benchmark clusters at several chunk widths.
A mutant that drops the cross-chunk term must fail.
"""
import numpy as np
import pytest

from ed_inputs import workloads as wl
from oracle import bruteforce as bf


def image_bits(perm, n, m, X):
    """(target block, image bit of every substate bit j of block X)."""
    Y = perm[X * m] // m
    bits = []
    for j in range(m):
        o = X * m + (m - 1 - j)                     # substate bit j <-> orbital o
        bits.append(m - 1 - (perm[o] - Y * m))
    return Y, bits


def chunk_entry(bits, v, k, cb, width):
    img, par = 0, 0
    for a in range(width):
        if v >> a & 1:
            img |= 1 << bits[k * cb + a]
            for c in range(a):
                if (v >> c & 1) and bits[k * cb + a] < bits[k * cb + c]:
                    par ^= 1
    return img, par


def chunked_parity(perm, n, m, cb, s, cross=True):
    ns = n // m
    nc = -(-m // cb)
    par, seen = 0, 0
    for X in range(ns):
        sx = (s >> (n - (X + 1) * m)) & ((1 << m) - 1)
        Y, bits = image_bits(perm, n, m, X)
        earlier = 0
        for k in range(nc - 1, -1, -1):
            width = min(cb, m - k * cb)
            v = (sx >> (k * cb)) & ((1 << width) - 1)
            img, pbit = chunk_entry(bits, v, k, cb, width)
            px = earlier
            for sh in (1, 2, 4, 8):
                px ^= px << sh
            par ^= pbit
            if cross:
                par ^= bin(img & (px << 1)).count("1") & 1
            earlier |= img
        odd = bin(sx).count("1") & 1
        par ^= odd & (bin(seen >> (Y + 1)).count("1") & 1)
        seen |= odd << Y
    return par


CLUSTERS = [
    ("triangular36", lambda: wl.triangular_36(n_sub=4).cluster, [3, 5, 9]),
    ("square40", lambda: wl.square_40_j1j2(n_sub=4).cluster, [2, 5, 10]),
    ("square32", lambda: wl.square_32_disorder(n_sub=8).cluster, [2, 4]),
]


def _random_states(n, count, rng):
    out = []
    for _ in range(count):
        k = int(rng.integers(0, n + 1))
        occ = rng.choice(n, size=k, replace=False)
        out.append(int(sum(1 << (n - 1 - int(o)) for o in occ)))
    return out


@pytest.mark.parametrize("name,make,widths", CLUSTERS, ids=[c[0] for c in CLUSTERS])
def test_chunked_rule_matches_pair_count(name, make, widths):
    c = make()
    n, m = c.n_sites, c.n_sites // c.n_sublat
    rng = np.random.default_rng(7)
    gs = rng.choice(c.n_elems, size=min(24, c.n_elems), replace=False)
    states = _random_states(n, 40, rng)
    for g in gs:
        perm = [int(v) for v in c.perm[g]]
        for cb in widths:
            for s in states:
                assert chunked_parity(perm, n, m, cb, s) == bf.fsign(n, np.asarray(perm), s), (name, g, cb, s)


def test_dropping_the_cross_chunk_term_fails():
    c = wl.triangular_36(n_sub=4).cluster
    n, m = c.n_sites, c.n_sites // c.n_sublat
    rng = np.random.default_rng(8)
    states = _random_states(n, 40, rng)
    bad = 0
    for g in range(0, c.n_elems, 37):
        perm = [int(v) for v in c.perm[g]]
        for s in states:
            bad += chunked_parity(perm, n, m, 3, s, cross=False) != bf.fsign(n, np.asarray(perm), s)
    assert bad > 0
