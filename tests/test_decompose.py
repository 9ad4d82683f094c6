"""Sublattice decompositions: enumeration of the stable superlattices and
their ranking by estimated representative-search cost (host only)."""
import numpy as np
import pytest

from ed_inputs import lattice as lat
from ed_inputs import workloads as wl
from paper_1804_05028_amd import _lib as L
from paper_1804_05028_amd import decompose as dc


def test_known_decompositions_are_found():
    c = lat.square((6, 2), (-2, 6), j2=True, spin_flip=True, name="sq40")
    found = {M for _, M in lat.sublattice_decompositions((6, 2), (-2, 6), c.point_group, 40, 12)}
    for sup in (wl.SQ_2X2, wl.SQ_5, wl.SQ_8, wl.SQ_10):
        assert lat._hnf(*sup) in found
    t = lat.triangular((6, 0), (0, 6), spin_flip=True)
    found = {M for _, M in lat.sublattice_decompositions((6, 0), (0, 6), t.point_group, 36, 12)}
    for sup in (wl.TRI_3, wl.TRI_4, wl.TRI_9):
        assert lat._hnf(*sup) in found
    # a two-sublattice split of the triangular lattice is never C6-stable
    assert lat.stable_superlattices((6, 0), (0, 6), t.point_group, 2) == []


def _all_superlattices(L1, L2, n):
    out = []
    for a in range(1, n + 1):
        if n % a:
            continue
        d = n // a
        for b in range(a):
            if lat._in_lattice(L1, a, b, d) and lat._in_lattice(L2, a, b, d):
                out.append(((a, 0), (b, d)))
    return out


@pytest.mark.parametrize("n", [2, 4, 8])
def test_enumeration_agrees_with_library_validation(n):
    """Every index-n superlattice containing the periods: the library accepts
    the decomposition exactly when the enumeration calls it stable."""
    base = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True, name="sq16")
    stable = set(lat.stable_superlattices((4, 0), (0, 4), base.point_group, n))
    cands = _all_superlattices((4, 0), (0, 4), n)
    assert stable <= set(cands) and len(cands) > len(stable) > 0
    for M in cands:
        c = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True, superlattice=M, name="sq16")
        arrays = L.ModelArrays(16, c.bonds, c.n_sublat, c.perm, c.flip, lat.characters(c, 0))
        if M in stable:
            L.ed_validate(arrays, 8)
        else:
            with pytest.raises(L.EDError) as e:
                L.ed_validate(arrays, 8)
            assert e.value.name == "ED_ERR_NOT_SUBLATTICE_STABLE"


def test_hnf_is_a_lattice_invariant():
    rng = np.random.default_rng(3)
    for M in [((2, 0), (1, 1)), ((5, 0), (3, 1)), ((4, 0), (2, 2))]:
        a, b = M
        for _ in range(20):
            U = rng.integers(-3, 4, size=(2, 2))
            while round(abs(np.linalg.det(U))) != 1:
                U = rng.integers(-3, 4, size=(2, 2))
            v1 = (U[0, 0] * a[0] + U[0, 1] * b[0], U[0, 0] * a[1] + U[0, 1] * b[1])
            v2 = (U[1, 0] * a[0] + U[1, 1] * b[0], U[1, 0] * a[1] + U[1, 1] * b[1])
            assert lat._hnf(v1, v2) == lat._hnf(*M)


def test_ranking_prefers_four_sublattices_on_the_large_clusters():
    c = lat.square((6, 2), (-2, 6), j2=True, spin_flip=True, name="sq40")
    decs = lat.sublattice_decompositions((6, 2), (-2, 6), c.point_group, 40, 12)
    r = dc.rank_decompositions(lambda M: lat.square((6, 2), (-2, 6), j2=True, spin_flip=True, superlattice=M),
                               decs, 20, samples=1000)
    assert r[0]["n_sub"] == 4 and r[0]["fits"]
    assert all(x["fits"] for x in r)
    t = lat.triangular((6, 0), (0, 6), spin_flip=True)
    decs = lat.sublattice_decompositions((6, 0), (0, 6), t.point_group, 36, 12)
    r = dc.rank_decompositions(lambda M: lat.triangular((6, 0), (0, 6), spin_flip=True, superlattice=M), decs, 18,
                               samples=1000)
    assert r[0]["n_sub"] == 4
    assert [x for x in r if x["n_sub"] == 3][0]["fits"] is False   # 12-site blocks overflow LDS
