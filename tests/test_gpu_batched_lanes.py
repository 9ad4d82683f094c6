"""Batched H.v with 1, 2 and 4 lanes per row.

Every lane of a row runs the same searches and accumulates its own sectors
in the same term order, so the result must not depend on the number of lanes
per row, bit for bit; the one-lane result is checked against the oracle of
each sector.  K = 5 leaves one lane of four without sectors; K = 12 gives two
lanes 6 sectors each and four lanes 3 each.
"""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _sectors(K):
    c = wl.square_4x4().cluster
    return [wl.Workload(f"sq16_k{k}", c, lat.characters(c, k), 8, np.ones(c.n_bonds)) for k in range(K)]


def _x(dim, K, seed):
    re = vec.normal_vector(dim * K, seed=seed, normalise=False)
    im = vec.normal_vector(dim * K, seed=seed + 1000, normalise=False)
    return (re + 1j * im).reshape(dim, K)


@pytest.mark.parametrize("K", [5, 12, 16])
def test_lanes_per_row_bit_identical(K):
    ed = _ed()
    ws = _sectors(K)
    ys, alphas, betas, x, masks = {}, {}, {}, None, None
    for lanes in (1, 2, 4):
        print(f"[lanes] K={K} lanes={lanes}", flush=True)
        mb = ed.MultiBasis.from_workloads(ws, {"lanes_per_row": lanes})
        try:
            assert mb.info()["lanes_per_row"] == lanes
            if x is None:
                x = _x(mb.dim, mb.K, 31)
                masks = mb.masks()
            ys[lanes] = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
            res = mb.lanczos(ws[0].J, torch.as_tensor(x).cuda(), 20)
            alphas[lanes], betas[lanes] = res["alpha"], res["beta"]
        finally:
            mb.close()
    for lanes in (2, 4):
        assert np.array_equal(ys[lanes], ys[1]), lanes
        assert np.array_equal(alphas[lanes], alphas[1]), lanes
        assert np.array_equal(betas[lanes], betas[1]), lanes
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        ref, _, _ = bf.apply(m, st, stab, x[sel, k])
        assert np.linalg.norm(ys[1][sel, k] - ref) <= RTOL * np.linalg.norm(ref), k
        assert np.all(ys[1][~sel, k] == 0)


def test_automatic_lanes_per_row():
    ed = _ed()
    c = lat.triangular((2, 2), (-2, 4), rotations=False, mirrors=False, spin_flip=True, superlattice=wl.TRI_3,
                       name="triangular12Tf")
    tri24 = [wl.Workload("tri12", c, lat.characters(c, k, flip_parity=f), 6, np.ones(c.n_bonds))
             for k in range(12) for f in (1, -1)]
    for ws, want in ((_sectors(2), 1), (_sectors(3), 2), (_sectors(8), 2), (_sectors(9), 4), (_sectors(16), 4),
                     (tri24, 4)):
        mb = ed.MultiBasis.from_workloads(ws)
        try:
            assert mb.info()["lanes_per_row"] == want, len(ws)
        finally:
            mb.close()


def test_lane_count_raised_for_character_tables_in_hbm():
    """16 full-group sectors of the 4x4 lattice carry a 64 KB character table,
    which is read from HBM; a forced single lane is raised to 2, and the
    result equals that of the automatic choice bit for bit."""
    ed = _ed()
    c = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True, superlattice=wl.SQ_2X2,
                   name="square16full")
    U, det = lat.momenta(c)
    ks = [0, U.index((det // 2, det // 2))]
    pcs = lat.point_group_chars_1d(c.point_group)
    ws = [wl.Workload("sq16full", c, lat.characters(c, k, p, f), 8, np.ones(c.n_bonds))
          for k in ks for p in pcs for f in (1, -1)]
    ys = {}
    for lanes in (1, 0):
        mb = ed.MultiBasis.from_workloads(ws, {"lanes_per_row": lanes})
        try:
            assert mb.info()["lanes_per_row"] == (2 if lanes == 1 else 4)
            x = _x(mb.dim, mb.K, 41)
            ys[lanes] = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
        finally:
            mb.close()
    assert np.array_equal(ys[1], ys[0])


def _tri12_gamma():
    """The eight Gamma irreps of the 12-site triangular full group (12 T x C6v
    x flip, 288 elements) with four 3-site sublattices: 36 KB of characters,
    read from HBM, as in the 36-site triangular Gamma benchmark."""
    c = lat.triangular((2, 2), (-2, 4), spin_flip=True, superlattice=wl.TRI_4, name="triangular12_4sub")
    return wl.gamma_irreps(wl.Workload("tri12", c, lat.characters(c, 0), 6, np.ones(c.n_bonds)))


# Cases that run the compile-time batched instances of the benchmarks: four
# sublattices with two action-table chunks (NSC 34, the all-momentum launches)
# and three chunks (NSC 35, the Gamma-irrep launch), 2-byte entries, the
# two-stage search, 2 and 4 lanes per row.
BENCH_INSTANCES = [
    ("sq16_allk_nsc34", lambda: _sectors(16), {"chunk_bits": 2}, 2, True),
    ("sq16_k4_nsc34", lambda: _sectors(4), {"chunk_bits": 2}, 2, True),
    ("tri12_gamma_nsc35", _tri12_gamma, {"chunk_bits": 1}, 3, False),
]


@pytest.mark.parametrize("lanes", [2, 4])
@pytest.mark.parametrize("name,make,tune,chunks,chi_lds", BENCH_INSTANCES, ids=[c[0] for c in BENCH_INSTANCES])
def test_benchmark_instances_match_oracle(name, make, tune, chunks, chi_lds, lanes):
    ed = _ed()
    ws = make()
    tuning = dict(tune, table_entry_bytes=2, search_mode=2, lanes_per_row=lanes)
    print(f"[lanes] {name} lanes={lanes}", flush=True)
    mb = ed.MultiBasis.from_workloads(ws, tuning)
    try:
        info = mb.info()
        assert info["n_sublat"] == 4 and info["table_entry_bytes"] == 2
        assert info["lanes_per_row"] == lanes and info["chi_in_lds"] == int(chi_lds)
        # the 8 Gamma irreps have characters +-1: above 32 KB, one sign bit each
        assert info["chi_signs"] == int(not chi_lds)
        m_bits = ws[0].cluster.n_sites // 4
        assert -(-m_bits // info["chunk_bits"]) == chunks
        x = _x(mb.dim, mb.K, 61)
        y = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
        masks = mb.masks()
    finally:
        mb.close()
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        assert np.array_equal(np.nonzero(sel)[0].size, len(st)), k
        if len(st) == 0:
            assert np.all(y[:, k] == 0)
            continue
        ref, _, _ = bf.apply(m, st, stab, x[sel, k])
        assert np.linalg.norm(y[sel, k] - ref) <= RTOL * np.linalg.norm(ref), (name, k)
        assert np.abs(y[sel, k] - ref).max() <= 10 * RTOL * max(np.abs(ref).max(), 1e-300), (name, k)
        assert np.all(y[~sel, k] == 0)



MANY = [("chain36_k36", 36, 3, 4), ("chain40_k40", 40, 3, 4)]


@pytest.mark.parametrize("name,n,n_up,period", MANY, ids=[m[0] for m in MANY])
def test_more_than_32_sectors(name, n, n_up, period):
    """All momenta of a 36- and a 40-site ring in one batched basis: sector
    masks beyond bit 31 come from the per-row mask array; every sector of
    H.v against the oracle, term counts against the single-sector path, and
    the batched Lanczos (one graph-replayed call for all sectors) against the
    dense spectrum of each sector."""
    ed = _ed()
    c = lat.chain(n, superlattice_period=period)
    ws = [wl.Workload(f"{name}_{k}", c, lat.characters(c, k), n_up, np.ones(c.n_bonds)) for k in range(n)]
    mb = ed.MultiBasis.from_workloads(ws)
    try:
        info = mb.info()
        assert info["n_sectors"] == n and info["lanes_per_row"] == 4 and info["chi_in_lds"] == 1
        x = _x(mb.dim, mb.K, 71)
        y = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
        masks = mb.masks()
        terms, _ = mb.stats()
        res = mb.lanczos(ws[0].J, torch.as_tensor(x).cuda(), 160)
    finally:
        mb.close()
    total = 0
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        assert sel.sum() == len(st), k
        total += len(st)
        assert np.all(y[~sel, k] == 0)
        if len(st) == 0:
            assert res["n_done"][k] == 0
            continue
        ref, kept, _ = bf.apply(m, st, stab, x[sel, k])
        assert np.linalg.norm(y[sel, k] - ref) <= RTOL * np.linalg.norm(ref), k
        assert terms[k] == len(st) + kept, k
        H = bf.dense_matrix(m, st)
        e0 = np.linalg.eigvalsh((H + H.conj().T) / 2)[0]
        assert abs(res["eigenvalues"][k][0] - e0) <= 1e-10 * max(1.0, abs(e0)), k
    from math import comb
    assert total == comb(n, n_up)
