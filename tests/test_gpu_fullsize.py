"""Full-size configurations, in the launch configuration the benchmark uses.

At these sizes the oracle cannot apply H in full, so the checks are the ones
it can make one item at a time, plus size-independent properties:
  * the dimension equals the character formula;
  * the whole basis and every stabiliser size match the oracle's brute-force
    enumeration bit for bit, through per-piece SHA-256 digests that
    tests/golden/make_basis_digests.py wrote from the oracle alone;
  * sampled rows are representatives with the right stabiliser size, and
    seeded random representatives found by brute force are in the basis;
  * 20,000 rows of y = H x per configuration (x a fixed hash of each
    representative's bits) match the oracle's row evaluation (1e-12): the
    first and last 1,000 rows, the 1,000 rows with the most terms, and a
    seeded random sample;
  * batched launches of the benchmarks' own sector groups (the eight Gamma
    irreps of the 36-site triangular full group, and sixteen of its momentum
    sectors), sector by sector against the oracle on sampled rows;
  * 200 Lanczos steps on the 40-site J1-J2 Gamma sector leave converged Ritz
    values, the lowest with residual below 1e-8; smaller sectors converge to
    the same lowest energy from two start vectors.
The 40-site J1-J2 basis is built once and shared by its tests.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import dimension as odim
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

N_EDGE = 1000      # first, last and heaviest rows
N_ROWS = 20000     # sampled rows per configuration, all strata together
N_REPS = 1000
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "basis_digests.json")


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _disorder():
    w = wl.square_32_disorder(n_sub=4)
    orbit = lat.bond_orbits(w.cluster)
    return wl.Workload(w.name, w.cluster, w.chi, w.n_up, lat.orbit_mean(w.J, orbit), w.description)


FULL = [
    ("triangular36", lambda: wl.triangular_36(n_sub=4), 10_524_036),
    ("square32_disorder", _disorder, 18_784_998),
    ("triangular36_k1", lambda: wl.triangular_36_momentum(1, n_sub=4), None),
    ("square40_j1j2", lambda: wl.square_40_j1j2(n_sub=4), 430_909_650),
    ("square40_j1j2j3", lambda: wl.square_40_j1j2j3(n_sub=4), 430_909_650),
]
SHARED = "square40_j1j2"


@pytest.fixture(scope="module")
def shared_basis():
    """The 40-site J1-J2 Gamma basis, built once for every test that needs it."""
    ed = _ed()
    w = wl.square_40_j1j2(n_sub=4)
    print(f"[fullsize] {SHARED}: building (shared)", flush=True)
    b = ed.Basis.from_workload(w)
    yield w, b
    b.close()
    torch.cuda.empty_cache()


def _term_counts(states, cluster):
    """Antiparallel bonds of every state (int16), computed on the device."""
    n = cluster.n_sites
    cnt = torch.zeros(states.shape[0], dtype=torch.int16, device=states.device)
    for p, q in np.asarray(cluster.bonds):
        cnt += (((states >> (n - 1 - int(p))) ^ (states >> (n - 1 - int(q)))) & 1).to(torch.int16)
    return cnt


def _stratified_rows(states, cluster, rng):
    """First and last N_EDGE rows, the N_EDGE rows with the most terms, and
    N_ROWS seeded random rows, without repeats, ascending."""
    D = states.shape[0]
    if D <= N_ROWS + 3 * N_EDGE:
        return np.arange(D)
    cnt = _term_counts(states, cluster)
    heavy = torch.topk(cnt, N_EDGE, sorted=False).indices.cpu().numpy()
    del cnt
    rand = rng.choice(D, size=N_ROWS, replace=False)
    return np.unique(np.concatenate([np.arange(N_EDGE), np.arange(D - N_EDGE, D), heavy, rand]))


def _check_rows(name, w, b, states=None):
    c = w.cluster
    D = b.dim
    assert D == odim.sector_dimension(c.perm, c.flip, w.chi, w.n_up)
    m = bf.Model.from_workload(w)
    st = b.states_device() if states is None else states
    assert bool((st[1:] > st[:-1]).all())
    rng = np.random.default_rng(vec.SEED_ROWS)
    rows = _stratified_rows(st, c, rng)
    rows_t = torch.as_tensor(rows).cuda()
    s_rows = st[rows_t].cpu().numpy().astype(np.uint64)
    # sampled rows are representatives, compatible, with the right |Stab|
    r, _, stab, comp = bf.rep_many(m, s_rows)
    assert np.array_equal(r, s_rows) and comp.all()
    norms = b.norms()
    assert np.array_equal(norms[rows].astype(np.int64), stab.astype(np.int64))
    del norms
    # brute-force representatives are present
    reps = bf.random_representatives(m, w.n_up, N_REPS, vec.SEED_ROWS + 1)
    reps_t = torch.as_tensor(reps.astype(np.int64)).cuda()
    pos = torch.searchsorted(st, reps_t)
    assert bool((pos < D).all())
    assert bool((st[pos.clamp(max=D - 1)] == reps_t).all())
    # sampled rows of H.v against the oracle's row evaluation
    print(f"[fullsize] {name}: H.v, {len(rows)} rows", flush=True)
    x = vec.hashed_amplitudes_torch(st, salt=1, complex_=b.is_complex)
    y = b.apply(w.J, x)
    x_rows = x[rows_t].cpu().numpy()
    assert np.array_equal(x_rows, vec.hashed_amplitudes(s_rows, 1, b.is_complex))
    y_rows = y[rows_t].cpu().numpy()
    del x, y
    ref, kept, _, rc = bf.rows_apply(m, s_rows, lambda s: vec.hashed_amplitudes(s, 1, b.is_complex))
    assert rc.all()
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(y_rows - ref).max()
    print(f"[fullsize] {name}: D={D} rows={len(rows)} terms={kept} max row error {err:.3e} (scale {scale:.3e})",
          flush=True)
    assert err <= 1e-12 * scale * 10
    assert np.linalg.norm(y_rows - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,make,dim", FULL, ids=[f[0] for f in FULL])
def test_fullsize_basis_and_sampled_rows(name, make, dim, shared_basis):
    if name == SHARED:
        w, b = shared_basis
        assert b.dim == dim
        _check_rows(name, w, b)
        return
    ed = _ed()
    w = make()
    print(f"[fullsize] {name}: building", flush=True)
    b = ed.Basis.from_workload(w)
    try:
        if dim is not None:
            assert b.dim == dim
        _check_rows(name, w, b)
    finally:
        b.close()
        torch.cuda.empty_cache()


def _golden():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as f:
        return json.load(f)["configs"]


DIGESTS = [("square32_disorder", _disorder), ("triangular36", lambda: wl.triangular_36(n_sub=4)),
           ("square40_j1j2", None)]


@pytest.mark.parametrize("name,make", DIGESTS, ids=[d[0] for d in DIGESTS])
def test_fullsize_basis_bit_exact(name, make, shared_basis):
    """Every representative and stabiliser size, piece by piece, against the
    SHA-256 digests of the oracle's enumeration."""
    cfg = _golden().get(name)
    if cfg is None or len(cfg["pieces"]) != cfg["n_pieces"]:
        pytest.skip(f"no complete oracle digest for {name} in tests/golden/basis_digests.json")
    if make is None:
        w, b = shared_basis
        own = False
    else:
        w, b, own = make(), None, True
        b = _ed().Basis.from_workload(w)
    try:
        assert b.dim == cfg["dim"]
        states = b.states()
        stab = b.norms().astype("<u2")
        assert states.dtype == np.uint64 and len(states) == cfg["dim"]
        bounds = [int(p["first_state"]) for p in cfg["pieces"]] + [None]
        cuts = [0] + [int(np.searchsorted(states, np.uint64(v))) for v in bounds[1:-1]] + [len(states)]
        bad = []
        for p, piece in enumerate(cfg["pieces"]):
            lo, hi = cuts[p], cuts[p + 1]
            hs = hashlib.sha256(np.ascontiguousarray(states[lo:hi], dtype="<u8").tobytes()).hexdigest()
            ht = hashlib.sha256(np.ascontiguousarray(stab[lo:hi]).tobytes()).hexdigest()
            if hi - lo != piece["count"] or hs != piece["sha256_states"] or ht != piece["sha256_stab"]:
                bad.append(p)
        print(f"[fullsize] {name}: {cfg['n_pieces']} pieces, {len(bad)} differ", flush=True)
        assert not bad, f"pieces {bad[:10]} differ from the oracle's enumeration"
    finally:
        if own:
            b.close()
            torch.cuda.empty_cache()


def test_fullsize_lanczos_200_steps(shared_basis):
    """200 FP64 Lanczos steps on the 40-site J1-J2 Gamma sector from the
    seeded start vector the benchmark uses."""
    w, b = shared_basis
    g = torch.Generator(device="cuda")
    g.manual_seed(vec.SEED_VECTOR)
    v0 = torch.randn(b.dim, dtype=torch.float64, device="cuda", generator=g)
    print(f"[fullsize] {SHARED}: 200 Lanczos steps", flush=True)
    res = b.lanczos(w.J, v0, 200)
    del v0
    assert res["n_done"] == 200
    w_all, resid = olz.ritz_residuals(res["alpha"], res["beta"])
    conv = olz.converged_ritz(res["alpha"], res["beta"], resid_tol=1e-8)
    print(f"[fullsize] {SHARED}: E0 = {res['eigenvalues'][0]:.12f} residual {resid[0]:.2e}, "
          f"{len(conv)} converged Ritz values", flush=True)
    assert len(conv) > 0
    assert resid[0] < 1e-8
    assert abs(conv[0] - res["eigenvalues"][0]) <= 1e-10 * abs(conv[0])
    assert np.allclose(w_all, res["eigenvalues"], rtol=0, atol=1e-10 * abs(conv[0]))


LANCZOS = [("triangular36", lambda: wl.triangular_36(n_sub=4)), ("square32_disorder", _disorder)]


@pytest.mark.parametrize("name,make", LANCZOS, ids=[f[0] for f in LANCZOS])
def test_fullsize_lanczos_two_start_vectors(name, make):
    ed = _ed()
    w = make()
    b = ed.Basis.from_workload(w)
    try:
        e0 = []
        for seed in (vec.SEED_VECTOR, 17):
            g = torch.Generator(device="cuda")
            g.manual_seed(seed)
            v0 = torch.randn(b.dim, dtype=torch.float64, device="cuda", generator=g)
            res = b.lanczos(w.J, v0, 200)
            conv = olz.converged_ritz(res["alpha"], res["beta"], resid_tol=1e-8)
            assert len(conv) > 0 and abs(conv[0] - res["eigenvalues"][0]) < 1e-10
            e0.append(res["eigenvalues"][0])
        print(f"[fullsize] {name}: E0 = {e0[0]:.12f} / {e0[1]:.12f} (per site {e0[0] / w.cluster.n_sites:.10f})",
              flush=True)
        assert abs(e0[0] - e0[1]) <= 1e-10 * abs(e0[0])
    finally:
        b.close()


# ---- batched launches at the benchmarks' own shapes ------------------------
BATCHED = [
    # the eight Gamma irreps of 36 T x C6v x flip: characters read from HBM, one
    # lane per row (the benchmark's instance), and two lanes per row
    ("triangular36_gamma", lambda: wl.triangular_36_gamma(n_sub=4), None, 1, 5000),
    ("triangular36_gamma_2lanes", lambda: wl.triangular_36_gamma(n_sub=4), {"lanes_per_row": 2}, 2, 2000),
    # the first sixteen momentum sectors, as the all-momentum benchmark groups them
    ("triangular36_allk16", lambda: wl.triangular_36_all_momenta(n_sub=4)[:16], None, 4, 1500),
    # eight Gamma irreps of 36 T x C6 x flip (no mirrors): complex characters
    # (sixth roots of unity), 55 KB of them, read from HBM as complex numbers
    ("triangular36_c6_gamma_complex", lambda: _tri36_c6_gamma()[:8], None, 1, 1500),
]


def _tri36_c6_gamma():
    c = lat.triangular((6, 0), (0, 6), spin_flip=True, mirrors=False, superlattice=wl.TRI_4, name="triangular36_c6")
    return wl.gamma_irreps(wl.Workload("triangular36_c6", c, lat.characters(c, 0), 18, np.ones(c.n_bonds)))


def _expected_chi_placement(ws):
    """(chi_in_lds, chi_signs) as the library chooses them: the table in LDS up
    to 32 KB; above, sign bits when every character is +-1 and K <= 8."""
    chis = np.array([w.chi for w in ws])
    in_lds = chis.size * 16 <= 32768
    signs = (not in_lds) and len(ws) <= 8 and bool(np.all(np.isin(chis.real, (1.0, -1.0)) & (chis.imag == 0.0)))
    return int(in_lds), int(signs)


@pytest.mark.parametrize("name,make,tuning,lanes,n_rows", BATCHED, ids=[c[0] for c in BATCHED])
def test_fullsize_batched_sampled_rows(name, make, tuning, lanes, n_rows):
    """Sector k's input is the state hash with salt k on the rows of sector k
    and a different hash elsewhere, which the kernel must ignore; sampled rows
    of every sector are compared with the oracle's row evaluation."""
    ed = _ed()
    ws = make()
    print(f"[fullsize] {name}: building {len(ws)} sectors", flush=True)
    mb = ed.MultiBasis.from_workloads(ws, tuning)
    try:
        info = mb.info()
        assert info["lanes_per_row"] == lanes and info["n_sublat"] == 4
        assert (info["chi_in_lds"], info["chi_signs"]) == _expected_chi_placement(ws)
        print(f"[fullsize] {name}: chi_in_lds={info['chi_in_lds']} chi_signs={info['chi_signs']}", flush=True)
        dims = mb.sector_dims()
        for k, w in enumerate(ws):
            c = w.cluster
            assert dims[k] == odim.sector_dimension(c.perm, c.flip, w.chi, w.n_up), k
        st = torch.as_tensor(mb.states().view(np.int64)).cuda()
        masks = torch.as_tensor(mb.masks().view(np.int64)).cuda()
        x = mb.empty()
        for k in range(mb.K):
            inside = ((masks >> k) & 1).bool()
            good = vec.hashed_amplitudes_torch(st, salt=k, complex_=True)
            junk = vec.hashed_amplitudes_torch(st, salt=1000 + k, complex_=True)
            x[:, k] = torch.where(inside, good, junk)
            del inside, good, junk
        del masks
        print(f"[fullsize] {name}: D={mb.dim} K={mb.K} lanes={info['lanes_per_row']} H.v", flush=True)
        y = mb.apply(ws[0].J, x)
        del x
        rng = np.random.default_rng(vec.SEED_ROWS)
        D = mb.dim
        rows = np.unique(np.concatenate([np.arange(200), np.arange(D - 200, D), rng.choice(D, n_rows, replace=False)]))
        rows_t = torch.as_tensor(rows).cuda()
        s_rows = st[rows_t].cpu().numpy().astype(np.uint64)
        y_rows = y[rows_t].cpu().numpy()
        del y, st
        m_rows = mb.masks()[rows]
        worst = 0.0
        for k, w in enumerate(ws):
            sel = ((m_rows >> np.uint64(k)) & np.uint64(1)).astype(bool)
            assert np.all(y_rows[~sel, k] == 0), k
            if not sel.any():
                continue
            m = bf.Model.from_workload(w)
            ref, _, _, rc = bf.rows_apply(m, s_rows[sel], lambda s, k=k: vec.hashed_amplitudes(s, k, True))
            assert rc.all(), k
            got = y_rows[sel, k]
            err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
            worst = max(worst, err)
            assert np.abs(got - ref).max() <= 10e-12 * max(np.abs(ref).max(), 1e-300), (name, k)
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), (name, k)
        print(f"[fullsize] {name}: {len(rows)} rows x {mb.K} sectors, worst relative row error {worst:.2e}",
              flush=True)
    finally:
        mb.close()
        torch.cuda.empty_cache()
