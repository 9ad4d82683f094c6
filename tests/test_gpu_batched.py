"""Batched sectors: one launch for several 1-D irreps over shared representatives.

Each sector's slice of the batched result is compared with the CPU oracle of
that sector alone (its own brute-force basis and scatter-form H.v), and with
the single-sector HIP path: sector dimensions exactly (also against the
character formula), sector bases bit-exactly, H.v within 1e-12, term counts
exactly, and Lanczos coefficients and eigenvalues.  Entries of the input that
lie outside a sector hold random values, which the kernel must ignore.
"""
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

RTOL = 1e-12


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _cases():
    out = []
    c = wl.square_4x4().cluster
    out.append(("square16_allk", [wl.Workload(f"sq16_k{k}", c, lat.characters(c, k), 8, np.ones(c.n_bonds))
                                  for k in range(16)]))
    c = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True, superlattice=wl.SQ_2X2,
                   name="square16full")
    U, det = lat.momenta(c)
    ks = [0, U.index((det // 2, det // 2))]
    pcs = lat.point_group_chars_1d(c.point_group)
    out.append(("square16_full_GM", [wl.Workload("sq16full", c, lat.characters(c, k, p, f), 8, np.ones(c.n_bonds))
                                     for k in ks for p in pcs for f in (1, -1)]))
    c = lat.triangular((2, 2), (-2, 4), rotations=False, mirrors=False, spin_flip=True, superlattice=wl.TRI_3,
                       name="triangular12Tf")
    out.append(("tri12_T_flip", [wl.Workload("tri12", c, lat.characters(c, k, flip_parity=f), 6, np.ones(c.n_bonds))
                                 for k in range(12) for f in (1, -1)]))
    c = lat.chain(4, superlattice_period=2, reflection=False, spin_flip=True)
    out.append(("ring4_flip_empty", [wl.Workload("ring4", c, lat.characters(c, k, flip_parity=f), 2, np.ones(4))
                                     for k in range(4) for f in (1, -1)]))
    return out


CASES = _cases()
IDS = [n for n, _ in CASES]


@pytest.fixture(scope="module")
def built():
    ed = _ed()
    cache = {}
    for name, ws in CASES:
        print(f"[build] {name} K={len(ws)}", flush=True)
        cache[name] = ed.MultiBasis.from_workloads(ws)
    yield cache
    for mb in cache.values():
        mb.close()


def _oracle_sector(w):
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    return m, st, stab


@pytest.mark.parametrize("name", IDS)
def test_masks_dims_and_sector_bases(built, name):
    ws = dict(CASES)[name]
    mb = built[name]
    states = mb.states()
    masks = mb.masks()
    dims = mb.sector_dims()
    assert np.all(masks >> np.uint64(len(ws)) == 0)
    for k, w in enumerate(ws):
        c = w.cluster
        assert dims[k] == odim.sector_dimension(c.perm, c.flip, w.chi, w.n_up)
        _, st, _ = _oracle_sector(w)
        sel = states[((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)]
        assert np.array_equal(sel, st), (name, k)
    # the shared rows are exactly the trivial-irrep representatives
    c = ws[0].cluster
    triv = bf.Model(c.n_sites, c.perm, c.flip, np.ones(c.n_elems))
    st0, _ = bf.basis(triv, ws[0].n_up)
    assert np.array_equal(states, st0)


def _garbage_x(mb, seed):
    """Random complex [dim][K] with random values also outside every sector."""
    re = vec.normal_vector(mb.dim * mb.K, seed=seed, normalise=False)
    im = vec.normal_vector(mb.dim * mb.K, seed=seed + 1000, normalise=False)
    return (re + 1j * im).reshape(mb.dim, mb.K)


@pytest.mark.parametrize("name", IDS)
def test_batched_apply_matches_oracle_per_sector(built, name):
    ws = dict(CASES)[name]
    mb = built[name]
    x = _garbage_x(mb, 21)
    y = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
    masks = mb.masks()
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        assert np.all(y[~sel, k] == 0)
        m, st, stab = _oracle_sector(w)
        ref, _, _ = bf.apply(m, st, stab, x[sel, k])
        got = y[sel, k]
        if len(st) == 0:
            continue
        scale = np.abs(ref).max()
        assert np.linalg.norm(got - ref) <= RTOL * max(np.linalg.norm(ref), 1e-300), (name, k)
        assert np.abs(got - ref).max() <= RTOL * max(scale, 1e-300) * 10, (name, k)


@pytest.mark.parametrize("name", IDS)
def test_batched_matches_single_sector_path(built, name):
    ed = _ed()
    ws = dict(CASES)[name]
    mb = built[name]
    x = _garbage_x(mb, 33)
    y = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
    terms, shared = mb.stats()
    masks = mb.masks()
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        b = ed.Basis.from_workload(w)
        try:
            if b.dim == 0:
                assert terms[k] == 0
                continue
            n_diag, kept, _ = b.stats()
            assert terms[k] == n_diag + kept, (name, k)
            xs = x[sel, k]
            if b.is_complex:
                ys = b.apply(w.J, torch.as_tensor(xs).cuda()).cpu().numpy()
            else:
                yr = b.apply(w.J, torch.as_tensor(xs.real.copy()).cuda()).cpu().numpy()
                yi = b.apply(w.J, torch.as_tensor(xs.imag.copy()).cuda()).cpu().numpy()
                ys = yr + 1j * yi
            assert np.linalg.norm(y[sel, k] - ys) <= RTOL * np.linalg.norm(ys), (name, k)
        finally:
            b.close()
    # each shared off-diagonal term is counted once however many sectors use it
    assert shared >= max(terms[k] - d for k, d in enumerate(mb.sector_dims()))


@pytest.mark.parametrize("name", IDS)
def test_batched_lanczos_graph_replays_match_eager(built, name):
    """Graph-captured steps against the same kernels launched directly."""
    ws = dict(CASES)[name]
    mb = built[name]
    v0 = torch.as_tensor(_garbage_x(mb, 41)).cuda()
    eager = mb.lanczos(ws[0].J, v0, 40, use_graph=False)
    for rep in range(3):
        # eager work and synchronisation between the graph runs
        y = mb.apply(ws[0].J, v0)
        torch.cuda.synchronize()
        assert torch.isfinite(y.real).all()
        g = mb.lanczos(ws[0].J, v0, 40, use_graph=True)
        assert np.array_equal(g["n_done"], eager["n_done"]), rep
        for k in range(mb.K):
            n = int(eager["n_done"][k])
            assert np.array_equal(g["alpha"][k, :n], eager["alpha"][k, :n]), (rep, k)
            assert np.array_equal(g["beta"][k, :n], eager["beta"][k, :n]), (rep, k)


@pytest.mark.parametrize("name", IDS)
def test_batched_lanczos_matches_oracle(built, name):
    ws = dict(CASES)[name]
    mb = built[name]
    x0 = _garbage_x(mb, 51)
    res = mb.lanczos(ws[0].J, torch.as_tensor(x0).cuda(), 120)
    masks = mb.masks()
    dims = mb.sector_dims()
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        n = int(res["n_done"][k])
        if dims[k] == 0:
            assert n == 0
            continue
        m, st, stab = _oracle_sector(w)
        Hk = _dense_sector(m, st, stab)
        ref = olz.lanczos(lambda v: Hk @ v, x0[sel, k], 120)
        # same recurrence on the same start vector: early coefficients agree
        nn = min(n, ref["n_done"], 6)
        assert np.allclose(res["alpha"][k, :nn], ref["alpha"][:nn], rtol=1e-10, atol=1e-10), (name, k)
        assert np.allclose(res["beta"][k, :nn], ref["beta"][:nn], rtol=1e-10, atol=1e-10), (name, k)
        # the lowest Ritz value is the sector's ground energy (eigenvalues to 1e-10)
        dense = np.linalg.eigvalsh((Hk + Hk.conj().T) / 2)
        assert abs(res["eigenvalues"][k][0] - dense[0]) <= 1e-10 * max(1.0, abs(dense[0])), (name, k)


def _dense_sector(m, st, stab):
    return bf.dense_matrix(m, st)


def test_batched_rejects_bad_input(built):
    ed = _ed()
    from paper_1804_05028_amd import _lib as L
    ws = dict(CASES)["square16_allk"]
    mb = built["square16_allk"]
    x = mb.empty()
    with pytest.raises(L.EDError) as e:
        L.ed_apply_H_batched(mb.handle, ws[0].J, x, x)
    assert e.value.name == "ED_ERR_ARG"
    # non-invariant couplings
    J = ws[0].J.copy()
    J[0] = 1.5
    with pytest.raises(L.EDError) as e:
        mb.apply(J, x)
    assert e.value.name == "ED_ERR_NONINVARIANT_H"
    # more than 64 sectors
    c = ws[0].cluster
    with pytest.raises(L.EDError) as e:
        ed.MultiBasis(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, [ws[0].chi] * 65, 8)
    assert e.value.name == "ED_ERR_UNSUPPORTED"
    # a character table that is not a homomorphism
    bad = ws[1].chi.copy()
    bad[1] *= -1
    with pytest.raises(L.EDError) as e:
        ed.MultiBasis(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, [ws[0].chi, bad], 8)
    assert e.value.name == "ED_ERR_BAD_IRREP"
