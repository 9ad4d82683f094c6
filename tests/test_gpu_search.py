"""GPU: the two-stage representative search against the one-stage search and
the oracle.

Both searches return the minimal image and the first minimiser in Sym-list
order, so H.v must agree bit for bit between them, and both must match the
oracle within 1e-12 relative.  The cases cover two, three and four
sublattices, one to three compile-time action-table chunks and run-time
chunk counts, 1-, 2- and 4-byte table entries, real and complex irreps, the
counting pass and the fused Lanczos kernel.
"""
import numpy as np
import pytest
import torch

from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

RTOL = 1e-12
ONE, TWO = 1, 2   # ED_SEARCH_ONE_STAGE, ED_SEARCH_TWO_STAGE


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _cases():
    return [
        ("square16_k0", wl.square_4x4(), {}),
        ("square16_k5", wl.square_4x4(momentum_index=5), {}),
        ("square16_full_n2", wl.square_4x4(n_sub=2, group="full"), {}),
        ("square16_full_n2_c2", wl.square_4x4(n_sub=2, group="full"), {"chunk_bits": 2}),
        ("tri12_A1_even_n3", wl.triangular_12(), {}),
        ("tri12_A1_even_n3_e1", wl.triangular_12(), {"table_entry_bytes": 1, "chunk_bits": 2}),
        ("tri12_k2_n3_complex", wl.triangular_12(momentum_index=2, spin_flip=False, rotations=False, mirrors=False),
         {}),
        ("sq20_j1j2_n4", wl.square_20_j1j2(n_sub=4), {}),
        ("sq20_j1j2_n4_e4_c2", wl.square_20_j1j2(n_sub=4), {"table_entry_bytes": 4, "chunk_bits": 2}),
        ("square16_k5_e4_c1", wl.square_4x4(momentum_index=5), {"table_entry_bytes": 4, "chunk_bits": 1}),
    ]


CASES = _cases()


def _supported(w):
    return 2 <= w.cluster.n_sublat <= 4


@pytest.mark.parametrize("name,w,tuning", CASES, ids=[n for n, _, _ in CASES])
def test_two_stage_matches_one_stage_and_oracle(name, w, tuning):
    ed = _ed()
    if not _supported(w):
        pytest.skip("two-stage search needs 2 to 4 sublattices")
    print(f"[search] {name} n_sub={w.cluster.n_sublat} {tuning}", flush=True)
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    x = vec.normal_vector(len(st), seed=11, complex_=w.is_complex)
    y_ref, kept, dropped = bf.apply(m, st, stab, x)
    ys = {}
    for mode in (ONE, TWO):
        b = ed.Basis.from_workload(w, dict(tuning, search_mode=mode))
        try:
            info = b.info()
            assert info["search_mode"] == mode
            assert info["mean_candidates"] >= 1.0
            assert np.array_equal(b.states(), st)
            ys[mode] = b.apply(w.J, torch.as_tensor(x).cuda()).cpu().numpy()
            assert b.stats() == (len(st), kept, dropped)
        finally:
            b.close()
    assert np.array_equal(ys[ONE], ys[TWO])
    assert np.linalg.norm(ys[TWO] - y_ref) <= RTOL * np.linalg.norm(y_ref)


def test_two_stage_lanczos_matches_oracle():
    ed = _ed()
    w = wl.triangular_12()
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    v0 = vec.normal_vector(len(st))
    n_steps = min(100, len(st) + 5)
    ref = olz.lanczos(lambda v: bf.apply(m, st, stab, v)[0], v0, n_steps)
    res = {}
    for mode in (ONE, TWO):
        b = ed.Basis.from_workload(w, {"search_mode": mode})
        try:
            res[mode] = b.lanczos(w.J, torch.as_tensor(v0).cuda(), n_steps)
        finally:
            b.close()
    assert np.array_equal(res[ONE]["alpha"], res[TWO]["alpha"])
    assert np.array_equal(res[ONE]["beta"], res[TWO]["beta"])
    k = min(10, res[TWO]["n_done"], ref["n_done"])
    assert np.abs(res[TWO]["alpha"][:k] - ref["alpha"][:k]).max() < 1e-11
    assert abs(res[TWO]["eigenvalues"][0] - ref["eigenvalues"][0]) < 1e-10


def test_automatic_choice_follows_the_candidate_count():
    ed = _ed()
    for w in (wl.triangular_12(), wl.square_4x4(), wl.square_20_j1j2(n_sub=5)):
        b = ed.Basis.from_workload(w)
        try:
            info = b.info()
            want = TWO if (_supported(w) and info["mean_candidates"] >= 3.0) else ONE
            assert info["search_mode"] == want, (w.name, info["mean_candidates"])
        finally:
            b.close()


def test_batched_two_stage_matches_one_stage_and_oracle():
    """The batched kernel runs the two-stage search through a run-time flag.
    16 sectors of the 4x4 full space group (Gamma and M, every 1-D point-group
    irrep, both flip parities): their 256 x 16 character table exceeds the LDS
    share and is read from HBM."""
    from ed_inputs import lattice as lat
    ed = _ed()
    c = lat.square((4, 0), (0, 4), rotations=True, mirrors=True, spin_flip=True, superlattice=wl.SQ_2X2,
                   name="square16full")
    U, det = lat.momenta(c)
    ks = [0, U.index((det // 2, det // 2))]
    pcs = lat.point_group_chars_1d(c.point_group)
    ws = [wl.Workload("sq16full", c, lat.characters(c, k, p, f), 8, np.ones(c.n_bonds))
          for k in ks for p in pcs for f in (1, -1)]
    assert len(ws) == 16 and c.n_elems * len(ws) * 16 > 32768
    ys, x, masks = {}, None, None
    for mode in (ONE, TWO):
        mb = ed.MultiBasis.from_workloads(ws, {"search_mode": mode})
        try:
            if x is None:
                re = vec.normal_vector(mb.dim * mb.K, seed=17, normalise=False)
                x = (re + 0.25j * re[::-1]).reshape(mb.dim, mb.K)
                masks = mb.masks()
            ys[mode] = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
        finally:
            mb.close()
    assert np.array_equal(ys[ONE], ys[TWO])
    for k, w in enumerate(ws):
        sel = ((masks >> np.uint64(k)) & np.uint64(1)).astype(bool)
        if not sel.any():
            continue
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        ref, _, _ = bf.apply(m, st, stab, x[sel, k])
        assert np.linalg.norm(ys[TWO][sel, k] - ref) <= RTOL * np.linalg.norm(ref), k
