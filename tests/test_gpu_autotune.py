"""Launch-configuration search: every candidate computes the same H.v, and the
chosen configuration reproduces the oracle."""
import numpy as np
import pytest
import torch

from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_valid_configuration():
    from paper_1804_05028_amd import autotune as at
    from paper_1804_05028_amd import ed
    best, results = at.autotune(lambda ns: wl.square_20_j1j2(n_sub=ns), [4, 5, 10], reps=2)
    assert any("hv_ms" in r for r in results)
    assert best["hv_ms"] == min(r["hv_ms"] for r in results if "hv_ms" in r)
    tab = at.speedup_table(results)
    assert tab[0][3] == 1.0 and all(t[3] >= 1.0 for t in tab)
    w = wl.square_20_j1j2(n_sub=best["n_sub"])
    b = ed.Basis.from_workload(w, best["tuning"])
    try:
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        assert np.array_equal(b.states(), st)
        x = vec.normal_vector(len(st), seed=9)
        y = b.apply(w.J, torch.as_tensor(x).cuda()).cpu().numpy()
        ref, _, _ = bf.apply(m, st, stab, x)
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    finally:
        b.close()


def test_autotune_over_enumerated_decompositions():
    """Host ranking of the stable decompositions, then GPU timing of the best two."""
    from paper_1804_05028_amd import autotune as at
    from paper_1804_05028_amd import ed
    from ed_inputs import lattice as lat

    def make(M):
        c = lat.square((4, 2), (-2, 4), j2=True, spin_flip=True, superlattice=M, name="square20")
        J = np.array([1.0, 0.5])[c.bond_kind]
        return wl.Workload("square20_j1j2", c, lat.characters(c, 0), 10, J)

    base = lat.square((4, 2), (-2, 4), j2=True, spin_flip=True, name="square20")
    decs = lat.sublattice_decompositions((4, 2), (-2, 4), base.point_group, 20, 12)
    best, results, ranking = at.autotune_decompositions(make, decs, 10, top=2, reps=2)
    assert len({r["n_sub"] for r in results}) <= 2
    w = make(best["n_sub"][1])
    b = ed.Basis.from_workload(w, best["tuning"])
    try:
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        x = vec.normal_vector(len(st), seed=12)
        y = b.apply(w.J, torch.as_tensor(x).cuda()).cpu().numpy()
        ref, _, _ = bf.apply(m, st, stab, x)
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    finally:
        b.close()


def test_autotune_batched_schedule_covers_every_sector():
    """The batched schedule tiles the sectors in order, picks a timed lane count
    for each group, and its launches reproduce the oracle of every sector."""
    from paper_1804_05028_amd import autotune as at
    from paper_1804_05028_amd import ed
    from ed_inputs import lattice as lat
    c = wl.square_4x4().cluster
    ws = [wl.Workload(f"sq16_k{k}", c, lat.characters(c, k), 8, np.ones(c.n_bonds)) for k in range(16)]
    tuned = at.autotune_batched(ws, batches=(4, 6, 16), reps=2)
    groups = tuned["groups"]
    assert [g[0] for g in groups] == list(range(0, 16, tuned["batch"]))
    assert sum(g[1] for g in groups) == 16 and all(g[2] in (1, 2, 4) for g in groups)
    # sizes timed: 4, 6, 16 and the remainder 4 of batch 6
    assert {t["K"] for t in tuned["trials"]} == {4, 6, 16}
    for first, k, lanes in groups:
        mb = ed.MultiBasis.from_workloads(ws[first:first + k], {"lanes_per_row": lanes})
        try:
            re = vec.normal_vector(mb.dim * k, seed=5, normalise=False)
            x = (re + 0.5j * re[::-1]).reshape(mb.dim, k)
            y = mb.apply(ws[0].J, torch.as_tensor(x).cuda()).cpu().numpy()
            masks = mb.masks()
            for j in range(k):
                w = ws[first + j]
                sel = ((masks >> np.uint64(j)) & np.uint64(1)).astype(bool)
                m = bf.Model.from_workload(w)
                st, stab = bf.basis(m, w.n_up)
                ref, _, _ = bf.apply(m, st, stab, x[sel, j])
                assert np.linalg.norm(y[sel, j] - ref) <= 1e-12 * np.linalg.norm(ref)
        finally:
            mb.close()
