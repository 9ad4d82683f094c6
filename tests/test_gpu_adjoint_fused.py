"""The fused adjoint pass (gx = H gy and the per-bond sums gJ in one pass
over the terms, reading x_j and gy_j from one adjoint slot: 32 bytes for
real sectors, 64 for complex ones)
against the separate products: gx against ed_apply_H on gy, gJ against the
per-bond kernel alone (ed_apply_H_backward without gx).  Both are formed
term by term in the same order and form, so they must agree bit for bit.
Covers real and complex sectors, 1-, 2- and 4-byte tables, one to three
compile-time chunks, the run-time search loops, 512- and 1024-thread blocks
(rows on the second and later waves of every SIMD), and the 32-site
disorder workload of the adjoint benchmark at full size."""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl

pytestmark = pytest.mark.gpu

CASES = [
    ("square16_k0", lambda: wl.square_4x4(), None),
    ("sq20_n4_2chunks", lambda: wl.square_20_j1j2(n_sub=4), {"chunk_bits": 3}),
    ("sq20_n4_u8", lambda: wl.square_20_j1j2(n_sub=4), {"table_entry_bytes": 1}),
    ("sq20_n4_u32_3chunks", lambda: wl.square_20_j1j2(n_sub=4), {"table_entry_bytes": 4, "chunk_bits": 2}),
    ("sq20_n5", lambda: wl.square_20_j1j2(n_sub=5), None),
    ("tri12_full", lambda: wl.triangular_12(), None),
    ("square32_disorder", lambda: _disorder32(), None),
    ("square16_k3_complex", lambda: wl.square_4x4(momentum_index=3), None),
    ("sq20_n4_k1_complex", lambda: _sq20_momentum(1), {"chunk_bits": 3}),
    ("square16_k5_complex_u8", lambda: wl.square_4x4(momentum_index=5), {"table_entry_bytes": 1}),
    # 1024-thread blocks: rows on the second and later waves of each SIMD
    ("square16_k0_1024", lambda: wl.square_4x4(), {"block_threads": 1024}),
    ("square16_k3_complex_1024", lambda: wl.square_4x4(momentum_index=3), {"block_threads": 1024}),
    ("square16_k5_complex_u8_1024", lambda: wl.square_4x4(momentum_index=5), {"table_entry_bytes": 1, "block_threads": 1024}),
    ("sq20_n4_u8_1024", lambda: wl.square_20_j1j2(n_sub=4), {"table_entry_bytes": 1, "block_threads": 1024}),
    ("sq20_n4_k1_complex_1024", lambda: _sq20_momentum(1), {"chunk_bits": 3, "block_threads": 1024}),
]


def _sq20_momentum(k):
    """The 20-site J1-J2 cluster, translations only, momentum sector k (complex)."""
    w = wl.square_20_j1j2(n_sub=4)
    c = lat.square((4, 2), (-2, 4), j2=True, rotations=False, mirrors=False, superlattice=wl.SQ_2X2, name="sq20T")
    return wl.Workload("sq20T_k", c, lat.characters(c, k), w.n_up, np.array([1.0, 0.5])[c.bond_kind])


def _disorder32():
    """The 32-site disorder workload with its couplings averaged over bond
    orbits (a translation sector sees only the orbit means)."""
    w = wl.square_32_disorder(n_sub=4)
    J = lat.orbit_mean(w.J, lat.bond_orbits(w.cluster))
    return wl.Workload(w.name, w.cluster, w.chi, w.n_up, J, w.description)


@pytest.mark.parametrize("name,make,tuning", CASES, ids=[c[0] for c in CASES])
def test_fused_adjoint_equals_separate_products(name, make, tuning):
    from paper_1804_05028_amd import _lib as L
    from paper_1804_05028_amd import ed
    w = make()
    b = ed.Basis.from_workload(w, tuning)
    try:
        J = np.asarray(w.J, dtype=np.float64)
        x = torch.as_tensor(vec.normal_vector(b.dim, seed=11, complex_=b.is_complex)).cuda()
        gy = torch.as_tensor(vec.normal_vector(b.dim, seed=12, complex_=b.is_complex)).cuda()
        print(f"[fused] {name}: D={b.dim}", flush=True)
        gx = b.empty()
        gJ = L.ed_apply_H_backward(b.handle, J, x, gy, gx, True, None)        # fused pass
        hx = b.apply(J, gy)                                                   # H gy alone
        gJ_sep = L.ed_apply_H_backward(b.handle, J, x, gy, None, True, None)  # per-bond kernel alone
        torch.cuda.synchronize()
        assert torch.equal(gx, hx)
        assert np.array_equal(gJ, gJ_sep)
        # a second fused call reuses the adjoint slots
        gx2 = b.empty()
        gJ2 = L.ed_apply_H_backward(b.handle, J, gy, x, gx2, True, None)
        hx2 = b.apply(J, x)
        gJ2_sep = L.ed_apply_H_backward(b.handle, J, gy, x, None, True, None)
        torch.cuda.synchronize()
        assert torch.equal(gx2, hx2) and np.array_equal(gJ2, gJ2_sep)
    finally:
        b.close()


def test_fused_adjoint_rejects_aliased_output():
    from paper_1804_05028_amd import _lib as L
    from paper_1804_05028_amd import ed
    w = wl.square_4x4()
    b = ed.Basis.from_workload(w)
    try:
        x = torch.as_tensor(vec.normal_vector(b.dim, seed=1)).cuda()
        gy = torch.as_tensor(vec.normal_vector(b.dim, seed=2)).cuda()
        with pytest.raises(L.EDError) as e:
            L.ed_apply_H_backward(b.handle, np.asarray(w.J, np.float64), x, gy, x, True, None)
        assert e.value.name == "ED_ERR_ARG"
    finally:
        b.close()
