"""The allocation-free adjoint entry point against ed_apply_H_backward.

ed_apply_H_backward_noalloc keeps its per-bond partial sums in the library's
static device array instead of per-call buffers.  Two calls in a row, the
second on a smaller basis (fewer blocks and bonds, so stale partial sums of
the first call remain in the array beyond what the second writes), must each
give the gradients of ed_apply_H_backward on the same inputs: gx = H gy and
the per-bond sums, within 1e-12 relative.
"""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import workloads as wl

pytestmark = pytest.mark.gpu


def _disorder32():
    w = wl.square_32_disorder(n_sub=4)
    return w, lat.orbit_mean(w.J, lat.bond_orbits(w.cluster))


def _square16():
    w = wl.square_4x4()
    return w, w.J


def _compare(make, seed):
    from paper_1804_05028_amd import _lib as L
    from paper_1804_05028_amd import ed
    w, J = make()
    b = ed.Basis.from_workload(w)
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        x = torch.randn(b.dim, dtype=b.dtype, device="cuda", generator=g)
        gy = torch.randn(b.dim, dtype=b.dtype, device="cuda", generator=g)
        gx_ref, gx_new = b.empty(), b.empty()
        gJ_ref = L.ed_apply_H_backward(b.handle, J, x, gy, gx_ref, True, None)
        gJ_new = L.ed_apply_H_backward_noalloc(b.handle, J, x, gy, gx_new, True, None)
        torch.cuda.synchronize()
        err_j = np.abs(gJ_new - gJ_ref).max() / np.abs(gJ_ref).max()
        err_x = float((gx_new - gx_ref).abs().max() / gx_ref.abs().max())
        same = np.array_equal(gJ_new, gJ_ref) and bool(torch.equal(gx_new, gx_ref))
        print(f"[no_alloc] {w.name}: D={b.dim} bonds={len(J)} gJ rel {err_j:.2e} gx rel {err_x:.2e} "
              f"bit-identical={same}", flush=True)
        assert err_j <= 1e-12 and err_x <= 1e-12
        # per-bond sums only, without gx
        gJ_only = L.ed_apply_H_backward_noalloc(b.handle, J, x, gy, None, True, None)
        assert np.abs(gJ_only - gJ_ref).max() <= 1e-12 * np.abs(gJ_ref).max()
    finally:
        b.close()


def test_noalloc_backward_matches_allocating_entry_point():
    _compare(_disorder32, 5)   # 18.8M rows, 64 bonds
    _compare(_square16, 6)     # then 822 rows, 32 bonds
