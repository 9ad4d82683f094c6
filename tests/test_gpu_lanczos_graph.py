"""ed_lanczos replays its step from HIP graphs (one per buffer assignment);
with tuning lanczos_direct = 1 it launches the same kernels directly.  Both
must give the same coefficients and ground state bit for bit, on repeated
calls on one basis, and the graph run must match the oracle recurrence."""
import numpy as np
import pytest
import torch

from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu


def _ed():
    from paper_1804_05028_amd import ed
    return ed


@pytest.mark.parametrize("name,w", [("square16_k0", wl.square_4x4()), ("tri12_A1_even", wl.triangular_12()),
                                    ("square16_k5", wl.square_4x4(momentum_index=5))])
def test_graph_replay_matches_direct_launches(name, w):
    ed = _ed()
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    v0 = vec.normal_vector(len(st), seed=7, complex_=w.is_complex)
    n_steps = min(80, len(st) + 3)
    runs = {}
    for direct in (0, 1):
        b = ed.Basis.from_workload(w, {"lanczos_direct": direct})
        try:
            first = b.lanczos(w.J, torch.as_tensor(v0).cuda(), n_steps, want_psi0=True)
            again = b.lanczos(w.J, torch.as_tensor(v0).cuda(), n_steps, want_psi0=True)
            for key in ("alpha", "beta"):
                assert np.array_equal(first[key], again[key]), (name, direct, key)
            assert torch.equal(first["psi0"], again["psi0"])
            runs[direct] = first
        finally:
            b.close()
    g, d = runs[0], runs[1]
    assert g["n_done"] == d["n_done"]
    assert np.array_equal(g["alpha"], d["alpha"]) and np.array_equal(g["beta"], d["beta"])
    assert torch.equal(g["psi0"], d["psi0"])
    ref = olz.lanczos(lambda v: bf.apply(m, st, stab, v)[0], v0, n_steps)
    k = min(10, g["n_done"], ref["n_done"])
    assert np.abs(g["alpha"][:k] - ref["alpha"][:k]).max() < 1e-11
    assert abs(g["eigenvalues"][0] - ref["eigenvalues"][0]) < 1e-10
