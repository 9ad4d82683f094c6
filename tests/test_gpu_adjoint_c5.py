"""Hellmann-Feynman at the 32-site disorder workload (D = 18,784,998).

L(J) = <psi0|H(Jbar)|psi0> with psi0 frozen has dL/dJbar_c = sum_{b in c} A_b
(the adjoint's per-bond sums), and by Hellmann-Feynman this equals dE0/dJbar_c.
E0 itself is linear-homogeneous in J, so sum_c Jbar_c dE0/dJbar_c = E0.  The
finite difference of E0 (h = 1e-4, two Lanczos runs per orbit) is the looser
check: its error is the Lanczos convergence of E0 over h plus O(h^2).
"""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl

pytestmark = pytest.mark.gpu


def test_hellmann_feynman_32_site_disorder():
    from paper_1804_05028_amd import ed
    w = wl.square_32_disorder(n_sub=4)
    orbit = lat.bond_orbits(w.cluster)
    Jbar = lat.orbit_mean(w.J, orbit)
    b = ed.Basis.from_workload(wl.Workload(w.name, w.cluster, w.chi, w.n_up, Jbar))
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(vec.SEED_VECTOR)
        v0 = torch.randn(b.dim, dtype=torch.float64, device="cuda", generator=g)
        res = b.lanczos(Jbar, v0, 200, want_psi0=True)
        e0 = res["eigenvalues"][0]
        psi = res["psi0"]
        # residual of the Ritz pair
        r = b.apply(Jbar, psi) - e0 * psi
        assert float(torch.linalg.norm(r)) < 1e-6
        _, A = b.backward(Jbar, psi, psi)
        hf = {o: A[orbit == o].sum() for o in np.unique(orbit)}
        assert abs(sum(Jbar[orbit == o][0] * hf[o] for o in hf) - e0) <= 1e-9 * abs(e0)
        h = 1e-4
        for o in np.unique(orbit):
            Jp, Jm = Jbar.copy(), Jbar.copy()
            Jp[orbit == o] += h
            Jm[orbit == o] -= h
            ep = b.lanczos(Jp, v0, 200)["eigenvalues"][0]
            em = b.lanczos(Jm, v0, 200)["eigenvalues"][0]
            fd = (ep - em) / (2 * h)
            print(f"[hf32] orbit {o}: HF {hf[o]:.10f} FD {fd:.10f}", flush=True)
            assert abs(fd - hf[o]) <= 1e-6 * abs(hf[o])
    finally:
        b.close()
