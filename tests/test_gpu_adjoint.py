"""Adjoint of the sector H.v: dL/dx = H^dagger g and per-bond dL/dJ_b.

Per-bond values A_b = Re(g^dagger dH/dJ_b x) follow the row form of the
kernel (terms generated from each row); they are compared with the same
quantity assembled by the CPU oracle's per-row matrix elements.  Sums over
a bond orbit -- the derivative with respect to an orbit coupling, which is
all a symmetric sector depends on -- are checked against finite
differences (exact for a loss linear in J) and, for the ground-state
energy, against Hellmann-Feynman and finite differences of E0.
"""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf

pytestmark = pytest.mark.gpu


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _oracle_per_bond(w, st, stab, x, gy):
    """A_b = Re sum_i conj(gy_i) (dH/dJ_b x)_i, row form, from oracle matrix elements."""
    c = w.cluster
    m = bf.Model(c.n_sites, c.perm, c.flip, w.chi, c.bonds, np.ones(c.n_bonds))
    t = bf.row_terms(m, st)
    nb = c.n_bonds
    A = np.zeros(nb)
    xc = np.asarray(x, dtype=np.complex128)
    gc = np.asarray(gy, dtype=np.complex128)
    for b in range(nb):
        flag = t["tgt_flag"][:, b]
        diag = np.where(flag == 0, 0.25, -0.25)
        contrib = diag * xc
        kept = flag == 1
        j = np.searchsorted(st, t["tgt"][kept, b])
        assert np.array_equal(st[j], t["tgt"][kept, b])
        contrib[kept] += t["coef"][kept, b] * xc[j]
        A[b] = np.real(np.vdot(gc, contrib))
    return A


SMALL = [
    ("square16_k0", lambda: wl.square_4x4()),
    ("square16_k3", lambda: wl.square_4x4(momentum_index=3)),
    ("tri12_full", lambda: wl.triangular_12()),
    ("sq20_j1j2", lambda: wl.square_20_j1j2(n_sub=5)),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[n for n, _ in SMALL])
def test_backward_matches_oracle(name, make):
    ed = _ed()
    w = make()
    b = ed.Basis.from_workload(w)
    try:
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        cplx = w.is_complex
        x = vec.normal_vector(len(st), seed=5, complex_=cplx)
        gy = vec.normal_vector(len(st), seed=6, complex_=cplx)
        gx, gJ = b.backward(w.J, torch.as_tensor(x).cuda(), torch.as_tensor(gy).cuda())
        # dL/dx = H^dagger gy = H gy
        ref_gx, _, _ = bf.apply(m, st, stab, gy)
        assert np.linalg.norm(gx.cpu().numpy() - ref_gx) <= 1e-12 * np.linalg.norm(ref_gx)
        A = _oracle_per_bond(w, st, stab, x, gy)
        assert np.abs(gJ - A).max() <= 1e-12 * max(1.0, np.abs(A).max())
        # linearity: sum_b J_b A_b = Re(gy^dagger H x)
        hx, _, _ = bf.apply(m, st, stab, x)
        assert abs(np.dot(w.J, gJ) - np.real(np.vdot(gy, hx))) <= 1e-11 * max(1.0, abs(np.real(np.vdot(gy, hx))))
    finally:
        b.close()


def test_backward_limits_index_matches_hash():
    ed = _ed()
    w = wl.square_20_j1j2(n_sub=5)
    bh = ed.Basis.from_workload(w)
    bl = ed.Basis.from_workload(w, {"index_mode": 1})
    try:
        x = torch.as_tensor(vec.normal_vector(bh.dim, seed=7)).cuda()
        gy = torch.as_tensor(vec.normal_vector(bh.dim, seed=8)).cuda()
        _, a = bh.backward(w.J, x, gy)
        _, c = bl.backward(w.J, x, gy)
        assert np.abs(a - c).max() <= 1e-13 * np.abs(a).max()
    finally:
        bh.close()
        bl.close()


def _orbit_ids(w):
    return lat.bond_orbits(w.cluster)


def test_autograd_fit_loss_matches_finite_differences():
    """L = |H(J) x - t|^2 on the 32-site disorder workload (orbit-averaged J)."""
    ed = _ed()
    w = wl.square_32_disorder(n_sub=4)
    orbit = _orbit_ids(w)
    Jraw = torch.as_tensor(vec.random_couplings(w.cluster.n_bonds, vec.SEED_COUPLING))
    b = ed.Basis.from_workload(wl.Workload(w.name, w.cluster, w.chi, w.n_up, lat.orbit_mean(Jraw.numpy(), orbit)))
    try:
        D = b.dim
        assert D == 18_784_998
        x = torch.as_tensor(vec.normal_vector(D, seed=vec.SEED_VECTOR)).cuda()
        t = torch.as_tensor(vec.normal_vector(D, seed=vec.SEED_TARGET)).cuda() * 3.0

        def loss(Jv, xv):
            y = ed.apply_H(b, Jv, xv, orbit=orbit)
            return ((y - t) ** 2).sum()

        J = Jraw.clone().requires_grad_(True)
        xg = x.clone().requires_grad_(True)
        L = loss(J, xg)
        L.backward()
        gJ = J.grad.numpy()
        # finite differences on individual bonds (they move the orbit mean)
        h = 1e-6
        for bidx in (0, 5, 40, 63):
            Jp = Jraw.clone()
            Jm = Jraw.clone()
            Jp[bidx] += h
            Jm[bidx] -= h
            with torch.no_grad():
                fd = (loss(Jp, x).item() - loss(Jm, x).item()) / (2 * h)
            assert abs(gJ[bidx] - fd) <= 1e-6 * max(abs(fd), 1e-3), (bidx, gJ[bidx], fd)
        # bonds of one orbit share the same gradient (orbit mean)
        for o in np.unique(orbit):
            sel = gJ[orbit == o]
            assert np.abs(sel - sel[0]).max() <= 1e-12 * max(1.0, abs(sel[0]))
        # directional derivative in x: dL/dx . d
        d = torch.as_tensor(vec.normal_vector(D, seed=11)).cuda()
        eps = 1e-6
        with torch.no_grad():
            fdx = (loss(Jraw, x + eps * d).item() - loss(Jraw, x - eps * d).item()) / (2 * eps)
        an = float(torch.dot(xg.grad, d))
        assert abs(an - fdx) <= 1e-6 * max(abs(fdx), 1e-3), (an, fdx)
    finally:
        b.close()


def test_hellmann_feynman_and_energy_finite_differences():
    """dE0/dJbar_c = <psi0|H_c|psi0> (sum of A_b over the orbit) = FD of E0."""
    ed = _ed()
    w = wl.square_4x4()          # non-degenerate ground state in the k=0 sector
    orbit = _orbit_ids(w)
    J0 = w.J.copy()
    b = ed.Basis.from_workload(w)
    try:
        v0 = torch.as_tensor(vec.normal_vector(b.dim)).cuda()
        res = b.lanczos(J0, v0, 250, want_psi0=True)
        psi = res["psi0"]
        _, A = b.backward(J0, psi, psi)
        hf = {o: A[orbit == o].sum() for o in np.unique(orbit)}
        # <psi|H|psi> = E0 and sum_c Jbar_c hf_c = E0 (H linear in J)
        e0 = res["eigenvalues"][0]
        assert abs(sum(J0[orbit == o][0] * hf[o] for o in hf) - e0) <= 1e-9 * abs(e0)
        h = 1e-5
        for o in np.unique(orbit):
            Jp, Jm = J0.copy(), J0.copy()
            Jp[orbit == o] += h
            Jm[orbit == o] -= h
            ep = b.lanczos(Jp, v0, 250)["eigenvalues"][0]
            em = b.lanczos(Jm, v0, 250)["eigenvalues"][0]
            fd = (ep - em) / (2 * h)
            assert abs(fd - hf[o]) <= 1e-6 * max(abs(hf[o]), 1e-3), (o, fd, hf[o])
    finally:
        b.close()
