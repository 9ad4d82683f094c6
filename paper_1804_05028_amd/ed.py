"""PyTorch-facing API over the C ABI.

PyTorch provides device memory and streams only; every operation of the path
(basis build, H.v, Lanczos, adjoint) runs in the HIP kernels of libed.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the H.v path runs on an AMD GPU (gfx950) only; no GPU is visible")


class Basis:
    """A sector basis resident on the current GPU.

    Parameters mirror the C ABI: site count, bonds, sublattice count (sites
    must be numbered sublattice by sublattice), group permutations and
    flips, the irrep's characters, and the number of up spins.  `tuning` is
    an optional dict with the fields of ed_tuning_t (all 0 = automatic):
    index_mode, limits_bits, block_threads, blocks_per_cu, chunk_bits,
    hash_load_pct, table_entry_bytes, search_mode (1 one-stage, 2 two-stage
    representative search) and lanczos_direct (1 = no graph replay).
    """

    _build = staticmethod(L.ed_build_basis)

    def __init__(self, n_sites, bonds, n_sublat, perm, flip, chi, n_up, tuning=None):
        _require_gpu()
        self.arrays = L.ModelArrays(n_sites, bonds, n_sublat, perm, flip, chi)
        self.n_up = int(n_up)
        self.handle = self._build(self.arrays, n_up, tuning, _stream())
        self.dim = L.ed_basis_dim(self.handle)
        self.is_complex = L.ed_basis_is_complex(self.handle)
        self.n_bonds = int(self.arrays.bonds.shape[0])

    @classmethod
    def from_workload(cls, w, tuning=None):
        c = w.cluster
        return cls(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, w.chi, w.n_up, tuning)

    # -- housekeeping ------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            L.ed_free_basis(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return L.ed_basis_info(self.handle)

    @property
    def dtype(self):
        return torch.complex128 if self.is_complex else torch.float64

    def empty(self):
        return torch.empty(self.dim, dtype=self.dtype, device="cuda")

    # -- basis contents ----------------------------------------------------
    def states(self):
        out = np.empty(self.dim, np.uint64)
        L.ed_basis_copy_states(self.handle, out, _stream())
        return out

    def states_device(self):
        out = torch.empty(self.dim, dtype=torch.int64, device="cuda")
        L.ed_basis_copy_states_device(self.handle, out, _stream())
        return out

    def norms(self):
        out = np.empty(self.dim, np.uint16)
        L.ed_basis_copy_norms(self.handle, out, _stream())
        return out

    # -- operators ---------------------------------------------------------
    def _check_vec(self, v, name):
        if not (v.is_cuda and v.is_contiguous() and v.dtype == self.dtype and v.numel() == self.dim):
            raise ValueError(f"{name} must be a contiguous CUDA {self.dtype} tensor of length {self.dim}")

    def apply(self, J, x, out=None, Jz=None):
        """y = H(J) x (J on the host, constant on bond orbits); with Jz the
        XXZ Hamiltonian (exchange J, Ising part Jz)."""
        self._check_vec(x, "x")
        y = self.empty() if out is None else out
        self._check_vec(y, "out")
        if Jz is None:
            L.ed_apply_H(self.handle, np.asarray(J, np.float64), x, y, _stream())
        else:
            L.ed_apply_H_xxz(self.handle, np.asarray(J, np.float64), np.asarray(Jz, np.float64), x, y, _stream())
        return y

    def stats(self):
        return L.ed_apply_H_stats(self.handle, _stream())

    def apply_timed(self, J, x, out=None, reps=5, Jz=None):
        """reps launches of y = H x; returns (y, mean scatter ms, mean H.v kernel ms).
        For fermionic bases J and Jz are the hoppings t and interactions V."""
        self._check_vec(x, "x")
        y = self.empty() if out is None else out
        self._check_vec(y, "out")
        pack_ms, kernel_ms = L.ed_apply_H_timed(self.handle, np.asarray(J, np.float64),
                                                None if Jz is None else np.asarray(Jz, np.float64), x, y, reps,
                                                _stream())
        return y, pack_ms, kernel_ms

    def lanczos(self, J, v0, n_steps, want_psi0=False, Jz=None):
        self._check_vec(v0, "v0")
        psi = self.empty() if want_psi0 else None
        if Jz is None:
            a, b, n = L.ed_lanczos(self.handle, np.asarray(J, np.float64), v0, n_steps, psi, _stream())
        else:
            a, b, n = L.ed_lanczos_xxz(self.handle, np.asarray(J, np.float64), np.asarray(Jz, np.float64), v0,
                                       n_steps, psi, _stream())
        ev, _ = L.ed_tridiag_eigh(a, b, want_vec=False) if n else (np.array([]), None)
        return dict(alpha=a, beta=b, n_done=n, eigenvalues=ev, psi0=psi)

    def backward(self, J, x, gy, want_gx=True, want_gJ=True):
        self._check_vec(gy, "gy")
        if want_gJ:
            self._check_vec(x, "x")
        gx = self.empty() if want_gx else None
        gJ = L.ed_apply_H_backward(self.handle, np.asarray(J, np.float64), x if want_gJ else None, gy, gx,
                                   want_gJ, _stream())
        return gx, gJ


class FermionBasis(Basis):
    """A sector of spinless fermions (or of spinful ones written as two
    orbitals per site) in the occupation-number basis: orbitals take the
    place of sites and n_particles that of n_up; the group carries no spin
    flip.  H = sum_b [-t_b (c+_p c_q + h.c.) + V_b n_p n_q]."""

    _build = staticmethod(L.ed_build_basis_fermions)

    def __init__(self, n_orb, bonds, n_sublat, perm, chi, n_particles, tuning=None):
        perm = np.asarray(perm)
        super().__init__(n_orb, bonds, n_sublat, perm, np.zeros(perm.shape[0], np.uint8), chi, n_particles, tuning)

    @classmethod
    def from_workload(cls, w, tuning=None):
        c = w.cluster
        return cls(c.n_sites, c.bonds, c.n_sublat, c.perm, w.chi, w.n_up, tuning)

    def apply(self, t, x, out=None, V=None):
        self._check_vec(x, "x")
        y = self.empty() if out is None else out
        self._check_vec(y, "out")
        L.ed_apply_H_fermions(self.handle, np.asarray(t, np.float64), None if V is None else np.asarray(V, np.float64),
                              x, y, _stream())
        return y

    def lanczos(self, t, v0, n_steps, want_psi0=False, V=None):
        self._check_vec(v0, "v0")
        psi = self.empty() if want_psi0 else None
        a, b, n = L.ed_lanczos_fermions(self.handle, np.asarray(t, np.float64),
                                        None if V is None else np.asarray(V, np.float64), v0, n_steps, psi, _stream())
        ev, _ = L.ed_tridiag_eigh(a, b, want_vec=False) if n else (np.array([]), None)
        return dict(alpha=a, beta=b, n_done=n, eigenvalues=ev, psi0=psi)

    def backward(self, *args, **kwargs):
        raise NotImplementedError("the adjoint covers spin bases")


class MultiBasis:
    """Several 1-D irreps of one group over one shared set of representatives.

    Batched vectors are complex128 tensors of shape [dim, K] (sector index
    fastest); column k restricted to the rows of sector k is that sector's
    vector in the order of its own basis.  `tuning` takes the fields of
    ed_tuning_t that apply to the shared basis and the batched kernel,
    notably lanes_per_row (1, 2 or 4 lanes per row; 0 = automatic) and
    search_mode.
    """

    def __init__(self, n_sites, bonds, n_sublat, perm, flip, chis, n_up, tuning=None):
        _require_gpu()
        self.arrays = L.ModelArrays(n_sites, bonds, n_sublat, perm, flip, None)
        self.n_up = int(n_up)
        self.K = len(chis)
        self.handle = L.ed_build_multi(self.arrays, chis, n_up, tuning, _stream())
        self.dim = int(L.ed_multi_info(self.handle)["dim"])
        self.n_bonds = int(self.arrays.bonds.shape[0])

    @classmethod
    def from_workloads(cls, ws, tuning=None):
        """Workloads that share cluster, n_up and couplings, one per sector."""
        c = ws[0].cluster
        return cls(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, [w.chi for w in ws], ws[0].n_up, tuning)

    def close(self):
        if getattr(self, "handle", None):
            L.ed_free_multi(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return L.ed_multi_info(self.handle)

    def sector_dims(self):
        return L.ed_multi_sector_dims(self.handle, self.K)

    def states(self):
        out = np.empty(self.dim, np.uint64)
        L.ed_multi_copy_states(self.handle, out, _stream())
        return out

    def masks(self):
        out = np.empty(self.dim, np.uint64)
        L.ed_multi_copy_masks(self.handle, out, _stream())
        return out

    def empty(self):
        return torch.empty((self.dim, self.K), dtype=torch.complex128, device="cuda")

    def _check_vec(self, v, name):
        if not (v.is_cuda and v.is_contiguous() and v.dtype == torch.complex128 and tuple(v.shape) == (self.dim, self.K)):
            raise ValueError(f"{name} must be a contiguous CUDA complex128 tensor of shape ({self.dim}, {self.K})")

    def apply(self, J, x, out=None):
        self._check_vec(x, "x")
        y = self.empty() if out is None else out
        self._check_vec(y, "out")
        L.ed_apply_H_batched(self.handle, np.asarray(J, np.float64), x, y, _stream())
        return y

    def stats(self):
        """(per-sector terms D_k + kept_k, shared off-diagonal terms)."""
        return L.ed_apply_H_batched_stats(self.handle, self.K, _stream())

    def lanczos(self, J, v0, n_steps, use_graph=True):
        self._check_vec(v0, "v0")
        a, b, nd = L.ed_lanczos_batched(self.handle, np.asarray(J, np.float64), v0, n_steps, self.K,
                                        0 if use_graph else L.ED_LANCZOS_NO_GRAPH, _stream())
        evs = []
        for k in range(self.K):
            n = int(nd[k])
            evs.append(L.ed_tridiag_eigh(a[k, :n], b[k, :n], want_vec=False)[0] if n else np.array([]))
        return dict(alpha=a, beta=b, n_done=nd, eigenvalues=evs)


def bond_orbits_from(perm, bonds):
    """Orbit index of every bond under the site permutations."""
    perm = np.asarray(perm)
    bonds = np.asarray(bonds).reshape(-1, 2)
    key = {}
    for b, (p, q) in enumerate(bonds):
        key.setdefault((min(p, q), max(p, q)), []).append(b)
    orbit = -np.ones(len(bonds), dtype=np.int64)
    nxt = 0
    for b in range(len(bonds)):
        if orbit[b] >= 0:
            continue
        p, q = bonds[b]
        for g in range(perm.shape[0]):
            a, c = perm[g, p], perm[g, q]
            for m in key.get((min(a, c), max(a, c)), []):
                orbit[m] = nxt
        nxt += 1
    return orbit


class _ApplyH(torch.autograd.Function):
    """y = H(Jbar) x with the hand-written adjoint: dx = H gy, dJbar_b = Re(gy^H H_b x)."""

    @staticmethod
    def forward(ctx, Jbar, x, basis):
        y = basis.apply(Jbar.detach().cpu().numpy(), x.detach().contiguous())
        ctx.basis = basis
        ctx.save_for_backward(Jbar, x)
        return y

    @staticmethod
    def backward(ctx, gy):
        Jbar, x = ctx.saved_tensors
        basis = ctx.basis
        need_J, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gx, gJ = basis.backward(Jbar.detach().cpu().numpy(), x.detach().contiguous(), gy.contiguous(),
                                want_gx=need_x, want_gJ=need_J)
        gJt = torch.from_numpy(gJ).to(Jbar.dtype) if need_J else None
        return gJt, gx, None


def orbit_mean(J, orbit):
    """Differentiable average of J over bond orbits (torch, CPU float64)."""
    orbit_t = torch.as_tensor(orbit, dtype=torch.long)
    n_orb = int(orbit_t.max().item()) + 1 if orbit_t.numel() else 0
    sums = torch.zeros(n_orb, dtype=J.dtype).index_add(0, orbit_t, J)
    counts = torch.zeros(n_orb, dtype=J.dtype).index_add(0, orbit_t, torch.ones_like(J))
    return (sums / counts)[orbit_t]


def apply_H(basis: Basis, J, x, orbit=None):
    """Differentiable y = H(J) x.

    J is a CPU float64 tensor of per-bond couplings.  In a symmetry sector
    only the orbit average of J enters the sector Hamiltonian, so J is first
    averaged over bond orbits (``orbit`` from ``bond_orbits_from``); autograd
    then distributes dL/dJbar evenly over each orbit.
    """
    if not torch.is_tensor(J):
        J = torch.as_tensor(np.asarray(J, np.float64))
    if orbit is not None:
        J = orbit_mean(J, orbit)
    return _ApplyH.apply(J, x, basis)
