"""Plain Lanczos recurrence in NumPy (FP64), and dense diagonalisation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs Lanczos with its matrix-vector product as the dominant cost
(sec. "Distributed and hybrid memory parallelization") and states no
details.  The reading used here: start from the given vector normalised;
w = H v_j - beta_{j-1} v_{j-1}; alpha_j = Re<v_j, w>; w -= alpha_j v_j;
beta_j = ||w||; stop after n_steps or when beta_j <= 1e-12 * max_k(|alpha_k|,
beta_k); no reorthogonalisation.  Eigenpairs of the tridiagonal T come from
a dense symmetric eigensolver (numpy.linalg.eigh on T), which stays robust
when many Ritz values nearly coincide (ghost copies after loss of
orthogonality), where LAPACK's MRRR tridiagonal driver can fail.

Pins: closed-form ground energies and the dense spectrum at small N.
"""
from __future__ import annotations

import numpy as np

BREAKDOWN_TOL = 1e-12


def lanczos(matvec, v0, n_steps, want_vectors=False):
    v = np.asarray(v0)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alphas, betas, vecs = [], [], []
    scale = 0.0
    for _ in range(n_steps):
        if want_vectors:
            vecs.append(v.copy())
        w = matvec(v) - beta_prev * v_prev
        a = float(np.real(np.vdot(v, w)))
        w = w - a * v
        b = float(np.linalg.norm(w))
        alphas.append(a)
        betas.append(b)
        scale = max(scale, abs(a), b)
        if b <= BREAKDOWN_TOL * scale:
            break
        v_prev, v = v, w / b
        beta_prev = b
    out = dict(alpha=np.array(alphas), beta=np.array(betas), n_done=len(alphas))
    out["eigenvalues"] = tridiag_eigenvalues(out["alpha"], out["beta"])
    if want_vectors:
        out["vectors"] = vecs
    return out


def _tmatrix(alpha, beta):
    m = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if m > 1:
        b = np.asarray(beta[: m - 1], dtype=np.float64)
        T += np.diag(b, 1) + np.diag(b, -1)
    return T


def tridiag_eigenvalues(alpha, beta):
    if len(alpha) == 0:
        return np.array([])
    return np.linalg.eigvalsh(_tmatrix(alpha, beta))


def ground_state(matvec, v0, n_steps):
    """Lowest Ritz value and vector, by a second pass of the same recurrence."""
    res = lanczos(matvec, v0, n_steps, want_vectors=True)
    m = res["n_done"]
    if m == 1:
        return res["alpha"][0], res["vectors"][0]
    w, s = np.linalg.eigh(_tmatrix(res["alpha"], res["beta"]))
    psi = sum(s[k, 0] * res["vectors"][k] for k in range(m))
    return w[0], psi / np.linalg.norm(psi)


def converged_ritz(alpha, beta, resid_tol=1e-8):
    """Ritz values whose residual beta_m |s_m| is below resid_tol."""
    m = len(alpha)
    if m == 1:
        return np.array([alpha[0]])
    w, s = np.linalg.eigh(_tmatrix(alpha, beta))
    res = abs(beta[m - 1]) * np.abs(s[m - 1, :])
    return w[res < resid_tol]
