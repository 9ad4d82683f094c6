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

Pins: closed-form ground energies and the dense spectrum at small N
(tests/test_oracle.py); the Ritz residual rule against a closed-form
2x2 tridiagonal and against residuals ||H y - theta y|| formed from the
Lanczos vectors themselves (tests/test_oracle_lanczos.py).
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


def ritz_residuals(alpha, beta):
    """Ritz values of the m-step T and their residual norms.

    For a Ritz pair (theta, y = V s) of m Lanczos steps, H y - theta y =
    beta_m (e_m . s) v_{m+1}, so the residual norm is beta_m |s_m|, with s_m
    the last component of the unit eigenvector s of T and beta_m the last
    beta the recurrence produced.
    """
    m = len(alpha)
    if m == 0:
        return np.array([]), np.array([])
    w, s = np.linalg.eigh(_tmatrix(alpha, beta))
    return w, abs(beta[m - 1]) * np.abs(s[m - 1, :])


def converged_ritz(alpha, beta, resid_tol=1e-8):
    """Ritz values whose residual beta_m |s_m| is below resid_tol, ascending."""
    w, res = ritz_residuals(alpha, beta)
    return w[res < resid_tol]
