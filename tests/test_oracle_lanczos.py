"""Pins of the oracle's Lanczos helpers (CPU only).

The converged-Ritz filter decides which Lanczos eigenvalues the GPU tests
compare, so its residual rule is pinned on its own:
  * a 2x2 tridiagonal with closed-form eigenpairs, where the residual of each
    Ritz value is beta_2 |s_2| with a known last component;
  * residuals ||A y - theta y|| formed from the Lanczos vectors of a run on a
    diagonal matrix with a known spectrum, which do not use the rule at all;
  * a single step, whose Ritz value has residual |beta_1|.
Planted mistakes in a copy of the module (the first instead of the last
eigenvector component, the next-to-last beta) must fail a pin.
"""
import math
import os
import types

import numpy as np
import pytest

from oracle import lanczos as olz

SRC = os.path.join(os.path.dirname(olz.__file__), "lanczos.py")


def _two_by_two_pin(mod):
    # T = [[0, 2], [2, 3]]: eigenvalues -1 and 4, unit eigenvectors
    # (2, -1)/sqrt5 and (1, 2)/sqrt5, last components -1/sqrt5 and 2/sqrt5
    beta2 = 1.5e-8
    w, res = mod.ritz_residuals(np.array([0.0, 3.0]), np.array([2.0, beta2]))
    ok = np.allclose(w, [-1.0, 4.0], atol=1e-14)
    ok &= np.allclose(res, [beta2 / math.sqrt(5), 2 * beta2 / math.sqrt(5)], rtol=1e-12, atol=0)
    # with tol 1e-8 only the first residual (6.7e-9) passes; the second is 1.3e-8
    conv = mod.converged_ritz(np.array([0.0, 3.0]), np.array([2.0, beta2]), resid_tol=1e-8)
    ok &= len(conv) == 1 and abs(conv[0] + 1.0) < 1e-14
    return bool(ok)


def _single_step_pin(mod):
    a = np.array([-0.75])
    ok = np.array_equal(mod.converged_ritz(a, np.array([0.0])), a)
    ok &= len(mod.converged_ritz(a, np.array([1e-3]))) == 0
    return bool(ok)


def test_two_by_two_closed_form():
    assert _two_by_two_pin(olz)


def test_single_step():
    assert _single_step_pin(olz)


@pytest.mark.parametrize("m", [8, 25, 40])
def test_residuals_match_explicit_vectors(m):
    """beta_m |s_m| equals ||A y - theta y|| for y = V s built from the vectors."""
    rng = np.random.default_rng(11)
    lam = np.sort(rng.uniform(-3.0, 3.0, 60))
    lam[0] = -4.0                      # an isolated lowest eigenvalue
    A = np.diag(lam)
    v0 = rng.standard_normal(60)
    res = olz.lanczos(lambda v: A @ v, v0, m, want_vectors=True)
    assert res["n_done"] == m
    V = np.stack(res["vectors"], 1)
    w, s = np.linalg.eigh(np.diag(res["alpha"]) + np.diag(res["beta"][:m - 1], 1)
                          + np.diag(res["beta"][:m - 1], -1))
    w2, r2 = olz.ritz_residuals(res["alpha"], res["beta"])
    assert np.allclose(w, w2, atol=1e-13)
    for k in range(m):
        y = V @ s[:, k]
        true = np.linalg.norm(A @ y - w[k] * y)
        assert abs(true - r2[k]) < 1e-10, (k, true, r2[k])
    conv = olz.converged_ritz(res["alpha"], res["beta"], resid_tol=1e-8)
    if m == 40:
        # the isolated eigenvalue has converged, to machine precision
        assert len(conv) > 0 and abs(conv[0] - (-4.0)) < 1e-12


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("olz_mutant")
    exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    return mod


MUTANTS = {
    "first_component": ("np.abs(s[m - 1, :])", "np.abs(s[0, :])"),
    "previous_beta": ("abs(beta[m - 1])", "abs(beta[m - 2])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    mod = _mutant(*MUTANTS[name])
    assert not (_two_by_two_pin(mod) and _single_step_pin(mod))
