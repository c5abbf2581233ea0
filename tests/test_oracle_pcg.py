"""Pins of the oracle's preconditioned conjugate gradient (Sec. 6.3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from paper_2307_11648_amd import inputs


def _system(n=300, seed=3):
    x = inputs.uniform_points(n, 3, seed)
    kern = inputs.Kernel(1, 1.0)  # the experiment's kernel: nu = 1/2, l = 1
    th = oracle.covariance(x, kern)
    sol = np.random.default_rng(seed).standard_normal(n)
    return x, kern, th, sol, th @ sol


def test_exact_inverse_cholesky_preconditioner_converges_in_one_step():
    """With L L^T = Theta^{-1} exactly the preconditioned matrix is the
    identity: one iteration."""
    _, _, th, sol, y = _system()
    L = np.linalg.cholesky(np.linalg.inv(th))
    xs, it, res = oracle.pcg(th, y, L, rel_tol=1e-10)
    assert it == 1 and res <= 1e-10
    np.testing.assert_allclose(xs, sol, rtol=1e-6, atol=1e-6 * np.max(np.abs(sol)))


def test_plain_cg_matches_scipy_and_solves():
    _, _, th, sol, y = _system(n=200, seed=5)
    xs, it, res = oracle.pcg(th, y, None, rel_tol=1e-8, max_iter=5000)
    assert res <= 1e-8
    assert np.linalg.norm(y - th @ xs) <= 1e-7 * np.linalg.norm(y)
    count = {"n": 0}

    def cb(_):
        count["n"] += 1

    xr, info = spla.cg(th, y, rtol=1e-8, atol=0.0, maxiter=5000, callback=cb)
    assert info == 0
    assert abs(count["n"] - it) <= 1
    np.testing.assert_allclose(xs, xr, rtol=1e-5, atol=1e-5 * np.max(np.abs(xr)))


def test_factor_preconditioner_matches_scipy_pcg():
    """With the sparse factor of the greedy selection: the same iterate count
    and solution as scipy's cg with M = L L^T, and fewer iterations than
    without the preconditioner."""
    x, kern, th, sol, y = _system(n=400, seed=7)
    xo, _ = inputs.ordered_cloud(x)
    th = oracle.covariance(xo, kern)
    y = th @ sol
    pool, plen = inputs.later_knn_pools(xo, 24)
    f = oracle.select_and_factor(xo, kern, np.arange(len(xo)), pool, plen, 8)
    cp, ri, v = oracle.single_target_csc(len(xo), np.arange(len(xo)), f["sel"], f["factor"])
    L = oracle.dense_factor(len(xo), cp, ri, v)
    xs, it, res = oracle.pcg(th, y, L, rel_tol=1e-10)
    assert res <= 1e-10
    count = {"n": 0}

    def cb(_):
        count["n"] += 1

    M = spla.LinearOperator(th.shape, matvec=lambda r: L @ (L.T @ r))
    xr, info = spla.cg(th, y, rtol=1e-10, atol=0.0, M=M, maxiter=5000, callback=cb)
    assert info == 0 and abs(count["n"] - it) <= 1
    np.testing.assert_allclose(xs, xr, rtol=1e-6, atol=1e-6 * np.max(np.abs(xr)))
    _, it0, _ = oracle.pcg(th, y, None, rel_tol=1e-10, max_iter=20000)
    assert it < it0
