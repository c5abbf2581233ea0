"""Pins of the oracle's global greedy allocation of nonzeros (Sec. 5.4, eq.
global_obj) and of its per-step gains.

* The heap-based allocation equals the allocation taken straight from its
  definition (an argmax scan over all columns per nonzero) on small inputs
  with many ties.
* It equals the threshold rule the GPU computes (steps in decreasing order of
  their column's prefix-minimum gain, ties by column then step), written out
  here independently of both.
* The gains are the squared conditional correlations of dense linear algebra
  (1 - Theta_ii|I,j / Theta_ii|I), and they telescope into the factor's log
  conditional variance: log Theta_ii|s = log Theta_ii + sum log(1 - gain).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_11648_amd import inputs


def _random_gains(rng, T, K, levels):
    g = rng.integers(1, levels + 1, size=(T, K)).astype(np.float64) / levels
    for i in range(T):
        n = int(rng.integers(0, K + 1))
        g[i, n:] = np.nan
    return g


def _threshold_rule(gains, budget):
    """Allocation by the prefix-minimum threshold: sort all steps by
    (prefix-min desc, column asc, step asc) and take the first `budget`."""
    T, K = gains.shape
    keys = []
    for i in range(T):
        run = np.inf
        for t in range(K):
            if np.isnan(gains[i, t]):
                break
            run = min(run, gains[i, t])
            keys.append((-run, i, t))
    keys.sort()
    alloc = np.zeros(T, np.int64)
    for _, i, t in keys[:budget]:
        alloc[i] += 1
    return alloc


@pytest.mark.parametrize("seed", range(40))
def test_heap_equals_naive_and_threshold_rule(seed):
    rng = np.random.default_rng(seed)
    T, K = int(rng.integers(1, 9)), int(rng.integers(1, 7))
    g = _random_gains(rng, T, K, levels=int(rng.integers(1, 5)))
    total = int(np.sum(~np.isnan(g)))
    for budget in sorted({0, 1, total // 2, max(total - 1, 0), total, total + 3}):
        a = oracle.global_allocation(g, budget)
        assert np.array_equal(a, oracle.global_allocation_naive(g, budget)), (g, budget)
        assert np.array_equal(a, _threshold_rule(g, budget)), (g, budget)
        assert int(a.sum()) == min(budget, total)


def _cond_var(th, i, S):
    if len(S) == 0:
        return th[i, i]
    S = list(S)
    return th[i, i] - th[S, i] @ np.linalg.solve(th[np.ix_(S, S)], th[S, i])


def test_gains_are_dense_conditional_correlations_and_telescope():
    w = inputs.workload_plain_fp64(n=300, seed=5)
    th = oracle.covariance(w.points, w.kernel)
    k = 10
    idx = np.arange(0, 280, 13)
    o = oracle.select_and_factor_diag(w.points, w.kernel, w.targets[idx], w.pool[idx], w.pool_len[idx], k)
    g = oracle.step_gains(o["diag"], o["sel"])
    for r, c in enumerate(idx):
        i = int(w.targets[c])
        sel = [int(s) for s in o["sel"][r] if s >= 0]
        for t in range(len(sel)):
            ref = 1.0 - _cond_var(th, i, sel[: t + 1]) / _cond_var(th, i, sel[:t])
            assert g[r, t] == pytest.approx(ref, rel=1e-9, abs=1e-13)
        # telescoping into the column's log conditional variance
        lcv = math.log(th[i, i]) + float(np.sum(np.log1p(-g[r, : len(sel)])))
        assert lcv == pytest.approx(o["log_condvar"][r], rel=1e-9, abs=1e-10)
        assert np.all(np.isnan(g[r, len(sel):]))


def test_allocated_factor_is_the_prefix_column():
    """By prefix consistency the pattern of a column with k_i allocated
    nonzeros is its first k_i greedy picks, and its factor column is the k_i
    selection's: the KL data term falls by the allocated gains."""
    w = inputs.workload_plain_fp64(n=400, seed=8)
    T, K = len(w.targets), 12
    o = oracle.select_and_factor_diag(w.points, w.kernel, w.targets, w.pool, w.pool_len, K)
    g = oracle.step_gains(o["diag"], o["sel"])
    budget = 6 * T
    a = oracle.global_allocation(g, budget)
    assert int(a.sum()) == budget
    S = 0.0
    for c in range(0, T, 17):
        r = oracle.select_one(w.points, w.kernel, int(w.targets[c]), w.pool[c, : w.pool_len[c]], int(a[c]))
        assert np.array_equal(r["sel"], o["sel"][c, : a[c]])
        lcv = math.log(w.kernel.variance + w.kernel.nugget) + float(np.sum(np.log1p(-g[c, : a[c]])))
        assert r["log_condvar"] == pytest.approx(lcv, rel=1e-9, abs=1e-10)
        S += r["log_condvar"]
    assert np.isfinite(S)
