"""Pins of the partial (non-adjacent) aggregation oracle (Sec. 5.1 eq.
chol_partial, eq. partial_kl; App. A.3; App. C.3).

* eq. partial_kl: the log determinant of the partially conditioned covariance
  built from the glued factor [L_{:p}; L'_{p+1:}] equals the sum of the
  targets' log conditional variances on their own patterns (dense solves).
* Brute force: every step's scores are 1 - exp(-decrease of the dense group
  term), so the greedy pick is the dense argmax; the tracked group term is
  the dense one.
* Reductions: with every candidate after every target the selection is the
  multi-target (adjacent) selection of the C oracle; with one target it is
  the single-target selection.
* Telescoping: the member columns of the aggregated pattern (eq. L_col per
  member, solved on their own by the C oracle) give log conditional
  variances that sum to the group term.
* Candidates before every target condition nothing (score 0); bad inputs get
  status 3.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import partial
from paper_2307_11648_amd import inputs


def _cloud(n, d, seed):
    x = inputs.uniform_points(n, d, seed)
    xo, _ = inputs.ordered_cloud(x)
    return xo


@pytest.mark.parametrize("seed", range(6))
def test_glued_factor_log_det_is_the_partial_kl_term(seed):
    rng = np.random.default_rng(seed)
    x = _cloud(60, 2, 100 + seed)
    kern = inputs.Kernel(int(rng.choice([1, 3, 5])), 0.3, 1.3)
    T = np.sort(rng.choice(60, size=int(rng.integers(2, 7)), replace=False))
    rest = np.setdiff1d(np.arange(60), T)
    for j in rng.choice(rest, size=4, replace=False):
        G = partial.partially_conditioned_cov(x, kern, T, j)
        sign, ld = np.linalg.slogdet(G)
        assert sign > 0
        ref = partial.group_term_dense(x, kern, T, [j])
        assert ld == pytest.approx(ref, rel=1e-10, abs=1e-10)
        # and it is the oracle's tracked term after forcing j
        r = partial.partial_one(x, kern, T, [j], 1, forced=[j])
        if np.any(j > T):
            assert r["logdet"] == pytest.approx(ref, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("seed", range(8))
def test_scores_and_picks_match_dense_brute_force(seed):
    """Tiny groups with candidates interleaved between the targets."""
    rng = np.random.default_rng(seed)
    n = 80
    x = _cloud(n, int(rng.integers(1, 4)), 200 + seed)
    kern = inputs.Kernel(int(rng.choice([1, 3, 5])), 0.25, 1.0, 1e-8)
    T = np.sort(rng.choice(np.arange(10, 60), size=int(rng.integers(2, 6)), replace=False))
    pool = rng.permutation(np.setdiff1d(np.arange(int(T.min()) - 5, n), T))[:14]
    k = 6
    r = partial.partial_one(x, kern, T, pool, k)
    assert r["status"] == 0
    S = []
    for t in range(k):
        base = partial.group_term_dense(x, kern, T, S)
        dense = {}
        for j in pool:
            if j in S:
                continue
            dense[int(j)] = 1.0 - math.exp(partial.group_term_dense(x, kern, T, S + [int(j)]) - base)
        best = max(dense.values())
        # the oracle's pick attains the dense maximum (ties and near-ties aside)
        got = int(r["sel"][t])
        assert dense[got] == pytest.approx(best, rel=1e-8, abs=1e-12)
        assert r["best"][t] == pytest.approx(best, rel=1e-8, abs=1e-12)
        if r["gap"][t] > 1e-6:
            assert got == max(dense, key=lambda j: (dense[j], -list(pool).index(j)))
        S.append(got)
    assert r["logdet"] == pytest.approx(partial.group_term_dense(x, kern, T, S), rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_adjacent_pools_reduce_to_multi_target_selection(seed):
    w = inputs.workload_aggregated(n=3000, seed=20 + seed, C=40, k=10, mmin=2, mmax=6)
    for g in range(0, 30, 3):
        T = w.members[w.group_ptr[g]:w.group_ptr[g + 1]]
        pool = w.pool[g, : w.pool_len[g]]
        assert np.all(pool > T.max())
        a = partial.partial_one(w.points, w.kernel, T, pool, 10)
        b = oracle.multi_one(w.points, w.kernel, T, pool, 10)
        dec = np.where(b["gap"] < 1e-6)[0]
        upto = int(dec[0]) if len(dec) else 10
        assert np.array_equal(a["sel"][:upto], b["sel"][:upto])
        if upto == 10:
            assert a["logdet"] == pytest.approx(b["logdet"], rel=1e-10, abs=1e-10)


def test_single_target_reduces_to_single_target_selection():
    w = inputs.workload_plain_fp64(n=400, seed=11)
    for c in range(0, 380, 37):
        pool = w.pool[c, : w.pool_len[c]]
        a = partial.partial_one(w.points, w.kernel, [w.targets[c]], pool, 8)
        b = oracle.select_one(w.points, w.kernel, int(w.targets[c]), pool, 8)
        assert np.array_equal(a["sel"][: len(b["sel"])], b["sel"])
        assert a["logdet"] == pytest.approx(b["log_condvar"], rel=1e-10, abs=1e-10)


def test_member_columns_telescope_to_the_group_term():
    x = _cloud(400, 2, 7)
    kern = inputs.Kernel(3, 0.1, 1.0, 1e-9)
    rng = np.random.default_rng(3)
    for _ in range(5):
        T = np.sort(rng.choice(np.arange(50, 300), size=8, replace=False))
        pool = rng.permutation(np.setdiff1d(np.arange(int(T.min()) + 1, 400), T))[:60]
        r = partial.partial_one(x, kern, T, pool, 12)
        cols = oracle.aggregated_columns(x, kern, T, r["sel"])
        assert np.all(cols["member_status"] == 0)
        assert float(np.sum(cols["member_log_condvar"])) == pytest.approx(r["logdet"], rel=1e-9, abs=1e-9)
        # each target's factor diagonal is its tracked conditional variance
        np.testing.assert_allclose(np.exp(cols["member_log_condvar"]), r["target_var"], rtol=1e-9)


def test_candidates_before_every_target_are_never_useful():
    x = _cloud(200, 2, 9)
    kern = inputs.Kernel(1, 0.2)
    T = np.array([120, 140, 150])
    early = np.arange(0, 100, 7)
    late = np.array([160, 170, 130])
    r = partial.partial_one(x, kern, T, np.concatenate([early, late]), 3)
    assert set(r["sel"].tolist()) == set(late.tolist())
    # only early candidates: every score is 0, picks by slot order
    r2 = partial.partial_one(x, kern, T, early, 2)
    assert np.all(r2["best"][:2] == 0.0)
    assert list(r2["sel"]) == [early[0], early[1]]


def test_bad_inputs():
    x = _cloud(50, 2, 1)
    kern = inputs.Kernel(3, 0.2)
    assert partial.partial_one(x, kern, [10, 20], [30, 20], 2)["status"] == 3   # pool holds a target
    assert partial.partial_one(x, kern, [10, 20], [30, 30], 2)["status"] == 3   # repeated candidate
    assert partial.partial_one(x, kern, [10, 60], [30], 1)["status"] == 3       # target out of range
    assert partial.partial_one(x, kern, [], [30], 1)["status"] == 3             # empty group
