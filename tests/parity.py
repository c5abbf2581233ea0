"""Parity helpers: compare GPU outputs with the FP64 oracle.

Where several greedy runs are correct (near-ties), only what is unique is
compared: the selection must agree on every decisive step (oracle top-two
relative gap above a threshold) up to the first non-decisive step of that
column; factor values are compared on columns whose whole selection agrees.
"""
from __future__ import annotations

import math

import numpy as np


def decisive_prefix(gap_row, thr):
    """Number of leading steps whose oracle top-two gap exceeds thr."""
    g = np.asarray(gap_row, dtype=np.float64)
    bad = np.where(~(g > thr))[0]
    return len(g) if len(bad) == 0 else int(bad[0])


def compare_single(gpu: dict, orc: dict, thr: float, factor_rtol: float, logcv_atol: float):
    """Returns a report dict; raises AssertionError on a parity violation.

    gpu/orc: numpy dicts with sel [T,k], factor [T,k+1], log_condvar [T],
    status [T]; orc also has gap [T,k] (float64, NaN padded)."""
    T, k = orc["sel"].shape
    assert gpu["sel"].shape == (T, k)
    np.testing.assert_array_equal(gpu["status"], orc["status"])
    n_match = n_decisive = 0
    worst_fac = 0.0
    worst_lcv = 0.0
    mismatched = []
    for t in range(T):
        if orc["status"][t] >= 2:
            continue
        p = decisive_prefix(orc["gap"][t], thr)
        # compare the decisive prefix; the step at p itself may go either way
        if not np.array_equal(gpu["sel"][t, :p], orc["sel"][t, :p]):
            raise AssertionError(f"column {t}: decisive selection differs\n gpu {gpu['sel'][t]}\n orc {orc['sel'][t]}"
                                 f"\n gap {orc['gap'][t]}")
        nsel = int(np.sum(orc["sel"][t] >= 0))
        if p >= nsel:
            n_decisive += 1
        if np.array_equal(gpu["sel"][t], orc["sel"][t]):
            n_match += 1
            a = gpu["factor"][t, : nsel + 1]
            b = orc["factor"][t, : nsel + 1]
            e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
            worst_fac = max(worst_fac, e)
            worst_lcv = max(worst_lcv, abs(float(gpu["log_condvar"][t]) - float(orc["log_condvar"][t])))
        else:
            mismatched.append(t)
    assert worst_fac <= factor_rtol, f"factor column error {worst_fac:.3e} > {factor_rtol:.1e}"
    assert worst_lcv <= logcv_atol, f"log condvar error {worst_lcv:.3e} > {logcv_atol:.1e}"
    return {"columns": T, "identical": n_match, "fully_decisive": n_decisive, "worst_factor_rel": worst_fac,
            "worst_logcv_abs": worst_lcv, "mismatched": mismatched}


def kl_rel_error(S_gpu: float, S_orc: float, logdet: float) -> float:
    """Relative error of KL = (S - logdet)/2 given the two data terms S."""
    kl = 0.5 * (S_orc - logdet)
    return abs(0.5 * (S_gpu - S_orc)) / abs(kl)


def replay_check(gpu: dict, points, kernel, targets, pool, pool_len, k, cols, tau: float, factor_rtol: float):
    """Replay the GPU's own selection of each column in ``cols`` in FP64.

    Every GPU pick must be a valid candidate whose exact score (the decrease
    of the target's conditional variance it brings, eq. obj_gp) falls short of
    the best exact score by at most tau times the target's current
    conditional variance -- i.e. each step loses at most a fraction tau of
    the variance, so log Theta_ii|s moves by at most ~tau per step -- and the
    GPU's factor column must equal eq. L_col on its own selected set.  Returns
    the largest normalised shortfall seen and the worst factor error."""
    import oracle

    worst_short = 0.0
    worst_fac = 0.0
    for t in cols:
        sel = gpu["sel"][t]
        r = oracle.replay_one(points, kernel, int(targets[t]), pool[t, : pool_len[t]], k, sel)
        assert r["status"] != 5, f"column {t}: a GPU pick is not a valid candidate"
        n = int(np.sum(sel >= 0))
        for s in range(n):
            short = (r["best"][s] - r["pick"][s]) / r["target_var"][s]
            worst_short = max(worst_short, short)
            assert short <= tau, (f"column {t} step {s}: pick score {r['pick'][s]} vs best {r['best'][s]}, "
                                  f"target variance {r['target_var'][s]}")
        a = gpu["factor"][t, : n + 1]
        b = r["factor"][: n + 1]
        e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        worst_fac = max(worst_fac, e)
        assert e <= factor_rtol, f"column {t}: factor error {e:.3e} on its own selected set"
    return worst_short, worst_fac


# FP32 unit roundoff
U32 = 2.0 ** -24


def mixed_decisive_prefix(diag_row, prior: float, k: int) -> int:
    """Number of leading steps of a column whose pick an FP32 evaluation and
    GEMV (the mixed-precision kernel) cannot flip, by a first-order error
    model of the FP64 oracle's own run on the same pool.

    diag_row [k, 5]: per step, the tracked (var, cov) of the best and of the
    second-best candidate (oracle.select_and_factor_diag).  The model:

    * the FP32 column of pick s has an absolute error per row of at most
      e_s = (s + 9) u32 prior / sqrt(var_pick_s): the evaluation (a few
      roundings of a value <= prior), an s-term GEMV whose terms sum to at
      most prior in magnitude (Cauchy-Schwarz on the factor rows), and the
      scaling by the pick's 1/sqrt(var);
    * a downdate adds u_s * (error of u_s) to a tracked variance or
      covariance; as sum_s u_s^2 <= prior for every row (the downdates never
      exceed the prior), Cauchy-Schwarz bounds the accumulated error by
      sqrt(prior) * sqrt(sum_s e_s^2); with the initial FP32 covariances and
      the target row's share this gives, for every tracked value,
      E_t = 8 u32 prior + 4 sqrt(prior) sqrt(sum_{s<t} e_s^2);
    * a score s = cov^2 / var then moves by at most s (E_t (2/|cov| + 1/var)
      + 8 u32) (the last term: the FP32 score and its key).

    A step is decisive when s1 - s2 exceeds twice the two scores' bounds; the
    prefix ends at the first step that is not (there either pick is valid, and
    the paths may part)."""
    e2 = 0.0
    for t in range(k):
        v1, c1, v2, c2 = (float(a) for a in diag_row[t][:4])
        if not np.isfinite(v1):
            return t  # no candidate: the run stopped
        E = 8.0 * U32 * prior + 4.0 * math.sqrt(prior * e2)
        if np.isfinite(v2):
            s1 = c1 * c1 / v1
            s2 = c2 * c2 / v2
            d1 = s1 * (E * (2.0 / max(abs(c1), 1e-300) + 1.0 / v1) + 8.0 * U32)
            d2 = s2 * (E * (2.0 / max(abs(c2), 1e-300) + 1.0 / v2) + 8.0 * U32)
            if not (s1 - s2 > 2.0 * (d1 + d2)):
                return t
        e2 += ((t + 9) * U32 * prior / math.sqrt(v1)) ** 2
    return k


def mixed_decisive_check(gpu_sel, orc: dict, prior: float, k: int):
    """Assert that the mixed GPU run picks exactly the oracle's candidates on
    every step of each column's decisive prefix (mixed_decisive_prefix).
    Returns (decisive steps, all steps, the largest oracle relative gap at a
    step where the paths parted)."""
    dec = tot = 0
    worst_gap = 0.0
    for t in range(len(gpu_sel)):
        if orc["status"][t] >= 2:
            continue
        n = int(np.sum(orc["sel"][t] >= 0))
        p = mixed_decisive_prefix(orc["diag"][t], prior, k)
        p = min(p, n)
        if not np.array_equal(gpu_sel[t, :p], orc["sel"][t, :p]):
            s = int(np.where(gpu_sel[t, :p] != orc["sel"][t, :p])[0][0])
            raise AssertionError(f"column {t}: mixed pick {s} differs on a decisive step (oracle gap "
                                 f"{orc['gap'][t][s]:.3e})\n gpu {gpu_sel[t]}\n orc {orc['sel'][t]}")
        dec += p
        tot += n
        diff = np.where(gpu_sel[t, :n] != orc["sel"][t, :n])[0]
        if len(diff):
            worst_gap = max(worst_gap, float(orc["gap"][t][diff[0]]))
    return dec, tot, worst_gap
