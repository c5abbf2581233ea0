"""FP64 oracle of partial (non-adjacent) aggregated selection (Sec. 5.1 eq.
chol_partial and eq. partial_kl; App. A.3; App. C.3 eq. chol_partial_update,
eq. partial_diag, eq. obj_partial and eq. partial_induct).

TEST INFRASTRUCTURE ONLY (imported by ``tests/``; never by the product
package).  Plain numpy in FP64, written from the paper's definitions; it
shares no code with the HIP library.

Setting.  A group of targets T (ids; points are in ordering-position order, so
a larger id is a later point) selects points one at a time from a pool of
candidates that may lie between the targets: candidate j enters the pattern
s_q of every target q before it (j > q) and of no other, so j conditions only
the targets it follows.  The group's KL term is
    sum_{q in T} log Theta_{qq | s_q \\ q},   s_q = {j in T u S : j >= q}
(eq. partial_kl), the log determinant of the partially conditioned target
covariance.  With the selected and target points sorted by decreasing id,
the Cholesky factor L of Theta over those columns (rows: every target and
candidate) holds it on its diagonal: L_qq^2 = Theta_{qq | s_q \\ q}, because
the columns before q's are exactly the points after q.

One step.  For every candidate j, walking the columns c in order with
v = Theta_{jj | columns before c} (eq. partial_diag: Theta_{cc|:c-1} =
L_cc^2, Theta_{jc|:c-1} = L_jc L_cc):
  * at a target column that j conditions (j > q_c), the target's variance
    conditioned also on j is Theta_{cc|:c-1} - Theta_{jc|:c-1}^2 / v
    (eq. obj_partial), i.e. it falls by the factor 1 - L_jc^2 / v;
  * then v -= L_jc^2 (eq. partial_induct).
The pick maximizes the decrease of the group term, sum -log(1 - L_jc^2 / v)
over the conditioned targets, taken here as the score 1 - prod (1 - L_jc^2 /
v) in [0, 1] (a monotone image; with every target conditioned it is the
multi-target score 1 - Theta_{jj|I,T} / Theta_{jj|I} of eq. greedy_mult).
Eligible: not selected and v > 1e-12 times the prior variance after the last
column (the multi-target rule on Theta_{jj | I, T}).  Ties go to the smaller
pool slot.  The pick is inserted as a column after every column with a
larger id (eq. chol_partial_update); here the factor is then rebuilt by
left-looking over the new column order, its definition (the kernels update
it by a rank-one downdate instead).
"""
from __future__ import annotations

import math

import numpy as np

from . import covariance

STATUS_OK, STATUS_STOPPED, STATUS_NOT_PD, STATUS_BAD = 0, 1, 2, 3


def _factor(K, cols):
    """Left-looking Cholesky of K over the columns `cols` (row indices into K,
    in column order): L[:, c] = (K[:, r_c] - L[:, :c] L[r_c, :c]^T) / sqrt(pivot);
    rows of earlier columns are 0 in later columns.  None if a pivot is not
    positive."""
    R = K.shape[0]
    L = np.zeros((R, len(cols)))
    for c, rc in enumerate(cols):
        v = K[:, rc] - L[:, :c] @ L[rc, :c]
        d = v[rc]
        if not d > 0.0:
            return None
        L[:, c] = v / math.sqrt(d)
        L[cols[:c], c] = 0.0
    return L


def _scores(K, L, cols, ids, is_target, cand_rows, thr):
    """Scores (eq. obj_partial / eq. partial_induct) and eligibility of the
    candidate rows."""
    v = K[cand_rows, cand_rows].copy()
    prod = np.ones(len(cand_rows))
    cid = ids[cand_rows]
    for c, rc in enumerate(cols):
        lc = L[cand_rows, c]
        if is_target[rc]:
            cond = cid > ids[rc]
            with np.errstate(divide="ignore", invalid="ignore"):
                f = np.clip(1.0 - lc * lc / v, 0.0, 1.0)
            prod = np.where(cond & (v > 0.0), prod * f, prod)
        v = v - lc * lc
    score = np.clip(1.0 - prod, 0.0, 1.0)
    return score, v > thr


def _valid(n, members, pool):
    if len(members) == 0 or np.any(members < 0) or np.any(members >= n) or np.any(pool < 0) or np.any(pool >= n):
        return False
    if len(np.unique(members)) != len(members) or len(np.unique(pool)) != len(pool):
        return False
    return not np.any(np.isin(pool, members))


def partial_one(x, kernel, members, pool, k: int, forced=None) -> dict:
    """One group.  Returns the picks (pool ids, selection order), the per-step
    relative top-two gap, the per-step best score and (with `forced`, a
    sequence of pool ids to follow instead of the argmax) the forced pick's
    score, the group term sum_q log Theta_{qq | s_q \\ q} after the picks, the
    per-target conditional variances and the status."""
    x = np.asarray(x, np.float64)
    T = np.asarray(members, np.int64)
    P = np.asarray(pool, np.int64)
    n = x.shape[0]
    m, C = len(T), len(P)
    out = {"sel": np.full(k, -1, np.int32), "gap": np.full(k, np.nan), "best": np.full(k, np.nan),
           "pick": np.full(k, np.nan), "logdet": np.nan, "target_var": np.full(m, np.nan), "status": STATUS_BAD}
    if not _valid(n, T, P):
        return out
    ids = np.concatenate([T, P])
    K = covariance(x[ids], kernel)
    prior = kernel.variance + kernel.nugget
    thr = 1e-12 * prior
    is_target = np.zeros(m + C, bool)
    is_target[:m] = True
    cols = sorted(range(m), key=lambda r: -ids[r])
    L = _factor(K, cols)
    if L is None:
        out["status"] = STATUS_NOT_PD
        return out
    chosen = np.zeros(m + C, bool)
    kk = min(k, C)
    status = STATUS_OK
    for t in range(kk):
        cand = np.array([r for r in range(m, m + C) if not chosen[r]], np.int64)
        score, elig = _scores(K, L, cols, ids, is_target, cand, thr) if len(cand) else (np.zeros(0), np.zeros(0, bool))
        if not np.any(elig):
            if forced is not None and t < len(forced) and forced[t] >= 0:
                status = 5  # a forced pick that is not a valid candidate
            else:
                status = STATUS_STOPPED
            break
        es, ec = score[elig], cand[elig]
        order = np.lexsort((ec, -es))  # score descending, then slot ascending
        best = ec[order[0]]
        out["best"][t] = es[order[0]]
        out["gap"][t] = 1.0 if len(order) == 1 else ((es[order[0]] - es[order[1]]) / es[order[0]]
                                                      if es[order[0]] > 0 else 0.0)
        if forced is not None:
            if t >= len(forced) or forced[t] < 0:
                break
            hit = np.where((ids[ec] == forced[t]))[0]
            if len(hit) == 0:
                status = 5
                break
            best = ec[hit[0]]
            out["pick"][t] = es[hit[0]]
        chosen[best] = True
        out["sel"][t] = ids[best]
        p = sum(1 for rc in cols if ids[rc] > ids[best])
        cols = cols[:p] + [int(best)] + cols[p:]
        L = _factor(K, cols)
        if L is None:
            out["status"] = STATUS_NOT_PD
            return out
    tv = np.array([L[r, cols.index(r)] ** 2 for r in range(m)])
    out["target_var"] = tv
    out["logdet"] = float(np.sum(np.log(tv)))
    out["status"] = status
    return out


def partial_select(x, kernel, group_ptr, members, pool, pool_len, k: int) -> dict:
    """Every group (serial).  sel [G][k], gap [G][k], logdet [G], status [G]."""
    gp = np.asarray(group_ptr, np.int64)
    G = len(gp) - 1
    sel = np.full((G, k), -1, np.int32)
    gap = np.full((G, k), np.nan)
    ld = np.full(G, np.nan)
    st = np.zeros(G, np.uint8)
    for g in range(G):
        r = partial_one(x, kernel, members[gp[g]:gp[g + 1]], pool[g, : pool_len[g]], k)
        sel[g], gap[g], ld[g], st[g] = r["sel"], r["gap"], r["logdet"], r["status"]
    return {"sel": sel, "gap": gap, "logdet": ld, "status": st}


# --------------------------------------------------------------------------
# dense definitions used by the pins
# --------------------------------------------------------------------------
def group_term_dense(x, kernel, members, selected) -> float:
    """sum_{q in T} log Theta_{qq | s_q \\ q} with s_q = {j in T u S : j > q}
    (eq. partial_kl's left side), by dense solves."""
    x = np.asarray(x, np.float64)
    T = [int(q) for q in members]
    S = [int(j) for j in selected if j >= 0]
    pts = sorted(set(T) | set(S))
    K = covariance(x[pts], kernel)
    at = {v: i for i, v in enumerate(pts)}
    tot = 0.0
    for q in T:
        cond = [at[j] for j in pts if j > q]
        i = at[q]
        v = K[i, i]
        if cond:
            v -= K[i, cond] @ np.linalg.solve(K[np.ix_(cond, cond)], K[cond, i])
        tot += math.log(v)
    return tot


def partially_conditioned_cov(x, kernel, members, j) -> np.ndarray:
    """Theta_{TT || j} of eq. chol_partial for one point j: the targets in
    decreasing id order, the first p of them (those after j) unconditioned and
    the rest conditioned on j, as the product of the glued factor
    [L_{:p}; L'_{p+1:}] with L = chol(Theta_TT), L' = chol(Theta_{TT | j})."""
    x = np.asarray(x, np.float64)
    T = sorted((int(q) for q in members), reverse=True)
    pts = T + [int(j)]
    K = covariance(x[pts], kernel)
    m = len(T)
    Ktt = K[:m, :m]
    Kc = Ktt - np.outer(K[:m, m], K[m, :m]) / K[m, m]
    L = np.linalg.cholesky(Ktt)
    Lc = np.linalg.cholesky(Kc)
    p = sum(1 for q in T if q > j)
    G = np.vstack([L[:p], Lc[p:]])
    return G @ G.T
