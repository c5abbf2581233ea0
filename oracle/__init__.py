"""FP64 CPU oracle of the greedy conditional-selection hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP library.  ``oracle.c`` holds the method in plain
loops (selection, eq. L_col entries, multi-target selection, aggregated
columns, factor products); this module adds ctypes marshalling and the dense
numpy quantities (log-determinant and KL of eq. kl / eq. obj_chol).

Kernel arguments are duck-typed: anything with ``two_nu``, ``length_scale``,
``variance`` and ``nugget`` attributes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)
_c = ctypes


def build() -> str:
    """Compile oracle.c with gcc (FP64, OpenMP over columns only)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_matern.argtypes = [_c.c_int, _c.c_double, _c.c_double, _c.c_double]
    lib.orc_matern.restype = _c.c_double
    kern = [_c.c_int32, _c.c_double, _c.c_double, _c.c_double]
    lib.orc_select_one.argtypes = [_f64p, _c.c_int32] + kern + [_c.c_int32, _i32p, _c.c_int32, _c.c_int32, _i32p,
                                                               _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_select_one.restype = _c.c_int
    lib.orc_select_and_factor.argtypes = [_f64p, _c.c_int32] + kern + [_c.c_int64, _i32p, _i32p, _i32p, _c.c_int32,
                                                                      _c.c_int32, _i32p, _f64p, _f64p, _f64p, _u8p,
                                                                      _c.c_int32]
    lib.orc_select_and_factor.restype = None
    lib.orc_select_and_factor_diag.argtypes = [_f64p, _c.c_int32] + kern + [_c.c_int64, _i32p, _i32p, _i32p,
                                                                           _c.c_int32, _c.c_int32, _i32p, _f64p,
                                                                           _f64p, _f64p, _u8p, _f64p, _c.c_int32]
    lib.orc_select_and_factor_diag.restype = None
    lib.orc_replay_one.argtypes = [_f64p, _c.c_int32] + kern + [_c.c_int32, _i32p, _c.c_int32, _c.c_int32, _i32p,
                                                               _f64p, _f64p, _f64p, _f64p]
    lib.orc_replay_one.restype = _c.c_int
    lib.orc_multi_one.argtypes = [_f64p, _c.c_int32] + kern + [_i32p, _c.c_int32, _i32p, _c.c_int32, _c.c_int32,
                                                              _i32p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_multi_one.restype = _c.c_int
    lib.orc_multi_replay_one.argtypes = [_f64p, _c.c_int32] + kern + [_i32p, _c.c_int32, _i32p, _c.c_int32,
                                                                     _c.c_int32, _i32p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_multi_replay_one.restype = _c.c_int
    lib.orc_aggregated_one.argtypes = [_f64p, _c.c_int32] + kern + [_i32p, _c.c_int32, _i32p, _c.c_int32, _i32p,
                                                                   _f64p, _f64p, _u8p]
    lib.orc_aggregated_one.restype = _c.c_int64
    lib.orc_aggregated_select.argtypes = [_f64p, _c.c_int32] + kern + [_c.c_int64, _i32p, _i32p, _i32p, _i32p,
                                                                      _c.c_int32, _c.c_int32, _i32p, _f64p, _f64p,
                                                                      _f64p, _i64p, _i32p, _f64p, _f64p, _u8p,
                                                                      _c.c_int32]
    lib.orc_aggregated_select.restype = None
    lib.orc_apply_factor.argtypes = [_c.c_int64, _i64p, _i32p, _f64p, _c.c_int32, _f64p, _f64p]
    lib.orc_apply_factor.restype = None
    lib.orc_covariance.argtypes = [_f64p, _c.c_int32, _c.c_int32] + kern + [_f64p]
    lib.orc_covariance.restype = None
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _kargs(kernel):
    return (int(kernel.two_nu), float(kernel.length_scale), float(kernel.variance), float(kernel.nugget))


def _pts(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    return x


# --------------------------------------------------------------------------
# kernel and dense covariance
# --------------------------------------------------------------------------
def matern(two_nu: int, ell: float, s2: float, r: float) -> float:
    return _load().orc_matern(two_nu, ell, s2, r)


def covariance(x, kernel) -> np.ndarray:
    """Dense Theta for small point sets (n x n, FP64)."""
    x = _pts(x)
    n, d = x.shape
    out = np.empty((n, n), np.float64)
    _load().orc_covariance(_p(x, _f64p), n, d, *_kargs(kernel), _p(out, _f64p))
    return out


# --------------------------------------------------------------------------
# single-target selection + eq. L_col
# --------------------------------------------------------------------------
def select_one(x, kernel, target: int, pool, k: int) -> dict:
    """One column: greedy selection over ``pool`` and its factor column."""
    x = _pts(x)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    C = len(pool)
    sel = np.empty(max(k, 1), np.int32)
    gap = np.empty(max(k, 1), np.float64)
    fac = np.empty(k + 1, np.float64)
    lcv = np.empty(1, np.float64)
    var = np.empty(max(C, 1), np.float64)
    cov = np.empty(max(C, 1), np.float64)
    st = _load().orc_select_one(_p(x, _f64p), x.shape[1], *_kargs(kernel), int(target), _p(pool, _i32p), C, k,
                                _p(sel, _i32p), _p(gap, _f64p), _p(fac, _f64p), _p(lcv, _f64p), _p(var, _f64p),
                                _p(cov, _f64p))
    return {"sel": sel[:k], "gap": gap[:k], "factor": fac, "log_condvar": float(lcv[0]), "var": var[:C],
            "cov": cov[:C], "status": int(st)}


def replay_one(x, kernel, target: int, pool, k: int, forced) -> dict:
    """Replay another run's selection sequence ``forced`` (ids, -1 padded) in
    FP64: per step the best valid score, the forced pick's score and the
    target's conditional variance before the step, and the eq. L_col column on
    [target, forced...].  Status 5: a forced pick was not
    a valid candidate."""
    x = _pts(x)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    forced = np.ascontiguousarray(forced, dtype=np.int32)
    best = np.empty(max(2 * k, 1), np.float64)
    pick = np.empty(max(k, 1), np.float64)
    fac = np.empty(k + 1, np.float64)
    lcv = np.empty(1, np.float64)
    st = _load().orc_replay_one(_p(x, _f64p), x.shape[1], *_kargs(kernel), int(target), _p(pool, _i32p), len(pool),
                                k, _p(forced, _i32p), _p(best, _f64p), _p(pick, _f64p), _p(fac, _f64p),
                                _p(lcv, _f64p))
    return {"best": best[:k], "pick": pick[:k], "target_var": best[k:2 * k], "factor": fac,
            "log_condvar": float(lcv[0]), "status": int(st)}


def select_and_factor(x, kernel, targets, pool, pool_len, k: int, nthreads: int = 0) -> dict:
    """All columns (OpenMP over columns).  Same output layout as the library:
    sel [T, k] (-1 padded), factor [T, k+1] ([0] = L_ii), log_condvar [T],
    gap [T, k], status [T]."""
    x = _pts(x)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    pool_len = np.ascontiguousarray(pool_len, dtype=np.int32)
    T = len(targets)
    stride = pool.shape[1] if pool.ndim == 2 else 0
    sel = np.empty((T, k), np.int32)
    gap = np.empty((T, k), np.float64)
    fac = np.empty((T, k + 1), np.float64)
    lcv = np.empty(T, np.float64)
    st = np.empty(T, np.uint8)
    _load().orc_select_and_factor(_p(x, _f64p), x.shape[1], *_kargs(kernel), T, _p(targets, _i32p),
                                  _p(pool, _i32p), _p(pool_len, _i32p), stride, k, _p(sel, _i32p), _p(gap, _f64p),
                                  _p(fac, _f64p), _p(lcv, _f64p), _p(st, _u8p), int(nthreads))
    return {"sel": sel, "gap": gap, "factor": fac, "log_condvar": lcv, "status": st}


def select_and_factor_diag(x, kernel, targets, pool, pool_len, k: int, nthreads: int = 0) -> dict:
    """select_and_factor plus, per column and step, the tracked FP64 state
    before the pick: diag [T, k, 5] = (var, cov) of the best candidate, (var,
    cov) of the second best (NaN where there is none), and the target's
    conditional variance."""
    x = _pts(x)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    pool_len = np.ascontiguousarray(pool_len, dtype=np.int32)
    T = len(targets)
    stride = pool.shape[1] if pool.ndim == 2 else 0
    sel = np.empty((T, k), np.int32)
    gap = np.empty((T, k), np.float64)
    fac = np.empty((T, k + 1), np.float64)
    lcv = np.empty(T, np.float64)
    st = np.empty(T, np.uint8)
    diag = np.empty((T, max(k, 1), 5), np.float64)
    _load().orc_select_and_factor_diag(_p(x, _f64p), x.shape[1], *_kargs(kernel), T, _p(targets, _i32p),
                                       _p(pool, _i32p), _p(pool_len, _i32p), stride, k, _p(sel, _i32p),
                                       _p(gap, _f64p), _p(fac, _f64p), _p(lcv, _f64p), _p(st, _u8p), _p(diag, _f64p),
                                       int(nthreads))
    return {"sel": sel, "gap": gap, "factor": fac, "log_condvar": lcv, "status": st, "diag": diag[:, :k]}


# --------------------------------------------------------------------------
# global greedy allocation of nonzeros (Sec. 5.4, eq. global_obj)
# --------------------------------------------------------------------------
def step_gains(diag, sel):
    """Per column and step, the fraction of the target's conditional variance
    that the greedy pick removes: its score cov^2/var (eq. obj_gp) over the
    target's conditional variance before the step -- the squared conditional
    correlation of eq. global_obj.  NaN past the column's picks."""
    diag = np.asarray(diag, np.float64)
    g = diag[..., 1] ** 2 / diag[..., 0] / diag[..., 4]
    return np.where(np.asarray(sel) >= 0, g, np.nan)


def global_allocation(gains, budget: int) -> np.ndarray:
    """Global greedy allocation with an array-backed binary heap, as Sec. 5.4
    describes: the queue holds each column's next greedy step keyed by its
    gain; the largest is removed (equal gains: the smaller column) and the
    column's following step, if any, is inserted, `budget` times.  Returns the
    nonzeros per column.  gains [T, k] with NaN past each column's picks."""
    import heapq

    gains = np.asarray(gains, np.float64)
    T, K = gains.shape
    npick = np.array([int(np.sum(~np.isnan(gains[i]))) for i in range(T)])
    alloc = np.zeros(T, np.int64)
    heap = [(-gains[i, 0], i) for i in range(T) if npick[i] > 0]
    heapq.heapify(heap)
    for _ in range(int(budget)):
        if not heap:
            break
        _, i = heapq.heappop(heap)
        alloc[i] += 1
        if alloc[i] < npick[i]:
            heapq.heappush(heap, (-gains[i, alloc[i]], i))
    return alloc


def global_allocation_naive(gains, budget: int) -> np.ndarray:
    """The same allocation straight from its definition, for small inputs:
    each of the `budget` nonzeros goes to the column whose next step has the
    largest gain (a scan over all columns; the first column wins a tie)."""
    gains = np.asarray(gains, np.float64)
    T, K = gains.shape
    alloc = np.zeros(T, np.int64)
    for _ in range(int(budget)):
        best, bi = -np.inf, -1
        for i in range(T):
            t = alloc[i]
            if t < K and not np.isnan(gains[i, t]) and gains[i, t] > best:
                best, bi = gains[i, t], i
        if bi < 0:
            break
        alloc[bi] += 1
    return alloc


# --------------------------------------------------------------------------
# multi-target / aggregated
# --------------------------------------------------------------------------
def multi_one(x, kernel, members, pool, k: int) -> dict:
    """One group: multi-target selection with the two partial factors."""
    x = _pts(x)
    T = np.ascontiguousarray(members, dtype=np.int32)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    m, C = len(T), len(pool)
    sel = np.empty(max(k, 1), np.int32)
    gap = np.empty(max(k, 1), np.float64)
    ld = np.empty(1, np.float64)
    pv = np.empty(m, np.float64)
    v1 = np.empty(m, np.float64)
    st = _load().orc_multi_one(_p(x, _f64p), x.shape[1], *_kargs(kernel), _p(T, _i32p), m, _p(pool, _i32p), C, k,
                               _p(sel, _i32p), _p(gap, _f64p), _p(ld, _f64p), _p(pv, _f64p), _p(v1, _f64p))
    return {"sel": sel[:k], "gap": gap[:k], "logdet": float(ld[0]), "post_var": pv, "var1_targets": v1,
            "status": int(st)}


def multi_replay_one(x, kernel, members, pool, k: int, forced) -> dict:
    """Replay a multi-target selection sequence in FP64: per step the best
    valid score and the forced pick's score (1 - var2/var1), the log det of
    the targets' conditional covariance and the posterior variances after the
    forced sequence.  Status 5: a forced pick was not a valid candidate."""
    x = _pts(x)
    T = np.ascontiguousarray(members, dtype=np.int32)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    forced = np.ascontiguousarray(forced, dtype=np.int32)
    m = len(T)
    best = np.empty(max(k, 1), np.float64)
    pick = np.empty(max(k, 1), np.float64)
    ld = np.empty(1, np.float64)
    pv = np.empty(m, np.float64)
    st = _load().orc_multi_replay_one(_p(x, _f64p), x.shape[1], *_kargs(kernel), _p(T, _i32p), m, _p(pool, _i32p),
                                      len(pool), k, _p(forced, _i32p), _p(best, _f64p), _p(pick, _f64p),
                                      _p(ld, _f64p), _p(pv, _f64p))
    return {"best": best[:k], "pick": pick[:k], "logdet": float(ld[0]), "post_var": pv, "status": int(st)}


def aggregated_columns(x, kernel, members, sel) -> dict:
    """Member columns of an aggregated pattern (eq. L_col per member on
    s_q = {j in sort(T u sel) : j >= q}), each solved on its own."""
    x = _pts(x)
    T = np.ascontiguousarray(members, dtype=np.int32)
    sel = np.ascontiguousarray([s for s in sel if s >= 0], dtype=np.int32)
    m, ns = len(T), len(sel)
    tot = sum(m - a + ns for a in range(m))
    rows = np.empty(max(tot, 1), np.int32)
    vals = np.empty(max(tot, 1), np.float64)
    lcv = np.empty(m, np.float64)
    mst = np.empty(m, np.uint8)
    w = _load().orc_aggregated_one(_p(x, _f64p), x.shape[1], *_kargs(kernel), _p(T, _i32p), m, _p(sel, _i32p), ns,
                                   _p(rows, _i32p), _p(vals, _f64p), _p(lcv, _f64p), _p(mst, _u8p))
    return {"rows": rows[:w], "vals": vals[:w], "member_log_condvar": lcv, "member_status": mst}


def aggregated_select(x, kernel, group_ptr, members, pool, pool_len, k: int, want_factor: bool = True,
                      want_post_var: bool = False, nthreads: int = 0) -> dict:
    """All groups (OpenMP over groups).  Member a of a group with m members and
    n_sel selections owns m - a + n_sel values at val_ptr."""
    x = _pts(x)
    gp = np.ascontiguousarray(group_ptr, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    plen = np.ascontiguousarray(pool_len, dtype=np.int32)
    G = len(gp) - 1
    stride = pool.shape[1]
    sel = np.empty((G, k), np.int32)
    gap = np.empty((G, k), np.float64)
    ld = np.empty(G, np.float64)
    st = np.empty(G, np.uint8)
    pv = np.empty(len(mem), np.float64) if want_post_var else None
    out = {"sel": sel, "gap": gap, "logdet": ld, "status": st}
    vp = rows = vals = lcv = None
    if want_factor:
        vp = aggregated_val_ptr(gp, plen, k)
        rows = np.empty(max(int(vp[-1]), 1), np.int32)
        vals = np.empty(max(int(vp[-1]), 1), np.float64)
        lcv = np.empty(len(mem), np.float64)
    _load().orc_aggregated_select(_p(x, _f64p), x.shape[1], *_kargs(kernel), G, _p(gp, _i32p), _p(mem, _i32p),
                                  _p(pool, _i32p), _p(plen, _i32p), stride, k, _p(sel, _i32p), _p(gap, _f64p),
                                  _p(ld, _f64p), _p(pv, _f64p), _p(vp, _i64p), _p(rows, _i32p), _p(vals, _f64p),
                                  _p(lcv, _f64p), _p(st, _u8p), int(nthreads))
    if want_factor:
        out.update(val_ptr=vp, rows=rows, vals=vals, member_log_condvar=lcv)
    if want_post_var:
        out["post_var"] = pv
    return out


def aggregated_val_ptr(group_ptr, pool_len, k: int) -> np.ndarray:
    """Offsets of the member columns, assuming min(k, pool_len) selections."""
    gp = np.asarray(group_ptr, np.int64)
    plen = np.asarray(pool_len, np.int64)
    sizes = []
    for g in range(len(gp) - 1):
        m = gp[g + 1] - gp[g]
        ns = min(k, plen[g])
        sizes.extend(m - a + ns for a in range(m))
    vp = np.zeros(len(sizes) + 1, np.int64)
    vp[1:] = np.cumsum(sizes)
    return vp


# --------------------------------------------------------------------------
# factor products and KL
# --------------------------------------------------------------------------
def apply_factor(col_ptr, row_idx, val, xin, transpose: bool) -> np.ndarray:
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(row_idx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xin = np.ascontiguousarray(xin, dtype=np.float64)
    n = len(cp) - 1
    y = np.empty(n, np.float64)
    _load().orc_apply_factor(n, _p(cp, _i64p), _p(ri, _i32p), _p(v, _f64p), int(bool(transpose)), _p(xin, _f64p),
                             _p(y, _f64p))
    return y


def single_target_csc(n: int, targets, sel, factor):
    """CSC arrays of the sparse factor from single-target outputs: column i
    holds i first, then its selections in selection order."""
    targets = np.asarray(targets)
    cols = [[] for _ in range(n)]
    for t, i in enumerate(targets):
        rows = [int(i)] + [int(s) for s in sel[t] if s >= 0]
        cols[int(i)] = list(zip(rows, factor[t][: len(rows)]))
    cp = np.zeros(n + 1, np.int64)
    cp[1:] = np.cumsum([len(c) for c in cols])
    ri = np.array([r for c in cols for r, _ in c], np.int32)
    v = np.array([w for c in cols for _, w in c], np.float64)
    return cp, ri, v


def pcg(theta, y, L=None, rel_tol: float = 1e-12, max_iter: int = 1000, x0=None):
    """The preconditioned conjugate gradient for Theta x = y with the
    preconditioner z = L (L^T r) (L L^T ~ Theta^{-1}, Sec. 6.3), textbook
    form, dense FP64 numpy; L None is the plain conjugate gradient.  Stops
    when the recurred residual's norm is at most rel_tol ||y||.  Returns (x,
    iterations, relative residual)."""
    theta = np.asarray(theta, np.float64)
    y = np.asarray(y, np.float64)
    x = np.zeros_like(y) if x0 is None else np.array(x0, np.float64)
    r = y - theta @ x
    ynorm = float(np.linalg.norm(y))

    def prec(v):
        return v.copy() if L is None else L @ (L.T @ v)

    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    res = float(np.linalg.norm(r)) / ynorm if ynorm > 0 else 0.0
    it = 0
    while it < max_iter and res > rel_tol:
        q = theta @ p
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = prec(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        res = float(np.linalg.norm(r)) / ynorm
    return x, it, res


def dense_factor(n, col_ptr, row_idx, val):
    """The dense n x n matrix of a factor in CSC form (entries with a row
    outside [0, n) are padding)."""
    L = np.zeros((n, n))
    for j in range(n):
        for q in range(int(col_ptr[j]), int(col_ptr[j + 1])):
            r = int(row_idx[q])
            if 0 <= r < n:
                L[r, j] += val[q]
    return L


def logdet(theta: np.ndarray) -> float:
    """log det of an SPD matrix by dense Cholesky (numpy)."""
    return float(2.0 * np.sum(np.log(np.diag(np.linalg.cholesky(theta)))))


def kl_from_log_condvar(log_condvar, logdet_theta: float) -> float:
    """KL of eq. obj_chol: 2 KL = sum_i log Theta_{ii|s_i \\ i} - log det Theta."""
    return 0.5 * (float(np.sum(log_condvar)) - logdet_theta)


def kl_dense(theta: np.ndarray, L: np.ndarray) -> float:
    """KL of eq. kl between N(0, Theta) and N(0, (L L^T)^{-1}), dense."""
    n = theta.shape[0]
    tr = float(np.trace(L.T @ theta @ L))
    ld_p = 2.0 * float(np.sum(np.log(np.abs(np.diag(L)))))
    return 0.5 * (tr - ld_p - logdet(theta) - n)
