"""Seeded synthetic inputs for the selection hot path.

This module builds what the method consumes and nothing more: point clouds,
the reverse-maximin ordering (Sec. 2.2, eq. maximin), candidate pools of
nearest later-ordered points (Sec. 4), supernode groups (Sec. 5.3, grouping by
length scale with lambda = 1.5) and GP prediction batches.  It evaluates no
covariance and takes no selection decision, so it serves the GPU path and the
CPU oracle alike.  The heavy geometry runs in ``geometry.c`` (kd-trees), built
by ``paper_2307_11648_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcsel_geometry.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is not built; run paper_2307_11648_amd.build.build_all() first")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.csel_geo_reverse_maximin.argtypes = [_f64p, ctypes.c_int32, ctypes.c_int32, _i32p, _f64p]
    lib.csel_geo_reverse_maximin.restype = ctypes.c_int
    lib.csel_geo_later_knn.argtypes = [_f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
    lib.csel_geo_later_knn.restype = ctypes.c_int
    lib.csel_geo_later_knn_subset.argtypes = [_f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.csel_geo_later_knn_subset.restype = ctypes.c_int
    lib.csel_geo_make_groups.argtypes = [_f64p, _f64p, ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.c_int32,
                                         ctypes.c_double, _i32p, _i32p]
    lib.csel_geo_make_groups.restype = ctypes.c_int32
    lib.csel_geo_group_pools.argtypes = [_f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         _i32p, _i32p]
    lib.csel_geo_group_pools.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


# --------------------------------------------------------------------------
# point clouds
# --------------------------------------------------------------------------
def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [0,1]^d, row-major (n, d) float64."""
    return np.random.default_rng(seed).random((n, d))


def cluster_points(n: int, d: int, seed: int, n_clusters: int = 20, sigma: float = 0.03,
                   background: float = 0.2) -> np.ndarray:
    """Mixture of isotropic Gaussian clusters plus a uniform background.

    Centres are uniform in [0.1, 0.9]^d with equal weights; cluster points that
    fall outside the unit cube are redrawn so every point lies in [0,1]^d."""
    rng = np.random.default_rng(seed)
    centres = 0.1 + 0.8 * rng.random((n_clusters, d))
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    lab = rng.integers(0, n_clusters, size=n_cl)
    pts = centres[lab] + sigma * rng.standard_normal((n_cl, d))
    bad = np.any((pts < 0) | (pts > 1), axis=1)
    while bad.any():
        pts[bad] = centres[lab[bad]] + sigma * rng.standard_normal((int(bad.sum()), d))
        bad = np.any((pts < 0) | (pts > 1), axis=1)
    allp = np.concatenate([pts, rng.random((n_bg, d))], axis=0)
    return allp[rng.permutation(n)]


# --------------------------------------------------------------------------
# ordering and candidate sets
# --------------------------------------------------------------------------
def reverse_maximin(x: np.ndarray):
    """Reverse-maximin ordering (eq. maximin with p = 1).

    Returns (order, ell): order[pos] is the original id at ordering position
    pos, ell[pos] its distance to every later point (inf for the last).  The
    last point is point 0 and ties go to the smaller id."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    order = np.empty(n, np.int32)
    ell = np.empty(n, np.float64)
    rc = _load().csel_geo_reverse_maximin(_p(x, _f64p), n, d, _p(order, _i32p), _p(ell, _f64p))
    if rc != 0:
        raise ValueError("reverse_maximin: bad arguments")
    return order, ell


def later_knn_pools(x_ordered: np.ndarray, C: int):
    """pool[i] = the C nearest points with ordering position > i, ascending by
    (distance, position); pool_len[i] = min(C, n-1-i); pad -1."""
    x = np.ascontiguousarray(x_ordered, dtype=np.float64)
    n, d = x.shape
    pool = np.empty((n, C), np.int32)
    plen = np.empty(n, np.int32)
    rc = _load().csel_geo_later_knn(_p(x, _f64p), n, d, C, _p(pool, _i32p), _p(plen, _i32p))
    if rc != 0:
        raise ValueError("later_knn_pools: bad arguments")
    return pool, plen


def later_knn_pools_subset(x_ordered: np.ndarray, C: int, positions):
    """later_knn_pools for the given ordering positions only (rows follow
    `positions`)."""
    x = np.ascontiguousarray(x_ordered, dtype=np.float64)
    n, d = x.shape
    q = np.ascontiguousarray(positions, dtype=np.int32)
    pool = np.empty((len(q), C), np.int32)
    plen = np.empty(len(q), np.int32)
    rc = _load().csel_geo_later_knn_subset(_p(x, _f64p), n, d, C, len(q), _p(q, _i32p), _p(pool, _i32p),
                                           _p(plen, _i32p))
    if rc != 0:
        raise ValueError("later_knn_pools_subset: bad arguments")
    return pool, plen


def make_groups(x_ordered: np.ndarray, ell: np.ndarray, sizes: np.ndarray, lam: float = 1.5):
    """Supernodes: the earliest unassigned position p plus up to m_g - 1 of its
    nearest unassigned later positions j with ell_j <= lam * ell_p.
    Returns (group_ptr, members) in CSR form, members ascending per group."""
    x = np.ascontiguousarray(x_ordered, dtype=np.float64)
    n, d = x.shape
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    gp = np.empty(n + 1, np.int32)
    mem = np.empty(n, np.int32)
    g = _load().csel_geo_make_groups(_p(x, _f64p), _p(ell, _f64p), n, d, _p(sizes, _i32p), len(sizes), lam,
                                     _p(gp, _i32p), _p(mem, _i32p))
    if g < 0:
        raise ValueError("make_groups: bad arguments")
    return gp[: g + 1].copy(), mem


def group_pools(x: np.ndarray, group_ptr: np.ndarray, members: np.ndarray, C: int,
                later_only: bool | str = True, cand_range: tuple[int, int] | None = None):
    """Union pools: the C points nearest to any member of the group, either
    among positions after the group's last member (later_only True), among
    the points after at least one member, each member contributing its own
    later neighbours and the members themselves left out (later_only
    "member": the partial, non-adjacent case), or among the ids in
    cand_range = [c0, c1)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    gp = np.ascontiguousarray(group_ptr, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    G = len(gp) - 1
    c0, c1 = cand_range if cand_range is not None else (0, n)
    pool = np.empty((G, C), np.int32)
    plen = np.empty(G, np.int32)
    mode = 2 if later_only == "member" else int(bool(later_only))
    rc = _load().csel_geo_group_pools(_p(x, _f64p), n, d, G, _p(gp, _i32p), _p(mem, _i32p), mode,
                                      c0, c1, C, _p(pool, _i32p), _p(plen, _i32p))
    if rc != 0:
        raise ValueError("group_pools: bad arguments")
    return pool, plen


def spatial_batches(x_pred: np.ndarray, n_strips: int = 8, per_strip: int = 8):
    """Split prediction points into n_strips * per_strip spatial batches: sort
    by the first coordinate into strips, each strip by the second into
    batches.  Returns (group_ptr, members) with members as row ids of x_pred."""
    n = x_pred.shape[0]
    idx = np.argsort(x_pred[:, 0], kind="stable")
    strips = np.array_split(idx, n_strips)
    groups = []
    for s in strips:
        s2 = s[np.argsort(x_pred[s, 1], kind="stable")]
        groups.extend(np.array_split(s2, per_strip))
    gp = np.zeros(len(groups) + 1, np.int32)
    gp[1:] = np.cumsum([len(g) for g in groups])
    mem = np.concatenate([np.sort(g) for g in groups]).astype(np.int32)
    return gp, mem


# --------------------------------------------------------------------------
# kernel parameters and named workloads
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Kernel:
    """Matern kernel: smoothness nu = two_nu / 2, length scale, variance, and
    a nugget added on the diagonal by index."""
    two_nu: int
    length_scale: float
    variance: float = 1.0
    nugget: float = 0.0


@dataclass
class SingleTargetWorkload:
    name: str
    points: np.ndarray         # (n, d) float64, ordering-position order
    ell: np.ndarray            # (n,) maximin length scales
    kernel: Kernel
    targets: np.ndarray        # (T,) int32 columns to build
    pool: np.ndarray           # (T, C) int32, -1 padded
    pool_len: np.ndarray       # (T,) int32
    k: int
    meta: dict = field(default_factory=dict)


@dataclass
class GroupWorkload:
    name: str
    points: np.ndarray
    kernel: Kernel
    group_ptr: np.ndarray
    members: np.ndarray
    pool: np.ndarray
    pool_len: np.ndarray
    k: int
    later_only: bool
    meta: dict = field(default_factory=dict)


def ordered_cloud(x: np.ndarray):
    order, ell = reverse_maximin(x)
    return np.ascontiguousarray(x[order]), ell


def single_target(name: str, x: np.ndarray, kernel: Kernel, C: int, k: int, targets=None):
    xo, ell = ordered_cloud(x)
    pool, plen = later_knn_pools(xo, C)
    n = xo.shape[0]
    t = np.arange(n, dtype=np.int32) if targets is None else np.asarray(targets, np.int32)
    return SingleTargetWorkload(name, xo, ell, kernel, t, np.ascontiguousarray(pool[t]),
                                np.ascontiguousarray(plen[t]), k)


def workload_plain_fp64(n: int = 2000, seed: int = 1):
    """N points uniform in [0,1]^2, Matern 3/2, l = 0.1, pools of the 64
    nearest later points, k = 16."""
    return single_target(f"plain-fp64 n={n} d=2 nu=3/2 C=64 k=16", uniform_points(n, 2, seed),
                         Kernel(3, 0.1), 64, 16)


def workload_plain_batched(n: int = 100_000, seed: int = 2):
    """N points uniform in [0,1]^3, Matern 5/2, l = 0.05, nugget 1e-6, pools of
    the 256 nearest later points (uneven at the tail), k = 32."""
    return single_target(f"plain-batched n={n} d=3 nu=5/2 C=256 k=32", uniform_points(n, 3, seed),
                         Kernel(5, 0.05, 1.0, 1e-6), 256, 32)


def workload_clustered(n: int = 1_000_000, seed: int = 4, C: int = 512, k: int = 32):
    """Mixture of 20 Gaussian clusters (sigma 0.03) plus 20% uniform background
    in [0,1]^3, Matern 3/2, l = 0.05; pools of 512, k = 32."""
    return single_target(f"clustered n={n} d=3 nu=3/2 C={C} k={k}", cluster_points(n, 3, seed),
                         Kernel(3, 0.05), C, k)


def workload_clustered_training(n: int = 1_000_000, seed: int = 40, C: int = 512, k: int = 32,
                                n_columns: int = 50_000):
    """Training cloud for the learned screen: the clustered distribution with
    its own seed; n_columns seeded columns with full pools of C."""
    xo, ell = ordered_cloud(cluster_points(n, 3, seed))
    rng = np.random.default_rng(seed + 1)
    t = np.sort(rng.choice(n, size=min(n_columns, n), replace=False)).astype(np.int32)
    pool, plen = later_knn_pools_subset(xo, C, t)
    return SingleTargetWorkload(f"clustered-training n={n} d=3 nu=3/2 C={C} k={k}", xo, ell, Kernel(3, 0.05), t,
                                pool, plen, k)


def workload_aggregated(n: int = 1_000_000, seed: int = 3, C: int = 512, k: int = 64,
                        mmin: int = 8, mmax: int = 32):
    """N uniform points in [0,1]^2, Matern 1/2, l = 0.02; supernodes of m
    uniform in {mmin..mmax}; union pools of the C nearest points after each
    group's last member; k per group."""
    x = uniform_points(n, 2, seed)
    xo, ell = ordered_cloud(x)
    sizes = np.random.default_rng(seed + 1000).integers(mmin, mmax + 1, size=n // mmin + 1).astype(np.int32)
    gp, mem = make_groups(xo, ell, sizes)
    pool, plen = group_pools(xo, gp, mem, C, later_only=True)
    return GroupWorkload(f"aggregated n={n} d=2 nu=1/2 m={mmin}..{mmax} C={C} k={k}", xo, Kernel(1, 0.02),
                         gp, mem, pool, plen, k, True, {"ell": ell})


def workload_partial(n: int = 1_000_000, seed: int = 3, C: int = 512, k: int = 32, mmin: int = 8, mmax: int = 32,
                     d: int = 2, two_nu: int = 1, ell: float = 0.02):
    """The aggregated workload's groups with unmodified candidate sets (Sec.
    5.3): N uniform points in [0,1]^d, Matern, supernodes of m uniform in
    {mmin..mmax}; each group's pool is the C points nearest to it among the
    later neighbours of its members (a candidate may precede some members
    and conditions only those it follows); k per group."""
    x = uniform_points(n, d, seed)
    xo, el = ordered_cloud(x)
    sizes = np.random.default_rng(seed + 1000).integers(mmin, mmax + 1, size=n // mmin + 1).astype(np.int32)
    gp, mem = make_groups(xo, el, sizes)
    pool, plen = group_pools(xo, gp, mem, C, later_only="member")
    return GroupWorkload(f"partial n={n} d={d} nu={two_nu}/2 m={mmin}..{mmax} C={C} k={k}", xo,
                         Kernel(two_nu, ell), gp, mem, pool, plen, k, False, {"ell": el})


def workload_gp(n_train: int = 500_000, n_pred: int = 4096, seed: int = 5, C: int = 2048, k: int = 128,
                n_strips: int = 8, per_strip: int = 8):
    """GP prediction: training points uniform in [0,1]^2 (ids [0, n_train)),
    prediction points uniform in [0,1]^2 (ids [n_train, n_train + n_pred)) in
    n_strips * per_strip spatial batches; Matern 5/2, l = 0.03; pool = the C
    training points nearest to any batch member; k per batch."""
    xt = uniform_points(n_train, 2, seed)
    xp = uniform_points(n_pred, 2, seed * 10)
    gp, mem = spatial_batches(xp, n_strips, per_strip)
    x = np.ascontiguousarray(np.concatenate([xt, xp], axis=0))
    mem = (mem + n_train).astype(np.int32)
    pool, plen = group_pools(x, gp, mem, C, later_only=False, cand_range=(0, n_train))
    return GroupWorkload(f"gp n_train={n_train} n_pred={n_pred} d=2 nu=5/2 C={C} k={k}", x, Kernel(5, 0.03),
                         gp, mem, pool, plen, k, False, {"n_train": n_train})
