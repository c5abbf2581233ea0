#!/usr/bin/env python3
"""Benchmark of the selection hot path: selected factor columns per second,
plain full-pool selection against learned-screened selection.

Default workload (--workload screened): N = 1,000,000 points in [0,1]^3 (20
Gaussian clusters with sigma 0.03 plus 20% uniform background), Matern 3/2,
l = 0.05, pools of the 512 nearest later-ordered points, k = 32.  The screen's
MLP is first trained on the GPU (untimed set-up) on exact selections of a
separate cloud.  One timed step is one csel_screened_select call, replayed
from its captured HIP graph: screen every column (features, BF16 MLP,
top-128 and the fallback flag), exact greedy selection with the factor column
(Sec. 3.1, eq. L_col) on the kept pools, and full-pool selection of the
fallback columns.  The credited leg computes the selection in FP64, the
paper's arithmetic; the mixed-precision leg (FP32 evaluation and GEMV) is
reported beside it with its difference from FP64.  Plain full-pool selection
and the selection on the 128 nearest candidates (the free screen) are timed
the same way.  Times are medians of the timed steps; inputs are resident in
HBM before timing; ordering, pools and training are set-up.

Other workloads: plain (N = 100,000 uniform in [0,1]^3, Matern 5/2, pools of
256, k = 32, replayed as a HIP graph), aggregated, gp (plain and screened) and
apply (products with a built factor, L^T x and L x).

Prints ONE JSON line (rank 0, N = 1 GPU).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "selected factor columns/s at fixed KL gap; plain vs learned-screened"
PEAK_ALU_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, unpacked FP32 = FP64 vector rate
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 MFMA


def eval_flops(dim: int, two_nu: int) -> int:
    """Flops of one covariance evaluation: per dimension a subtraction and an
    FMA (3), then sqrt, scale, exp (1 each) and the Matern polynomial."""
    poly = {1: 1, 3: 3, 5: 5}[two_nu]
    return 3 * dim + 3 + poly


def column_work(C, k, dim, two_nu, from_pivots=False):
    """Algorithmic flops and bytes of one column (numpy arrays C, k).
    from_pivots: the factor column is one back-substitution with the picks'
    Cholesky rows (FP64, pools up to 256); otherwise Theta_ss over the picks
    and the target is built and factored first."""
    import numpy as np

    C = np.asarray(C, np.float64)
    kk = np.minimum(k, C)
    fe = eval_flops(dim, two_nu)
    evals = C + C * kk                            # initial covariances + one per candidate per pick
    gemv = 2.0 * C * kk * (kk - 1) / 2.0          # left-looking GEMV, 2 flops per FMA
    down = 4.0 * C * kk                           # two FP64 FMAs per candidate per pick
    score = 2.0 * C * kk                          # cov^2 and the division
    m = kk + 1
    if from_pivots:
        tss = m * m                                # back-substitution
    else:
        tss = fe * m * (m + 1) / 2.0 + m ** 3 / 3.0 + m * m   # Theta_ss build, Cholesky, back-substitution
    flops = fe * evals + gemv + down + score + tss
    # bytes: target + pool_len + pool indices read, outputs written
    # (sel int32 k, factor fp64 k+1, log_condvar fp64, status u8)
    byt = 8.0 + 4.0 * C + 4.0 * k + 8.0 * (k + 1) + 8.0 + 1.0
    return flops, byt


def group_work(group_ptr, pool_len, k, dim, two_nu, want_factor):
    """Algorithmic flops and bytes of one aggregated group (numpy arrays)."""
    import numpy as np

    m = np.diff(np.asarray(group_ptr, np.float64))
    C = np.asarray(pool_len, np.float64)
    kk = np.minimum(k, C)
    R = C + m
    fe = eval_flops(dim, two_nu)
    # target conditioning: m left-looking columns over all rows
    init = fe * R * m + 2.0 * R * m * (m - 1) / 2.0 + 2.0 * R * m
    # picks: one evaluation, GEMV over the A (t) and B (m + t) columns, two FP64 downdates, score
    picks = fe * R * kk + 2.0 * R * (kk * (kk - 1) / 2.0 + m * kk + kk * (kk - 1) / 2.0) + 4.0 * R * kk + 3.0 * C * kk
    flops = init + picks
    if want_factor:
        M = m + kk
        flops = flops + fe * M * (M + 1) / 2.0 + M ** 3 / 3.0 + m * M * M
    byt = 8.0 + 4.0 * C + 4.0 * m + 4.0 * k + 8.0 + 1.0 + 8.0 * m
    if want_factor:
        byt = byt + 12.0 * (m * (m + 1) / 2.0 + m * kk) + 8.0 * m
    return flops, byt


def cpu_baseline(w, k, seconds, threads):
    """Time the FP64 oracle on a bounded seeded sample of the same columns."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(12345)
    T = len(w.targets)
    probe = np.sort(rng.choice(T, size=min(T, 512), replace=False))
    t0 = time.perf_counter()
    oracle.select_and_factor(w.points, w.kernel, w.targets[probe], w.pool[probe], w.pool_len[probe], k,
                             nthreads=threads)
    dt = time.perf_counter() - t0
    m = int(min(T, max(len(probe), len(probe) * seconds / max(dt, 1e-6))))
    idx = np.sort(rng.choice(T, size=m, replace=False))
    t0 = time.perf_counter()
    oracle.select_and_factor(w.points, w.kernel, w.targets[idx], w.pool[idx], w.pool_len[idx], k, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "columns/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} of {T} columns (seeded uniform sample), FP64 C oracle with OpenMP over columns, "
                      f"{dt:.1f} s"}


def cpu_baseline_groups(w, k, seconds, threads, want_factor, want_post_var):
    """Time the FP64 oracle on a bounded seeded sample of the groups."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(12345)
    G = len(w.group_ptr) - 1

    def run(idx):
        gp = np.zeros(len(idx) + 1, np.int32)
        sizes = np.diff(w.group_ptr)[idx]
        gp[1:] = np.cumsum(sizes)
        mem = np.concatenate([w.members[w.group_ptr[g]:w.group_ptr[g + 1]] for g in idx])
        t0 = time.perf_counter()
        oracle.aggregated_select(w.points, w.kernel, gp, mem, w.pool[idx], w.pool_len[idx], k,
                                 want_factor=want_factor, want_post_var=want_post_var, nthreads=threads)
        return time.perf_counter() - t0, int(sizes.sum())

    probe = np.sort(rng.choice(G, size=min(G, 64), replace=False))
    dt, _ = run(probe)
    m = int(min(G, max(len(probe), len(probe) * seconds / max(dt, 1e-6))))
    idx = np.sort(rng.choice(G, size=m, replace=False))
    dt, cols = run(idx)
    return {"value": cols / dt, "unit": "columns/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} of {G} groups ({cols} member columns, seeded uniform sample), FP64 C oracle with "
                      f"OpenMP over groups, {dt:.1f} s"}


def bench_groups(args):
    """Aggregated (supernodal) selection or GP prediction batches."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs

    print("bench: building inputs", file=sys.stderr, flush=True)
    if args.workload == "aggregated":
        w = inputs.workload_aggregated(n=args.n or 1_000_000)
        want_factor, want_post_var = True, False
        desc = (f"aggregated selection, N={len(w.points)} uniform in [0,1]^2, Matern 1/2, l=0.02, supernodes of "
                f"m uniform in 8..32, union pools of 512 later points, k=64, {args.precision}, member columns")
    else:
        w = inputs.workload_gp(n_train=args.n or 500_000)
        # posterior variances are FP64-only (the mixed run is compared with FP64 below)
        want_factor, want_post_var = False, args.precision == "fp64"
        desc = (f"GP prediction, {w.meta['n_train']} training points uniform in [0,1]^2, 4096 prediction points "
                f"in 64 batches of 64, Matern 5/2, l=0.03, pools of 2048, k=128, {args.precision}, "
                f"posterior variances")
    k = w.k
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    pts = t(w.points, torch.float64)
    gp_t, mem_t = t(w.group_ptr, torch.int32), t(w.members, torch.int32)
    pl, ln = t(w.pool, torch.int32), t(w.pool_len, torch.int32)
    mm = int(np.max(np.diff(w.group_ptr)))
    # the schedule the tuner picks for this shape class (set-up: each candidate
    # schedule timed once)
    from paper_2307_11648_amd import autotune

    tuner = autotune.SelectTuner()
    out = tuner.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, args.precision,
                                  want_factor=want_factor, want_post_var=want_post_var)
    torch.cuda.synchronize()
    ws = out["workspace"]
    tuned = next(iter(tuner.choices.values()), None)
    sched = tuned["schedule"] if tuned else "auto"

    def step():
        csel.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, args.precision,
                               want_factor=want_factor, want_post_var=want_post_var, out=out, workspace=ws,
                               schedule=sched)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        ev[i][0].record()
        step()
        ev[i][1].record()
    torch.cuda.synchronize()
    times = [a.elapsed_time(b_) for a, b_ in ev]
    ms = float(np.mean(times))
    cols = len(w.members)
    flops, byt = group_work(w.group_ptr, w.pool_len, k, w.points.shape[1], w.kernel.two_nu, want_factor)
    achieved = float(np.sum(flops)) / (ms * 1e-3) / 1e12
    st = out["status"].cpu().numpy()
    # the kernel the chosen schedule runs
    reg = args.precision == "mixed" and not want_post_var and w.pool.shape[1] <= 512 and mm <= 32 and k <= 64
    if sched.startswith("split"):
        coop = True
    elif sched == "one_group":
        coop = False
    else:  # the library's rule
        coop = (not want_factor and not reg and len(w.group_ptr) - 1 <= 128 and w.pool.shape[1] + mm > 256)
    sel_kernel = ("agg_select_coop_kernel" if coop else "agg_select_reg_kernel" if reg else "agg_select_kernel") + (
        " (+ agg_factor_kernel)" if want_factor else "")
    res = {
        "metric": METRIC, "value": cols / (ms * 1e-3), "unit": "columns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": desc, "groups": len(w.group_ptr) - 1, "columns": cols, "k": k,
                   "status_counts": {int(v): int((st == v).sum()) for v in np.unique(st)},
                   "schedule": sched, "schedule_tuning_ms": tuned["ms"] if tuned else None},
        "roofline": {"bound": "alu", "kernel": sel_kernel, "achieved": achieved,
                     "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": None, "kernel_ms": ms,
                     "algorithmic_gflop_per_launch": float(np.sum(flops)) / 1e9,
                     "algorithmic_mb_per_launch": float(np.sum(byt)) / 1e6},
    }
    if coop:
        # the left-looking updates read each row's factor entries once per
        # target column and per pick (8 bytes per FP64 fused multiply-add, 4
        # for the FP32 picks-only factor of mixed runs): factor B's first
        # columns from LDS, the rest from the per-group slabs
        sa = 8 if args.precision == "fp64" else 4
        gsz = np.diff(w.group_ptr).astype(np.int64)
        rows = w.pool_len.astype(np.int64) + gsz
        kk = np.minimum(k, w.pool_len).astype(np.int64)
        per_row = (8 * gsz * (gsz - 1) // 2 + 8 * (gsz * kk + kk * (kk - 1) // 2) + sa * kk * (kk - 1) // 2
                   + 8 * (gsz + kk) + sa * kk)
        stream = float(np.sum(per_row * rows))
        res["roofline"]["factor_stream_gb_per_launch"] = stream / 1e9
        res["roofline"]["factor_stream_tb_per_s"] = stream / (ms * 1e-3) / 1e12
    if args.workload == "gp" and args.precision == "mixed":
        # the same batches in FP64: selections, posterior variances and time
        o64 = csel.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, "fp64", want_factor=False,
                                     want_post_var=True)
        torch.cuda.synchronize()
        ev64 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev64[0].record()
        csel.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, "fp64", want_factor=False, want_post_var=True,
                               out=o64, workspace=o64["workspace"])
        ev64[1].record()
        torch.cuda.synchronize()
        ld, ld64 = out["logdet"].cpu().numpy(), o64["logdet"].cpu().numpy()
        res["config"]["mixed_vs_fp64"] = {
            "fp64_ms": ev64[0].elapsed_time(ev64[1]),
            "groups_identical": int(np.sum(np.all(out["sel"].cpu().numpy() == o64["sel"].cpu().numpy(), axis=1))),
            "logdet_sum": float(ld.sum()), "logdet_sum_fp64": float(ld64.sum()),
            "logdet_max_abs_difference": float(np.max(np.abs(ld - ld64))),
            "note": "posterior variances are FP64-only (CSEL_EUNSUPPORTED in mixed precision)"}
    if args.workload == "gp" and args.precision == "fp64":
        res["config"].update(gp_screened(args, w, pts, gp_t, mem_t, mm, pl, ln, out, ms))
    if args.cpu_seconds > 0:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        res["cpu_baseline"] = cpu_baseline_groups(w, k, args.cpu_seconds, threads, want_factor, want_post_var)
    print(json.dumps(res), flush=True)


def bench_knn(args):
    """The set-up of the default workload's cloud on the GPU (Sec. 2.2, Sec.
    4): N = 1e6 clustered points in [0,1]^3, their reverse-maximin ordering
    (csel_reverse_maximin) and the later-ordered pools of 512
    (csel_later_knn).  Timed: each whole call (grids, rounds, queries),
    medians; checked: the full ordering and a seeded sample of pool rows
    against the host definitions; beside it the host C kd-trees on all of
    the machine's cores for the same ordering and pools."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs

    n = args.n or 1_000_000
    C = 512
    x = inputs.cluster_points(n, 3, 4)
    print("bench: ordering the cloud (host)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ho, hell = inputs.reverse_maximin(x)
    host_order_s = time.perf_counter() - t0
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    lib = csel.load()
    mws = torch.empty(max(lib.csel_reverse_maximin_workspace_size(n, 3), 1), dtype=torch.uint8, device="cuda")
    gorder, gell, rounds = csel.reverse_maximin(xd, workspace=mws)
    order_identical = bool(np.array_equal(gorder.cpu().numpy(), ho)) and bool(
        np.array_equal(gell.cpu().numpy().view(np.uint64), hell.view(np.uint64)))
    xo = np.ascontiguousarray(x[ho])
    pts = torch.from_numpy(xo).cuda()
    pool, plen = csel.later_knn_pools(pts, C)
    ws = torch.empty(max(lib.csel_later_knn_workspace_size(n, 3), 1), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t_ord, t_knn = [], []
    for i in range(args.warmup + args.steps):
        # the ordering call returns after its stream drained (it reads a progress counter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        csel.reverse_maximin(xd, out=(gorder, gell), workspace=mws)
        t1 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        csel.later_knn_pools(pts, C, out=(pool, plen), workspace=ws, check=False)
        e1.record()
        torch.cuda.synchronize()
        if i >= args.warmup:
            t_ord.append((t1 - t0) * 1e3)
            t_knn.append(e0.elapsed_time(e1))
    ms_ord = float(np.median(t_ord))
    ms_knn = float(np.median(t_knn))
    ms = ms_ord + ms_knn
    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(n, size=4096, replace=False)).astype(np.int32)
    hp, hl = inputs.later_knn_pools_subset(xo, C, rows)
    gp = pool[torch.from_numpy(rows).long().cuda()].cpu().numpy()
    gl = plen.cpu().numpy()[rows]
    identical = int(np.sum(np.all(gp == hp, axis=1) & (gl == hl)))
    res = {"metric": "ordered candidate pools/s (reverse-maximin order + later-ordered 512-nearest pools)",
           "value": n / (ms * 1e-3), "unit": "pools/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"N={n} points in [0,1]^3 (20 Gaussian clusters sigma 0.03 + 20% uniform): "
                                  f"reverse-maximin ordering, then the 512 nearest later-ordered points of each; "
                                  f"medians of {args.steps} calls",
                      "ordering_ms": ms_ord, "ordering_rounds": rounds,
                      "ordering_identical_to_host": order_identical, "pools_ms": ms_knn,
                      "pool_rows_checked": len(rows), "pool_rows_identical_to_host": identical,
                      "min_pool_len": int(gl.min())}}
    if args.cpu_seconds > 0:
        print("bench: host kd-tree pools", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        inputs.later_knn_pools(xo, C)
        dt = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        res["cpu_baseline"] = {"value": n / (dt + host_order_s), "unit": "pools/s", "cores": threads,
                               "kind": "host kd-tree",
                               "sample": f"the whole cloud by the library's host C kd-trees: ordering "
                                         f"{host_order_s:.1f} s (one core, a sequential heap), pools {dt:.1f} s "
                                         f"(OpenMP)"}
    print(json.dumps(res), flush=True)


def partial_work(group_ptr, members, pool, pool_len, sel, k, dim, two_nu):
    """Algorithmic flops of partial selection per group (numpy), from the
    picks the run made: per step t with ncol = m + t columns and the pick
    inserted after p of them, every remaining candidate's score (2 flops per
    column, 4 more per member it conditions), every row's new column (one
    evaluation and p FMAs) and the rank-one downdate of the ncol - p later
    columns (6 flops per row and column); the member columns' Theta_sg,
    Cholesky and back-substitutions as in the aggregated count."""
    import numpy as np

    fe = eval_flops(dim, two_nu)
    G = len(group_ptr) - 1
    out = np.zeros(G)
    for g in range(G):
        T = members[group_ptr[g]:group_ptr[g + 1]]
        m = len(T)
        P = pool[g, : pool_len[g]]
        C = len(P)
        R = C + m
        cond = float(np.mean(np.searchsorted(np.sort(T), P))) if C else 0.0
        f = fe * R * m + R * m * m  # the members' columns
        picks = [int(v) for v in sel[g] if v >= 0]
        for t, j in enumerate(picks):
            ncol = m + t
            pp = int(np.sum(T > j)) + sum(1 for v in picks[:t] if v > j)
            f += (C - t) * (2.0 * ncol + 4.0 * cond) + R * (fe + 2.0 * pp) + 6.0 * R * (ncol - pp)
        M = m + len(picks)
        f += fe * M * (M + 1) / 2.0 + M ** 3 / 3.0 + m * M * M
        out[g] = f
    return out


def bench_partial(args):
    """Partial (non-adjacent) aggregated selection (Sec. 5.1, App. C.3) on
    the aggregated workload's groups with unmodified candidate sets: N = 1e6
    uniform in [0,1]^2, Matern 1/2, l = 0.02, groups of 8-32 members, pools of
    the 512 points nearest to the group among its members' later neighbours,
    k = 32, FP64, member columns.  Beside it, the adjacent selection the
    multi-target algorithm needs (pools cut to the points after the group's
    last member; csel_aggregated_select, FP64, same k): its time and its KL
    term, against the partial one's (Sec. 5.3: forcing adjacency loses
    accuracy)."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs

    n = args.n or 1_000_000
    k = 32
    print("bench: building inputs", file=sys.stderr, flush=True)
    w = inputs.workload_partial(n=n, k=k)
    pool_adj, plen_adj = inputs.group_pools(w.points, w.group_ptr, w.members, 512, later_only=True)
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    pts = t(w.points, torch.float64)
    gp_t, mem_t = t(w.group_ptr, torch.int32), t(w.members, torch.int32)
    pl, ln = t(w.pool, torch.int32), t(w.pool_len, torch.int32)
    pla, lna = t(pool_adj, torch.int32), t(plen_adj, torch.int32)
    mm = int(np.max(np.diff(w.group_ptr)))
    G = len(w.group_ptr) - 1
    out = csel.partial_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, want_factor=True)
    sel_only = csel.partial_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, want_factor=False)
    adj = csel.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pla, lna, k, "fp64", want_factor=True)
    torch.cuda.synchronize()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for i in range(args.steps):
            ev[i][0].record()
            fn()
            ev[i][1].record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b_) for a, b_ in ev]))

    print("bench: timing partial selection", file=sys.stderr, flush=True)
    ms = timed(lambda: csel.partial_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, want_factor=True, out=out))
    ms_sel = timed(lambda: csel.partial_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, want_factor=False,
                                               out=sel_only))
    ws = adj["workspace"]
    ms_adj = timed(lambda: csel.aggregated_select(pts, w.kernel, gp_t, mem_t, mm, pla, lna, k, "fp64",
                                                  want_factor=True, out=adj, workspace=ws))
    st = out["status"].cpu().numpy()
    sel = out["sel"].cpu().numpy()
    S_part = float(out["member_log_condvar"].sum())
    S_adj = float(adj["member_log_condvar"].sum())
    # the members' term with no selected point: sum over groups of log det Theta_TT, by k = 0
    zero = csel.partial_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, 0)
    torch.cuda.synchronize()
    S_0 = float(zero["logdet"].sum())
    cols = len(w.members)
    flops = partial_work(w.group_ptr, w.members, w.pool, w.pool_len, sel, k, 2, w.kernel.two_nu)
    M = np.diff(w.group_ptr) + np.sum(sel >= 0, axis=1)
    fe = eval_flops(2, w.kernel.two_nu)
    m_ = np.diff(w.group_ptr)
    fac_flops = fe * M * (M + 1) / 2.0 + M ** 3 / 3.0 + m_ * M * M
    sel_flops = float(np.sum(flops - fac_flops))
    achieved = sel_flops / (ms_sel * 1e-3) / 1e12
    res = {
        "metric": "member factor columns/s (partial aggregated selection)", "value": cols / (ms * 1e-3),
        "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"partial aggregated selection, N={n} uniform in [0,1]^2, Matern 1/2, l=0.02, "
                               f"supernodes of m uniform in 8..32, pools of the 512 points nearest to the group "
                               f"among its members' later neighbours, k={k}, FP64, member columns; medians of "
                               f"{args.steps} steps",
                   "groups": G, "columns": cols, "k": k,
                   "status_counts": {int(v): int((st == v).sum()) for v in np.unique(st)},
                   "select_ms": ms_sel, "factor_ms": ms - ms_sel,
                   "groups_with_interleaved_picks": int(sum(
                       np.any((sel[g][sel[g] >= 0] < w.members[w.group_ptr[g + 1] - 1])) for g in range(G))),
                   "adjacent": {"ms": ms_adj, "S": S_adj,
                                "note": "csel_aggregated_select FP64 on pools cut to the points after the "
                                        "group's last member, same k"},
                   "S_partial": S_part, "S_no_selection": S_0,
                   "kl_term_reduction": {"partial": S_0 - S_part, "adjacent": S_0 - S_adj,
                                         "partial_over_adjacent": (S_0 - S_part) / (S_0 - S_adj)
                                         if S_0 != S_adj else None}},
        "roofline": {"bound": "alu", "kernel": "partial_select_kernel<1>", "achieved": achieved,
                     "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": None, "kernel_ms": ms_sel,
                     "algorithmic_gflop_per_launch": sel_flops / 1e9},
    }
    if args.cpu_seconds > 0:
        print("bench: cpu baseline (partial oracle)", file=sys.stderr, flush=True)
        from oracle import partial as opartial

        rng = np.random.default_rng(12345)
        done = ncols = 0
        t0 = time.perf_counter()
        order = rng.permutation(G)
        while time.perf_counter() - t0 < args.cpu_seconds and done < G:
            g = int(order[done])
            opartial.partial_one(w.points, w.kernel, w.members[w.group_ptr[g]:w.group_ptr[g + 1]],
                                 w.pool[g, : w.pool_len[g]], k)
            ncols += int(w.group_ptr[g + 1] - w.group_ptr[g])
            done += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": ncols / dt, "unit": "columns/s", "cores": 1, "kind": "oracle",
                               "sample": f"{done} of {G} groups ({ncols} member columns, seeded order), the numpy "
                                         f"FP64 partial-selection oracle (factor rebuilt by left-looking after "
                                         f"each pick), one process, {dt:.1f} s"}
    print(json.dumps(res), flush=True)


def gp_screened(args, w, pts, gp_t, mem_t, mm, pl, ln, plain, ms_plain, keeps=(512, 1024)):
    """The learned-screened GP runs beside the plain one: the group screen is
    trained (untimed set-up) on the exact multi-target selections of GP
    batches of four separate training clouds of the same distribution and
    batch geometry; then each batch's 2048 candidates are screened to `keep`
    (no fallback) before the selection.  For each keep: time, and the gap of
    the screened selection to the plain one, sum_g (log det Theta_TT|s_screen
    - log det Theta_TT|s_plain) relative to sum_g (log det Theta_TT - log det
    Theta_TT|s_plain), plus the largest relative change of a posterior
    variance."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs, screen_train

    dev = pts.device
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    k = w.k
    print("bench: gp screen training", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    clouds = [inputs.workload_gp(n_train=w.meta["n_train"], n_pred=len(w.members), C=w.pool.shape[1], k=k, seed=sd)
              for sd in (8, 9, 10, 11)]
    sets = [screen_train.group_training_set(t(tr.points, torch.float64), tr.kernel, t(tr.group_ptr, torch.int32),
                                            t(tr.members, torch.int32), 64, t(tr.pool, torch.int32),
                                            t(tr.pool_len, torch.int32), k, "fp64") for tr in clouds]
    X = torch.cat([a for a, _ in sets])
    y = torch.cat([b for _, b in sets])
    del sets
    p, pb, losses = screen_train.train(X, y, steps=3000, batch=8192, lr=3e-3, seed=1, log_every=1000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    rows = int(X.shape[0])
    del X, y
    # log det Theta_TT of every batch (dense FP64 Cholesky on the GPU)
    G = len(w.group_ptr) - 1
    ld_prior = 0.0
    for g in range(G):
        xm = pts[w.members[w.group_ptr[g]:w.group_ptr[g + 1]]]
        a = torch.sqrt(torch.tensor(float(w.kernel.two_nu), dtype=torch.float64, device=dev)) * \
            torch.cdist(xm, xm) / w.kernel.length_scale
        th = w.kernel.variance * _matern_torch(w.kernel.two_nu, a) + \
            w.kernel.nugget * torch.eye(len(xm), dtype=torch.float64, device=dev)
        ld_prior += float(2.0 * torch.log(torch.diagonal(torch.linalg.cholesky(th))).sum().item())
    ld_plain = float(plain["logdet"].sum().item())
    prior = float(w.kernel.variance + w.kernel.nugget)
    pv_p = plain["post_var"].cpu().numpy()
    runs = {}
    for keep in keeps:
        out, scr, nfb = screen_train.screened_group_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, p, pb, keep,
                                                           args.precision, fallback_threshold=1e30)

        def step():
            screen_train.screened_group_select(pts, w.kernel, gp_t, mem_t, mm, pl, ln, k, p, pb, keep,
                                               args.precision, fallback_threshold=1e30, scr=scr, out=out)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.mean(times))
        pv_s = out["post_var"].cpu().numpy()
        runs[str(keep)] = {
            "screened_ms": ms, "speedup_vs_plain": ms_plain / ms,
            "groups_identical_to_plain": int(np.sum(np.all(out["sel"].cpu().numpy() == plain["sel"].cpu().numpy(),
                                                           axis=1))),
            "logdet_gap_relative": (float(out["logdet"].sum().item()) - ld_plain) / (ld_prior - ld_plain),
            "post_var_max_rel_change": float(np.max(np.abs(pv_s - pv_p) / pv_p)),
            "post_var_mean_rel_change": float(np.mean((pv_s - pv_p) / pv_p)),
            "post_var_max_change_over_prior": float(np.max(np.abs(pv_s - pv_p))) / prior}
    return {"plain_ms": ms_plain, "screened": runs,
            "screen_training": f"{rows} rows from {4 * G} exact FP64 batch selections of four separate clouds "
                               f"(seeds 8-11), {t_train:.1f} s set-up; losses {losses}"}


def _matern_torch(two_nu, a):
    import torch
    e = torch.exp(-a)
    if two_nu == 1:
        return e
    if two_nu == 3:
        return (1 + a) * e
    return (1 + a + a * a / 3.0) * e


def kl_gap_estimate(w, targets_sample, lcv_plain, lcv_screen, dS, n_ref=2048):
    """Relative KL gap of the screened factor, (S_screen - S_plain) / (2 KL_plain).

    2 KL_plain = sum_i [log Theta_ii|s_i - log Theta_ii|i+1:] (eq. obj_chol);
    the second term is estimated on a seeded sample of columns by conditioning
    on the n_ref nearest later points (dense FP64 Cholesky on the GPU; the
    screening effect makes the rest negligible) and scaled to all columns."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import inputs

    pool, plen = inputs.later_knn_pools_subset(w.points, n_ref, targets_sample)
    X = torch.from_numpy(w.points).cuda()
    c = math.sqrt(w.kernel.two_nu) / w.kernel.length_scale
    terms = []
    for r, i in enumerate(targets_sample):
        S = torch.from_numpy(pool[r, : plen[r]].astype(np.int64)).cuda()
        if len(S) == 0:
            ref = w.kernel.variance + w.kernel.nugget
        else:
            xs = X[S]
            K = w.kernel.variance * _matern_torch(w.kernel.two_nu, c * torch.cdist(xs, xs))
            K += w.kernel.nugget * torch.eye(len(S), dtype=K.dtype, device=K.device)
            k = w.kernel.variance * _matern_torch(w.kernel.two_nu, c * torch.linalg.norm(xs - X[int(i)], dim=1))
            Lc = torch.linalg.cholesky(K)
            z = torch.linalg.solve_triangular(Lc, k[:, None], upper=False)
            ref = float(w.kernel.variance + w.kernel.nugget - (z * z).sum())
        terms.append(float(lcv_plain[r]) - math.log(ref))
    kl2_plain = np.mean(terms) * len(w.targets)
    return dS / kl2_plain, kl2_plain / 2.0, len(targets_sample)


def cpu_baseline_screened(w, k, keep, fbt, p_np, seconds, threads):
    """The oracle's screened pipeline on a bounded seeded sample of the same
    columns: FP64 numpy features (batched over columns) and the MLP on the
    BF16-rounded weights, the exact top-keep with the fallback rule, then the
    FP64 C oracle's selection on the kept (or full) pools with OpenMP over
    columns.  The median of three runs on `threads` host threads, and one run
    on a single thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle import screen as so

    rng = np.random.default_rng(4321)
    T = len(w.targets)

    def run(idx, nthreads):
        t0 = time.perf_counter()
        pools = np.full((len(idx), w.pool.shape[1]), -1, np.int32)
        lens = np.zeros(len(idx), np.int32)
        with threadpool_limits(nthreads):
            for a in range(0, len(idx), 1024):
                ii = idx[a:a + 1024]
                f = so.features_batch(w.points, w.kernel, w.targets[ii], w.pool[ii], w.pool_len[ii])
                z, _ = so.mlp_forward(f.reshape(-1, 16), p_np, bf16=True)
                z = z.reshape(len(ii), -1)
                for r, t in enumerate(ii):
                    L = int(w.pool_len[t])
                    kept, fb = so.screen_keep(z[r], L, keep, fbt)
                    if fb:
                        pools[a + r, :L], lens[a + r] = w.pool[t, :L], L
                    else:
                        pools[a + r, : len(kept)], lens[a + r] = w.pool[t, kept], len(kept)
            oracle.select_and_factor(w.points, w.kernel, w.targets[idx], pools, lens, k, nthreads=nthreads)
        return time.perf_counter() - t0

    probe = np.sort(rng.choice(T, size=min(T, 1024), replace=False))
    dt = run(probe, threads)
    m = int(min(T, max(len(probe), len(probe) * seconds / 4.0 / max(dt, 1e-6))))
    idx = np.sort(rng.choice(T, size=m, replace=False))
    runs = sorted(run(idx, threads) for _ in range(3))
    dt_med = runs[1]
    m1 = max(256, m // max(threads, 1))
    dt1 = run(idx[:m1], 1)
    return {"value": m / dt_med, "unit": "columns/s", "cores": threads, "kind": "oracle",
            "one_core_value": m1 / dt1,
            "sample": f"{m} of {T} columns (seeded uniform sample), median of 3 runs ({', '.join(f'{r:.2f}' for r in runs)} "
                      f"s): FP64 numpy features and MLP on BF16-rounded weights (batched over 1024 columns; BLAS "
                      f"limited to {threads} threads), exact top-{keep} with the fallback rule, FP64 C oracle "
                      f"selection with OpenMP over columns on {threads} threads; one_core_value: {m1} columns on "
                      f"one thread, {dt1:.1f} s"}


def kl_ref_bound(pts, kernel, tg, pl, ln, S_plain_cols, dS, k_ref=128, sample=None):
    """Conservative relative KL gap of a screened selection: S_ref from the
    greedy selection of k_ref candidates from the same pools (FP64, through
    the multi-target selection with one member per group, whose picks are
    the single-target picks).  By prefix consistency those patterns contain
    the plain k-patterns, so S_ref <= S_plain and log det Theta <= S_ref:
    dS / (S_plain - S_ref) bounds dS / (2 KL_plain) from above.  On a seeded
    column sample when `sample` is given (scaled to all columns)."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel

    T = tg.shape[0]
    idx = np.arange(T) if not sample or sample >= T else \
        np.sort(np.random.default_rng(91).choice(T, size=sample, replace=False))
    ii = torch.from_numpy(idx.astype(np.int64)).to(pl.device)
    m = len(idx)
    gp = torch.arange(m + 1, dtype=torch.int32, device=pl.device)
    members = tg[ii].contiguous()
    out = csel.aggregated_select(pts, kernel, gp, members, 1, pl[ii].contiguous(), ln[ii].contiguous(), k_ref,
                                 "fp64")
    torch.cuda.synchronize()
    S_ref = out["logdet"].double().cpu().numpy()
    S_pl = np.asarray(S_plain_cols)[idx]
    st = out["status"].cpu().numpy()
    ok = st == 0
    diff = float(np.sum(S_pl[ok] - S_ref[ok])) * (T / max(int(ok.sum()), 1))
    return {"k_ref": k_ref, "columns": m, "status_nonzero": int((~ok).sum()),
            "prefix_violations": int(np.sum(S_ref[ok] > S_pl[ok] + 1e-9 * np.abs(S_pl[ok]))),
            "S_plain_minus_S_ref": diff, "gap_relative_upper": dS / diff if diff > 0 else None}


def _source_digest(*names):
    """Digest of the named sources and of the compiler flags of the units
    built from them (a flag change alters the kernel as much as an edit)."""
    import hashlib

    from paper_2307_11648_amd import build

    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2307_11648_amd", "csrc", n), "rb") as f:
            h.update(f.read())
        h.update(repr(sorted(repr(d) for src, d in build.HIP_UNITS if src == n)).encode())
    h.update(repr(build.HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


# HBM traffic per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# this script (copy-probe calibrated), keyed by the kernel, its column schedule
# and the digest of its sources at measurement time; a changed kernel reports
# null.
MEASURED_TRAFFIC = {
    # FETCH_SIZE x 1.9999 (a 1 GiB device copy reads as 524,315 KiB) + WRITE_SIZE x 1.0, in bytes; medians of
    # the launches of the default run (learned-screened workload, N = 1e6)
    ("select_factor_kernel<double> (kept pools)", "spatial", "5b36f12868af78eb"): (540572 * 1.9999 + 471876) * 1024,
    ("screen_kernel", "spatial", "a84e86504bb655a5"): (2114127 * 1.9999 + 564042) * 1024,
}


def bench_screened(args):
    """Plain full-pool selection vs learned-screened selection on the clustered
    1e6-point workload (pools of 512, keep 128, k = 32), in FP64 (the credited
    leg) and in mixed precision."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import autotune, csel, inputs, screen_train

    n = args.n or 1_000_000
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    print("bench: training cloud", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tr = inputs.workload_clustered_training(n=n, n_columns=min(50_000, n))
    P, Tg, Pl, Ln = t(tr.points, torch.float64), t(tr.targets, torch.int32), t(tr.pool, torch.int32), \
        t(tr.pool_len, torch.int32)
    X, y = screen_train.training_set(P, tr.kernel, Tg, Pl, Ln, 32, "fp64")
    del P, Tg, Pl, Ln
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p, pb, losses = screen_train.train(X, y, steps=args.train_steps, batch=8192, lr=3e-3, seed=1, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    rows = int(X.shape[0])
    del X, y
    print(f"bench: trained on {rows} rows in {t_train:.1f} s (set-up {t1 - t0:.1f} s); losses {losses}",
          file=sys.stderr, flush=True)
    print("bench: building inputs", file=sys.stderr, flush=True)
    w = inputs.workload_clustered(n=n)
    k, keep = 32, 128
    pts, tg, pl, ln = t(w.points, torch.float64), t(w.targets, torch.int32), t(w.pool, torch.int32), \
        t(w.pool_len, torch.int32)
    T = len(w.targets)
    fbt = args.fallback_threshold
    # the free screen: the 128 nearest candidates of every pool
    near_pl, near_ln = pl[:, :keep].contiguous(), torch.clamp(ln, max=keep).contiguous()
    order, _ = csel.spatial_order(pts, tg)
    tuner = autotune.SelectTuner()
    torch.cuda.synchronize()

    def timed(fn, nev):
        """Median over the K timed steps of the span between the first and last
        of `nev` HIP events fn records on the current stream, and of each
        consecutive pair; plus the host wall time per step."""
        for _ in range(args.warmup):
            fn()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for e in evs:
            fn(e)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_a) * 1e3 / args.steps
        parts = [float(np.median([e[j].elapsed_time(e[j + 1]) for e in evs])) for j in range(nev - 1)]
        total = float(np.median([e[0].elapsed_time(e[-1]) for e in evs]))
        return total, parts, wall

    kernel_ms = {}
    legs = {}
    outs = {}
    for prec in ("fp64", "mixed"):
        print(f"bench: {prec} legs", file=sys.stderr, flush=True)
        plain = tuner.select_and_factor(pts, w.kernel, tg, pl, ln, k, prec, order=order)
        near = tuner.select_and_factor(pts, w.kernel, tg, near_pl, near_ln, k, prec, order=order)
        plan = csel.Plan(T, pl.shape[1], keep, k, prec, graph=True)
        plan.set_order(pts, tg)
        scr = plan.step(pts, w.kernel, tg, pl, ln, p, pb, fbt)  # the first step tunes the kept-pool schedule
        plan.step(pts, w.kernel, tg, pl, ln, p, pb, fbt, out=scr)  # captures the graph
        torch.cuda.synchronize()
        kept_schedule = plan.info()

        def plain_step(ev=None):
            if ev is not None:
                ev[0].record()
            tuner.select_and_factor(pts, w.kernel, tg, pl, ln, k, prec, order=order, out=plain)
            if ev is not None:
                ev[1].record()

        def near_step(ev=None):
            if ev is not None:
                ev[0].record()
            tuner.select_and_factor(pts, w.kernel, tg, near_pl, near_ln, k, prec, order=order, out=near)
            if ev is not None:
                ev[1].record()

        def screened_step(ev=None):
            # one library call: screen, kept-pool selection, fallback columns
            # (a graph replay on the current stream)
            if ev is not None:
                ev[0].record()
            plan.step(pts, w.kernel, tg, pl, ln, p, pb, fbt, out=scr)
            if ev is not None:
                ev[1].record()

        # the same kernels launched one by one, for their separate times
        sep = csel.screen(pts, w.kernel, tg, pl, ln, p, pb, keep, fbt, order=order)
        sep_out = csel.select_and_factor(pts, w.kernel, tg, sep["kept"], sep["kept_len"], k, prec)
        kept_sched = kept_schedule["schedule"]
        n_all = torch.tensor([T], dtype=torch.int32, device=dev)

        def parts_step(ev=None):
            if ev is not None:
                ev[0].record()
            csel.screen(pts, w.kernel, tg, pl, ln, p, pb, keep, fbt, out=sep, order=order)
            if ev is not None:
                ev[1].record()
            if kept_sched == "spatial":
                csel.select_and_factor_list(pts, w.kernel, tg, sep["kept"], sep["kept_len"], k, prec, order, n_all,
                                            T, sep_out)
            else:
                csel.select_and_factor(pts, w.kernel, tg, sep["kept"], sep["kept_len"], k, prec, out=sep_out)
            if ev is not None:
                ev[2].record()
            csel.select_and_factor_list(pts, w.kernel, tg, pl, ln, k, prec, sep["fallback_list"],
                                        sep["fallback_count"], T, sep_out)
            if ev is not None:
                ev[3].record()

        print(f"bench: timing {prec} plain", file=sys.stderr, flush=True)
        ms_plain, _, _ = timed(plain_step, 2)
        print(f"bench: timing {prec} screened", file=sys.stderr, flush=True)
        ms_scr, _, wall_scr = timed(screened_step, 2)
        ms_near, _, _ = timed(near_step, 2)
        _, (ms_screen_k, ms_kept_k, ms_fb_k), _ = timed(parts_step, 4)
        torch.cuda.synchronize()
        so = plan.screen_outputs()
        nfb = int(so["fallback_count"].item())
        S_plain = float(plain["log_condvar"].sum().item())
        S_scr = float(scr["log_condvar"].sum().item())
        S_near = float(near["log_condvar"].sum().item())
        kl_len = so["kept_len"].cpu().numpy()
        fb_cols = so["fallback"].cpu().numpy() >= 1
        legs[prec] = {
            "plain_ms": ms_plain, "screened_ms": ms_scr, "screened_wall_ms_per_step": wall_scr,
            "nearest128_ms": ms_near, "speedup_vs_plain": ms_plain / ms_scr,
            "nearest128_speedup_vs_plain": ms_plain / ms_near,
            "screen_kernel_ms": ms_screen_k, "kept_select_ms": ms_kept_k, "fallback_select_ms": ms_fb_k,
            "fallback_columns": nfb, "kept_pool_schedule": kept_schedule,
            "status_nonzero": int(np.count_nonzero(scr["status"].cpu().numpy())),
            "delta_S": S_scr - S_plain, "delta_S_nearest128": S_near - S_plain,
            "S_plain": S_plain,
        }
        outs[prec] = {"plain": plain, "scr": scr, "near": near}
        kernel_ms[prec] = (ms_screen_k, ms_kept_k, kl_len, fb_cols)
        del plan, sep, sep_out
        torch.cuda.empty_cache()
    # operating points in FP64 at other keep sizes: the learned screen (its
    # fallback off, so the screen alone decides) and the nearest truncation
    # through the same kernels, each with its time and data-term change (the
    # KL gaps follow below)
    sweep = {}
    for kp in args.keep_sweep:
        if kp == keep or kp < k or kp > pl.shape[1]:
            continue
        print(f"bench: keep {kp} operating points", file=sys.stderr, flush=True)
        plan = csel.Plan(T, pl.shape[1], kp, k, "fp64", graph=True)
        plan.set_order(pts, tg)
        o = plan.step(pts, w.kernel, tg, pl, ln, p, pb, 1e30)
        plan.step(pts, w.kernel, tg, pl, ln, p, pb, 1e30, out=o)
        npl, nln = pl[:, :kp].contiguous(), torch.clamp(ln, max=kp).contiguous()
        no = tuner.select_and_factor(pts, w.kernel, tg, npl, nln, k, "fp64", order=order)

        def lstep(ev=None):
            if ev is not None:
                ev[0].record()
            plan.step(pts, w.kernel, tg, pl, ln, p, pb, 1e30, out=o)
            if ev is not None:
                ev[1].record()

        def nstep(ev=None):
            if ev is not None:
                ev[0].record()
            tuner.select_and_factor(pts, w.kernel, tg, npl, nln, k, "fp64", order=order, out=no)
            if ev is not None:
                ev[1].record()

        ms_l, _, _ = timed(lstep, 2)
        ms_n, _, _ = timed(nstep, 2)
        sweep[str(kp)] = {"learned_ms": ms_l, "nearest_ms": ms_n, "learned_fallback": "off",
                          "learned_delta_S": float(o["log_condvar"].sum()) - legs["fp64"]["S_plain"],
                          "nearest_delta_S": float(no["log_condvar"].sum()) - legs["fp64"]["S_plain"]}
        del plan, o, no, npl, nln
        torch.cuda.empty_cache()
    tune_choices = tuner.choices

    # quality: the KL gap of the screened and the nearest-128 selections
    print("bench: KL gap estimates", file=sys.stderr, flush=True)
    rng = np.random.default_rng(77)
    samp = np.sort(rng.choice(T, size=96, replace=False)).astype(np.int32)
    lcv_p64 = outs["fp64"]["plain"]["log_condvar"].cpu().numpy()
    for prec in ("fp64", "mixed"):
        lg = legs[prec]
        lcv_p = outs[prec]["plain"]["log_condvar"].cpu().numpy()
        gap, kl_plain, ns = kl_gap_estimate(w, samp, lcv_p[samp], None, lg["delta_S"])
        lg["kl_gap_relative_estimate"] = gap
        lg["kl_gap_relative_estimate_nearest128"] = lg["delta_S_nearest128"] / (2.0 * kl_plain)
        lg["kl_plain_estimate"] = kl_plain
        lg["kl_estimate_sample_columns"] = ns
    print("bench: KL bound with k_ref = 128", file=sys.stderr, flush=True)
    bound = kl_ref_bound(pts, w.kernel, tg, pl, ln, lcv_p64, legs["fp64"]["delta_S"], sample=args.kl_ref_sample)
    legs["fp64"]["kl_bound_k128"] = bound
    if bound["S_plain_minus_S_ref"] > 0:
        den = bound["S_plain_minus_S_ref"]
        legs["fp64"]["kl_gap_relative_upper_nearest128"] = legs["fp64"]["delta_S_nearest128"] / den
        for v in sweep.values():
            v["learned_kl_gap_relative_upper"] = v["learned_delta_S"] / den
            v["nearest_kl_gap_relative_upper"] = v["nearest_delta_S"] / den
            v["learned_speedup_vs_plain"] = legs["fp64"]["plain_ms"] / v["learned_ms"]
            v["nearest_speedup_vs_plain"] = legs["fp64"]["plain_ms"] / v["nearest_ms"]
    # mixed precision against FP64 (same workload, same screen)
    m64, mmx = outs["fp64"], outs["mixed"]
    for key in ("plain", "scr"):
        a, b = m64[key], mmx[key]
        same = torch.all(a["sel"] == b["sel"], dim=1)
        fa, fb_ = a["factor"][same], b["factor"][same]
        err = float((torch.max(torch.abs(fa - fb_), dim=1).values / torch.max(torch.abs(fa), dim=1).values).max()) \
            if bool(same.any()) else None
        legs["mixed"][f"{key}_vs_fp64"] = {
            "columns_identical": int(same.sum().item()), "columns": T,
            "S_relative_difference": (float(b["log_condvar"].sum()) - float(a["log_condvar"].sum()))
            / abs(float(a["log_condvar"].sum())),
            "worst_factor_rel_error_on_identical_columns": err}

    flops_kept, _ = column_work(kernel_ms["fp64"][2], k, 3, 3, from_pivots=True)
    mlp_flops = 2.0 * (16 * 64 + 64 * 64 + 64) * float(np.sum(w.pool_len))
    sched = legs["fp64"]["kept_pool_schedule"]["schedule"]
    kernels = {
        "select_factor_kernel<double> (kept pools)": {
            "bound": "alu", "ms": kernel_ms["fp64"][1], "work": float(np.sum(flops_kept)), "peak": PEAK_ALU_TFLOPS,
            "src": ("select_kernel.hpp", "select_inst.hip", "device_common.hpp"), "schedule": sched},
        "screen_kernel": {"bound": "mfma", "ms": kernel_ms["fp64"][0], "work": mlp_flops, "peak": PEAK_BF16_TFLOPS,
                          "src": ("screen.hip", "device_common.hpp"), "schedule": "spatial"},
    }
    dom = max(kernels, key=lambda kname: kernels[kname]["ms"])

    def roof(kname):
        kd = kernels[kname]
        ach = kd["work"] / (kd["ms"] * 1e-3) / 1e12
        tr_ = MEASURED_TRAFFIC.get((kname, kd["schedule"], _source_digest(*kd["src"])))
        return {"bound": kd["bound"], "kernel": kname, "achieved": ach, "peak": kd["peak"], "unit": "TFLOP/s",
                "frac": ach / kd["peak"], "traffic": tr_, "traffic_unit": "HBM bytes per launch (rocprofv3 "
                "FETCH_SIZE + WRITE_SIZE, copy-calibrated)", "schedule": kd["schedule"], "kernel_ms": kd["ms"],
                "algorithmic_tflop_per_launch": kd["work"] / 1e12}

    f64 = legs["fp64"]
    flops_plain, _ = column_work(w.pool_len, k, 3, 3)
    for prec in ("fp64", "mixed"):
        legs[prec]["plain_roofline_frac"] = float(np.sum(flops_plain)) / (legs[prec]["plain_ms"] * 1e-3) / 1e12 / \
            PEAK_ALU_TFLOPS
    res = {
        "metric": METRIC, "value": T / (f64["screened_ms"] * 1e-3), "unit": "columns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f64["screened_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": f"learned-screened selection, N={n} in [0,1]^3 (20 Gaussian clusters sigma 0.03 + 20% "
                               f"uniform), Matern 3/2, l=0.05, pools of 512 -> keep {keep}, k={k}; FP64 selection "
                               f"(the credited leg; mixed precision reported beside it); MLP 16-64-64-1 trained on "
                               f"the GPU on {rows} rows from {len(tr.targets)} exact selections; one "
                               f"csel_screened_select graph replay per step; medians of {args.steps} steps",
                   "columns": T, "fallback_threshold": fbt, "legs": legs, "fp64_keep_sweep": sweep,
                   "autotuned_schedules": tune_choices,
                   "speedup_vs_plain": f64["speedup_vs_plain"], "train_seconds": t_train},
        "roofline": roof(dom),
        "roofline_other": [roof(kname) for kname in kernels if kname != dom],
    }
    if args.cpu_seconds > 0:
        print("bench: cpu baseline (screened oracle)", file=sys.stderr, flush=True)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        res["cpu_baseline"] = cpu_baseline_screened(w, k, keep, fbt, p.cpu().numpy().astype(np.float64),
                                                    args.cpu_seconds, threads)
    print(json.dumps(res), flush=True)


def bench_apply(args):
    """Products with a built factor (csel_apply_factor): y = L^T x and y = L x
    for the sparse inverse-Cholesky factor of N = 1e6 clustered points (pools of
    the 64 nearest later points, k = 32, mixed precision; built untimed).  L x
    runs as the gather on L^T (csel_transpose_factor, built once, its time
    reported as set-up); the atomic scatter is timed beside it.  HBM-bound:
    the roofline counts the algorithmic bytes of each product."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs

    n = args.n or 1_000_000
    print("bench: building the factor", file=sys.stderr, flush=True)
    w = inputs.workload_clustered(n=n, C=64, k=32)
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    pts, tg = t(w.points, torch.float64), t(w.targets, torch.int32)
    f = csel.select_and_factor(pts, w.kernel, tg, t(w.pool, torch.int32), t(w.pool_len, torch.int32), 32,
                               args.precision)
    col_ptr, rows, vals = csel.single_target_csc(tg, f["sel"], f["factor"])
    nnz = int((rows >= 0).sum().item())
    # L^T in CSC form, built once (set-up): L x then runs as a gather
    tf = csel.transpose_factor(col_ptr, rows, vals)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    tf = csel.transpose_factor(col_ptr, rows, vals, out=tf)
    e1.record()
    torch.cuda.synchronize()
    ms_transpose = e0.elapsed_time(e1)
    x = torch.from_numpy(np.random.default_rng(3).standard_normal(n)).to(dev)
    y = torch.empty_like(x)
    slots = int(rows.numel())
    # algorithmic bytes: per stored entry its row index and value (12 B) and
    # one gathered x (8 B); per column one y write (8 B).  The atomic L x reads
    # x once per column and read-modify-writes y per entry, after clearing y.
    cases = {"lt": (col_ptr, rows, vals, True, 12 * slots + 8 * nnz + 8 * n),
             "l": (tf[0], tf[1], tf[2], True, 12 * slots + 8 * nnz + 8 * n),
             "l_atomic": (col_ptr, rows, vals, False, 12 * slots + 16 * nnz + 16 * n)}
    res = {}
    for name, (cp_, r_, v_, tr, byt) in cases.items():
        for _ in range(args.warmup):
            csel.apply_factor(cp_, r_, v_, x, tr, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            csel.apply_factor(cp_, r_, v_, x, tr, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = {"ms": ms, "bytes": byt, "gbs": byt / (ms * 1e-3) / 1e9}
    ms = res["lt"]["ms"] + res["l"]["ms"]
    dom = max(("lt", "l"), key=lambda key: res[key]["ms"])
    out = {
        "metric": "factor columns applied/s (y = L^T x then y = L x)", "value": n / (ms * 1e-3),
        "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"apply_factor, N={n} clustered points in [0,1]^3, factor from pools of the 64 "
                               f"nearest later points, k=32, {args.precision}", "columns": n, "nnz": nnz,
                   "stored_slots": slots, "lt_ms": res["lt"]["ms"], "l_ms": res["l"]["ms"],
                   "l_atomic_ms": res["l_atomic"]["ms"], "transpose_setup_ms": ms_transpose},
        "roofline": {"bound": "hbm", "kernel": f"apply_lt_kernel ({'L^T x' if dom == 'lt' else 'L x on L^T'})",
                     "achieved": res[dom]["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": res[dom]["gbs"] / PEAK_HBM_GBS, "traffic": None, "kernel_ms": res[dom]["ms"],
                     "algorithmic_bytes_per_launch": res[dom]["bytes"]},
        "roofline_other": [{"bound": "hbm", "kernel": name, "achieved": res[key]["gbs"], "peak": PEAK_HBM_GBS,
                            "unit": "GB/s", "frac": res[key]["gbs"] / PEAK_HBM_GBS, "kernel_ms": res[key]["ms"]}
                           for key, name in (("lt", "apply_lt_kernel (L^T x)"), ("l", "apply_lt_kernel (L x on L^T)"),
                                             ("l_atomic", "apply_l_kernel (L x, atomic scatter)")) if key != dom],
    }
    print(json.dumps(out), flush=True)


def bench_pcg(args):
    """The factor as a preconditioner (Sec. 6.3): N = 2^16 points uniform in
    [0,1]^3, Matern 1/2, l = 1, y = Theta x for a Gaussian x; the conjugate
    gradient to a relative residual of 1e-12 with the factor of greedy
    selection (k of 3k later neighbours, FP64), with the factor on the k
    nearest later neighbours, and without a preconditioner (capped)."""
    import numpy as np
    import torch

    from paper_2307_11648_amd import csel, inputs

    n = args.n or (1 << 16)
    k = 16
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    kern = inputs.Kernel(1, 1.0)
    print("bench: building inputs", file=sys.stderr, flush=True)
    xo, _ = inputs.ordered_cloud(inputs.uniform_points(n, 3, 6))
    pts = t(xo, torch.float64)
    tg = t(np.arange(n, dtype=np.int32), torch.int32)
    sol = t(np.random.default_rng(6).standard_normal(n), torch.float64)
    y, mv_ws = csel.kernel_matvec(pts, kern, sol)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        csel.kernel_matvec(pts, kern, sol, out=y, workspace=mv_ws)
    e1.record()
    torch.cuda.synchronize()
    ms_mv = e0.elapsed_time(e1) / 3
    out = {}
    for name, C in (("conditional", 3 * k), ("knn", k)):
        pool, plen = inputs.later_knn_pools(xo, C)
        pl, ln = t(pool, torch.int32), t(plen, torch.int32)
        f = csel.select_and_factor(pts, kern, tg, pl, ln, k, "fp64")
        cp, rows, vals = csel.single_target_csc(tg, f["sel"], f["factor"])
        ft = csel.transpose_factor(cp, rows, vals)[:3]  # a first build: allocations and first launches
        torch.cuda.synchronize()
        e0.record()
        f = csel.select_and_factor(pts, kern, tg, pl, ln, k, "fp64", out=f)
        cp, rows, vals = csel.single_target_csc(tg, f["sel"], f["factor"])
        ft = csel.transpose_factor(cp, rows, vals)[:3]
        e1.record()
        torch.cuda.synchronize()
        ms_build = e0.elapsed_time(e1)
        t0 = time.perf_counter()
        x, it, rel = csel.pcg(pts, kern, y, (cp, rows, vals), ft, rel_tol=1e-12, max_iter=2000)
        torch.cuda.synchronize()
        s_cg = time.perf_counter() - t0
        err = float(torch.linalg.norm(x - sol) / torch.linalg.norm(sol))
        out[name] = {"iterations": it, "rel_residual": rel, "solution_rel_error": err, "factor_ms": ms_build,
                     "cg_seconds": s_cg, "ms_per_iteration": s_cg * 1e3 / max(it, 1)}
    t0 = time.perf_counter()
    _, it0, rel0 = csel.pcg(pts, kern, y, None, None, rel_tol=1e-12, max_iter=args.pcg_plain_iters)
    torch.cuda.synchronize()
    out["none"] = {"iterations": it0, "rel_residual": rel0, "cg_seconds": time.perf_counter() - t0,
                   "capped": it0 >= args.pcg_plain_iters}
    # the kernel matvec: n^2 evaluations of the FP64 Matern (each counted as
    # in column_work) plus the multiply-add
    flops_mv = float(n) * n * (eval_flops(3, 1) + 2)
    ach = flops_mv / (ms_mv * 1e-3) / 1e12
    c = out["conditional"]
    res = {"metric": "conjugate-gradient solves/s (relative residual 1e-12, preconditioned by the factor)",
           "value": 1.0 / (c["cg_seconds"] + c["factor_ms"] * 1e-3), "unit": "solves/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": c["cg_seconds"] * 1e3 + c["factor_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"PCG, N={n} uniform in [0,1]^3, Matern 1/2, l=1, y = Theta x with x Gaussian; "
                                  f"factor of greedy selection k={k} of {3 * k} later neighbours vs the factor on the "
                                  f"{k} nearest later neighbours vs none", "k": k, "runs": out,
                      "kernel_matvec_ms": ms_mv},
           "roofline": {"bound": "alu", "kernel": "kmatvec_partial_kernel<1>", "achieved": ach,
                        "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_ALU_TFLOPS, "traffic": None,
                        "kernel_ms": ms_mv, "algorithmic_tflop_per_launch": flops_mv / 1e12}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="screened",
                    choices=["screened", "plain", "aggregated", "gp", "apply", "pcg", "partial", "knn"])
    ap.add_argument("--pcg-plain-iters", type=int, default=300,
                    help="pcg workload: iteration cap of the unpreconditioned run")
    ap.add_argument("--train-steps", type=int, default=3000, help="screened workload: Adam steps")
    ap.add_argument("--fallback-threshold", type=float, default=2.0,
                    help="screened workload: fall back to the full pool when the dropped candidates' summed "
                         "selection probability exceeds this")
    ap.add_argument("--n", type=int, default=0, help="number of points (0 = the workload's full size)")
    ap.add_argument("--precision", default="", choices=["", "mixed", "fp64"],
                    help="default: mixed, except fp64 for the GP workload (its conditional variances fall "
                         "below the FP32 error floor)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="CPU-baseline budget (0 = skip)")
    ap.add_argument("--keep-sweep", type=lambda v: [int(a) for a in v.split(",") if a], default=[48, 64, 96],
                    help="screened workload: further keep sizes timed in FP64, learned and nearest")
    ap.add_argument("--kl-ref-sample", type=int, default=200_000,
                    help="screened workload: columns of the k_ref = 128 KL bound (seeded sample; 0 = all)")
    ap.add_argument("--graph", type=int, default=1, help="plain workload: replay the step as a captured HIP graph")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run one 1 GiB device copy first (profiler byte-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (its columns would shard with "
              "no communication but an 8-byte sum).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2307_11648_amd import build as b
    if not (os.path.exists(b.LIB) and os.path.exists(b.GEO_LIB)):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2307_11648_amd import csel, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if not args.precision:
        args.precision = "fp64" if args.workload == "gp" else "mixed"
    if args.copy_probe:
        # a plain copy of known size (1 GiB read + 1 GiB written) for calibrating
        # the HBM byte counters of a profiler run
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "screened":
        return bench_screened(args)
    if args.workload == "apply":
        return bench_apply(args)
    if args.workload == "pcg":
        return bench_pcg(args)
    if args.workload == "partial":
        return bench_partial(args)
    if args.workload == "knn":
        return bench_knn(args)
    if args.workload != "plain":
        return bench_groups(args)
    args.n = args.n or 100_000
    print("bench: building inputs", file=sys.stderr, flush=True)
    w = inputs.workload_plain_batched(n=args.n)
    k = w.k
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    pts = t(w.points, torch.float64)
    tg = t(w.targets, torch.int32)
    pl = t(w.pool, torch.int32)
    ln = t(w.pool_len, torch.int32)
    T = len(w.targets)
    out = csel.select_and_factor(pts, w.kernel, tg, pl, ln, k, args.precision)
    s_out = torch.empty(1, dtype=torch.float64, device=dev)
    # the column schedule (natural or Morton order), tuned once here (set-up)
    from paper_2307_11648_amd import autotune

    order, _ = csel.spatial_order(pts, tg)
    tuner = autotune.SelectTuner()
    tuner.select_and_factor(pts, w.kernel, tg, pl, ln, k, args.precision, order=order, out=out)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def step(i=None):
        if i is not None:
            ev[i][0].record()
        tuner.select_and_factor(pts, w.kernel, tg, pl, ln, k, args.precision, order=order, out=out)
        if i is not None:
            ev[i][1].record()
        csel.sum(out["log_condvar"], out=s_out)

    graph = None
    if args.graph:
        # capture one step (no events inside) and check replays against eager
        step()
        torch.cuda.synchronize()
        ref = {key: v.clone() for key, v in out.items()}
        ref_s = s_out.clone()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            step()
        torch.cuda.current_stream().wait_stream(cs)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(2):
            for v in out.values():
                v.zero_()
            graph.replay()
            torch.cuda.synchronize()
            for key in out:
                assert torch.equal(out[key], ref[key]), f"graph replay differs from eager in {key}"
            assert torch.equal(s_out, ref_s)

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        graph.replay() if graph is not None else step()
    torch.cuda.synchronize()

    # timed region: K steps; inside each step the select kernel is bracketed by
    # events on its own stream (the current stream)
    print("bench: timing", file=sys.stderr, flush=True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for i in range(args.steps):
        if graph is not None:
            ev[i][0].record()
            graph.replay()
            ev[i][1].record()
        else:
            step(i)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    # with a graph the per-step events bracket select + sum; the sum kernel is
    # a single 1024-thread block over T doubles (a few microseconds)
    kern_ms = float(np.mean([a.elapsed_time(b_) for a, b_ in ev]))

    flops, byt = column_work(w.pool_len, k, w.points.shape[1], w.kernel.two_nu,
                             from_pivots=args.precision == "fp64" and pl.shape[1] <= 256)
    plain_schedule = tuner.choices[autotune.shape_key(pts.shape[1], int(w.kernel.two_nu), T, pl.shape[1], k,
                                                      args.precision)]["schedule"]
    flops_launch = float(np.sum(flops))
    bytes_launch = float(np.sum(byt)) + w.points.nbytes
    achieved = flops_launch / (kern_ms * 1e-3) / 1e12
    st = out["status"].cpu().numpy()
    S = float(s_out.item())

    res = {
        "metric": METRIC,
        "value": T / (ms_step * 1e-3),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"plain greedy selection, N={args.n} uniform in [0,1]^3, Matern 5/2, l=0.05, nugget 1e-6, "
                        f"pools of 256 nearest later points (uneven at the tail), k={k}, {args.precision}",
            "columns": T,
            "k": k,
            "pool": 256,
            "precision": args.precision,
            "graph": bool(args.graph),
            "autotuned_schedules": tuner.choices,
            "sum_log_condvar": S,
            "status_nonzero": int(np.count_nonzero(st)),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "select_factor_kernel",
            "achieved": achieved,
            "peak": PEAK_ALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU_TFLOPS,
            "traffic": MEASURED_TRAFFIC.get(("select_factor_kernel (plain batched)", plain_schedule,
                                             _source_digest("select_kernel.hpp", "select_inst.hip",
                                                            "device_common.hpp"))),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "schedule": plain_schedule,
            "kernel_ms": kern_ms,
            "algorithmic_gflop_per_launch": flops_launch / 1e9,
            "algorithmic_mb_per_launch": bytes_launch / 1e6,
            "hbm_frac_at_algorithmic_bytes": bytes_launch / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        },
    }
    if args.cpu_seconds > 0:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        res["cpu_baseline"] = cpu_baseline(w, k, args.cpu_seconds, threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
