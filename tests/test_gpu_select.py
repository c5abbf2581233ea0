"""GPU parity of csel_select_and_factor against the FP64 oracle (through the C ABI)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2307_11648_amd import csel, inputs
from parity import compare_single, kl_rel_error, replay_check

pytestmark = pytest.mark.gpu

# decisive-step threshold on the oracle's top-two relative score gap
THR = 1e-6
# Mixed precision evaluates covariances and the GEMV in FP32 (unit roundoff
# u32 = 6e-8).  The absolute error of a downdated conditional variance is then
# about u32 * prior, so its relative error is u32 * prior / var; after 16-32
# picks var/prior reaches 1e-5..1e-6 on these workloads, which puts score
# perturbations in the 1e-2 range.  A mixed run can therefore follow another
# valid greedy path; it is checked by replaying its own picks in FP64: each
# pick's exact score may fall short of the best exact score by at most
# TAU_MIXED times the target's current conditional variance (a per-step loss of
# at most 1e-4 in log Theta_ii|s, i.e. a KL effect far below the 1e-3 mixed
# factor tolerance), and its factor must equal eq. L_col on its own selected
# set (Theta_ss is FP64).
TAU_MIXED = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run_gpu(w, k, precision, targets=None, pool=None, pool_len=None, points=None):
    pts = _dev(w.points if points is None else points, torch.float64)
    tg = _dev(w.targets if targets is None else targets, torch.int32)
    pl = _dev(w.pool if pool is None else pool, torch.int32)
    ln = _dev(w.pool_len if pool_len is None else pool_len, torch.int32)
    out = csel.select_and_factor(pts, w.kernel, tg, pl, ln, k, precision, want_gap=True)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def run_orc(w, k, targets=None, pool=None, pool_len=None, points=None):
    return oracle.select_and_factor(w.points if points is None else points, w.kernel,
                                    w.targets if targets is None else targets, w.pool if pool is None else pool,
                                    w.pool_len if pool_len is None else pool_len, k)


@pytest.fixture(scope="module")
def c1():
    return inputs.workload_plain_fp64()


def test_plain_fp64_parity_and_kl(c1):
    """N=2000 uniform in [0,1]^2, Matern 3/2, l=0.1, C=64, k=16, FP64."""
    print("case: plain fp64 n=2000 C=64 k=16", flush=True)
    g = run_gpu(c1, 16, "fp64")
    o = run_orc(c1, 16)
    rep = compare_single(g, o, THR, factor_rtol=1e-5, logcv_atol=1e-8)
    print(rep["identical"], "of", rep["columns"], "columns identical; worst factor", rep["worst_factor_rel"])
    assert rep["identical"] >= rep["fully_decisive"]
    ld = oracle.logdet(oracle.covariance(c1.points, c1.kernel))
    assert kl_rel_error(float(np.sum(g["log_condvar"])), float(np.sum(o["log_condvar"])), ld) <= 1e-6
    # the GPU gaps agree with the oracle's on identical columns
    for t in range(0, 2000, 37):
        if np.array_equal(g["sel"][t], o["sel"][t]):
            m = o["sel"][t] >= 0
            np.testing.assert_allclose(g["gap"][t][m], o["gap"][t][m], rtol=1e-3, atol=1e-6)


def check(precision, g, w, k, cols=None, targets=None, pool=None, pool_len=None):
    """FP64: strict comparison with the oracle's own greedy run.  Mixed: replay
    of the GPU's picks in FP64 (see TAU_MIXED) plus agreement statistics."""
    targets = w.targets if targets is None else targets
    pool = w.pool if pool is None else pool
    pool_len = w.pool_len if pool_len is None else pool_len
    cols = np.arange(len(targets)) if cols is None else cols
    o = oracle.select_and_factor(w.points, w.kernel, targets[cols], pool[cols], pool_len[cols], k)
    gs = {key: v[cols] for key, v in g.items()}
    if precision == "fp64":
        rep = compare_single(gs, o, THR, factor_rtol=1e-5, logcv_atol=1e-8)
        assert rep["identical"] >= rep["fully_decisive"]
    else:
        np.testing.assert_array_equal(gs["status"] >= 2, o["status"] >= 2)
        short, fac = replay_check(g, w.points, w.kernel, targets, pool, pool_len, k, cols, TAU_MIXED, 1e-3)
        same = np.all(gs["sel"] == o["sel"], axis=1)
        rep = {"columns": len(cols), "identical": int(same.sum()), "worst_shortfall": short,
               "worst_factor_rel": fac}
    print(precision, rep, flush=True)
    return rep, o


def test_plain_mixed_parity(c1):
    print("case: plain mixed n=2000 C=64 k=16", flush=True)
    g = run_gpu(c1, 16, "mixed")
    rep, o = check("mixed", g, c1, 16)
    assert rep["identical"] >= 0.95 * rep["columns"]
    ld = oracle.logdet(oracle.covariance(c1.points, c1.kernel))
    e = kl_rel_error(float(np.sum(g["log_condvar"])), float(np.sum(o["log_condvar"])), ld)
    print("mixed KL rel err", e)
    assert e <= 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_reduced_parity(precision):
    """The batched workload's distribution at reduced N (uniform [0,1]^3,
    Matern 5/2, l=0.05, nugget 1e-6, C=256 uneven at the tail, k=32)."""
    print(f"case: batched n=12000 C=256 k=32 {precision}", flush=True)
    w = inputs.workload_plain_batched(n=12000, seed=22)
    g = run_gpu(w, 32, precision)
    rep, _ = check(precision, g, w, 32)
    assert rep["identical"] >= 0.95 * rep["columns"]


def test_batched_full_size_sampled():
    """Full N = 100,000 in the benchmark's launch configuration (mixed, one
    launch over all columns); the oracle recomputes a seeded sample of 1500
    columns one by one."""
    print("case: batched n=100000 C=256 k=32 mixed, sampled", flush=True)
    w = inputs.workload_plain_batched()
    g = run_gpu(w, 32, "mixed")
    rng = np.random.default_rng(7)
    idx = np.sort(np.concatenate([rng.choice(len(w.targets) - 400, 1100, replace=False),
                                  np.arange(len(w.targets) - 400, len(w.targets))]))
    rep, _ = check("mixed", g, w, 32, cols=idx)
    assert rep["identical"] >= 0.95 * rep["columns"]
    assert np.all(g["status"] == 0)


def test_edge_cases_ragged_empty_k0_k1():
    print("case: edge cases", flush=True)
    w = inputs.workload_plain_fp64(n=500, seed=3)
    rng = np.random.default_rng(1)
    plen = w.pool_len.copy()
    plen[::3] = np.minimum(plen[::3], rng.integers(0, 20, size=len(plen[::3])))
    plen[5] = 0
    for k in (0, 1, 7, 16):
        for prec in ("fp64", "mixed"):
            g = run_gpu(w, k, prec, pool_len=plen)
            check(prec, g, w, k, pool_len=plen)
    # k = 0: L_ii = 1/sqrt(Theta_ii)
    g = run_gpu(w, 0, "fp64")
    np.testing.assert_allclose(g["factor"][:, 0], 1.0, rtol=1e-14)


def test_large_pool_and_odd_stride():
    """Pool stride 512 (8 rows per lane) and a stride that is not a power of two."""
    print("case: stride 512 / 100", flush=True)
    x = inputs.uniform_points(3000, 2, 12)
    for C, k in ((512, 32), (100, 9)):
        w = inputs.single_target("t", x, inputs.Kernel(3, 0.05), C, k, targets=np.arange(0, 3000, 5))
        for prec in ("fp64", "mixed"):
            g = run_gpu(w, k, prec)
            rep, _ = check(prec, g, w, k)
            assert rep["identical"] >= 0.9 * rep["columns"]


def test_status_codes():
    print("case: status codes", flush=True)
    # duplicated points, no nugget: the twin becomes ineligible (status 1)
    x = np.array([[0.0, 0.0], [0.1, 0.0], [0.1, 0.0], [0.5, 0.5]])
    w = inputs.SingleTargetWorkload("dup", x, np.zeros(4), inputs.Kernel(3, 0.3), np.array([0], np.int32),
                                    np.array([[1, 2, -1, -1]], np.int32), np.array([2], np.int32), 2)
    for prec in ("fp64", "mixed"):
        g = run_gpu(w, 2, prec)
        assert g["status"][0] == 1
        assert g["sel"][0, 1] == -1
        o = run_orc(w, 2)
        assert o["status"][0] == 1
        assert g["sel"][0, 0] == o["sel"][0, 0]
        np.testing.assert_allclose(g["factor"][0, :2], o["factor"][0, :2], rtol=1e-6)
    # the target's own location in its pool, no nugget: the copy is picked first
    # (score 1, the largest possible), and Theta' over [copy, ..., target] is
    # singular -- its last pivot is exactly 0 -- so the column is not defined
    # (status 2, all NaN), in the oracle's Cholesky and in the kernel's L D L^T
    x3 = np.array([[0.2, 0.2], [0.2, 0.2], [0.6, 0.1], [0.9, 0.9]])
    w3 = inputs.SingleTargetWorkload("twin", x3, np.zeros(4), inputs.Kernel(3, 0.3), np.array([0], np.int32),
                                     np.array([[1, 2, -1, -1]], np.int32), np.array([2], np.int32), 2)
    o3 = run_orc(w3, 2)
    assert o3["status"][0] == 2 and o3["sel"][0, 0] == 1
    for prec in ("fp64", "mixed"):
        g3 = run_gpu(w3, 2, prec)
        assert g3["status"][0] == 2, (prec, g3["status"])
        assert g3["sel"][0, 0] == 1
        assert np.all(np.isnan(g3["factor"][0])) and np.isnan(g3["log_condvar"][0])
    # out-of-range pool index and target: status 3, nothing read out of bounds
    w2 = inputs.SingleTargetWorkload("bad", x, np.zeros(4), inputs.Kernel(3, 0.3), np.array([0, 7, 1], np.int32),
                                     np.array([[1, 9, -1, -1], [1, 2, 3, -1], [2, 3, -1, -1]], np.int32),
                                     np.array([2, 3, 5], np.int32), 2)
    g = run_gpu(w2, 2, "fp64")
    assert list(g["status"]) == [3, 3, 3]
    assert np.all(g["sel"] == -1)


def test_deterministic_and_sum():
    print("case: determinism + sum", flush=True)
    w = inputs.workload_plain_fp64(n=1500, seed=4)
    a = run_gpu(w, 16, "mixed")
    b = run_gpu(w, 16, "mixed")
    for key in a:
        assert np.array_equal(a[key], b[key], equal_nan=True), key
    x = torch.from_numpy(np.random.default_rng(0).standard_normal(100003)).cuda()
    s1 = csel.sum(x).item()
    s2 = csel.sum(x).item()
    assert s1 == s2
    assert s1 == pytest.approx(float(np.sum(x.cpu().numpy())), rel=1e-12, abs=1e-9)


def test_host_validation_errors():
    x = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(csel.CselError):
        csel.select_and_factor(x, inputs.Kernel(4, 0.1), t, p, t, 2)
    with pytest.raises(csel.CselError):
        csel.select_and_factor(x, inputs.Kernel(3, 0.1), t, p, t, 40)
    with pytest.raises(ValueError):
        csel.select_and_factor(x.cpu(), inputs.Kernel(3, 0.1), t, p, t, 2)
    # a column list shorter than the capacity it claims is refused before launch
    out = csel.select_and_factor(x, inputs.Kernel(3, 0.1), t, p, t, 2)
    with pytest.raises(ValueError):
        csel.select_and_factor_list(x, inputs.Kernel(3, 0.1), t, p, t, 2, "mixed", t, t, 5, out)


@pytest.mark.parametrize("C", [256, 128, 512])
def test_gap_and_no_gap_variants_agree(C):
    """Asking for top2_gap does not change the answer: the kernel without it
    (a plain maximum instead of the top-two reduction) takes the same
    decisions and computes the same values bit for bit, in FP64 (both rank
    by the FP64 score) and in mixed precision (both rank by the FP32 score of
    the FP64 state, equal scores to the smallest slot).  The mixed run also
    passes the FP64 replay; the gaps lie in [0, 1]."""
    print(f"case: gap vs no-gap variants C={C}", flush=True)
    w = inputs.workload_plain_batched(n=6000, seed=9) if C == 256 else \
        inputs.single_target("g", inputs.cluster_points(6000, 3, 9), inputs.Kernel(3, 0.05), C, 32,
                             targets=np.arange(0, 6000, 2))
    pts = _dev(w.points, torch.float64)
    args = (_dev(w.targets, torch.int32), _dev(w.pool, torch.int32), _dev(w.pool_len, torch.int32))
    for prec in ("fp64", "mixed"):
        a = csel.select_and_factor(pts, w.kernel, *args, 32, prec, want_gap=True)
        b = csel.select_and_factor(pts, w.kernel, *args, 32, prec, want_gap=False)
        torch.cuda.synchronize()
        for key in ("sel", "factor", "log_condvar", "status"):
            assert torch.equal(a[key], b[key]), (prec, key)
        gap = a["gap"].cpu().numpy()
        ok = ~np.isnan(gap)
        assert np.all((gap[ok] >= 0) & (gap[ok] <= 1))
        assert np.array_equal(ok, a["sel"].cpu().numpy() >= 0)
        if prec == "mixed" and C == 256:
            ga = {key: v.cpu().numpy() for key, v in a.items()}
            cols = np.arange(len(w.targets))
            short, fac = replay_check(ga, w.points, w.kernel, w.targets, w.pool, w.pool_len, 32, cols, TAU_MIXED,
                                      1e-3)
            print("mixed replay worst shortfall", short, "factor", fac)


@pytest.mark.parametrize("prec,C", [("mixed", 128), ("fp64", 128), ("mixed", 512)])
def test_list_variant_matches_full_run(prec, C):
    """csel_select_and_factor_list on an odd-length random subset of the
    columns (capacity larger than the count, list positions split over the
    eight XCD segments) reproduces the full run bit for bit on the listed
    columns and leaves every other column's outputs untouched."""
    print(f"case: list variant {prec} C={C}", flush=True)
    x = inputs.cluster_points(6001, 3, 21)
    w = inputs.single_target("list", x, inputs.Kernel(3, 0.05), C, 32, targets=np.arange(0, 6001, 3))
    k, T = 32, len(w.targets)
    pts, tg = _dev(w.points, torch.float64), _dev(w.targets, torch.int32)
    pl, ln = _dev(w.pool, torch.int32), _dev(w.pool_len, torch.int32)
    ref = {key: v.cpu().numpy() for key, v in csel.select_and_factor(pts, w.kernel, tg, pl, ln, k, prec).items()}
    cols = np.random.default_rng(8).choice(T, 333, replace=False).astype(np.int32)
    lst = np.full(T, -1, np.int32)
    lst[: len(cols)] = cols
    out = {
        "sel": torch.full((T, k), -7, dtype=torch.int32, device="cuda"),
        "factor": torch.full((T, k + 1), 7.0, dtype=torch.float64, device="cuda"),
        "log_condvar": torch.full((T,), 7.0, dtype=torch.float64, device="cuda"),
        "status": torch.full((T,), 9, dtype=torch.uint8, device="cuda"),
    }
    csel.select_and_factor_list(pts, w.kernel, tg, pl, ln, k, prec, _dev(lst, torch.int32),
                                _dev(np.array([len(cols)], np.int32), torch.int32), T, out)
    g = {key: v.cpu().numpy() for key, v in out.items()}
    for key in ("sel", "factor", "log_condvar", "status"):
        assert np.array_equal(g[key][cols], ref[key][cols], equal_nan=True), key
    rest = np.setdiff1d(np.arange(T), cols)
    assert np.all(g["sel"][rest] == -7) and np.all(g["status"][rest] == 9)
    assert np.all(g["factor"][rest] == 7.0) and np.all(g["log_condvar"][rest] == 7.0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_pool_selection_at_capacity(prec):
    """k = 32 (the largest pick capacity) on pools of exactly 32 and 33
    candidates: with C = k every candidate is selected, so the column is the
    exact KL-optimal column on the whole pool, checked against a dense FP64
    solve; with C = k + 1 one candidate is left out."""
    print(f"case: k = C = 32 {prec}", flush=True)
    x = inputs.uniform_points(1200, 2, 77)
    for C in (32, 33):
        w = inputs.single_target("cap", x, inputs.Kernel(3, 0.05), C, 32, targets=np.arange(0, 1100, 7))
        g = run_gpu(w, 32, prec)
        rep, _ = check(prec, g, w, 32)
        full = w.pool_len == 32
        if C == 32:
            assert np.all(np.sum(g["sel"][full] >= 0, axis=1) == 32)
            for t in np.where(full)[0][:12]:
                s = np.concatenate([[w.targets[t]], g["sel"][t]])
                th = oracle.covariance(w.points[s], w.kernel)
                e = np.zeros(len(s))
                e[0] = 1.0
                col = np.linalg.solve(th, e)
                col /= math.sqrt(col[0])
                tol = 1e-9 if prec == "fp64" else 1e-6
                np.testing.assert_allclose(g["factor"][t], col, rtol=0, atol=tol * np.max(np.abs(col)))


def test_list_variant_with_zero_count():
    """A column list whose device count is 0 writes nothing."""
    print("case: list variant, count 0", flush=True)
    w = inputs.workload_plain_fp64(n=300, seed=6)
    T = len(w.targets)
    out = {
        "sel": torch.full((T, 16), -7, dtype=torch.int32, device="cuda"),
        "factor": torch.full((T, 17), 7.0, dtype=torch.float64, device="cuda"),
        "log_condvar": torch.full((T,), 7.0, dtype=torch.float64, device="cuda"),
        "status": torch.full((T,), 9, dtype=torch.uint8, device="cuda"),
    }
    csel.select_and_factor_list(_dev(w.points, torch.float64), w.kernel, _dev(w.targets, torch.int32),
                                _dev(w.pool, torch.int32), _dev(w.pool_len, torch.int32), 16, "mixed",
                                _dev(np.arange(T, dtype=np.int32), torch.int32),
                                _dev(np.array([0], np.int32), torch.int32), T, out)
    torch.cuda.synchronize()
    assert torch.all(out["sel"] == -7) and torch.all(out["status"] == 9)
    assert torch.all(out["factor"] == 7.0) and torch.all(out["log_condvar"] == 7.0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("C,k", [(64, 16), (128, 32), (200, 32), (512, 32), (512, 7)])
def test_multi_wave_schedule_matches_one_wave(prec, C, k):
    """csel_select_and_factor_sched with the pool split over 2 or 4 waves per
    column gives the one-wave kernel's outputs bit for bit -- in natural order
    and through a column list -- on ragged pools, empty pools, bad rows
    (status 3) and a column count that does not fill the last workgroup; the
    FP64 run also matches the oracle."""
    print(f"case: multi-wave schedule {prec} C={C} k={k}", flush=True)
    x = inputs.cluster_points(5003, 3, 61)
    w = inputs.single_target("mw", x, inputs.Kernel(5, 0.06), C, k, targets=np.arange(0, 5003, 4))
    plen = w.pool_len.copy()
    plen[::7] = np.minimum(plen[::7], np.random.default_rng(2).integers(0, C + 1, size=len(plen[::7])))
    plen[3] = 0
    pool = w.pool.copy()
    tg = w.targets.copy()
    tg[10] = -4                            # bad target
    pool[20, min(3, plen[20] - 1)] = 99999  # bad pool id
    T = len(tg)
    pts = _dev(w.points, torch.float64)
    args = (pts, w.kernel, _dev(tg, torch.int32), _dev(pool, torch.int32), _dev(plen, torch.int32), k, prec)
    ref = {key: v.cpu().numpy() for key, v in csel.select_and_factor(*args).items()}
    waves = csel.select_waves_per_column(C)
    assert waves == (2 if C <= 128 else 4)
    got = {key: v.cpu().numpy() for key, v in csel.select_and_factor_sched(*args, waves=waves).items()}
    torch.cuda.synchronize()
    for key in ("sel", "factor", "log_condvar", "status"):
        assert np.array_equal(got[key], ref[key], equal_nan=True), key
    assert got["status"][10] == 3 and got["status"][20] == 3
    # through a column list (a random subset, capacity above the count)
    cols = np.random.default_rng(3).choice(T, 301, replace=False).astype(np.int32)
    lst = np.full(T, -1, np.int32)
    lst[: len(cols)] = cols
    out = {"sel": torch.full((T, k), -7, dtype=torch.int32, device="cuda"),
           "factor": torch.full((T, k + 1), 7.0, dtype=torch.float64, device="cuda"),
           "log_condvar": torch.full((T,), 7.0, dtype=torch.float64, device="cuda"),
           "status": torch.full((T,), 9, dtype=torch.uint8, device="cuda")}
    csel.select_and_factor_sched(*args, waves=waves, col_list=_dev(lst, torch.int32),
                                 col_count=_dev(np.array([len(cols)], np.int32), torch.int32), max_cols=T, out=out)
    g2 = {key: v.cpu().numpy() for key, v in out.items()}
    for key in ("sel", "factor", "log_condvar", "status"):
        assert np.array_equal(g2[key][cols], ref[key][cols], equal_nan=True), key
    rest = np.setdiff1d(np.arange(T), cols)
    assert np.all(g2["status"][rest] == 9) and np.all(g2["sel"][rest] == -7)
    if prec == "fp64":
        good = np.setdiff1d(np.arange(T), [10, 20])
        o = oracle.select_and_factor(w.points, w.kernel, tg[good], pool[good], plen[good], k)
        gg = {key: v[good] for key, v in got.items()}
        gg["gap"] = o["gap"]
        rep = compare_single(gg, o, THR, factor_rtol=1e-5, logcv_atol=1e-8)
        assert rep["identical"] >= rep["fully_decisive"]
    # unsupported wave counts are refused on the host
    with pytest.raises(csel.CselError):
        csel.select_and_factor_sched(*args, waves=3)
