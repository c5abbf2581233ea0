"""GPU parity of csel_aggregated_select (multi-target selection, aggregated
columns, GP posterior variances) and csel_apply_factor against the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2307_11648_amd import csel, inputs
from parity import decisive_prefix

pytestmark = pytest.mark.gpu

THR = 1e-6
# Mixed precision: a GPU pick may lose at most this much log-determinant
# (log(1 - s_pick) - log(1 - s_best), exact FP64 scores on the GPU's own path)
# per step; FP32 covariances perturb 1 - var2/var1 by about u32 * prior / var2.
TAU_LOGDET = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run_gpu(w, k, precision, want_factor=True, want_post_var=True, max_members=None, pool=None, members=None):
    mm = int(np.max(np.diff(w.group_ptr))) if max_members is None else max_members
    out = csel.aggregated_select(_t(w.points, torch.float64), w.kernel, _t(w.group_ptr, torch.int32),
                                 _t(w.members if members is None else members, torch.int32), mm,
                                 _t(w.pool if pool is None else pool, torch.int32), _t(w.pool_len, torch.int32), k,
                                 precision, want_factor=want_factor, want_post_var=want_post_var, want_gap=True)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items() if key != "workspace"}


@pytest.fixture(scope="module")
def agg_small():
    return inputs.workload_aggregated(n=6000, seed=31, C=128, k=24, mmin=4, mmax=12)


def _compare_groups(g, o, w, thr, check_values=True, vtol=1e-5):
    G = len(w.group_ptr) - 1
    np.testing.assert_array_equal(g["status"], o["status"])
    same = 0
    worst = 0.0
    for gi in range(G):
        if o["status"][gi] >= 2:
            continue
        p = decisive_prefix(o["gap"][gi], thr)
        assert np.array_equal(g["sel"][gi, :p], o["sel"][gi, :p]), f"group {gi}: decisive picks differ"
        if not np.array_equal(g["sel"][gi], o["sel"][gi]):
            continue
        same += 1
        assert g["logdet"][gi] == pytest.approx(o["logdet"][gi], rel=1e-9 if thr == THR else 1e-3, abs=1e-9)
        if check_values:
            b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
            for a in range(b, e):
                gv = g["vals"][g["val_ptr"][a]:g["val_ptr"][a + 1]]
                ov = o["vals"][o["val_ptr"][a]:o["val_ptr"][a + 1]]
                gr = g["rows"][g["val_ptr"][a]:g["val_ptr"][a + 1]]
                orr = o["rows"][o["val_ptr"][a]:o["val_ptr"][a + 1]]
                n = len(ov)
                assert np.array_equal(gr[:n], orr)
                err = float(np.max(np.abs(gv[:n] - ov)) / np.max(np.abs(ov)))
                worst = max(worst, err)
                assert err <= vtol, f"group {gi} member {a}: column error {err}"
    return same, worst


def test_aggregated_fp64_parity(agg_small):
    print("case: aggregated fp64 n=6000 C=128 k=24 m=4..12", flush=True)
    w = agg_small
    g = run_gpu(w, w.k, "fp64")
    o = oracle.aggregated_select(w.points, w.kernel, w.group_ptr, w.members, w.pool, w.pool_len, w.k,
                                 want_factor=True, want_post_var=True)
    same, worst = _compare_groups(g, o, w, THR)
    G = len(w.group_ptr) - 1
    print(f"fp64: {same} of {G} groups identical, worst column error {worst:.2e}")
    assert same >= 0.97 * G
    np.testing.assert_allclose(g["member_log_condvar"], o["member_log_condvar"], rtol=1e-8, atol=1e-9)
    # telescoping (eq. obj_mult): member log condvars sum to the tracked log det
    for gi in range(G):
        b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
        assert np.sum(g["member_log_condvar"][b:e]) == pytest.approx(g["logdet"][gi], rel=1e-8, abs=1e-8)
    np.testing.assert_allclose(g["post_var"], o["post_var"], rtol=1e-7, atol=1e-12)


def test_aggregated_mixed_replay(agg_small):
    print("case: aggregated mixed n=6000 C=128 k=24 m=4..12", flush=True)
    w = agg_small
    g = run_gpu(w, w.k, "mixed", want_post_var=False)
    G = len(w.group_ptr) - 1
    worst_loss = 0.0
    worst_val = 0.0
    for gi in range(G):
        b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
        T = w.members[b:e]
        pool = w.pool[gi, : w.pool_len[gi]]
        r = oracle.multi_replay_one(w.points, w.kernel, T, pool, w.k, g["sel"][gi])
        assert r["status"] != 5, f"group {gi}: a GPU pick is not a valid candidate"
        n = int(np.sum(g["sel"][gi] >= 0))
        for s in range(n):
            loss = math.log1p(-r["pick"][s]) - math.log1p(-r["best"][s])
            worst_loss = max(worst_loss, loss)
            assert loss <= TAU_LOGDET, f"group {gi} step {s}: log det loss {loss}"
        cols = oracle.aggregated_columns(w.points, w.kernel, T, g["sel"][gi])
        for a in range(b, e):
            gv = g["vals"][g["val_ptr"][a]:g["val_ptr"][a + 1]]
            off = sum(len(T) - q + n for q in range(a - b))
            ov = cols["vals"][off: off + len(T) - (a - b) + n]
            err = float(np.max(np.abs(gv[: len(ov)] - ov)) / np.max(np.abs(ov)))
            worst_val = max(worst_val, err)
            assert err <= 1e-3
        # mixed tracked log det vs FP64 log det on the same selection
        assert g["logdet"][gi] == pytest.approx(r["logdet"], rel=1e-3, abs=1e-3)
    print(f"mixed: worst per-step log det loss {worst_loss:.2e}, worst column error {worst_val:.2e}")


def test_gp_posterior_variance():
    """GP prediction batches: training points uniform in [0,1]^2, 4 spatial
    batches of 64 prediction points, Matern 5/2, l = 0.03, pools of the 512
    training points nearest to any batch member, k = 64 (reduced sizes),
    FP64: selections and posterior variances against the oracle."""
    print("case: gp n_train=20000 m=64 C=512 k=64 fp64", flush=True)
    w = inputs.workload_gp(n_train=20000, n_pred=256, C=512, k=64, n_strips=2, per_strip=2)
    g = run_gpu(w, w.k, "fp64", want_factor=False)
    G = len(w.group_ptr) - 1
    o = oracle.aggregated_select(w.points, w.kernel, w.group_ptr, w.members, w.pool, w.pool_len, w.k,
                                 want_factor=False, want_post_var=True)
    same, _ = _compare_groups(g, o, w, THR, check_values=False)
    assert same >= G - 1
    for gi in range(G):
        if np.array_equal(g["sel"][gi], o["sel"][gi]):
            b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
            np.testing.assert_allclose(g["post_var"][b:e], o["post_var"][b:e], rtol=1e-7, atol=1e-13)


def test_gp_full_shape_sample_matches_oracle():
    """The GP prediction workload at its full shape: 500,000 training points,
    64 batches of 64 prediction points, pools of 2,048, k = 128, FP64 (the
    batches' rows split over cooperatively launched workgroups of 1,024
    threads).  Four batches against the oracle: picks up to the first top-two
    gap below 1e-6; on batches whose picks all agree, posterior variances to
    1e-7 relative and log det to 1e-8 relative.  (64 clustered targets under
    the smooth kernel drive their conditional variances to about 1e-7 of the
    prior, where one FP64 rounding moves the log of a variance by about
    1e-16 * 1e7 = 1e-9; log det sums some 200 such terms, about 800 in
    magnitude.)"""
    print("case: gp full shape n_train=500000 G=64 m=64 C=2048 k=128 fp64", flush=True)
    w = inputs.workload_gp(n_train=500_000)
    g = run_gpu(w, w.k, "fp64", want_factor=False)
    assert np.all(g["status"] == 0)
    same = 0
    worst_pv = 0.0
    sample = (0, 21, 42, 63)
    for gi in sample:
        b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
        o = oracle.aggregated_select(w.points, w.kernel, np.array([0, e - b], np.int32), w.members[b:e],
                                     w.pool[gi: gi + 1], w.pool_len[gi: gi + 1], w.k, want_factor=False,
                                     want_post_var=True)
        p = decisive_prefix(o["gap"][0], THR)
        assert np.array_equal(g["sel"][gi, :p], o["sel"][0, :p]), gi
        if not np.array_equal(g["sel"][gi], o["sel"][0]):
            continue
        same += 1
        assert g["logdet"][gi] == pytest.approx(o["logdet"][0], rel=1e-8, abs=1e-9)
        pv = g["post_var"][b:e]
        np.testing.assert_allclose(pv, o["post_var"], rtol=1e-7, atol=1e-13)
        worst_pv = max(worst_pv, float(np.max(np.abs(pv - o["post_var"]) / o["post_var"])))
    print(f"{same} of {len(sample)} batches identical; worst posterior variance error {worst_pv:.2e}", flush=True)
    assert same >= len(sample) - 1


def test_gp_split_rows_match_one_workgroup_per_group():
    """FP64 runs with at most 128 groups and more than 256 rows a group split
    each group's rows over several workgroups (cooperative launch; 1,024,
    512 or 256 threads a workgroup depending on how many groups share the
    chip); larger runs give each group one workgroup.  Both round alike and
    groups are independent, so the first H groups run alone reproduce what
    the full run of 144 gives them bit for bit: picks, gaps, log det and
    posterior variances.  H = 64, 50 and 20 take the three block sizes
    (groups of 1,040 rows on 256 CUs).  The set includes an out-of-range pool
    id (status 3), an empty pool and a pool shorter than k."""
    print("case: gp split rows n_train=30000 G=144 m=16 C=1024 k=48 fp64", flush=True)
    w = inputs.workload_gp(n_train=30000, n_pred=2304, C=1024, k=48, n_strips=12, per_strip=12)
    G = len(w.group_ptr) - 1
    assert G == 144
    pool = w.pool.copy()
    plen = w.pool_len.copy()
    pool[3, 5] = len(w.points) + 7
    plen[5] = 0
    plen[6] = 10
    w.pool_len[:] = plen
    full = run_gpu(w, w.k, "fp64", want_factor=False, pool=pool)
    assert full["status"][3] == 3
    for H in (64, 50, 20):
        print(f"case: first {H} groups", flush=True)
        sub = inputs.GroupWorkload(w.name, w.points, w.kernel, w.group_ptr[: H + 1].copy(),
                                   w.members[: w.group_ptr[H]].copy(), pool[:H].copy(), plen[:H].copy(), w.k,
                                   w.later_only, w.meta)
        part = run_gpu(sub, w.k, "fp64", want_factor=False, pool=sub.pool,
                       max_members=int(np.max(np.diff(w.group_ptr))))
        np.testing.assert_array_equal(part["status"], full["status"][:H])
        assert np.all(part["sel"][3] == -1) and np.isnan(part["logdet"][3])
        assert np.all(part["sel"][5] == -1) and part["status"][5] == 0
        assert np.sum(part["sel"][6] >= 0) == 10
        np.testing.assert_array_equal(part["sel"], full["sel"][:H])
        np.testing.assert_array_equal(part["gap"], full["gap"][:H])
        np.testing.assert_array_equal(part["logdet"], full["logdet"][:H])
        # (a status-3 group's posterior variances are left unwritten)
        for gi in range(H):
            if full["status"][gi] < 2:
                b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
                np.testing.assert_array_equal(part["post_var"][b:e], full["post_var"][b:e])


def test_group_slab_caches_keep_the_split_schedule_bits():
    """Pools of 512 with groups of 8-32 (one 576-thread workgroup per group):
    the slab kernel keeps the first columns of both factors in LDS column
    caches, the split-row schedule keeps every column in global memory; both
    take the same multiply-adds in the same order, so picks, gaps, log
    determinants (and in FP64 posterior variances) agree bit for bit."""
    # pools of 512 (part of each factor cached), and pools of 64 with k = 4,
    # where the caches hold every column and the slab is never touched
    for name, w, split in (("n=2000 C=512 k=64 m=8..32", inputs.workload_aggregated(n=2000, C=512, k=64), "split512"),
                           ("n=500 C=64 k=4 m=2..8",
                            inputs.workload_aggregated(n=500, seed=7, C=64, k=4, mmin=2, mmax=8), "split256")):
        print(f"case: slab caches vs split rows, aggregated {name}", flush=True)
        # few enough groups for the split schedule's cooperative launch
        assert len(w.group_ptr) - 1 <= 128
        dev = dict(pts=_t(w.points, torch.float64), gp=_t(w.group_ptr, torch.int32), mem=_t(w.members, torch.int32),
                   pl=_t(w.pool, torch.int32), ln=_t(w.pool_len, torch.int32))
        mm = int(np.max(np.diff(w.group_ptr)))

        def run(precision, schedule, post_var):
            o = csel.aggregated_select(dev["pts"], w.kernel, dev["gp"], dev["mem"], mm, dev["pl"], dev["ln"], w.k,
                                       precision, want_post_var=post_var, want_gap=True, schedule=schedule)
            torch.cuda.synchronize()
            return {key: v.cpu().numpy() for key, v in o.items() if key != "workspace"}

        for precision, post_var in (("fp64", True), ("mixed", False)):
            ref = run(precision, split, post_var)
            got = run(precision, "one_group", post_var)
            assert np.mean(ref["status"] == 0) > 0.9
            for key in ref:
                np.testing.assert_array_equal(got[key], ref[key], err_msg=f"{name} {precision} {key}")
            print(f"{precision}: slab with LDS caches == split rows ({len(w.group_ptr) - 1} groups)", flush=True)


def test_explicit_schedules_are_bit_identical():
    """csel_aggregated_select_sched: one workgroup per group and the three
    split-row block sizes give the same bits (FP64 with posterior variances
    and gaps; mixed without); the tuner picks one of them and its result is
    the same again.  Schedules outside their range are refused."""
    from paper_2307_11648_amd import autotune

    print("case: explicit schedules gp n_train=20000 G=16 m=64 C=1024 k=64", flush=True)
    w = inputs.workload_gp(n_train=20000, n_pred=1024, C=1024, k=64, n_strips=4, per_strip=4)
    dev = dict(pts=_t(w.points, torch.float64), gp=_t(w.group_ptr, torch.int32), mem=_t(w.members, torch.int32),
               pl=_t(w.pool, torch.int32), ln=_t(w.pool_len, torch.int32))
    mm = int(np.max(np.diff(w.group_ptr)))

    def run(precision, schedule, post_var):
        o = csel.aggregated_select(dev["pts"], w.kernel, dev["gp"], dev["mem"], mm, dev["pl"], dev["ln"], w.k,
                                   precision, want_post_var=post_var, want_gap=True, schedule=schedule)
        torch.cuda.synchronize()
        return {key: v.cpu().numpy() for key, v in o.items() if key != "workspace"}

    for precision, post_var in (("fp64", True), ("mixed", False)):
        ref = run(precision, "one_group", post_var)
        assert np.all(ref["status"] == 0)
        for schedule in ("split256", "split512", "split1024", "auto"):
            got = run(precision, schedule, post_var)
            for key in ref:
                np.testing.assert_array_equal(got[key], ref[key], err_msg=f"{precision} {schedule} {key}")
        print(f"{precision}: one_group, split256/512/1024 and auto identical", flush=True)
    tuner = autotune.SelectTuner()
    t = tuner.aggregated_select(dev["pts"], w.kernel, dev["gp"], dev["mem"], mm, dev["pl"], dev["ln"], w.k, "fp64",
                                want_post_var=True, want_gap=True)
    torch.cuda.synchronize()
    (key, choice), = tuner.choices.items()
    print("tuned", key, choice, flush=True)
    assert choice["schedule"] in autotune.AGG_SCHEDULES
    ref = run("fp64", "one_group", True)
    for k_ in ref:
        np.testing.assert_array_equal(t[k_].cpu().numpy(), ref[k_])
    # out of range: the register kernel with posterior variances; a split with factor output
    with pytest.raises(csel.CselError):
        run("mixed", "register", True)
    with pytest.raises(csel.CselError):
        csel.aggregated_select(dev["pts"], w.kernel, dev["gp"], dev["mem"], mm, dev["pl"], dev["ln"], w.k, "fp64",
                               want_factor=True, schedule="split256")


def test_gp_mixed_selection_runs_to_k():
    """The same batches in mixed precision: 64 clustered targets under a
    smooth kernel drive var2 / prior to 1e-4..1e-7, below what an FP32
    evaluation resolves, so the slab kernel keeps the target-conditioned
    factor (var2) in FP64 and the selection runs to k (no early stop); each
    pick loses at most TAU_LOGDET of log det (FP64 replay).  Posterior
    variances are FP64-only: asking for them in mixed precision is refused."""
    print("case: gp n_train=20000 m=64 C=512 k=64 mixed", flush=True)
    w = inputs.workload_gp(n_train=20000, n_pred=256, C=512, k=64, n_strips=2, per_strip=2)
    g = run_gpu(w, w.k, "mixed", want_factor=False, want_post_var=False)
    assert np.all(g["status"] == 0)
    worst_loss = 0.0
    for gi in range(len(w.group_ptr) - 1):
        b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
        r = oracle.multi_replay_one(w.points, w.kernel, w.members[b:e], w.pool[gi, : w.pool_len[gi]], w.k,
                                    g["sel"][gi])
        assert r["status"] != 5
        for s in range(int(np.sum(g["sel"][gi] >= 0))):
            loss = math.log1p(-r["pick"][s]) - math.log1p(-r["best"][s])
            worst_loss = max(worst_loss, loss)
            assert loss <= TAU_LOGDET
        assert g["logdet"][gi] == pytest.approx(r["logdet"], rel=1e-6, abs=1e-6)
    print(f"mixed: worst per-step log det loss {worst_loss:.2e}")
    with pytest.raises(csel.CselError):
        run_gpu(w, w.k, "mixed", want_factor=False, want_post_var=True)


def test_aggregated_status_codes(agg_small):
    print("case: aggregated status codes", flush=True)
    w = agg_small
    # a pool that reaches before the group's last member -> status 4 with factor output
    pool = w.pool.copy()
    pool[0, 0] = w.members[w.group_ptr[0]]
    g = run_gpu(w, w.k, "fp64", pool=pool)
    assert g["status"][0] == 4 and np.all(g["sel"][0] == -1)
    assert np.all(g["status"][1:] <= 1)
    # the same pool without factor output is a valid multi-target problem
    g2 = run_gpu(w, w.k, "fp64", pool=pool, want_factor=False)
    assert g2["status"][0] in (0, 1)
    # group larger than max_members -> status 3 for that group only
    m = np.diff(w.group_ptr)
    g3 = run_gpu(w, w.k, "fp64", max_members=int(m.min()))
    assert np.all((g3["status"] == 3) == (m > m.min()))
    # aggregated pattern beyond the block size -> status 5, selection still valid
    w5 = inputs.workload_aggregated(n=4000, seed=5, C=128, k=80, mmin=20, mmax=24)
    g5 = run_gpu(w5, 80, "fp64")
    assert np.all(g5["status"][np.diff(w5.group_ptr) + np.minimum(80, w5.pool_len) > 96] == 5)


def test_apply_factor():
    print("case: apply_factor", flush=True)
    w = inputs.workload_plain_fp64(n=2000, seed=8)
    pts = _t(w.points, torch.float64)
    out = csel.select_and_factor(pts, w.kernel, _t(w.targets, torch.int32), _t(w.pool, torch.int32),
                                 _t(w.pool_len, torch.int32), 16, "fp64")
    cp, rows, vals = csel.single_target_csc(_t(w.targets, torch.int32), out["sel"], out["factor"])
    x = torch.from_numpy(np.random.default_rng(1).standard_normal(2000)).cuda()
    ylt = csel.apply_factor(cp, rows, vals, x, True)
    yl = csel.apply_factor(cp, rows, vals, x, False)
    torch.cuda.synchronize()
    cp_n, rows_n, vals_n = cp.cpu().numpy(), rows.cpu().numpy(), vals.cpu().numpy()
    xn = x.cpu().numpy()
    np.testing.assert_allclose(ylt.cpu().numpy(), oracle.apply_factor(cp_n, rows_n, vals_n, xn, True), rtol=1e-12,
                               atol=1e-10)
    np.testing.assert_allclose(yl.cpu().numpy(), oracle.apply_factor(cp_n, rows_n, vals_n, xn, False), rtol=1e-12,
                               atol=1e-10)
    # L^T x is deterministic
    assert torch.equal(ylt, csel.apply_factor(cp, rows, vals, x, True))


def test_transpose_factor_and_gather_products():
    """L^T in CSC form (csel_transpose_factor) equals scipy's CSR of L entry
    for entry (padding slots dropped, columns ascending inside a row), and
    the gather on it, y = (L^T)^T x, equals L x from the dense product and
    from the atomic scatter."""
    import scipy.sparse as sp

    print("case: transpose factor", flush=True)
    w = inputs.workload_plain_fp64(n=900, seed=13)
    plen = w.pool_len.copy()
    plen[::5] = np.minimum(plen[::5], 3)  # short pools: padding slots in the [T][k+1] layout
    g = csel.select_and_factor(_t(w.points, torch.float64), w.kernel, _t(w.targets, torch.int32),
                               _t(w.pool, torch.int32), _t(plen, torch.int32), 16, "fp64")
    cp, rows, vals = csel.single_target_csc(_t(w.targets, torch.int32), g["sel"], g["factor"])
    n = len(w.targets)
    tcp, trow, tval = csel.transpose_factor(cp, rows, vals)
    torch.cuda.synchronize()
    tcp, trow, tval = tcp.cpu().numpy(), trow.cpu().numpy(), tval.cpu().numpy()
    r, v = rows.cpu().numpy(), vals.cpu().numpy()
    cols = np.repeat(np.arange(n), 17)
    keep = r >= 0
    L = sp.csc_matrix((v[keep], (r[keep], cols[keep])), shape=(n, n))
    csr = L.tocsr()
    csr.sort_indices()
    nnz = int(keep.sum())
    np.testing.assert_array_equal(tcp, csr.indptr.astype(np.int64))
    np.testing.assert_array_equal(trow[:nnz], csr.indices)
    np.testing.assert_array_equal(tval[:nnz], csr.data)
    assert np.all(trow[nnz:] == -1) and np.all(tval[nnz:] == 0.0)
    x = np.random.default_rng(5).standard_normal(n)
    xt = torch.from_numpy(x).cuda()
    tcp_d, trow_d, tval_d = csel.transpose_factor(cp, rows, vals)
    y_gather = csel.apply_factor(tcp_d, trow_d, tval_d, xt, True).cpu().numpy()
    y_atomic = csel.apply_factor(cp, rows, vals, xt, False).cpu().numpy()
    ref = L @ x
    np.testing.assert_allclose(y_gather, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
    np.testing.assert_allclose(y_atomic, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
    # deterministic: the same bits on a second run
    y2 = csel.apply_factor(tcp_d, trow_d, tval_d, xt, True).cpu().numpy()
    assert np.array_equal(y2, y_gather)
    # an empty factor and one without stored slots
    e0 = csel.transpose_factor(torch.zeros(1, dtype=torch.int64, device="cuda"),
                               torch.zeros(0, dtype=torch.int32, device="cuda"),
                               torch.zeros(0, dtype=torch.float64, device="cuda"))
    e1 = csel.transpose_factor(torch.zeros(4, dtype=torch.int64, device="cuda"),
                               torch.zeros(0, dtype=torch.int32, device="cuda"),
                               torch.zeros(0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert e0[0].cpu().tolist() == [0] and e1[0].cpu().tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("want_gap", [True, False])
def test_aggregated_mixed_register_kernel(want_gap):
    """Mixed precision without posterior variances, pools <= 512, groups <= 32,
    k <= 64 (the register-resident kernel): FP64 replay of every pick, the
    tracked log det against FP64 on the same selection, and the aggregated
    columns; with and without the gap output the picks agree."""
    print(f"case: aggregated mixed register kernel gap={want_gap}", flush=True)
    w = inputs.workload_aggregated(n=9000, seed=33, C=256, k=48, mmin=8, mmax=32)
    mm = int(np.max(np.diff(w.group_ptr)))
    args = (_t(w.points, torch.float64), w.kernel, _t(w.group_ptr, torch.int32), _t(w.members, torch.int32), mm,
            _t(w.pool, torch.int32), _t(w.pool_len, torch.int32), w.k, "mixed")
    out = csel.aggregated_select(*args, want_factor=True, want_post_var=False, want_gap=want_gap)
    other = csel.aggregated_select(*args, want_factor=False, want_post_var=False, want_gap=not want_gap)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "workspace"}
    assert np.array_equal(g["sel"], other["sel"].cpu().numpy())
    G = len(w.group_ptr) - 1
    assert np.all(g["status"] <= 1)
    worst_loss = worst_val = 0.0
    for gi in range(0, G, 3):
        b, e = w.group_ptr[gi], w.group_ptr[gi + 1]
        T = w.members[b:e]
        r = oracle.multi_replay_one(w.points, w.kernel, T, w.pool[gi, : w.pool_len[gi]], w.k, g["sel"][gi])
        assert r["status"] != 5, f"group {gi}: a GPU pick is not a valid candidate"
        n = int(np.sum(g["sel"][gi] >= 0))
        for s in range(n):
            loss = math.log1p(-r["pick"][s]) - math.log1p(-r["best"][s])
            worst_loss = max(worst_loss, loss)
            assert loss <= TAU_LOGDET, f"group {gi} step {s}: log det loss {loss}"
        assert g["logdet"][gi] == pytest.approx(r["logdet"], rel=1e-3, abs=1e-3)
        cols = oracle.aggregated_columns(w.points, w.kernel, T, g["sel"][gi])
        for a in range(b, e):
            gv = g["vals"][g["val_ptr"][a]:g["val_ptr"][a + 1]]
            off = sum(len(T) - q + n for q in range(a - b))
            ov = cols["vals"][off: off + len(T) - (a - b) + n]
            err = float(np.max(np.abs(gv[: len(ov)] - ov)) / np.max(np.abs(ov)))
            worst_val = max(worst_val, err)
            assert err <= 1e-3
        if want_gap:
            assert np.all(np.isfinite(g["gap"][gi, :n])) and np.all(np.isnan(g["gap"][gi, n:]))
    print(f"mixed register kernel: worst per-step log det loss {worst_loss:.2e}, worst column error {worst_val:.2e}")
