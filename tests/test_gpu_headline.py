"""The benchmark's configurations, checked against the FP64 oracle exactly as
they run: the learned-screened step (csel_screened_select: screen, kept-pool
selection and the fallback columns' full-pool selection, mixed precision, no
gap output, replayed from its captured graph), the plain selection on pools
of 512, and the aggregated register kernel on union pools of 512.

Mixed-precision runs are held to two bars:
* a replay of every GPU pick in FP64 (each pick may fall short of the best
  exact score by at most TAU_MIXED of the target's conditional variance, and
  the factor column equals eq. L_col on the GPU's own set);
* the decisive bar: on every step that an FP32 evaluation and GEMV cannot
  flip (parity.mixed_decisive_prefix, an error model of the oracle's own
  run), the GPU's pick is the oracle's.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2307_11648_amd import csel, inputs, screen_train
from parity import compare_single, mixed_decisive_check, replay_check

pytestmark = pytest.mark.gpu

TAU_MIXED = 1e-4
TAU_LOGDET = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _dev(w):
    return _t(w.points, torch.float64), _t(w.targets, torch.int32), _t(w.pool, torch.int32), \
        _t(w.pool_len, torch.int32)


@pytest.fixture(scope="module")
def trained():
    """A screen trained on the GPU on exact FP64 selections of a separate
    clustered cloud (the benchmark's recipe at reduced size)."""
    tr = inputs.workload_clustered(n=12000, seed=40, C=512, k=32)
    P, Tg, Pl, Ln = _dev(tr)
    X, y = screen_train.training_set(P, tr.kernel, Tg, Pl, Ln, 32, "fp64")
    p, pb, _ = screen_train.train(X, y, steps=1000, batch=8192, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    return p, pb


def _mixed_checks(g, w, targets, pool, plen, k, label):
    """Status, replay and decisive bar of a mixed run against the oracle on
    the given per-column pools."""
    T = len(targets)
    o = oracle.select_and_factor_diag(w.points, w.kernel, targets, pool, plen, k)
    np.testing.assert_array_equal(g["status"], o["status"])
    short, fac = replay_check(g, w.points, w.kernel, targets, pool, plen, k, np.arange(T), TAU_MIXED, 1e-3)
    prior = w.kernel.variance + w.kernel.nugget
    dec, tot, gap_parted = mixed_decisive_check(g["sel"], o, prior, k)
    same = int(np.sum(np.all(g["sel"] == o["sel"], axis=1)))
    S_g, S_o = float(np.sum(g["log_condvar"])), float(np.sum(o["log_condvar"]))
    print(f"{label}: {same} of {T} columns identical; decisive steps {dec} of {tot}; largest oracle gap where "
          f"the paths parted {gap_parted:.2e}; worst replay shortfall {short:.2e}; worst factor error on own set "
          f"{fac:.2e}; S mixed - S fp64 = {S_g - S_o:.3e} ({(S_g - S_o) / abs(S_o):.2e} rel)", flush=True)
    assert dec >= 0.3 * tot  # the bound is worst case: late steps with small variances are left to the replay
    return o


def test_screened_step_mixed_as_benchmarked(trained):
    """Clustered cloud, n = 20,000, pools of 512 -> keep 128, k = 32, mixed, no
    gap output; the threshold sends the columns with the 2% largest dropped
    mass to their full pools; one csel_screened_select call per step, with
    the Morton order, the tuned schedule and the graph replay the benchmark
    times."""
    print("case: screened step, mixed, n=20000 C=512 keep=128 k=32", flush=True)
    p, pb = trained
    w = inputs.workload_clustered(n=20000, seed=15, C=512, k=32)
    P, Tg, Pl, Ln = _dev(w)
    T, k, keep = len(w.targets), 32, 128
    z = csel.screen(P, w.kernel, Tg, Pl, Ln, p, pb, keep, 1e30, want_logits=True)["logits"].cpu().double()
    zs = torch.sort(z, dim=1, descending=True).values
    drop = np.array([float(torch.sigmoid(zs[t, keep:int(w.pool_len[t])]).sum()) for t in range(T)])
    thr = float(np.quantile(drop[w.pool_len > keep], 0.98))
    plan = csel.Plan(T, 512, keep, k, "mixed", graph=True)
    plan.set_order(P, Tg)
    out = None
    for _ in range(3):  # the first step tunes the schedule, the next capture and replay the graph
        out, scr = screen_train.screened_select(P, w.kernel, Tg, Pl, Ln, k, p, pb, keep, "mixed",
                                                fallback_threshold=thr, out=out, plan=plan)
    torch.cuda.synchronize()
    assert "gap" not in out
    g = {key: v.cpu().numpy() for key, v in out.items()}
    fb = scr["fallback"].cpu().numpy()
    kept, kl = scr["kept"].cpu().numpy(), scr["kept_len"].cpu().numpy()
    nfb = int(scr["fallback_count"].item())
    assert nfb == int(np.sum(fb >= 1)) and 0 < nfb < T
    pool = np.full((T, 512), -1, np.int32)
    plen = np.zeros(T, np.int32)
    for t in range(T):
        if fb[t]:
            pool[t], plen[t] = w.pool[t], w.pool_len[t]
        else:
            pool[t, : kl[t]], plen[t] = kept[t, : kl[t]], kl[t]
    _mixed_checks(g, w, w.targets, pool, plen, k, f"screened mixed ({nfb} fallback columns)")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_plain_pools_of_512_no_gap(precision):
    """The plain leg of the benchmark: clustered cloud, n = 20,000, Matern 3/2,
    l = 0.05, pools of 512, k = 32, no gap output (the kernel the benchmark
    runs), in both precisions."""
    print(f"case: plain pools of 512, {precision}, n=20000 k=32", flush=True)
    w = inputs.workload_clustered(n=20000, seed=16, C=512, k=32)
    P, Tg, Pl, Ln = _dev(w)
    out = csel.select_and_factor(P, w.kernel, Tg, Pl, Ln, 32, precision)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items()}
    if precision == "mixed":
        _mixed_checks(g, w, w.targets, w.pool, w.pool_len, 32, "plain mixed C=512")
        return
    o = oracle.select_and_factor(w.points, w.kernel, w.targets, w.pool, w.pool_len, 32)
    g["gap"] = o["gap"]
    rep = compare_single(g, o, 1e-6, factor_rtol=1e-5, logcv_atol=1e-8)
    print("plain fp64 C=512:", rep["identical"], "of", rep["columns"], "identical; worst factor",
          rep["worst_factor_rel"], flush=True)
    assert rep["identical"] >= rep["fully_decisive"]
    # the FP64 path's own accuracy (its covariances, square roots and
    # exponentials within a few ulp), far inside the 1e-5 parity bar
    assert rep["worst_factor_rel"] <= 1e-10
    S_g, S_o = float(np.sum(g["log_condvar"])), float(np.sum(o["log_condvar"]))
    assert abs(S_g - S_o) <= 1e-9 * abs(S_o)


def _multi_replay_checks(g, w, groups):
    worst_loss = worst_val = 0.0
    for gi in groups:
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
            assert err <= 1e-3, f"group {gi} member {a}: column error {err}"
    return worst_loss, worst_val


def test_aggregated_register_kernel_pools_of_512():
    """The aggregated configuration's shape: supernodes of m uniform in 8..32,
    union pools of 512 later points (one pool row per thread of the 512-thread
    register kernel), k = 64, mixed, with member columns."""
    print("case: aggregated mixed register kernel, pools of 512, k=64", flush=True)
    w = inputs.workload_aggregated(n=30000, seed=34, C=512, k=64, mmin=8, mmax=32)
    mm = int(np.max(np.diff(w.group_ptr)))
    out = csel.aggregated_select(_t(w.points, torch.float64), w.kernel, _t(w.group_ptr, torch.int32),
                                 _t(w.members, torch.int32), mm, _t(w.pool, torch.int32), _t(w.pool_len, torch.int32),
                                 w.k, "mixed", want_factor=True, want_post_var=False)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "workspace"}
    G = len(w.group_ptr) - 1
    assert np.all(g["status"] <= 1)
    full = np.where(w.pool_len == 512)[0]
    assert len(full) > 0.8 * G
    groups = np.concatenate([full[::7], np.where(w.pool_len < 512)[0][:40]])
    loss, val = _multi_replay_checks(g, w, groups)
    print(f"register kernel, pools of 512: {len(groups)} groups replayed; worst per-step log det loss {loss:.2e}, "
          f"worst column error {val:.2e}", flush=True)


def test_aggregated_rejects_unsorted_or_repeated_members():
    """With factor output, a group whose members are not strictly ascending
    (the factor columns are laid out by member rank) is reported with status
    3 by both selection kernels, and its neighbours are unaffected."""
    print("case: aggregated groups with unsorted / repeated members", flush=True)
    for C, prec in ((64, "mixed"), (64, "fp64")):  # register kernel, slab kernel
        w = inputs.workload_aggregated(n=3000, seed=35, C=C, k=8, mmin=3, mmax=6)
        mem = w.members.copy()
        gp = w.group_ptr
        bad = []
        for gi in (2, 5, 9):
            b = gp[gi]
            if gi == 5:
                mem[b + 1] = mem[b]  # repeated member
            else:
                mem[b], mem[b + 1] = mem[b + 1], mem[b]  # unsorted
            bad.append(gi)
        mm = int(np.max(np.diff(gp)))
        args = (_t(w.points, torch.float64), w.kernel, _t(gp, torch.int32), _t(mem, torch.int32), mm,
                _t(w.pool, torch.int32), _t(w.pool_len, torch.int32), w.k, prec)
        out = csel.aggregated_select(*args, want_factor=True, want_post_var=False)
        ref = csel.aggregated_select(_t(w.points, torch.float64), w.kernel, _t(gp, torch.int32),
                                     _t(w.members, torch.int32), mm, _t(w.pool, torch.int32),
                                     _t(w.pool_len, torch.int32), w.k, prec, want_factor=True, want_post_var=False)
        torch.cuda.synchronize()
        st = out["status"].cpu().numpy()
        assert all(st[gi] == 3 for gi in bad), (prec, st[bad])
        good = np.setdiff1d(np.arange(len(gp) - 1), bad)
        assert np.array_equal(st[good], ref["status"].cpu().numpy()[good])
        assert np.array_equal(out["sel"].cpu().numpy()[good], ref["sel"].cpu().numpy()[good])
