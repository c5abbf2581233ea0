"""GPU parity of the learned screen (features, MLP forward/backward, Adam,
top-keep, fallback) against the screen oracle, and the screen's gain."""
import numpy as np
import pytest
import torch

import oracle
from oracle import screen as so
from paper_2307_11648_amd import csel, inputs, screen_train
from parity import compare_single

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def clustered():
    w = inputs.workload_clustered(n=8000, seed=14, C=512, k=32)
    dev = {"pts": _t(w.points, torch.float64), "tg": _t(w.targets, torch.int32), "pl": _t(w.pool, torch.int32),
           "ln": _t(w.pool_len, torch.int32)}
    return w, dev


def _rand_params(seed):
    p = torch.from_numpy((np.random.default_rng(seed).standard_normal(so.N_PARAMS) * 0.25).astype(np.float32))
    p = p.cuda()
    return p, csel.mlp_to_bf16(p)


def test_features_match_oracle(clustered):
    print("case: screen features n=8000 C=512", flush=True)
    w, d = clustered
    f = csel.screen_features(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"]).cpu().numpy()
    worst = 0.0
    for t in list(range(0, 7800, 131)) + [7990, 7999]:
        C = int(w.pool_len[t])
        ref = so.features(w.points, w.kernel, int(w.targets[t]), w.pool[t, :C])
        err = np.abs(f[t, :C] - ref)
        worst = max(worst, float(err.max()) if C else 0.0)
        np.testing.assert_allclose(f[t, :C], ref, rtol=2e-4, atol=2e-5)
        assert np.all(f[t, C:] == 0)
    print("worst feature error", worst)


def test_bf16_conversion_matches_oracle():
    p, pb = _rand_params(5)
    ref = so.bf16_round(p.cpu().numpy())
    got = (pb.cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
    np.testing.assert_array_equal(got.view(np.float32).astype(np.float64), ref)


def test_mlp_forward_and_gradient_match_oracle(clustered):
    print("case: mlp forward/backward", flush=True)
    w, d = clustered
    f = csel.screen_features(d["pts"], w.kernel, d["tg"][:200], d["pl"][:200], d["ln"][:200])
    X = f.view(-1, 16)[: 200 * 512 - 77].contiguous()  # a ragged number of rows
    y = (torch.rand(X.shape[0], generator=torch.Generator().manual_seed(3)) < 0.07).to(torch.uint8).cuda()
    p, pb = _rand_params(7)
    z = csel.mlp_forward(p, pb, X).cpu().numpy()
    Xn, yn, pn = X.cpu().numpy().astype(np.float64), y.cpu().numpy(), p.cpu().numpy().astype(np.float64)
    zr, _ = so.mlp_forward(Xn, pn, bf16=True)
    rel = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    print("logit normwise rel err", rel, "max abs", np.max(np.abs(z - zr)))
    assert rel <= 1e-3
    g, _ = csel.mlp_grad(p, pb, X, y, 4.0)
    g = g.cpu().numpy()
    loss, gr = so.bce_loss_and_grad(Xn, yn, pn, pos_weight=4.0, bf16=True)
    assert g[-1] / X.shape[0] == pytest.approx(loss, rel=1e-3)
    relg = np.linalg.norm(g[:-1] - gr) / np.linalg.norm(gr)
    print("gradient normwise rel err", relg)
    assert relg <= 2e-2
    # per block of parameters too (each block is a separate backward product)
    for a, b in ((so.OFF_W1, so.OFF_B1), (so.OFF_B1, so.OFF_W2), (so.OFF_W2, so.OFF_B2), (so.OFF_B2, so.OFF_W3),
                 (so.OFF_W3, so.OFF_B3), (so.OFF_B3, so.N_PARAMS)):
        assert np.linalg.norm(g[a:b] - gr[a:b]) <= 3e-2 * np.linalg.norm(gr[a:b]) + 1e-7
    # deterministic reduction
    g2, _ = csel.mlp_grad(p, pb, X, y, 4.0)
    assert np.array_equal(g2.cpu().numpy(), g)


def test_adam_matches_oracle():
    p, pb = _rand_params(11)
    g = torch.from_numpy(np.random.default_rng(12).standard_normal(so.N_PARAMS).astype(np.float32)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    pn, mn, vn = p.cpu().numpy().astype(np.float64), np.zeros(so.N_PARAMS), np.zeros(so.N_PARAMS)
    for step in (1, 2, 3):
        csel.mlp_adam(p, pb, g, m, v, 1e-2, step)
        pn, mn, vn = so.adam_step(pn, g.cpu().numpy().astype(np.float64), mn, vn, step, 1e-2)
    np.testing.assert_allclose(p.cpu().numpy(), pn, rtol=1e-5, atol=1e-6)
    ref = so.bf16_round(p.cpu().numpy())
    got = ((pb.cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16).view(np.float32)
    np.testing.assert_array_equal(got.astype(np.float64), ref)


def test_screen_keep_and_fallback_match_oracle(clustered):
    print("case: screen top-keep", flush=True)
    w, d = clustered
    p, pb = _rand_params(21)
    keep = 128
    out = csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, keep, 0.5, want_logits=True)
    torch.cuda.synchronize()
    z = out["logits"].cpu().numpy()
    kept = out["kept"].cpu().numpy()
    kl = out["kept_len"].cpu().numpy()
    fb = out["fallback"].cpu().numpy()
    nfb = int(out["fallback_count"].item())
    assert nfb == int(np.sum(fb >= 1))
    assert set(out["fallback_list"].cpu().numpy()[:nfb].tolist()) == set(np.where(fb >= 1)[0].tolist())
    for t in range(len(w.targets)):
        C = int(w.pool_len[t])
        ks, f = so.screen_keep(z[t], C, keep, 0.5)
        # integer work on the GPU's own logits: bit-exact
        assert kl[t] == len(ks)
        assert np.array_equal(kept[t, : kl[t]], w.pool[t, ks])
        assert np.all(kept[t, kl[t]:] == -1)
        if C > keep:
            drop = np.sort(np.setdiff1d(np.arange(C), ks))
            s = float(np.sum(1.0 / (1.0 + np.exp(-z[t, drop].astype(np.float64)))))
            if abs(s - 0.5) > 1e-4:
                assert bool(fb[t]) == f
    # GPU logits against the oracle's end-to-end logits (oracle features, FP64 MLP)
    for t in range(0, len(w.targets), 397):
        C = int(w.pool_len[t])
        fr = so.features(w.points, w.kernel, int(w.targets[t]), w.pool[t, :C])
        zr, _ = so.mlp_forward(fr, p.cpu().numpy().astype(np.float64), bf16=True)
        assert np.linalg.norm(z[t, :C] - zr) <= 5e-3 * np.linalg.norm(zr) + 1e-5


def test_screened_selection_parity(clustered):
    """Exact selection on the kept pools plus full-pool selection for the
    fallback columns equals the oracle run on the same per-column pools."""
    print("case: screened selection parity", flush=True)
    w, d = clustered
    p, pb = _rand_params(33)
    # a threshold at the median dropped mass sends about half the columns to the full pool
    z = csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, 128, 0.5, want_logits=True)["logits"]
    zs = torch.sort(z.cpu(), dim=1, descending=True).values.double()
    drop = [float(torch.sigmoid(zs[t, 128:int(w.pool_len[t])]).sum()) for t in range(len(w.targets))]
    thr = float(np.median([v for v, L in zip(drop, w.pool_len) if L > 128]))
    out, scr = screen_train.screened_select(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], 32, p, pb, 128,
                                            precision="fp64", fallback_threshold=thr)
    torch.cuda.synchronize()
    fb = scr["fallback"].cpu().numpy()
    kept = scr["kept"].cpu().numpy()
    kl = scr["kept_len"].cpu().numpy()
    assert 0 < fb.sum() < len(fb)  # both paths exercised
    pool = np.full((len(w.targets), 512), -1, np.int32)
    plen = np.zeros(len(w.targets), np.int32)
    for t in range(len(w.targets)):
        if fb[t]:
            pool[t] = w.pool[t]
            plen[t] = w.pool_len[t]
        else:
            pool[t, : kl[t]] = kept[t, : kl[t]]
            plen[t] = kl[t]
    o = oracle.select_and_factor(w.points, w.kernel, w.targets, pool, plen, 32)
    g = {key: v.cpu().numpy() for key, v in out.items()}
    g["gap"] = o["gap"]  # not requested from the GPU
    rep = compare_single(g, o, 1e-6, factor_rtol=1e-5, logcv_atol=1e-8)
    print(rep["identical"], "of", rep["columns"], "identical")
    assert rep["identical"] >= 0.97 * rep["columns"]


def _composed_step(d, w, p, pb, keep, k, prec, thr, order=None):
    """The screened step composed from the separate entry points: csel_screen,
    csel_select_and_factor on the kept pools, csel_select_and_factor_list on
    the full pools of the listed fallback columns (capacity: every column)."""
    T = len(w.targets)
    scr = csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, keep, thr, order=order)
    out = csel.select_and_factor(d["pts"], w.kernel, d["tg"], scr["kept"], scr["kept_len"], k, prec)
    csel.select_and_factor_list(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], k, prec, scr["fallback_list"],
                                scr["fallback_count"], T, out)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}, scr


@pytest.mark.parametrize("thr,spatial,graph", [(0.6, False, False), (0.6, True, True), (1e30, True, True),
                                               (0.0, False, True)])
def test_plan_step_matches_composed_step(clustered, thr, spatial, graph):
    """csel_screened_select (one call: screen, kept-pool selection, the
    fallback columns over the device-side list, no host read) writes
    exactly what the composition of the separate entry points writes: with
    fallback columns, with none, and with every column falling back
    (threshold 0).  With a graph, the step is replayed three times into
    cleared outputs, with eager work and a synchronisation between replays;
    every replay must match."""
    print(f"case: plan step threshold {thr} spatial {spatial} graph {graph}", flush=True)
    w, d = clustered
    p, pb = _rand_params(37)
    T, k, keep = len(w.targets), 32, 128
    ref, scr_ref = _composed_step(d, w, p, pb, keep, k, "mixed", thr)
    nfb = int(scr_ref["fallback_count"].item())
    assert (nfb > 0) == (thr < 1.0)
    if thr == 0.0:
        assert nfb == int((w.pool_len > keep).sum())
    plan = csel.Plan(T, 512, keep, k, "mixed", graph=graph)
    if spatial:
        plan.set_order(d["pts"], d["tg"])
    out = None
    for rep in range(4):
        if out is not None:
            for v in out.values():
                v.zero_()
        out = plan.step(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, thr, out=out)
        scr = plan.screen_outputs()
        torch.cuda.synchronize()
        for key in ("sel", "factor", "log_condvar", "status"):
            assert np.array_equal(out[key].cpu().numpy(), ref[key], equal_nan=True), (rep, key)
        for key in ("kept", "kept_len", "fallback", "fallback_count"):
            assert torch.equal(scr[key], scr_ref[key]), (rep, key)
        assert sorted(scr["fallback_list"][:nfb].cpu().tolist()) == sorted(scr_ref["fallback_list"][:nfb].cpu().tolist())
        # unrelated eager work between the replays
        _composed_step(d, w, p, pb, keep, k, "fp64", 0.3)
    info = plan.info()
    print("plan schedule", info, flush=True)
    assert info["schedule"] in ("natural", "spatial", "natural/mw", "spatial/mw")
    # new output buffers: the graph is captured again and writes the new ones
    out2 = plan.step(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, thr)
    torch.cuda.synchronize()
    assert np.array_equal(out2["sel"].cpu().numpy(), ref["sel"])
    plan.close()


def test_plan_rejects_bad_arguments(clustered):
    w, d = clustered
    p, pb = _rand_params(38)
    with pytest.raises(csel.CselError):
        csel.Plan(100, 513, 128, 32)
    with pytest.raises(csel.CselError):
        csel.Plan(100, 512, 600, 32)
    with pytest.raises(csel.CselError):
        csel.Plan(100, 512, 128, 40)
    plan = csel.Plan(len(w.targets), 512, 128, 32)
    with pytest.raises(ValueError):
        plan.step(d["pts"], w.kernel, d["tg"][:10], d["pl"], d["ln"], p, pb, 0.5)
    with pytest.raises(csel.CselError):
        plan.step(d["pts"], inputs.Kernel(4, 0.05), d["tg"], d["pl"], d["ln"], p, pb, 0.5)
    with pytest.raises(csel.CselError):
        plan.step(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, -1.0)
    plan.close()


def test_trained_screen_gains(tmp_path):
    """Train on a separate cloud of the same distribution (labels from exact
    greedy selections), then screen 512-candidate pools to 128 on a test cloud:
    the trained screen keeps the KL within 1% of full-pool selection and beats
    the untrained network, random screening and the 128-nearest screen.  KL is
    exact (dense log det on the GPU, FP64)."""
    print("case: trained screen gain, n=12000", flush=True)
    n = 12000
    tr = inputs.workload_clustered(n=n, seed=40, C=512, k=32)
    te = inputs.workload_clustered(n=n, seed=41, C=512, k=32)
    dt = lambda w: (_t(w.points, torch.float64), _t(w.targets, torch.int32), _t(w.pool, torch.int32),  # noqa: E731
                    _t(w.pool_len, torch.int32))
    P, Tg, Pl, Ln = dt(tr)
    X, y = screen_train.training_set(P, tr.kernel, Tg, Pl, Ln, 32, "fp64")
    print("training rows", X.shape[0], "positives", float(y.float().mean()))
    p, pb, losses = screen_train.train(X, y, steps=1500, batch=8192, lr=3e-3, seed=1, log_every=500)
    print("training losses", losses)
    p0, pb0 = _rand_params(99)
    P, Tg, Pl, Ln = dt(te)
    full = csel.select_and_factor(P, te.kernel, Tg, Pl, Ln, 32, "fp64")
    # exact log det of Theta on the GPU (evaluation only)
    th = torch.from_numpy(oracle.covariance(te.points, te.kernel)).cuda()
    ld = float(2.0 * torch.log(torch.diagonal(torch.linalg.cholesky(th))).sum().item())
    del th
    S_full = float(full["log_condvar"].sum().item())
    kl_full = 0.5 * (S_full - ld)

    def kl_of(pool_t, len_t):
        o = csel.select_and_factor(P, te.kernel, Tg, pool_t, len_t, 32, "fp64")
        return 0.5 * (float(o["log_condvar"].sum().item()) - ld)

    res = {}
    for name, (pp, ppb) in {"trained": (p, pb), "untrained": (p0, pb0)}.items():
        out, scr = screen_train.screened_select(P, te.kernel, Tg, Pl, Ln, 32, pp, ppb, 128, precision="fp64",
                                                fallback_threshold=1e9)  # no fallback: the screen alone
        res[name] = 0.5 * (float(out["log_condvar"].sum().item()) - ld)
    res["nearest128"] = kl_of(Pl[:, :128].contiguous(), torch.clamp(Ln, max=128))
    rng = np.random.default_rng(0)
    pr = te.pool.copy()
    for t in range(n):
        L = te.pool_len[t]
        if L > 128:
            pr[t, :128] = te.pool[t, np.sort(rng.choice(L, 128, replace=False))]
    res["random128"] = kl_of(_t(pr[:, :128], torch.int32), torch.clamp(Ln, max=128))
    gaps = {k: (v - kl_full) / kl_full for k, v in res.items()}
    print("KL full", kl_full, "relative gaps", gaps)
    assert gaps["trained"] <= 0.01
    assert gaps["trained"] < gaps["untrained"]
    assert gaps["trained"] < gaps["random128"]
    # the trained network beats the free truncation to the 128 nearest candidates
    assert gaps["trained"] < gaps["nearest128"]


@pytest.mark.parametrize("d,C,keep", [(1, 64, 16), (2, 128, 40), (3, 256, 128), (2, 512, 128)])
def test_screen_ragged_dims_and_bad_rows(d, C, keep):
    """Every pool width (one to eight candidates per lane), dimensions 1-3,
    ragged pool lengths (the ordering's tail, an empty pool), and rows the
    screen must reject (target or pool index out of range, pool length past
    the stride): kept lists and flags bit-exact on the GPU's own logits,
    logits against the oracle's features and MLP."""
    print(f"case: screen edge cases d={d} C={C} keep={keep}", flush=True)
    n = 1500
    w = inputs.single_target(f"edge d={d}", inputs.uniform_points(n, d, 50 + d + C), inputs.Kernel(3, 0.08), C, 8)
    pool = w.pool.copy()
    plen = w.pool_len.copy()
    tg = w.targets.copy()
    T = len(tg)
    bad = {3: "target", 10: "index", 17: "length"}
    tg[3] = -1
    pool[10, min(5, plen[10] - 1)] = n
    plen[17] = C + 1
    plen[25] = 0
    p, pb = _rand_params(60 + C)
    out = csel.screen(_t(w.points, torch.float64), w.kernel, _t(tg, torch.int32), _t(pool, torch.int32),
                      _t(plen, torch.int32), p, pb, keep, 0.7, want_logits=True)
    torch.cuda.synchronize()
    z = out["logits"].cpu().numpy()
    kept, kl = out["kept"].cpu().numpy(), out["kept_len"].cpu().numpy()
    fb = out["fallback"].cpu().numpy()
    nfb = int(out["fallback_count"].item())
    # fallback columns and rejected columns (fallback 3) are both listed
    assert set(out["fallback_list"].cpu().numpy()[:nfb].tolist()) == set(np.where(fb >= 1)[0].tolist())
    for t in range(T):
        if t in bad:
            assert kl[t] == 0 and fb[t] == 3, (t, bad[t])
            continue
        L = int(plen[t])
        ks, f = so.screen_keep(z[t], L, keep, 0.7)
        assert kl[t] == len(ks) and np.array_equal(kept[t, : kl[t]], pool[t, ks]), t
        assert np.all(kept[t, kl[t]:] == -1)
        if L > keep:
            drop = np.sort(np.setdiff1d(np.arange(L), ks))
            s = float(np.sum(1.0 / (1.0 + np.exp(-z[t, drop].astype(np.float64)))))
            if abs(s - 0.7) > 1e-4:
                assert bool(fb[t]) == f, t
        else:
            assert fb[t] == 0
    # the screened pipeline reports the rejected columns as bad input (status 3)
    # from their full-pool selection, instead of answering for an empty pool
    sel_out, _ = screen_train.screened_select(_t(w.points, torch.float64), w.kernel, _t(tg, torch.int32),
                                              _t(pool, torch.int32), _t(plen, torch.int32), 8, p, pb, keep,
                                              "mixed", fallback_threshold=0.7)
    torch.cuda.synchronize()
    st = sel_out["status"].cpu().numpy()
    for t in bad:
        assert st[t] == 3, (t, bad[t])
        assert np.all(sel_out["sel"][t].cpu().numpy() == -1)
    assert np.all(np.delete(st, list(bad)) < 2)
    pn = p.cpu().numpy().astype(np.float64)
    for t in list(range(0, T, 97)) + [T - 2, T - 5, T - 9, T - 70]:
        L = int(plen[t])
        if t in bad or L == 0:
            continue
        fr = so.features(w.points, w.kernel, int(tg[t]), pool[t, :L])
        zr, _ = so.mlp_forward(fr, pn, bf16=True)
        assert np.linalg.norm(z[t, :L] - zr) <= 5e-3 * np.linalg.norm(zr) + 1e-5, t


def _morton_reference(points, targets):
    """Morton codes as the schedule defines them (coordinates of in-range
    targets quantised over the targets' bounding box with separately rounded
    FP64 operations, bits interleaved coordinate-minor), stable-sorted."""
    n, dim = points.shape
    ok = (targets >= 0) & (targets < n)
    X = np.zeros((len(targets), 3))
    X[ok, :dim] = points[targets[ok]]
    bits = 10 if dim >= 3 else (15 if dim == 2 else 30)
    step = 3 if dim >= 3 else dim
    cells = float((1 << bits) - 1)
    code = np.zeros(len(targets), np.uint64)
    for c in range(dim):
        lo, hi = X[:, c].min(), X[:, c].max()
        ext = hi - lo
        u = (X[:, c] - lo) / ext if ext > 0 else np.zeros(len(targets))
        u = np.clip(u, 0.0, 1.0)
        q = np.floor(u * cells + 0.5).astype(np.uint64)  # numpy rounds the product, then the sum
        for b in range(bits):
            code |= ((q >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * step + c)
    return np.argsort(code, kind="stable").astype(np.int32)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_spatial_order_matches_reference(dim):
    print(f"case: spatial order d={dim}", flush=True)
    pts = inputs.uniform_points(3000, dim, 70 + dim)
    tg = np.random.default_rng(dim).permutation(3000)[:2500].astype(np.int32)
    tg[7] = -5  # out of range: placed at the origin of the box
    tg[8] = tg[9]  # a repeated target: equal codes keep column order
    order, ws = csel.spatial_order(_t(pts, torch.float64), _t(tg, torch.int32))
    got = order.cpu().numpy()
    assert np.array_equal(np.sort(got), np.arange(len(tg)))
    assert np.array_equal(got, _morton_reference(pts, tg))
    empty, _ = csel.spatial_order(_t(pts, torch.float64), _t(tg[:0], torch.int32))
    assert empty.numel() == 0


def test_screen_order_does_not_change_results(clustered):
    """Outputs under the spatial order, a random order and the natural order
    are identical; an order entry out of range is skipped and a column left
    out of the order keeps its outputs untouched."""
    print("case: screen processing orders", flush=True)
    w, d = clustered
    p, pb = _rand_params(44)
    T = len(w.targets)
    ref = csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, 128, 0.6, want_logits=True)
    sp, _ = csel.spatial_order(d["pts"], d["tg"])
    rnd = _t(np.random.default_rng(5).permutation(T).astype(np.int32), torch.int32)
    for name, order in (("spatial", sp), ("random", rnd)):
        o = csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, 128, 0.6, want_logits=True, order=order)
        torch.cuda.synchronize()
        for key in ("kept", "kept_len", "fallback", "logits", "fallback_count"):
            assert torch.equal(o[key], ref[key]), (name, key)
        nfb = int(ref["fallback_count"].item())
        assert set(o["fallback_list"][:nfb].cpu().tolist()) == set(ref["fallback_list"][:nfb].cpu().tolist())
    # the order in three slices (separate fallback outputs) covers every column once
    o = {key: torch.empty_like(v) for key, v in ref.items() if key != "logits"}
    fb_all = []
    for a, b in ((0, 1000), (1000, 5000), (5000, T)):
        part = dict(o, fallback_list=torch.empty(b - a, dtype=torch.int32, device="cuda"),
                    fallback_count=torch.empty(1, dtype=torch.int32, device="cuda"))
        csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, 128, 0.6, out=part, order=sp[a:b])
        torch.cuda.synchronize()
        fb_all += part["fallback_list"][: int(part["fallback_count"].item())].cpu().tolist()
    for key in ("kept", "kept_len", "fallback"):
        assert torch.equal(o[key], ref[key]), ("slices", key)
    nfb = int(ref["fallback_count"].item())
    assert sorted(fb_all) == sorted(ref["fallback_list"][:nfb].cpu().tolist())
    # drop column 11 from the order, put an out-of-range entry in its place
    od = sp.clone()
    pos = int(torch.nonzero(od == 11)[0].item())
    od[pos] = T + 3
    o = {"kept": torch.full((T, 128), -7, dtype=torch.int32, device="cuda"),
         "kept_len": torch.full((T,), -7, dtype=torch.int32, device="cuda"),
         "fallback": torch.full((T,), 9, dtype=torch.uint8, device="cuda"),
         "fallback_list": torch.empty(T, dtype=torch.int32, device="cuda"),
         "fallback_count": torch.empty(1, dtype=torch.int32, device="cuda")}
    csel.screen(d["pts"], w.kernel, d["tg"], d["pl"], d["ln"], p, pb, 128, 0.6, out=o, order=od)
    torch.cuda.synchronize()
    keep_rows = torch.ones(T, dtype=torch.bool, device="cuda")
    keep_rows[11] = False
    assert int(o["kept_len"][11].item()) == -7 and int(o["fallback"][11].item()) == 9
    assert bool(torch.all(o["kept"][11] == -7))
    for key in ("kept", "kept_len", "fallback"):
        assert torch.equal(o[key][keep_rows], ref[key][keep_rows]), key


def test_spatial_order_degenerate_inputs():
    """One target, all targets at one point (a zero-extent box: every code is
    0, so the order is the column order), and collinear targets along each
    axis of a 3-D cloud (one coordinate varies)."""
    print("case: spatial order degenerate inputs", flush=True)
    pts = inputs.uniform_points(500, 3, 91)
    one, _ = csel.spatial_order(_t(pts, torch.float64), _t(np.array([42], np.int32), torch.int32))
    assert one.cpu().numpy().tolist() == [0]
    same = np.full(37, 11, np.int32)
    o, _ = csel.spatial_order(_t(pts, torch.float64), _t(same, torch.int32))
    assert np.array_equal(o.cpu().numpy(), np.arange(37))
    for axis in range(3):
        line = np.zeros((200, 3))
        line[:, axis] = np.random.default_rng(axis).random(200)
        tg = np.arange(200, dtype=np.int32)
        o, _ = csel.spatial_order(_t(line, torch.float64), _t(tg, torch.int32))
        got = o.cpu().numpy()
        assert np.array_equal(got, _morton_reference(line, tg))
        # one coordinate varies: the order sorts its quantised value (ties by column)
        x = line[:, axis]
        q = np.floor((x - x.min()) / (x.max() - x.min()) * 1023 + 0.5)
        assert np.all(np.diff(q[got]) >= 0)
