"""GPU parity of the group screen (csel_screen_groups) against the oracle,
and the screened multi-target selection of GP prediction batches."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import screen as so
from paper_2307_11648_amd import csel, inputs, screen_train

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _rand_params(seed):
    p = torch.from_numpy((np.random.default_rng(seed).standard_normal(so.N_PARAMS) * 0.25).astype(np.float32))
    p = p.cuda()
    return p, csel.mlp_to_bf16(p)


def _ragged_groups(w, sizes, C):
    """Regroup the workload's prediction points into groups of `sizes`
    members (consecutive members of the spatial batches) with fresh pools."""
    mem = w.members[: int(np.sum(sizes))]
    gp = np.zeros(len(sizes) + 1, np.int32)
    gp[1:] = np.cumsum(sizes)
    n_train = w.meta["n_train"]
    pool, plen = inputs.group_pools(w.points, gp, mem, C, later_only=False, cand_range=(0, n_train))
    return gp, mem, pool, plen


@pytest.fixture(scope="module")
def gpw():
    """20,000 training points, 16 batches of 64 prediction points, Matern 5/2,
    l = 0.03, pools of 2048; regrouped into ragged groups (1..64 members) and
    with some pools cut short (0, 1, 300, 512, 513, 1500 candidates)."""
    w = inputs.workload_gp(n_train=20000, n_pred=1024, C=2048, k=64, n_strips=4, per_strip=4)
    sizes = np.array([64, 1, 63, 30, 34, 64, 2, 62, 64, 64, 17, 47, 64, 64], np.int32)
    gp, mem, pool, plen = _ragged_groups(w, sizes, 2048)
    for g, L in ((1, 0), (2, 1), (3, 300), (4, 512), (5, 513), (6, 1500)):
        plen[g] = L
        pool[g, L:] = -1
    return w, gp, mem, pool, plen


def _dev(w, gp, mem, pool, plen):
    return _t(w.points, torch.float64), _t(gp, torch.int32), _t(mem, torch.int32), _t(pool, torch.int32), \
        _t(plen, torch.int32)


def test_group_features_match_oracle(gpw):
    print("case: group screen features, 14 ragged groups, pools <= 2048", flush=True)
    w, gp, mem, pool, plen = gpw
    pts, gpt, memt, pl, ln = _dev(*gpw)
    f = csel.screen_groups(pts, w.kernel, gpt, memt, pl, ln, None, None, 0)["features"].cpu().numpy()
    worst = 0.0
    for g in range(len(gp) - 1):
        C = int(plen[g])
        ref = so.group_features(w.points, w.kernel, mem[gp[g]:gp[g + 1]], pool[g, :C])
        if C:
            worst = max(worst, float(np.max(np.abs(f[g, :C] - ref))))
        np.testing.assert_allclose(f[g, :C], ref, rtol=2e-4, atol=2e-5)
        assert np.all(f[g, C:] == 0)
    print("worst feature error", worst)


def test_group_keep_and_fallback_match_oracle(gpw):
    print("case: group screen top-keep", flush=True)
    w, gp, mem, pool, plen = gpw
    pts, gpt, memt, pl, ln = _dev(*gpw)
    p, pb = _rand_params(23)
    for keep, thr in ((512, 3.0), (100, 50.0), (2048, 0.5)):
        out = csel.screen_groups(pts, w.kernel, gpt, memt, pl, ln, p, pb, keep, thr, want_logits=True)
        torch.cuda.synchronize()
        z = out["logits"].cpu().numpy()
        kept, kl, fb = (out[key].cpu().numpy() for key in ("kept", "kept_len", "fallback"))
        for g in range(len(gp) - 1):
            C = int(plen[g])
            ks, f = so.screen_keep(z[g], C, keep, thr)
            # integer work on the GPU's own logits: bit-exact
            assert kl[g] == len(ks), (keep, g)
            assert np.array_equal(kept[g, : kl[g]], pool[g, ks]), (keep, g)
            assert np.all(kept[g, kl[g]:] == -1)
            if C > keep:
                drop = np.setdiff1d(np.arange(C), ks)
                s = float(np.sum(1.0 / (1.0 + np.exp(-z[g, drop].astype(np.float64)))))
                if abs(s - thr) > 1e-3 * thr:
                    assert bool(fb[g]) == f, (keep, g, s)
            else:
                assert fb[g] == 0
    # GPU logits against the oracle's end-to-end logits (oracle features, FP64 MLP)
    for g in range(len(gp) - 1):
        C = int(plen[g])
        if C == 0:
            continue
        fr = so.group_features(w.points, w.kernel, mem[gp[g]:gp[g + 1]], pool[g, :C])
        zr, _ = so.mlp_forward(fr, p.cpu().numpy().astype(np.float64), bf16=True)
        assert np.linalg.norm(z[g, :C] - zr) <= 5e-3 * np.linalg.norm(zr) + 1e-5


def test_group_screen_bad_groups(gpw):
    """A member id, a pool id or a member range out of bounds fails that group
    alone (fallback 3, kept_len 0); the other groups are unchanged."""
    print("case: group screen bad groups", flush=True)
    w, gp, mem, pool, plen = gpw
    pts, gpt, memt, pl, ln = _dev(*gpw)
    p, pb = _rand_params(29)
    ref = {key: v.cpu().numpy() for key, v in csel.screen_groups(pts, w.kernel, gpt, memt, pl, ln, p, pb, 256,
                                                                 1.0).items()}
    mem2 = mem.copy()
    mem2[gp[3]] = len(w.points) + 3
    pool2 = pool.copy()
    pool2[7, 5] = -4
    out = csel.screen_groups(pts, w.kernel, gpt, _t(mem2, torch.int32), _t(pool2, torch.int32), ln, p, pb, 256, 1.0)
    # the last group's member range runs past the member array
    gp3 = gp.copy()
    gp3[-1] = gp3[-1] + 5
    out3 = csel.screen_groups(pts, w.kernel, _t(gp3, torch.int32), memt, pl, ln, p, pb, 256, 1.0)
    torch.cuda.synchronize()
    got = {key: v.cpu().numpy() for key, v in out.items()}
    got3 = {key: v.cpu().numpy() for key, v in out3.items()}
    G = len(gp) - 1
    for g in range(G):
        if g in (3, 7):
            assert got["fallback"][g] == 3 and got["kept_len"][g] == 0
        else:
            for key in ("kept", "kept_len", "fallback"):
                assert np.array_equal(got[key][g], ref[key][g]), (g, key)
    assert got3["fallback"][G - 1] == 3 and got3["kept_len"][G - 1] == 0
    for key in ("kept", "kept_len", "fallback"):
        assert np.array_equal(got3[key][: G - 1], ref[key][: G - 1]), key
    # the screened selection reports the two bad groups from their full pools
    sel, _, _ = screen_train.screened_group_select(pts, w.kernel, gpt, _t(mem2, torch.int32), 64,
                                                   _t(pool2, torch.int32), ln, 16, p, pb, 256, "fp64",
                                                   fallback_threshold=1e30)
    st = sel["status"].cpu().numpy()
    assert st[3] == 3 and st[7] == 3
    assert np.all(np.delete(st, [3, 7]) < 2)


def test_screened_gp_selection_parity(gpw):
    """FP64 multi-target selection on the kept pools (random MLP, keep 512,
    with fallback groups re-selected on their full pools) equals the oracle's
    selection on the same pools, posterior variances included."""
    print("case: screened GP selection parity (fp64)", flush=True)
    w, gp, mem, pool, plen = gpw
    pts, gpt, memt, pl, ln = _dev(*gpw)
    p, pb = _rand_params(31)
    k, keep = 64, 512
    # a fallback threshold between the groups' dropped masses, so that some
    # groups fall back and the others run on their kept pools
    z = csel.screen_groups(pts, w.kernel, gpt, memt, pl, ln, p, pb, keep, 1e9, want_logits=True)["logits"]
    z = z.cpu().numpy()
    mass = []
    for gi in range(len(gp) - 1):
        C = int(plen[gi])
        if C > keep:
            ks, _ = so.screen_keep(z[gi], C, keep, 1e9)
            drop = np.setdiff1d(np.arange(C), ks)
            mass.append(float(np.sum(1.0 / (1.0 + np.exp(-z[gi, drop].astype(np.float64))))))
    mass = np.sort(mass)
    thr = float(0.5 * (mass[len(mass) // 2 - 1] + mass[len(mass) // 2]))
    out, scr, nfb = screen_train.screened_group_select(pts, w.kernel, gpt, memt, 64, pl, ln, k, p, pb, keep, "fp64",
                                                       fallback_threshold=thr)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "workspace"}
    kept, kl, fb = (scr[key].cpu().numpy() for key in ("kept", "kept_len", "fallback"))
    print("fallback groups", nfb, "threshold", thr)
    assert nfb == int(np.sum(fb == 1)) and 0 < nfb < len(gp) - 1
    G = len(gp) - 1
    # the pools each group was selected on
    sel_pool = np.full((G, 2048), -1, np.int32)
    sel_len = np.zeros(G, np.int32)
    for gi in range(G):
        if fb[gi] == 1:
            sel_pool[gi], sel_len[gi] = pool[gi], plen[gi]
        else:
            sel_pool[gi, : kl[gi]], sel_len[gi] = kept[gi, : kl[gi]], kl[gi]
    o = oracle.aggregated_select(w.points, w.kernel, gp, mem, sel_pool, sel_len, k, want_factor=False,
                                 want_post_var=True)
    np.testing.assert_array_equal(g["status"], o["status"])
    same = 0
    for gi in range(G):
        if np.array_equal(g["sel"][gi], o["sel"][gi]):
            same += 1
            b, e = gp[gi], gp[gi + 1]
            np.testing.assert_allclose(g["post_var"][b:e], o["post_var"][b:e], rtol=1e-7, atol=1e-13)
            assert g["logdet"][gi] == pytest.approx(o["logdet"][gi], rel=1e-9, abs=1e-9)
    print("identical groups", same, "of", G)
    assert same >= G - 1


def test_trained_group_screen_gains():
    """Train the group screen on GP batches of a separate training cloud
    (labels from exact multi-target selections), then screen 2048-candidate
    pools to 512 on a test cloud (k = 128): the trained screen's log det gap
    to full-pool selection is smaller than the untrained network's and random
    screening's, and is reported against the 512-nearest screen.  The gap is
    sum_g (log det Theta_TT|s_screen - log det Theta_TT|s_full), relative to
    sum_g (log det Theta_TT - log det Theta_TT|s_full)."""
    print("case: trained group screen gain", flush=True)
    k, keep = 128, 512
    tr = inputs.workload_gp(n_train=20000, n_pred=4096, C=2048, k=k, seed=8, n_strips=8, per_strip=8)
    te = inputs.workload_gp(n_train=20000, n_pred=1024, C=2048, k=k, seed=9, n_strips=4, per_strip=4)

    def dev(w):
        return (_t(w.points, torch.float64), _t(w.group_ptr, torch.int32), _t(w.members, torch.int32),
                _t(w.pool, torch.int32), _t(w.pool_len, torch.int32))

    P, GP, M, PL, LN = dev(tr)
    X, y = screen_train.group_training_set(P, tr.kernel, GP, M, 64, PL, LN, k, "fp64")
    print("training rows", X.shape[0], "positives", float(y.float().mean()), flush=True)
    p, pb, losses = screen_train.train(X, y, steps=1500, batch=8192, lr=3e-3, seed=1, log_every=500)
    print("training losses", losses, flush=True)
    p0, pb0 = _rand_params(98)
    P, GP, M, PL, LN = dev(te)
    full = csel.aggregated_select(P, te.kernel, GP, M, 64, PL, LN, k, "fp64")
    assert np.all(full["status"].cpu().numpy() == 0)
    ld_full = full["logdet"].cpu().numpy()
    G = len(te.group_ptr) - 1
    ld_prior = np.array([np.linalg.slogdet(oracle.covariance(te.points[te.members[te.group_ptr[g]:te.group_ptr[g + 1]]],
                                                               te.kernel))[1] for g in range(G)])
    den = float(np.sum(ld_prior - ld_full))

    def gap_of(pool_t, len_t):
        o = csel.aggregated_select(P, te.kernel, GP, M, 64, pool_t, len_t, k, "fp64")
        return float(np.sum(o["logdet"].cpu().numpy() - ld_full)) / den

    res = {}
    for name, (pp, ppb) in {"trained": (p, pb), "untrained": (p0, pb0)}.items():
        scr = csel.screen_groups(P, te.kernel, GP, M, PL, LN, pp, ppb, keep, 1e9)  # no fallback: the screen alone
        res[name] = gap_of(scr["kept"], scr["kept_len"])
    res["nearest512"] = gap_of(PL[:, :keep].contiguous(), torch.clamp(LN, max=keep))
    rng = np.random.default_rng(0)
    pr = np.full((G, keep), -1, np.int32)
    for g in range(G):
        L = int(te.pool_len[g])
        pr[g, : min(L, keep)] = te.pool[g, np.sort(rng.choice(L, min(L, keep), replace=False))]
    res["random512"] = gap_of(_t(pr, torch.int32), torch.clamp(LN, max=keep))
    print("log det gaps relative to the prior-to-full reduction", res, flush=True)
    assert res["trained"] < res["untrained"]
    assert res["trained"] < res["random512"]
    assert res["trained"] <= 0.01
    # against the free truncation to the 512 nearest candidates: at k = 128
    # the trained group screen does not beat it (measured 1.95e-4 against
    # 1.62e-4); the comparison is reported, and held to a factor of two so a
    # regression of the screen shows
    assert res["trained"] <= 2.0 * res["nearest512"] + 1e-6
