"""Pins of the screen oracle (features, MLP forward/backward, Adam, top-keep)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import screen as so
from paper_2307_11648_amd import inputs


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(so.N_PARAMS) * scale


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, so.F))
    y = (rng.random(40) < 0.3).astype(np.float64)
    p = _params(2)
    loss, g = so.bce_loss_and_grad(X, y, p, pos_weight=3.0, bf16=False)
    h = 1e-6
    for j in rng.choice(so.N_PARAMS, size=60, replace=False):
        e = np.zeros(so.N_PARAMS)
        e[j] = h
        lp, _ = so.bce_loss_and_grad(X, y, p + e, 3.0, bf16=False)
        lm, _ = so.bce_loss_and_grad(X, y, p - e, 3.0, bf16=False)
        fd = (lp - lm) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_gradient_matches_torch_autograd():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((64, so.F))
    y = (rng.random(64) < 0.2).astype(np.float64)
    p = _params(4)
    loss, g = so.bce_loss_and_grad(X, y, p, pos_weight=2.0, bf16=False)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    W1 = pt[so.OFF_W1:so.OFF_B1].view(so.F, so.H)
    b1 = pt[so.OFF_B1:so.OFF_W2]
    W2 = pt[so.OFF_W2:so.OFF_B2].view(so.H, so.H)
    b2 = pt[so.OFF_B2:so.OFF_W3]
    w3 = pt[so.OFF_W3:so.OFF_B3]
    b3 = pt[so.OFF_B3]
    Xt = torch.tensor(X)
    z = torch.relu(torch.relu(Xt @ W1 + b1) @ W2 + b2) @ w3 + b3
    yt = torch.tensor(y)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z, yt, pos_weight=torch.tensor(2.0))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.14159, 1e-3], np.float64)
    r = so.bf16_round(x)
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(r, t)


def test_adam_matches_closed_form_first_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.1])
    p1, m, v = so.adam_step(p, g, np.zeros(2), np.zeros(2), 1, lr=0.01)
    # first Adam step moves every coordinate by lr * sign(g) (up to eps)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=1e-7)


def test_adam_matches_torch_adam_over_several_steps():
    """Six FP64 Adam steps with changing gradients against torch.optim.Adam:
    past step 1 the bias corrections no longer cancel, so a wrong moment
    update, bias correction or epsilon placement shows."""
    rng = np.random.default_rng(11)
    p = rng.standard_normal(7)
    m = np.zeros(7)
    v = np.zeros(7)
    pt = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.03, betas=(0.8, 0.95), eps=1e-3)
    for step in range(1, 7):
        g = rng.standard_normal(7) * (0.1 + step)
        p, m, v = so.adam_step(p, g, m, v, step, lr=0.03, beta1=0.8, beta2=0.95, eps=1e-3)
        opt.zero_grad()
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_column_features_hand_worked():
    """Target at the origin of the plane; candidates (sorted by distance) at
    (1, 0), (0, 2), (2.5, 0) and (-3, 0); exponential kernel, l = 2, unit
    variance.  Every feature worked out by hand."""
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0], [2.5, 0.0], [-3.0, 0.0]])
    ker = inputs.Kernel(1, 2.0)
    f = so.features(x, ker, 0, [1, 2, 3, 4])
    rho = lambda r: math.exp(-r / 2.0)  # noqa: E731
    r = [1.0, 2.0, 2.5, 3.0]
    # distances between candidates: |p0 p1| = sqrt 5, |p0 p2| = 1.5, |p0 p3| = 4,
    # |p1 p2| = sqrt 10.25, |p1 p3| = sqrt 13, |p2 p3| = 5.5
    dj0 = [0.0, math.sqrt(5.0), 1.5, 4.0]
    nearest_other = [1.5, math.sqrt(5.0), 1.5, math.sqrt(13.0)]
    cos0 = [1.0, 0.0, 1.0, -1.0]
    # closer candidates within the 0.7 cone: only p0 for p2 (same direction)
    cone = [0, 0, 1, 0]
    for s in range(4):
        assert f[s, 0] == pytest.approx(math.log(r[s] / 1.0))
        assert f[s, 1] == pytest.approx(s / 4)
        assert f[s, 2] == pytest.approx(rho(r[s]))
        assert f[s, 3] == pytest.approx(r[s] / 2.0)
        assert f[s, 4] == pytest.approx(0.5)
        assert f[s, 5] == pytest.approx(cos0[s], abs=1e-15)
        assert f[s, 6] == pytest.approx(nearest_other[s] / r[s])
        assert f[s, 7] == pytest.approx(cone[s] / 8)
        assert f[s, 8] == pytest.approx(rho(dj0[s]))
        if s == 0:
            assert f[s, 9] == 1.0
        else:
            # after conditioning on p0: cov = rho(r) - rho(1) rho(dj0), var = 1 - rho(dj0)^2
            cov1 = rho(r[s]) - rho(1.0) * rho(dj0[s])
            var1 = 1.0 - rho(dj0[s]) ** 2
            assert f[s, 9] == pytest.approx(cov1 * cov1 / var1)
        assert f[s, 10] == (1.0 if s == 0 else 0.0)
        assert f[s, 11] == pytest.approx(math.log1p(s) / math.log1p(4))
    assert np.all(f[:, 12:] == 0.0)


def test_step1_feature_equals_oracle_conditional_score():
    """f9 is the decrease of the target's variance that candidate j brings once
    the nearest candidate is selected: the oracle's tracked cov^2/var after one
    pick, over the prior."""
    w = inputs.workload_plain_fp64(n=400, seed=7)
    for t in range(0, 350, 23):
        i = int(w.targets[t])
        pool = w.pool[t, : w.pool_len[t]]
        if len(pool) < 3:
            continue
        f = so.features(w.points, w.kernel, i, pool)
        r = oracle.select_one(w.points, w.kernel, i, pool, 1)
        assert r["sel"][0] == pool[0]
        prior = w.kernel.variance + w.kernel.nugget
        score = r["cov"] ** 2 / r["var"] / prior
        np.testing.assert_allclose(f[1:, 9], score[1:], rtol=1e-9, atol=1e-14)
        assert f[0, 9] == 1.0 and f[0, 10] == 1.0 and np.all(f[1:, 10] == 0)
        np.testing.assert_allclose(f[:, 2], [oracle.matern(w.kernel.two_nu, w.kernel.length_scale, 1.0,
                                                          np.linalg.norm(w.points[j] - w.points[i])) for j in pool],
                                   rtol=1e-12)


def test_features_invariant_under_rigid_motion():
    w = inputs.workload_plain_fp64(n=300, seed=2)
    ang = 0.4
    R = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    moved = w.points @ R.T + 0.7
    for t in (3, 50, 120):
        a = so.features(w.points, w.kernel, int(w.targets[t]), w.pool[t, : w.pool_len[t]])
        b = so.features(moved, w.kernel, int(w.targets[t]), w.pool[t, : w.pool_len[t]])
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-11)


def test_screen_keep_picks_largest_logits_in_slot_order():
    z = np.array([0.1, 2.0, -1.0, 2.0, 0.5, -3.0])
    kept, fb = so.screen_keep(z, 6, 3, fallback_threshold=10.0)
    assert list(kept) == [1, 3, 4] and not fb
    kept, fb = so.screen_keep(z, 6, 3, fallback_threshold=0.2)
    assert fb  # dropped sigmoids sum to 0.525 + 0.269 + 0.047
    kept, fb = so.screen_keep(z, 2, 3)
    assert list(kept) == [0, 1] and not fb


def _torch_st_bf16(t):
    """Round to bfloat16 in the forward pass, identity in the backward pass."""
    return t + (t.to(torch.bfloat16).to(t.dtype) - t).detach()


def test_bf16_forward_and_backward_match_torch_straight_through():
    """The rounded forward (inputs, weights and both hidden activations in
    BF16) and its gradient with the rounding taken as the identity, against
    torch's own bfloat16 casts and autograd."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((48, so.F))
    y = (rng.random(48) < 0.25).astype(np.float64)
    p = _params(9)
    loss, g = so.bce_loss_and_grad(X, y, p, pos_weight=2.5, bf16=True)
    z, _ = so.mlp_forward(X, p, bf16=True)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    W1 = _torch_st_bf16(pt[so.OFF_W1:so.OFF_B1].view(so.F, so.H))
    b1 = pt[so.OFF_B1:so.OFF_W2]
    W2 = _torch_st_bf16(pt[so.OFF_W2:so.OFF_B2].view(so.H, so.H))
    b2 = pt[so.OFF_B2:so.OFF_W3]
    w3 = _torch_st_bf16(pt[so.OFF_W3:so.OFF_B3])
    b3 = pt[so.OFF_B3]
    Xt = torch.tensor(X).to(torch.bfloat16).to(torch.float64)
    h1 = _torch_st_bf16(torch.relu(Xt @ W1 + b1))
    h2 = _torch_st_bf16(torch.relu(h1 @ W2 + b2))
    zt = h2 @ w3 + b3
    lt = torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.tensor(y), pos_weight=torch.tensor(2.5))
    lt.backward()
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-14)


# ---- group screen (multi-target) features and keys ---------------------------
def test_group_features_with_one_member_reduce_to_column_features():
    """With a single member the group features are the column screen's
    distance features of that member as the target."""
    x = inputs.uniform_points(400, 2, 17)
    ker = inputs.Kernel(5, 0.07)
    tgt = 11
    d = np.sqrt(np.sum((x - x[tgt]) ** 2, axis=1))
    pool = [j for j in np.argsort(d, kind="stable") if j != tgt][:60]
    fc = so.features(x, ker, tgt, pool)
    fg = so.group_features(x, ker, [tgt], pool)
    for gcol, ccol in ((0, 0), (1, 1), (2, 2), (3, 3), (9, 10), (10, 11)):
        np.testing.assert_allclose(fg[:, gcol], fc[:, ccol], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(fg[:, 4], fc[:, 2], rtol=1e-12)  # r2 = r1
    np.testing.assert_allclose(fg[:, 5], fc[:, 2], rtol=1e-12)  # mean over one member
    np.testing.assert_allclose(fg[:, 6], fc[:, 2] ** 2, rtol=1e-12)
    np.testing.assert_allclose(fg[:, 7], fc[:, 3], rtol=1e-12)
    assert np.all(fg[:, 8] == 1.0 / 64.0) and np.all(fg[:, 13:] == 0.0)
    # the member's nearest candidate is slot 0: ratio r_s / r_0
    np.testing.assert_allclose(fg[:, 11], fc[:, 0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(fg[:, 12], np.exp(1.0 - np.exp(fc[:, 0])), rtol=1e-12)


def test_group_features_hand_worked():
    """Members at 0 and 1 on a line, candidates at 0.25, 0.6 and 3 (sorted by
    the distance to the nearest member); exponential kernel, l = 0.5."""
    x = np.array([[0.0], [1.0], [0.25], [0.6], [3.0]])
    ker = inputs.Kernel(1, 0.5)
    f = so.group_features(x, ker, [0, 1], [2, 3, 4])
    rho = lambda r: math.exp(-r / 0.5)  # noqa: E731
    # slot 0: r = (0.25, 0.75); slot 1: r = (0.6, 0.4); slot 2: r = (3, 2)
    for s, (ra, rb) in enumerate(((0.25, 0.75), (0.6, 0.4), (3.0, 2.0))):
        r1, r2 = min(ra, rb), max(ra, rb)
        assert f[s, 0] == pytest.approx(math.log(r1 / 0.25))
        assert f[s, 1] == pytest.approx(s / 3)
        assert f[s, 2] == pytest.approx(rho(r1))
        assert f[s, 3] == pytest.approx(r1 / 0.5)
        assert f[s, 4] == pytest.approx(rho(r2))
        assert f[s, 5] == pytest.approx((rho(ra) + rho(rb)) / 2)
        assert f[s, 6] == pytest.approx((rho(ra) ** 2 + rho(rb) ** 2) / 2)
        assert f[s, 7] == pytest.approx((ra + rb) / 2 / 0.5)
        assert f[s, 8] == pytest.approx(2 / 64)
        assert f[s, 9] == (1.0 if s == 0 else 0.0)
        assert f[s, 10] == pytest.approx(math.log1p(s) / math.log1p(3))
        # nearest candidates: member 0 -> 0.25 (slot 0), member 1 -> 0.4 (slot 1)
        qa, qb = ra / 0.25, rb / 0.4
        assert f[s, 11] == pytest.approx(math.log(min(qa, qb)))
        assert f[s, 12] == pytest.approx((math.exp(1 - qa) + math.exp(1 - qb)) / 2)


def test_group_features_rigid_motion_invariant():
    rng = np.random.default_rng(5)
    x = rng.random((300, 3))
    ker = inputs.Kernel(3, 0.1)
    members = [3, 8, 21, 40]
    pool = list(range(100, 180))
    a = rng.standard_normal((3, 3))
    q, _ = np.linalg.qr(a)
    y = x @ q.T + np.array([0.3, -2.0, 5.0])
    np.testing.assert_allclose(so.group_features(y, ker, members, pool), so.group_features(x, ker, members, pool),
                               rtol=1e-9, atol=1e-12)


def test_screen_keep_is_exact_order_with_ties_to_smaller_slot():
    """The keep rule is the plain definition: logits that differ in their last
    bit are ordered by value, equal logits by slot, and -0 equals +0."""
    from itertools import combinations

    one_ulp = np.nextafter(np.float32(1.0), np.float32(2.0))
    z = np.array([1.0, one_ulp, 0.5, 1.0], np.float32)
    assert list(so.screen_keep(z, 4, 1, 10.0)[0]) == [1]
    assert list(so.screen_keep(z, 4, 2, 10.0)[0]) == [0, 1]
    assert list(so.screen_keep(z, 4, 3, 10.0)[0]) == [0, 1, 3]
    z2 = np.array([-0.0, 0.0, -1.0, 0.0], np.float32)
    assert list(so.screen_keep(z2, 4, 2, 10.0)[0]) == [0, 1]
    assert list(so.screen_keep(z2, 4, 3, 10.0)[0]) == [0, 1, 3]
    # brute force: of every subset of `keep` slots, the one whose sorted
    # (-z, slot) list is smallest
    rng = np.random.default_rng(5)
    for _ in range(50):
        C = int(rng.integers(2, 9))
        zz = rng.integers(-2, 3, size=C).astype(np.float32) * np.float32(0.5)
        keep = int(rng.integers(1, C))
        best = min((sorted((-float(zz[s]), s) for s in sub), sub) for sub in combinations(range(C), keep))
        assert list(so.screen_keep(zz, C, keep, 1e9)[0]) == list(best[1])


def test_features_batch_equals_per_column_features():
    """The batched features (used by the CPU baseline) are the per-column
    definition, column by column, including ragged and short pools."""
    w = inputs.workload_clustered(n=3000, seed=19, C=64, k=8)
    idx = np.array(list(range(0, 2900, 37)) + [2990, 2995, 2998, 2999])
    lens = w.pool_len[idx].copy()
    lens[3] = 5  # shorter than the eight neighbours
    lens[4] = 1
    fb = so.features_batch(w.points, w.kernel, w.targets[idx], w.pool[idx], lens)
    for b, t in enumerate(idx):
        L = int(lens[b])
        ref = so.features(w.points, w.kernel, int(w.targets[t]), w.pool[t, :L])
        np.testing.assert_allclose(fb[b, :L], ref, rtol=1e-12, atol=1e-14)
        assert np.all(fb[b, L:] == 0.0)
