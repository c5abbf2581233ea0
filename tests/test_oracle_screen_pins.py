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
