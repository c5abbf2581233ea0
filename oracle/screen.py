"""Oracle of the learned candidate screen: per-candidate features and the MLP.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy, FP64.

The screen is not part of the paper: it prunes a column's candidate pool to
the `keep` candidates an MLP scores highest, before the exact greedy
selection of Sec. 3.1 runs on the kept candidates.  Features describe a
candidate j of target i (pool sorted by distance, slot s, nearest slot 0):

  f0  log(r_s / r_0)                  f6  min_{l<8, l!=s} |x_j - x_l| / r_s
  f1  s / C                           f7  #{l<8, l!=s : r_l < r_s, cos(d_s, d_l) > 0.7} / 8
  f2  K(r_s) / var  (correlation)     f8  K(|x_j - x_{p0}|) / var
  f3  r_s / length_scale              f9  step-1 score: the variance decrease of
  f4  r_0 / length_scale                  the target from j after the nearest
  f5  cos(d_s, d_0)                       candidate is selected (eq. obj_gp), / prior
                                      f10 [s == 0]
                                      f11 log(1 + s) / log(1 + C)
  f12..f15 = 0
with d_s = x_{p_s} - x_i, r_s = |d_s|, guarded against zero distances.

MLP: 16 -> 64 -> 64 -> 1 with ReLU.  The GPU computes it with BF16 inputs,
BF16 weights and BF16 activations of both hidden layers (matrix-core
operands) and FP32 accumulation; `mlp_forward(..., bf16=True)` evaluates the
same rounded quantities in FP64 so the two sides differ only by accumulation
order.  The backward pass takes the rounding as the identity.
Parameters are one FP32 vector: W1[16][64], b1[64], W2[64][64], b2[64],
w3[64], b3 (5313 values).
"""
from __future__ import annotations

import numpy as np

F = 16
H = 64
N_PARAMS = F * H + H + H * H + H + H + 1
OFF_W1, OFF_B1 = 0, F * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H


def unpack(p):
    p = np.asarray(p, np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(F, H)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(H, H)
    b2 = p[OFF_B2:OFF_W3]
    w3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def matern_corr(two_nu, a):
    if two_nu == 1:
        return np.exp(-a)
    if two_nu == 3:
        return (1 + a) * np.exp(-a)
    return (1 + a + a * a / 3.0) * np.exp(-a)


def features(x, kernel, target, pool):
    """Features [C, 16] (FP64) of the candidates `pool` (sorted by distance)."""
    x = np.asarray(x, np.float64)
    pool = np.asarray(pool)
    C = len(pool)
    out = np.zeros((C, F))
    if C == 0:
        return out
    ell = float(kernel.length_scale)
    c = np.sqrt(float(kernel.two_nu)) / ell
    tiny = 1e-9 * ell
    a_diag = 1.0 + float(kernel.nugget) / float(kernel.variance)
    xi = x[target]
    d = x[pool] - xi
    r = np.sqrt(np.sum(d * d, axis=1))
    r0 = max(r[0], tiny)
    rs = np.maximum(r, tiny)
    s = np.arange(C)
    out[:, 0] = np.log(rs / r0)
    out[:, 1] = s / C
    rho_i = matern_corr(kernel.two_nu, c * r)
    out[:, 2] = rho_i
    out[:, 3] = r / ell
    out[:, 4] = r[0] / ell
    cos0 = (d @ d[0]) / (rs * r0)
    out[:, 5] = np.where(r > 0, cos0, 1.0)
    near = min(8, C)
    for j in range(C):
        best = np.inf
        cnt = 0
        for l in range(near):
            if l == j:
                continue
            dl = np.sqrt(np.sum((x[pool[j]] - x[pool[l]]) ** 2))
            best = min(best, dl / rs[j])
            if r[l] < r[j] and (d[j] @ d[l]) / (rs[j] * max(r[l], tiny)) > 0.7:
                cnt += 1
        out[j, 6] = best if np.isfinite(best) else 0.0
        out[j, 7] = cnt / 8.0
    dj0 = np.sqrt(np.sum((x[pool] - x[pool[0]]) ** 2, axis=1))
    rho_j0 = matern_corr(kernel.two_nu, c * dj0)
    rho_j0[0] = a_diag
    out[:, 8] = matern_corr(kernel.two_nu, c * dj0)
    cov1 = rho_i - rho_i[0] * rho_j0 / a_diag
    var1 = a_diag - rho_j0 * rho_j0 / a_diag
    f9 = np.where(var1 > 1e-12 * a_diag, cov1 * cov1 / np.maximum(var1, 1e-300) / a_diag, 0.0)
    f9[0] = 1.0
    out[:, 9] = f9
    out[0, 10] = 1.0
    out[:, 11] = np.log1p(s) / np.log1p(C)
    return out


def features_batch(x, kernel, targets, pools, lens):
    """`features` of many columns at once: pools [B, S] (-1 padded), lens [B]
    -> [B, S, 16], zeros past each pool's length.  The same definitions,
    written over a batch axis (numpy broadcasting instead of per-column
    calls); pinned to `features` column by column."""
    x = np.asarray(x, np.float64)
    pools = np.asarray(pools)
    lens = np.asarray(lens, np.int64)
    B, S = pools.shape
    out = np.zeros((B, S, F))
    if B == 0 or S == 0:
        return out
    ell = float(kernel.length_scale)
    c = np.sqrt(float(kernel.two_nu)) / ell
    tiny = 1e-9 * ell
    a_diag = 1.0 + float(kernel.nugget) / float(kernel.variance)
    s = np.arange(S)
    valid = s[None, :] < lens[:, None]
    P = np.where(valid, pools, 0)
    xp = x[P]                                    # [B, S, d]
    d = xp - x[np.asarray(targets)][:, None, :]
    r = np.sqrt(np.sum(d * d, axis=2))           # [B, S]
    r0 = np.maximum(r[:, 0], tiny)
    rs = np.maximum(r, tiny)
    Cf = np.maximum(lens, 1).astype(np.float64)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        out[..., 0] = np.log(rs / r0[:, None])
        out[..., 1] = s[None, :] / Cf
        rho_i = matern_corr(kernel.two_nu, c * r)
        out[..., 2] = rho_i
        out[..., 3] = r / ell
        out[..., 4] = (r[:, 0] / ell)[:, None]
        cos0 = np.sum(d * d[:, :1, :], axis=2) / (rs * r0[:, None])
        out[..., 5] = np.where(r > 0, cos0, 1.0)
        # neighbourhood terms over the (up to) 8 nearest candidates l != j
        L8 = min(8, S)
        near = np.minimum(8, lens)
        ls = np.arange(L8)
        ok = (ls[None, None, :] < near[:, None, None]) & (ls[None, None, :] != s[None, :, None])
        D = np.sqrt(np.sum((xp[:, :, None, :] - xp[:, None, :L8, :]) ** 2, axis=3))  # [B, S, L8]
        best = np.min(np.where(ok, D / rs[:, :, None], np.inf), axis=2)
        out[..., 6] = np.where(np.isfinite(best), best, 0.0)
        rl = r[:, None, :L8]
        dots = np.sum(d[:, :, None, :] * d[:, None, :L8, :], axis=3)
        cone = ok & (rl < r[:, :, None]) & (dots / (rs[:, :, None] * np.maximum(rl, tiny)) > 0.7)
        out[..., 7] = np.sum(cone, axis=2) / 8.0
        dj0 = np.sqrt(np.sum((xp - xp[:, :1, :]) ** 2, axis=2))
        rho_j0 = matern_corr(kernel.two_nu, c * dj0)
        out[..., 8] = rho_j0
        rho_j0 = rho_j0.copy()
        rho_j0[:, 0] = a_diag
        cov1 = rho_i - rho_i[:, :1] * rho_j0 / a_diag
        var1 = a_diag - rho_j0 * rho_j0 / a_diag
        f9 = np.where(var1 > 1e-12 * a_diag, cov1 * cov1 / np.maximum(var1, 1e-300) / a_diag, 0.0)
        f9[:, 0] = 1.0
        out[..., 9] = f9
        out[:, 0, 10] = 1.0
        out[..., 11] = np.log1p(s)[None, :] / np.log1p(Cf)
    out[~valid] = 0.0
    return out


def group_features(x, kernel, members, pool):
    """Features [C, 16] (FP64) of the candidates `pool` of a group of targets
    `members` (multi-target selection, Sec. 5; pool sorted by the distance to
    the nearest member, slot s, nearest slot 0).  With r_q = |x_j - x_q| over
    the m members, r1 and r2 the smallest and second smallest (r2 = r1 when
    m = 1) and rho the kernel correlation:

      f0  log(r1_s / r1_0)          f5  mean_q rho(r_q)
      f1  s / C                     f6  mean_q rho(r_q)^2
      f2  rho(r1)                   f7  mean_q r_q / length_scale
      f3  r1 / length_scale         f8  m / 64
      f4  rho(r2)                   f9  [s == 0]
                                    f10 log(1 + s) / log(1 + C)
      f11 log min_q (r_q / dmin_q)  f12 mean_q exp(1 - r_q / dmin_q)
      f13..f15 = 0
    with dmin_q the distance from member q to its nearest candidate of the
    pool (f11 = 0 for a candidate that is some member's nearest); distances
    guarded against zero as in `features`."""
    x = np.asarray(x, np.float64)
    pool = np.asarray(pool)
    members = np.asarray(members)
    C = len(pool)
    out = np.zeros((C, F))
    m = len(members)
    if C == 0 or m == 0:
        return out
    ell = float(kernel.length_scale)
    c = np.sqrt(float(kernel.two_nu)) / ell
    tiny = 1e-9 * ell
    d = x[pool][:, None, :] - x[members][None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))  # [C, m]
    rsort = np.sort(r, axis=1)
    r1 = rsort[:, 0]
    r2 = rsort[:, 1] if m > 1 else r1
    rho = matern_corr(kernel.two_nu, c * r)
    s = np.arange(C)
    out[:, 0] = np.log(np.maximum(r1, tiny) / max(r1[0], tiny))
    out[:, 1] = s / C
    out[:, 2] = matern_corr(kernel.two_nu, c * r1)
    out[:, 3] = r1 / ell
    out[:, 4] = matern_corr(kernel.two_nu, c * r2)
    out[:, 5] = np.mean(rho, axis=1)
    out[:, 6] = np.mean(rho * rho, axis=1)
    out[:, 7] = np.mean(r, axis=1) / ell
    out[:, 8] = m / 64.0
    out[0, 9] = 1.0
    out[:, 10] = np.log1p(s) / np.log1p(C)
    dmin = np.maximum(np.min(r, axis=0), tiny)  # [m]
    ratio = np.maximum(r, tiny) / dmin[None, :]
    out[:, 11] = np.log(np.min(ratio, axis=1))
    out[:, 12] = np.mean(np.exp(1.0 - ratio), axis=1)
    return out


def mlp_forward(X, p, bf16=True):
    """Logits [N] and the intermediate activations (FP64)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, np.float64)
    if bf16:
        X, W1, W2, w3 = bf16_round(X), bf16_round(W1), bf16_round(W2), bf16_round(w3)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    H1q = bf16_round(H1) if bf16 else H1
    Z2 = H1q @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    H2q = bf16_round(H2) if bf16 else H2
    z = H2q @ w3 + b3
    return z, {"X": X, "W1": W1, "W2": W2, "w3": w3, "H1": H1, "H1q": H1q, "H2": H2, "H2q": H2q}


def bce_loss_and_grad(X, y, p, pos_weight=1.0, bf16=True):
    """Mean weighted BCE-with-logits over the rows and its gradient with
    respect to the FP32 parameter vector (backpropagated through the same
    rounded forward quantities)."""
    y = np.asarray(y, np.float64)
    z, a = mlp_forward(X, p, bf16)
    N = len(y)
    wgt = np.where(y > 0.5, pos_weight, 1.0)
    # log(1 + exp(-|z|)) form of the BCE
    loss = wgt * (np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z))))
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = wgt * (sig - y) / N
    g = np.zeros(N_PARAMS)
    H2, H1q, H1 = a["H2"], a["H1q"], a["H1"]
    g[OFF_W3:OFF_B3] = a["H2q"].T @ dz
    g[OFF_B3] = dz.sum()
    dH2 = np.outer(dz, a["w3"]) * (H2 > 0)
    g[OFF_W2:OFF_B2] = (H1q.T @ dH2).ravel()
    g[OFF_B2:OFF_W3] = dH2.sum(axis=0)
    dH1 = (dH2 @ a["W2"].T) * (H1 > 0)
    g[OFF_W1:OFF_B1] = (a["X"].T @ dH1).ravel()
    g[OFF_B1:OFF_W2] = dH1.sum(axis=0)
    return float(loss.sum() / N), g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in FP64; returns new p, m, v."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def screen_keep(logits, pool_len, keep, fallback_threshold=0.5):
    """Kept slots (ascending) of one column (or group): the `keep` largest
    logits, equal logits ordered by the smaller slot; and the fallback flag:
    the expected number of true selections among the dropped candidates,
    sum sigmoid(logit), exceeds the threshold.  The rule is the plain
    definition, with no quantisation of the logits: two logits are equal only
    when their values are (so -0.0 equals +0.0)."""
    z = np.asarray(logits[:pool_len], np.float64)
    C = len(z)
    if C <= keep:
        return np.arange(C), False
    order = np.lexsort((np.arange(C), -z))  # by -z, then by slot
    kept = np.sort(order[:keep])
    dropped = np.array(order[keep:])
    fb = float(np.sum(1.0 / (1.0 + np.exp(-z[dropped])))) > fallback_threshold
    return kept, fb
