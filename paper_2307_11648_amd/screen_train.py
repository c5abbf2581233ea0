"""Training of the learned candidate screen, on the GPU, with the library's
own kernels.

Labels come from the exact method: a candidate is positive when the greedy
selection (csel_select_and_factor on the full pool) selects it.  Features
come from csel_screen_features.  Training is weighted BCE with logits by Adam
(csel_mlp_grad + csel_mlp_adam, FP32 master weights, BF16 copy for the
MFMA forward).  torch supplies memory, the random row sampling of each
minibatch and the bookkeeping; every forward, backward and update step runs
in libcsel.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import csel


def init_params(seed: int, device) -> torch.Tensor:
    """He-uniform weights, zero biases (FP32 vector, csel layout)."""
    F, H = 16, 64
    g = np.random.default_rng(seed)
    p = np.zeros(csel.mlp_num_params(), np.float32)
    o = 0
    p[o:o + F * H] = g.uniform(-1, 1, F * H) * math.sqrt(6.0 / F)
    o += F * H + H
    p[o:o + H * H] = g.uniform(-1, 1, H * H) * math.sqrt(6.0 / H)
    o += H * H + H
    p[o:o + H] = g.uniform(-1, 1, H) * math.sqrt(6.0 / H)
    return torch.from_numpy(p).to(device)


def training_set(points, kernel, targets, pool, pool_len, k: int, precision: str = "mixed"):
    """(X [rows, 16] float32, y [rows] uint8) for every valid pool slot of the
    given columns; y = 1 where the exact greedy selection picks the slot."""
    sel = csel.select_and_factor(points, kernel, targets, pool, pool_len, k, precision)["sel"]
    feats = csel.screen_features(points, kernel, targets, pool, pool_len)
    T, C = pool.shape
    valid = torch.arange(C, device=pool.device)[None, :] < pool_len[:, None]
    chosen = torch.zeros((T, C), dtype=torch.bool, device=pool.device)
    for t0 in range(0, T, 4096):
        t1 = min(T, t0 + 4096)
        chosen[t0:t1] = (pool[t0:t1, :, None] == sel[t0:t1, None, :]).any(-1)
    chosen &= valid
    X = feats[valid].contiguous()
    y = chosen[valid].to(torch.uint8).contiguous()
    return X, y


def train(X, y, steps: int = 3000, batch: int = 8192, lr: float = 2e-3, seed: int = 0, pos_weight: float = 1.0,
          log_every: int = 0):
    """Adam on minibatches of rows; returns (params FP32, params BF16, losses)."""
    dev = X.device
    p = init_params(seed, dev)
    pb = csel.mlp_to_bf16(p)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    n = X.shape[0]
    grad = None
    ws = None
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), device=dev, generator=gen)
        xb = X[idx].contiguous()
        yb = y[idx].contiguous()
        grad, ws = csel.mlp_grad(p, pb, xb, yb, pos_weight, grad=grad, workspace=ws)
        csel.mlp_adam(p, pb, grad[:-1], m, v, lr, step)
        if log_every and step % log_every == 0:
            losses.append(float(grad[-1].item()) / batch)
    return p, pb, losses


def mean_loss(p, pb, X, y, chunk: int = 1 << 20) -> float:
    tot = 0.0
    ws = None
    grad = None
    for a in range(0, X.shape[0], chunk):
        b = min(X.shape[0], a + chunk)
        grad, ws = csel.mlp_grad(p, pb, X[a:b].contiguous(), y[a:b].contiguous(), 1.0, grad=grad, workspace=ws)
        tot += float(grad[-1].item())
    return tot / X.shape[0]


def screened_select(points, kernel, targets, pool, pool_len, k: int, p, pb, keep: int, precision: str = "mixed",
                    fallback_threshold: float = 0.5, out=None, spatial_order: bool = False, plan=None):
    """The screened hot path as one library call (csel_screened_select):
    screen, exact selection on the kept candidates, exact selection on the
    full pool for the fallback columns, all inside the library with no host
    synchronisation.  `plan` (csel.Plan for this shape) is reused when given;
    otherwise one is made for the call, with the Morton processing order when
    `spatial_order`.  Returns (out, scr): the selection outputs and copies of
    the screen's outputs (kept, kept_len, fallback, fallback_list,
    fallback_count)."""
    T, stride = pool.shape
    if plan is None:
        plan = csel.Plan(T, stride, keep, k, precision)
        if spatial_order:
            plan.set_order(points, targets)
    out = plan.step(points, kernel, targets, pool, pool_len, p, pb, fallback_threshold, out=out)
    return out, plan.screen_outputs()


# ---------------------------------------------------------------------------
# groups (multi-target selection: GP prediction batches, supernodes)
# ---------------------------------------------------------------------------
def group_training_set(points, kernel, group_ptr, members, max_members: int, pool, pool_len, k: int,
                       precision: str = "fp64"):
    """(X [rows, 16] float32, y [rows] uint8) for every valid pool slot of the
    given groups; y = 1 where the exact multi-target greedy selection
    (csel_aggregated_select on the full pool) picks the slot."""
    sel = csel.aggregated_select(points, kernel, group_ptr, members, max_members, pool, pool_len, k, precision)["sel"]
    feats = csel.screen_groups(points, kernel, group_ptr, members, pool, pool_len, None, None, 0)["features"]
    G, C = pool.shape
    valid = torch.arange(C, device=pool.device)[None, :] < pool_len[:, None]
    chosen = torch.zeros((G, C), dtype=torch.bool, device=pool.device)
    for g0 in range(0, G, 64):
        g1 = min(G, g0 + 64)
        chosen[g0:g1] = (pool[g0:g1, :, None] == sel[g0:g1, None, :]).any(-1)
    chosen &= valid
    return feats[valid].contiguous(), chosen[valid].to(torch.uint8).contiguous()


def screened_group_select(points, kernel, group_ptr, members, max_members: int, pool, pool_len, k: int, p, pb,
                          keep: int, precision: str = "mixed", fallback_threshold: float = 0.5, want_post_var=True,
                          scr=None, out=None):
    """Screened multi-target selection: csel_screen_groups, then
    csel_aggregated_select on the kept pools; groups whose screen falls back
    (or rejects them as bad input) are selected again on their full pools
    (their count is read on the host, the one synchronisation of this path).
    Returns (out, scr, n_fallback)."""
    scr = csel.screen_groups(points, kernel, group_ptr, members, pool, pool_len, p, pb, keep, fallback_threshold,
                             out=scr)
    out = csel.aggregated_select(points, kernel, group_ptr, members, max_members, scr["kept"], scr["kept_len"], k,
                                 precision, want_post_var=want_post_var, out=out, workspace=(out or {}).get("workspace"))
    fb = torch.nonzero(scr["fallback"] >= 1).flatten()  # 1: fallback, 3: bad group (reported on its full pool)
    nfb = int(fb.numel())
    if nfb:
        # member ranges read on the host, so a bad range is never used to index
        gp = group_ptr.to(torch.int64).cpu()
        n_members = members.numel()
        ok, dead = [], []
        for g in fb.tolist():
            b, e = int(gp[g]), int(gp[g + 1])
            (ok if 0 <= b <= e <= n_members else dead).append(g)
        for g in dead:  # no member range to select for: reported as bad input
            out["sel"][g] = -1
            out["logdet"][g] = float("nan")
            out["status"][g] = 3
        if ok:
            sizes = [int(gp[g + 1] - gp[g]) for g in ok]
            sub_ptr = torch.zeros(len(ok) + 1, dtype=torch.int64)
            sub_ptr[1:] = torch.cumsum(torch.tensor(sizes, dtype=torch.int64), 0)
            idx = torch.cat([torch.arange(int(gp[g]), int(gp[g + 1]), dtype=torch.int64) for g in ok]).to(pool.device)
            okd = torch.tensor(ok, dtype=torch.int64, device=pool.device)
            sub = csel.aggregated_select(points, kernel, sub_ptr.to(torch.int32).to(pool.device),
                                         members[idx].contiguous(), max_members, pool[okd].contiguous(),
                                         pool_len[okd].contiguous(), k, precision, want_post_var=want_post_var)
            for key in ("sel", "logdet", "status"):
                out[key][okd] = sub[key]
            if want_post_var:
                out["post_var"][idx] = sub["post_var"]
    return out, scr, nfb

