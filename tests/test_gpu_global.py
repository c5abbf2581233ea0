"""GPU parity of csel_select_global (global greedy allocation of nonzeros,
Sec. 5.4, eq. global_obj) against the oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2307_11648_amd import csel, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("budget_per_column", [0, 7, 16, 40])
def test_global_allocation_matches_oracle(budget_per_column):
    """Clustered cloud (an inhomogeneous geometry, where columns differ in how
    much they gain), pools of 128, k_max = 32, FP64: the GPU's per-step gains
    against the oracle's; its allocation against the oracle's heap run on the
    GPU's own gains (bit-exact integer work on the same keys) and on the
    oracle's gains; the factor columns against the oracle's selection of the
    allocated number of picks."""
    print(f"case: global allocation, budget {budget_per_column} per column", flush=True)
    w = inputs.single_target("glob", inputs.cluster_points(6000, 3, 71), inputs.Kernel(3, 0.05), 128, 32,
                             targets=np.arange(0, 6000, 2))
    T, K = len(w.targets), 32
    tg = w.targets.copy()
    pool = w.pool.copy()
    tg[5] = 7000  # a bad column: status 3, no allocation
    budget = budget_per_column * T
    out = csel.select_global(_t(w.points, torch.float64), w.kernel, _t(tg, torch.int32), _t(pool, torch.int32),
                             _t(w.pool_len, torch.int32), K, budget, "fp64", want_gain=True)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "workspace"}
    assert g["status"][5] == 3 and g["k_alloc"][5] == 0 and np.all(g["sel"][5] == -1)
    assert np.all(np.isnan(g["factor"][5]))
    good = np.setdiff1d(np.arange(T), [5])
    assert np.all(g["status"][good] == 0)
    # the allocation is the heap's on the GPU's gains, exactly
    gains = g["gain"].copy()
    gains[5] = np.nan
    ref = oracle.global_allocation(gains, budget)
    assert np.array_equal(g["k_alloc"], ref)
    total = int(np.sum(~np.isnan(gains)))
    assert int(g["k_alloc"].sum()) == min(budget, total)
    # the oracle's own run: gains, and the allocation on its gains
    o = oracle.select_and_factor_diag(w.points, w.kernel, w.targets[good], w.pool[good], w.pool_len[good], K)
    og = oracle.step_gains(o["diag"], o["sel"])
    # gains on the allocated steps of columns whose allocated picks agree
    worst_gain = 0.0
    n_same = 0
    for r, c in enumerate(good):
        kk = int(g["k_alloc"][c])
        if not np.array_equal(g["sel"][c, :kk], o["sel"][r, :kk]):
            continue
        n_same += 1
        if kk:
            d = np.abs(gains[c, :kk] - og[r, :kk]) / np.maximum(og[r, :kk], 1e-300)
            worst_gain = max(worst_gain, float(np.max(d)))
    print(f"allocated picks identical on {n_same} of {len(good)} columns; worst gain relative difference "
          f"{worst_gain:.2e}", flush=True)
    assert n_same >= 0.99 * len(good)
    assert worst_gain <= 1e-9
    m = ~np.isnan(og)
    oa = oracle.global_allocation(np.where(m, og, np.nan), budget)
    agree = float(np.mean(oa == g["k_alloc"][good]))
    print(f"allocation identical on {agree:.4f} of the columns (oracle gains)", flush=True)
    assert agree >= 0.99
    # every column's pattern is the prefix of its greedy run; its column is eq. L_col on it
    worst = 0.0
    for c in list(good[::41]) + [good[-1]]:
        kk = int(g["k_alloc"][c])
        assert np.all(g["sel"][c, kk:] == -1)
        r = oracle.select_one(w.points, w.kernel, int(tg[c]), pool[c, : w.pool_len[c]], kk)
        if not np.array_equal(r["sel"], g["sel"][c, :kk]):
            continue
        a, b = g["factor"][c, : kk + 1], r["factor"][: kk + 1]
        worst = max(worst, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
        assert g["log_condvar"][c] == pytest.approx(r["log_condvar"], abs=1e-8)
    print("worst factor error", worst, flush=True)
    assert worst <= 1e-5
    if budget == 0:
        np.testing.assert_allclose(g["factor"][good, 0], 1.0 / math.sqrt(w.kernel.variance), rtol=1e-14)

