"""GPU parity of csel_kernel_matvec and csel_pcg (the conjugate gradient
preconditioned by the sparse factor, Sec. 6.3) against the oracle."""
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


@pytest.mark.parametrize("two_nu,d,n", [(1, 3, 3001), (3, 2, 1000), (5, 1, 257), (1, 3, 1)])
def test_kernel_matvec_matches_dense(two_nu, d, n):
    print(f"case: kernel matvec nu={two_nu}/2 d={d} n={n}", flush=True)
    x = inputs.uniform_points(n, d, 11 + n)
    kern = inputs.Kernel(two_nu, 0.3, 1.7, 1e-3)
    v = np.random.default_rng(2).standard_normal(n)
    y, _ = csel.kernel_matvec(_t(x, torch.float64), kern, _t(v, torch.float64))
    y2, _ = csel.kernel_matvec(_t(x, torch.float64), kern, _t(v, torch.float64))
    ref = oracle.covariance(x, kern) @ v
    got = y.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))
    assert np.array_equal(got, y2.cpu().numpy())  # deterministic


def _factor(xo, kern, C, k, knn=False):
    """The factor on the greedy selection of k from C later neighbours (or, with
    knn, on the k nearest later neighbours), FP64, and its transpose."""
    n = len(xo)
    pool, plen = inputs.later_knn_pools(xo, k if knn else C)
    pts = _t(xo, torch.float64)
    tg = _t(np.arange(n, dtype=np.int32), torch.int32)
    f = csel.select_and_factor(pts, kern, tg, _t(pool, torch.int32), _t(plen, torch.int32), k, "fp64")
    cp, rows, vals = csel.single_target_csc(tg, f["sel"], f["factor"])
    return pts, (cp, rows, vals), csel.transpose_factor(cp, rows, vals)[:3]


def test_pcg_matches_oracle_and_conditional_beats_knn():
    """N = 4000 uniform in [0,1]^3, Matern 1/2, l = 1 (the experiment's kernel
    at reduced N), y = Theta x for a Gaussian x: the GPU's iterations and
    solution against the oracle's PCG with the same factor (dense FP64); the
    conditional-selection factor converges in fewer iterations than the
    factor on the k nearest neighbours, and both beat no preconditioner."""
    print("case: pcg n=4000 nu=1/2 l=1", flush=True)
    n, k = 4000, 8
    kern = inputs.Kernel(1, 1.0)
    xo, _ = inputs.ordered_cloud(inputs.uniform_points(n, 3, 17))
    sol = np.random.default_rng(4).standard_normal(n)
    th = oracle.covariance(xo, kern)
    y = th @ sol
    res = {}
    for name, knn in (("conditional", False), ("knn", True)):
        pts, fac, fac_t = _factor(xo, kern, 3 * k, k, knn)
        xg, it, rel = csel.pcg(pts, kern, _t(y, torch.float64), fac, fac_t, rel_tol=1e-10, max_iter=2000)
        torch.cuda.synchronize()
        L = oracle.dense_factor(n, *(a.cpu().numpy() for a in fac))
        xo_, ito, relo = oracle.pcg(th, y, L, rel_tol=1e-10, max_iter=2000)
        print(f"{name}: GPU {it} iterations (rel residual {rel:.2e}), oracle {ito}", flush=True)
        assert rel <= 1e-10 and abs(it - ito) <= 1
        xg = xg.cpu().numpy()
        assert np.linalg.norm(xg - xo_) <= 1e-6 * np.linalg.norm(xo_)
        assert np.linalg.norm(y - th @ xg) <= 1e-9 * np.linalg.norm(y)
        res[name] = it
    _, it0, rel0 = csel.pcg(_t(xo, torch.float64), kern, _t(y, torch.float64), None, None, rel_tol=1e-10,
                            max_iter=5000)
    print("no preconditioner:", it0, "iterations", flush=True)
    assert res["conditional"] < res["knn"] < it0
