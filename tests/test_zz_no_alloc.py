"""The allocation-free gradient entry point (csel_mlp_grad_noalloc) against
csel_mlp_grad with its workspace, through the C ABI: bit-identical gradients
and loss on two calls in a row, the second with fewer rows, and the row limit
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from oracle import screen as so
from paper_2307_11648_amd import csel

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.standard_normal((n, 16)).astype(np.float32)).cuda()
    y = torch.from_numpy((rng.random(n) < 0.1).astype(np.uint8)).cuda()
    return x, y


def test_mlp_grad_noalloc_matches_workspace_variant():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    print("case: mlp_grad_noalloc, 20000 then 3001 rows", flush=True)
    p = torch.from_numpy((np.random.default_rng(2).standard_normal(so.N_PARAMS) * 0.2).astype(np.float32)).cuda()
    pb = csel.mlp_to_bf16(p)
    grad = torch.empty(csel.mlp_num_params() + 1, dtype=torch.float32, device="cuda")
    for n, seed in ((20000, 1), (3001, 2)):
        x, y = _batch(n, seed)
        ref, _ = csel.mlp_grad(p, pb, x, y, 3.0)
        grad.fill_(float("nan"))
        csel.mlp_grad_noalloc(p, pb, x, y, 3.0, grad)
        torch.cuda.synchronize()
        assert torch.equal(grad, ref), f"{n} rows: gradient differs from the workspace variant"
        assert torch.isfinite(grad).all()
    # the largest batch is accepted, one row more is refused on the host
    x, y = _batch(csel.MLP_GRAD_NOALLOC_MAX_ROWS, 3)
    ref, _ = csel.mlp_grad(p, pb, x, y, 1.0)
    csel.mlp_grad_noalloc(p, pb, x, y, 1.0, grad)
    torch.cuda.synchronize()
    assert torch.equal(grad, ref)
    x1, y1 = _batch(csel.MLP_GRAD_NOALLOC_MAX_ROWS + 1, 4)
    with pytest.raises(csel.CselError):
        csel.mlp_grad_noalloc(p, pb, x1, y1, 1.0, grad)
