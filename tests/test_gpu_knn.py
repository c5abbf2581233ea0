"""GPU later-ordered kNN pools (csel_later_knn, Sec. 4) against the host
definition (the C kd-tree pools of `inputs.later_knn_pools`, themselves
checked against brute force in test_inputs_geometry.py): bit-identical
pools and lengths, including integer grids with many distance ties,
duplicate points, the last positions (fewer later points than C) and
degenerate clouds."""
import numpy as np
import pytest
import torch

from paper_2307_11648_amd import csel, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    csel.load()


def _gpu_pools(xo, C):
    pool, plen = csel.later_knn_pools(torch.from_numpy(np.ascontiguousarray(xo)).cuda(), C)
    torch.cuda.synchronize()
    return pool.cpu().numpy(), plen.cpu().numpy()


def _compare(xo, C, label):
    print(f"case: later kNN {label} n={len(xo)} d={xo.shape[1]} C={C}", flush=True)
    hp, hl = inputs.later_knn_pools(xo, C)
    gp, gl = _gpu_pools(xo, C)
    np.testing.assert_array_equal(gl, hl)
    bad = np.where(np.any(gp != hp, axis=1))[0]
    assert len(bad) == 0, (label, bad[:5], gp[bad[0]][:12] if len(bad) else None, hp[bad[0]][:12] if len(bad) else None)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("C", [1, 17, 64])
def test_uniform_clouds(d, C):
    xo, _ = inputs.ordered_cloud(inputs.uniform_points(3001, d, 10 + d))
    _compare(xo, C, "uniform")


@pytest.mark.parametrize("d", [1, 2, 3])
def test_integer_grids_with_ties_and_duplicates(d):
    rng = np.random.default_rng(20 + d)
    x = rng.integers(0, 6 if d > 1 else 40, size=(2500, d)).astype(np.float64)
    xo, _ = inputs.ordered_cloud(x)
    _compare(xo, 23, "grid")


def test_clustered_cloud_pools_of_512():
    """The benchmark's distribution (Gaussian clusters plus uniform background,
    3-D) at 60,000 points with pools of 512: every row."""
    xo, _ = inputs.ordered_cloud(inputs.cluster_points(60000, 3, 4))
    _compare(xo, 512, "clustered")


def test_small_and_degenerate():
    for n in (1, 2, 3, 70):
        xo, _ = inputs.ordered_cloud(inputs.uniform_points(n, 2, n))
        _compare(xo, 5, f"tiny n={n}")
    # every point identical: all distances tie at 0, order by position
    xo = np.zeros((40, 3))
    _compare(xo, 8, "identical")
    # a line in 3-D (zero extent in two coordinates)
    t = np.linspace(0.0, 1.0, 500)
    xo, _ = inputs.ordered_cloud(np.stack([t, np.zeros_like(t), np.zeros_like(t)], axis=1))
    _compare(xo, 16, "line")
    # C = 0 and C larger than n
    xo, _ = inputs.ordered_cloud(inputs.uniform_points(300, 3, 5))
    gp, gl = _gpu_pools(xo, 0)
    assert gp.shape == (300, 0) and np.all(gl == 0)
    _compare(xo, 400, "C > n")


def test_rejects_oversized_pools():
    with pytest.raises(csel.CselError):
        _gpu_pools(np.zeros((10, 2)), 2049)
