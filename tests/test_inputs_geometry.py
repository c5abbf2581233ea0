"""Pins of the seeded inputs' geometry against O(n^2) brute force.

Both the oracle and the HIP path consume the ordering, the candidate pools and
the groups built by ``paper_2307_11648_amd.inputs`` (host kd-trees), so a
mistake there would be invisible to every parity test.  Here each is checked
against its definition written out directly:

* reverse-maximin ordering (Sec. 2.2, eq. maximin, p = 1): the last point is
  point 0; going backwards, each position takes the point farthest from all
  later ones, ties to the smaller id; ell is that distance;
* later-ordered kNN pools (Sec. 4): the C nearest points of larger position,
  by (distance, position);
* union pools of groups (Sec. 5): the C points nearest to any member;
* supernode groups: the earliest unassigned position and its nearest
  unassigned later points within the length-scale ratio.

Integer grids make exact distance ties common, so the tie rules are exercised.
"""
import numpy as np
import pytest

from paper_2307_11648_amd import inputs


def _d2(x, q):
    """Squared distances of every row of x to q, summed coordinate by
    coordinate in order (exact on integer grids)."""
    s = np.zeros(len(x))
    for k in range(x.shape[1]):
        e = x[:, k] - q[k]
        s = s + e * e
    return s


def _clouds():
    rng = np.random.default_rng(21)
    out = []
    for d in (1, 2, 3):
        out.append(("uniform", d, rng.random((300, d))))
        # integer grid with repeated distances (and a few duplicate points)
        g = rng.integers(0, 6 if d > 1 else 40, size=(250, d)).astype(np.float64)
        out.append(("grid", d, g))
    return out


def _brute_maximin(x):
    n = len(x)
    order = np.empty(n, np.int64)
    ell = np.empty(n)
    dist2 = _d2(x, x[0])
    done = np.zeros(n, bool)
    order[n - 1], ell[n - 1], done[0] = 0, np.inf, True
    for pos in range(n - 2, -1, -1):
        cand = np.where(~done)[0]
        best = cand[np.argmax(dist2[cand])]  # argmax returns the first (smallest id) of ties
        order[pos], ell[pos] = best, np.sqrt(dist2[best])
        done[best] = True
        dist2 = np.minimum(dist2, _d2(x, x[best]))
    return order, ell


@pytest.mark.parametrize("name,d,x", _clouds(), ids=lambda v: str(v) if not hasattr(v, "shape") else "pts")
def test_reverse_maximin_matches_brute_force(name, d, x):
    order, ell = inputs.reverse_maximin(x)
    bo, be = _brute_maximin(x)
    np.testing.assert_array_equal(order, bo)
    np.testing.assert_array_equal(ell, be)
    # each earlier position is at least as close to its later points
    assert np.all(np.diff(ell[:-1]) >= 0)


def _brute_later_pool(xo, i, C):
    later = np.arange(i + 1, len(xo))
    d2 = _d2(xo[later], xo[i])
    srt = later[np.lexsort((later, d2))]
    return srt[:C]


@pytest.mark.parametrize("name,d,x", _clouds(), ids=lambda v: str(v) if not hasattr(v, "shape") else "pts")
def test_later_knn_pools_match_brute_force(name, d, x):
    xo, _ = inputs.ordered_cloud(x)
    C = 17
    pool, plen = inputs.later_knn_pools(xo, C)
    for i in range(len(xo)):
        ref = _brute_later_pool(xo, i, C)
        assert plen[i] == len(ref) == min(C, len(xo) - 1 - i)
        np.testing.assert_array_equal(pool[i, : plen[i]], ref)
        assert np.all(pool[i, plen[i]:] == -1)
    q = np.array([0, 5, len(xo) - 1, 3, len(xo) - 2, -1, len(xo)], np.int32)
    ps, ls = inputs.later_knn_pools_subset(xo, C, q)
    for r, i in enumerate(q):
        if 0 <= i < len(xo):
            np.testing.assert_array_equal(ps[r, : ls[r]], pool[i, : plen[i]])
            assert ls[r] == plen[i]
        else:
            assert ls[r] == 0 and np.all(ps[r] == -1)


def _brute_group_pool(x, members, C, later_only, c0, c1):
    if later_only:
        cand = np.arange(max(members) + 1, len(x))
    else:
        cand = np.arange(c0, c1)
    d2 = np.full(len(cand), np.inf)
    for q in members:
        d2 = np.minimum(d2, _d2(x[cand], x[q]))
    return cand[np.lexsort((cand, d2))][:C]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("grid", [False, True])
def test_group_pools_match_brute_force(d, grid):
    rng = np.random.default_rng(30 + d + 10 * grid)
    n = 260
    x = rng.integers(0, 5, size=(n, d)).astype(np.float64) if grid else rng.random((n, d))
    # groups of 1-6 ascending members among the first 200 ids
    sizes = rng.integers(1, 7, size=25)
    gp = np.zeros(len(sizes) + 1, np.int32)
    gp[1:] = np.cumsum(sizes)
    mem = np.concatenate([np.sort(rng.choice(200, size=s, replace=False)) for s in sizes]).astype(np.int32)
    C = 23
    pool, plen = inputs.group_pools(x, gp, mem, C, later_only=True)
    for g in range(len(sizes)):
        ref = _brute_group_pool(x, mem[gp[g]:gp[g + 1]], C, True, 0, 0)
        assert plen[g] == len(ref)
        np.testing.assert_array_equal(pool[g, : plen[g]], ref)
    pool, plen = inputs.group_pools(x, gp, mem, C, later_only=False, cand_range=(60, 240))
    for g in range(len(sizes)):
        ref = _brute_group_pool(x, mem[gp[g]:gp[g + 1]], C, False, 60, 240)
        assert plen[g] == len(ref) == C
        np.testing.assert_array_equal(pool[g, : plen[g]], ref)


def _brute_member_pool(x, members, C):
    """Per member its C + m nearest later points (ties to the smaller id);
    their union without the members, by the smallest distance to a member
    that listed the point (then id); the first C."""
    m = len(members)
    best = {}
    for q in members:
        cand = np.arange(q + 1, len(x))
        d2 = _d2(x[cand], x[q])
        order = np.lexsort((cand, d2))[: C + m]
        for j, dj in zip(cand[order], d2[order]):
            if j not in best or dj < best[j]:
                best[int(j)] = float(dj)
    ids = np.array([j for j in best if j not in set(int(q) for q in members)], np.int64)
    dd = np.array([best[j] for j in ids])
    return ids[np.lexsort((ids, dd))][:C]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("grid", [False, True])
def test_member_later_group_pools_match_brute_force(d, grid):
    """The partial (non-adjacent) pools: every member's own later neighbours,
    so a candidate may precede some members; members never enter a pool."""
    rng = np.random.default_rng(50 + d + 10 * grid)
    n = 240
    x = rng.integers(0, 5, size=(n, d)).astype(np.float64) if grid else rng.random((n, d))
    sizes = rng.integers(1, 7, size=25)
    gp = np.zeros(len(sizes) + 1, np.int32)
    gp[1:] = np.cumsum(sizes)
    mem = np.concatenate([np.sort(rng.choice(220, size=s, replace=False)) for s in sizes]).astype(np.int32)
    C = 19
    pool, plen = inputs.group_pools(x, gp, mem, C, later_only="member")
    interleaved = 0
    for g in range(len(sizes)):
        T = mem[gp[g]:gp[g + 1]]
        ref = _brute_member_pool(x, T, C)
        assert plen[g] == len(ref)
        np.testing.assert_array_equal(pool[g, : plen[g]], ref)
        assert not np.any(np.isin(pool[g, : plen[g]], T))
        assert np.all(pool[g, : plen[g]] > T.min())
        interleaved += int(np.any(pool[g, : plen[g]] < T.max()))
    assert interleaved > 0


@pytest.mark.parametrize("d", [2, 3])
def test_make_groups_matches_brute_force(d):
    rng = np.random.default_rng(40 + d)
    x = rng.random((220, d))
    xo, ell = inputs.ordered_cloud(x)
    sizes = rng.integers(1, 6, size=30).astype(np.int32)
    lam = 1.5
    gp, mem = inputs.make_groups(xo, ell, sizes, lam)
    n = len(xo)
    taken = np.zeros(n, bool)
    ref_ptr, ref_mem = [0], []
    p, g = 0, 0
    while True:
        while p < n and taken[p]:
            p += 1
        if p >= n:
            break
        m = max(1, int(sizes[g % len(sizes)]))
        cand = np.array([j for j in range(p + 1, n) if not taken[j] and (not np.isfinite(ell[p])
                                                                          or ell[j] <= lam * ell[p])], np.int64)
        if len(cand):
            d2 = _d2(xo[cand], xo[p])
            cand = cand[np.lexsort((cand, d2))][: m - 1]
        grp = sorted([p] + [int(j) for j in cand])
        taken[grp] = True
        ref_mem.extend(grp)
        ref_ptr.append(len(ref_mem))
        g += 1
    np.testing.assert_array_equal(gp, ref_ptr)
    np.testing.assert_array_equal(mem[: len(ref_mem)], ref_mem)
