"""Pins of the group-by oracle: a dict-based brute force, invariants that any
correct grouping satisfies, and closed forms."""
import numpy as np
import pytest

import oracle

M64 = 1 << 64


def brute(keys, vals):
    g = {}
    for i, k in enumerate(int(x) for x in keys):
        c, s = g.get(k, (0, [0] * len(vals)))
        g[k] = (c + 1, [(a + int(v[i])) % M64 for a, v in zip(s, vals)])
    ks = sorted(g)
    to64 = lambda u: u - M64 if u >= 1 << 63 else u
    return ks, [g[k][0] for k in ks], [[to64(g[k][1][c]) for k in ks] for c in range(len(vals))]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_group_by_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 3000))
    keys = rng.integers(-50, 50, n).astype(np.int32) if seed % 2 else \
        rng.choice(np.array([-2**63, 2**63 - 1, 0, -1, 7], dtype=np.int64), n)
    vals = [rng.integers(-2**63, 2**63 - 1, n, dtype=np.int64), rng.integers(-2**31, 2**31, n).astype(np.int32)]
    gk, cnt, sums = oracle.group_by(keys, vals)
    bk, bc, bs = brute(keys, vals)
    assert gk.tolist() == bk and cnt.tolist() == bc
    assert [s.tolist() for s in sums] == bs


def test_group_by_invariants_and_closed_forms():
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 1000, 100000)
    v = rng.integers(-10**6, 10**6, 100000)
    gk, cnt, (s,) = oracle.group_by(keys, [v])
    assert cnt.sum() == keys.size and s.sum() == v.sum()
    assert np.array_equal(gk, np.unique(keys))
    # every row in one group: count n, sum of all values
    gk, cnt, (s,) = oracle.group_by(np.full(500, 42, np.int64), [np.arange(500)])
    assert gk.tolist() == [42] and cnt.tolist() == [500] and s.tolist() == [500 * 499 // 2]
    # all keys distinct: the groups are the rows, sorted
    perm = rng.permutation(1000)
    gk, cnt, (s,) = oracle.group_by(perm, [perm * 3])
    assert np.array_equal(gk, np.arange(1000)) and (cnt == 1).all() and np.array_equal(s, np.arange(1000) * 3)
    # empty input, and the mod-2^64 wrap of a sum
    gk, cnt, sums = oracle.group_by(np.zeros(0, np.int64), [np.zeros(0, np.int64)])
    assert gk.size == 0 and cnt.size == 0 and sums[0].size == 0
    gk, cnt, (s,) = oracle.group_by(np.array([1, 1]), [np.array([2**63 - 1, 2], dtype=np.int64)])
    assert s.tolist() == [-(2**63) + 1]
