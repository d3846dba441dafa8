"""Pins of the statistics oracle: min/max, the sketch hash, the registers and
the distinct-count estimate (Section 4: min, max and an HLL++ sketch of
intermediate data; Section 4.1 for the distinct count).

The estimate is held to HyperLogLog's standard error 1.04/sqrt(m) (0.8125% at
m = 2^14) over a wide range of true distinct counts, and to closed forms of
the estimator; the hash is pinned by inverting it.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

M = 1 << oracle.HLL_P
SIGMA = 1.04 / math.sqrt(M)
MASK = (1 << 64) - 1


def inverse_fmix64(h: int) -> int:
    """Undo each step of fmix64: xor-shift by 33 is its own inverse on 64 bits
    (33 > 32), and the multipliers are odd, so they have inverses mod 2^64."""
    inv1 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    inv2 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    h ^= h >> 33
    h = (h * inv1) & MASK
    h ^= h >> 33
    h = (h * inv2) & MASK
    h ^= h >> 33
    return h


def test_fmix64_is_the_invertible_finalizer():
    assert oracle.fmix64(0) == 0
    rng = np.random.default_rng(3)
    for x in [1, 2, MASK, 1 << 63, 0x0123456789ABCDEF] + [int(v) for v in rng.integers(0, 1 << 62, 200)]:
        h = oracle.fmix64(x)
        assert inverse_fmix64(h) == x
        assert h != x or x == 0


def test_fmix64_avalanche():
    """Flipping one input bit flips about half of the output bits."""
    rng = np.random.default_rng(5)
    flips = []
    for x in rng.integers(0, 1 << 63, 64):
        h = oracle.fmix64(int(x))
        for b in range(64):
            flips.append(bin(h ^ oracle.fmix64(int(x) ^ (1 << b))).count("1"))
    assert abs(np.mean(flips) - 32) < 0.5


def test_min_max_exact():
    for col in [synth.random_small(1, 1000, 1, -(1 << 63), (1 << 63) - 1, dtype=torch.int64).build_keys,
                synth.random_small(2, 777, 1, -5, 5).build_keys,
                torch.tensor([-(1 << 31), (1 << 31) - 1], dtype=torch.int32)]:
        st = oracle.column_stats(col)
        a = col.numpy()
        assert (st["n"], st["min"], st["max"]) == (a.size, int(a.min()), int(a.max()))


def test_empty_column():
    st = oracle.column_stats(torch.zeros(0, dtype=torch.int32))
    assert (st["n"], st["min"], st["max"], st["ndv"]) == (0, 0, 0, 0.0)
    assert not st["regs"].any()


def test_one_distinct_key():
    st = oracle.column_stats(torch.full((10000,), 12345, dtype=torch.int64))
    assert abs(st["ndv"] - 1.0) < 1e-3
    assert np.count_nonzero(st["regs"]) == 1


def test_registers_ignore_order_duplicates_and_width():
    v = synth.random_small(8, 5000, 1, -(1 << 31), (1 << 31) - 1).build_keys
    r32 = oracle.hll_registers(v)
    r64 = oracle.hll_registers(v.to(torch.int64))
    assert np.array_equal(r32, r64)
    perm = torch.randperm(v.numel(), generator=torch.Generator().manual_seed(1))
    assert np.array_equal(oracle.hll_registers(torch.cat([v[perm], v[:100]])), r32)


def test_registers_merge_by_max():
    a = synth.distinct_values(1, 3000, 3000)
    b = synth.distinct_values(2, 4000, 4000)
    merged = np.maximum(oracle.hll_registers(a), oracle.hll_registers(b))
    assert np.array_equal(oracle.hll_registers(torch.cat([a, b])), merged)


def test_register_values_in_range():
    regs = oracle.hll_registers(synth.distinct_values(3, 200000, 200000))
    assert regs.max() <= 64 - oracle.HLL_P + 1
    # for n >> m nearly every register is set, and about half of the ranks seen are 1
    assert np.count_nonzero(regs) == M


def test_estimator_closed_form_all_registers_equal():
    """With every register equal to k (1 <= k <= 64-p), the estimate reduces to
    alpha_inf * m * 2^k with alpha_inf = 1/(2 ln 2)."""
    for k in [1, 3, 10, 30]:
        est = oracle.hll_estimate(np.full(M, k, dtype=np.uint8))
        assert math.isclose(est, M * 2.0 ** k / (2 * math.log(2)), rel_tol=1e-12)


def test_estimator_close_to_linear_counting_when_sparse():
    """For n << m almost every non-empty register holds one key and the
    estimate approaches linear counting m ln(m/V)."""
    for n in [50, 500]:
        regs = oracle.hll_registers(synth.distinct_values(4, n, n))
        v = int(np.count_nonzero(regs == 0))
        lc = M * math.log(M / v)
        assert abs(oracle.hll_estimate(regs) / lc - 1) < 0.01


@pytest.mark.parametrize("n", [1000, 10000, 30000, 45000, 60000, 100000, 1000000, 5000000])
def test_estimate_within_three_sigma(n):
    for seed in (1, 2):
        st = oracle.column_stats(synth.distinct_values(seed, n, n + n // 3))
        assert abs(st["ndv"] / n - 1) < 3 * SIGMA, (n, seed, st["ndv"])


@pytest.mark.parametrize("n", [20000, 50000, 200000])
def test_estimate_mean_within_one_sigma(n):
    errs = [oracle.column_stats(synth.distinct_values(seed, n, n))["ndv"] / n - 1
            for seed in range(20)]
    assert abs(np.mean(errs)) < SIGMA
    assert np.std(errs) < 2 * SIGMA


def test_planted_mistake_is_caught():
    """Ranks off by one (no +1) halve the estimate: the 3-sigma bound catches it."""
    regs = oracle.hll_registers(synth.distinct_values(6, 300000, 300000))
    bad = np.where(regs > 0, regs - 1, 0).astype(np.uint8)
    assert abs(oracle.hll_estimate(bad) / 300000 - 1) > 3 * SIGMA
    assert abs(oracle.hll_estimate(regs) / 300000 - 1) < 3 * SIGMA
