"""Group-by on the GPU against the group-by oracle: group keys, counts and
per-column sums, for the hash-based and the partition-based algorithm, int32
and int64 keys and values, group counts from one to beyond an LDS table (the
spill path), the rule's HLL-guided choice, and the edge cases."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth

pytestmark = pytest.mark.gpu


def check(keys, vals, res):
    gk, cnt, sums = oracle.group_by(keys, vals)
    assert res.groups == len(gk)
    k = res.keys.cpu().numpy().astype(np.int64)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(k[order], gk)
    assert np.array_equal(res.counts.cpu().numpy()[order], cnt)
    for got, want in zip(res.sums, sums):
        assert np.array_equal(got.cpu().numpy()[order], want)


def forced(keys, variant, bits=0):
    return eg.groupby_plan(eg.stats(keys), eg.SEL_FORCED, eg.make_groupby_plan(variant, bits))


# part2: 4 partitions of ~250,000 rows, each aggregated in 4 slices merged globally
VARIANTS = [("hash", eg.GB_HASH, 0), ("part2", eg.GB_PARTITION, 2), ("part4", eg.GB_PARTITION, 4),
            ("part8", eg.GB_PARTITION, 8), ("part12p2", eg.GB_PARTITION, 12)]


@pytest.mark.parametrize("variant", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("groups", [1, 7, 1000, 50000, 300000])
def test_groupby_int32(gpu, variant, groups):
    keys, vals = synth.groupby_input(seed=groups, n=1_000_003, groups=groups, device=gpu)
    res = eg.groupby(keys, vals, forced(keys, variant[1], variant[2]))
    check(keys, vals, res)


@pytest.mark.parametrize("variant", VARIANTS[:3], ids=[v[0] for v in VARIANTS[:3]])
def test_groupby_int64_keys_and_values(gpu, variant):
    keys, vals = synth.groupby_input(seed=5, n=700_001, groups=200_000, key_dtype=torch.int64,
                                     val_dtype=torch.int64, device=gpu)
    vals = [vals[0], vals[1].to(torch.int32)]  # one 8-byte and one 4-byte value column
    res = eg.groupby(keys, vals, forced(keys, variant[1], variant[2]))
    check(keys, vals, res)


def test_groupby_rule_follows_the_estimate(gpu):
    small, sv = synth.groupby_input(seed=1, n=2_000_000, groups=600, device=gpu)
    big, bv = synth.groupby_input(seed=2, n=2_000_000, groups=1_500_000, device=gpu)
    ps, pb = eg.groupby_plan(eg.stats(small)), eg.groupby_plan(eg.stats(big))
    assert ps.variant == eg.GB_HASH and pb.variant == eg.GB_PARTITION
    assert abs(ps.predicted_groups - 600) < 600 * 0.05
    check(small, sv, eg.groupby(small, sv, ps))
    check(big, bv, eg.groupby(big, bv, pb))


def test_groupby_spill_and_small_table_retry(gpu):
    keys, vals = synth.groupby_input(seed=3, n=400_000, groups=300_000, device=gpu)
    # two partitions of ~150,000 groups each: far beyond one LDS table, so every
    # partition spills into the global table
    check(keys, vals, eg.groupby(keys, vals, forced(keys, eg.GB_PARTITION, 1)))
    # a table far smaller than the groups: the library refuses, the wrapper retries larger
    p = forced(keys, eg.GB_HASH)
    p.slots = 1024
    check(keys, vals, eg.groupby(keys, vals, p))


def test_groupby_edges(gpu):
    e = torch.zeros(0, dtype=torch.int32, device=gpu)
    for v, b in ((eg.GB_HASH, 0), (eg.GB_PARTITION, 4)):
        r = eg.groupby(e, [e], forced(e, v, b))
        assert r.groups == 0
    same = torch.full((100_000,), -5, dtype=torch.int32, device=gpu)
    vals = [torch.arange(100_000, dtype=torch.int64, device=gpu)]
    for v, b in ((eg.GB_HASH, 0), (eg.GB_PARTITION, 6)):
        check(same, vals, eg.groupby(same, vals, forced(same, v, b)))
        check(same, [], eg.groupby(same, [], forced(same, v, b)))
    # int64 keys including INT64_MIN: the plan marks empty slots with INT64_MAX
    k = torch.tensor([-(2**63), 5, -(2**63), 7, 5], dtype=torch.int64, device=gpu)
    p = forced(k, eg.GB_HASH)
    assert p.sentinel == 2**63 - 1
    check(k, [k], eg.groupby(k, [k], p))
    both = torch.tensor([-(2**63), 2**63 - 1, 0], dtype=torch.int64, device=gpu)
    with pytest.raises(eg.EigerError) as err:
        eg.groupby(both, [], forced(both, eg.GB_HASH))
    assert err.value.code == eg.EIGER_ERR_UNSUPPORTED


# PARTITION over every lane count (0-4 value words: none, int32, two int32,
# int64 + int32, two int64) and one to three partitioning passes (digits of at
# most 8 bits, narrower for wide rows: 7 bits for 12-byte rows, 6 for 24-byte).
LANES = [("none", torch.int32, []), ("i32", torch.int32, [torch.int32]),
         ("2xi32", torch.int32, [torch.int32, torch.int32]), ("i64+i32", torch.int64, [torch.int64, torch.int32]),
         ("2xi64", torch.int64, [torch.int64, torch.int64])]


@pytest.mark.parametrize("lanes", LANES, ids=[x[0] for x in LANES])
@pytest.mark.parametrize("bits", [3, 9, 15, 18])
def test_groupby_partition_lanes_and_passes(gpu, lanes, bits):
    _, key_dtype, val_dtypes = lanes
    keys, vals = synth.groupby_input(seed=bits, n=1_500_007, groups=400_000, key_dtype=key_dtype, n_vals=2,
                                     val_dtype=torch.int64, device=gpu)
    vals = [v.to(d) for v, d in zip(vals, val_dtypes)]
    check(keys, vals, eg.groupby(keys, vals, forced(keys, eg.GB_PARTITION, bits)))


@pytest.mark.parametrize("key_dtype", [torch.int32, torch.int64])
def test_groupby_row_group_and_per_row_loads(gpu, key_dtype):
    # aligned columns are read four rows at a time, views one row in per row;
    # partitions start anywhere, so the four-row groups also mask rows before
    # a partition's start (odd lengths give ragged ends)
    keys, vals = synth.groupby_input(seed=9, n=300_001, groups=5000, key_dtype=key_dtype, n_vals=2,
                                     val_dtype=torch.int64, device=gpu)
    vals = [vals[0], vals[1].to(torch.int32)]
    for view in (0, 1):
        k, v = keys[view:], [x[view:] for x in vals]
        for variant, bits in ((eg.GB_HASH, 0), (eg.GB_PARTITION, 3), (eg.GB_PARTITION, 9)):
            check(k, v, eg.groupby(k, v, forced(k, variant, bits)))
