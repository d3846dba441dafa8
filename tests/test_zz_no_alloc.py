"""eiger_join_noalloc (the join with the library's fixed scratch array as its
workspace) against eiger_join (caller workspace) through the C ABI: identical
count, checksum and canonical pair list, for two calls in a row on one GPU, the
second with a smaller input (the array keeps the first call's contents), for
each variant; the first call's result is also checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from joincheck import assert_exact, forced_plan, gpu_canonical

pytestmark = pytest.mark.gpu

SPECS = [
    ("direct", eg.DIRECT, 0, 0, 0.0),
    ("hash_lf50", eg.GLOBAL_HASH, 0, 0, 0.5),
    ("radix_b10p2", eg.RADIX, 10, 2, 0.5),
    ("cache_b6", eg.RADIX_CACHE, 6, 1, 0.75),
]


def both(inp, spec):
    plan = forced_plan(inp, spec)
    args = (inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan)
    need = eg.join_workspace_size(plan, *args[:4])
    assert need <= eg.NOALLOC_SCRATCH_BYTES, (spec[0], need)
    ref = eg.join(*args)
    cap = max(ref.count, 1)
    ob = torch.full((cap,), -1, dtype=torch.int32, device=inp.probe_keys.device)
    op = torch.full((cap,), -1, dtype=torch.int32, device=inp.probe_keys.device)
    got = eg.join_noalloc(*args, outputs=(ob, op))
    cnt_only = eg.join_noalloc(*args)
    return ref, got, cnt_only


def assert_same(ref, got, cnt_only):
    assert (got.count, got.checksum) == (ref.count, ref.checksum)
    assert (cnt_only.count, cnt_only.checksum) == (ref.count, ref.checksum)
    assert np.array_equal(gpu_canonical(got), gpu_canonical(ref))


@pytest.mark.parametrize("spec", SPECS, ids=[s[0] for s in SPECS])
def test_noalloc_matches_join_twice(gpu, spec):
    print(f"[noalloc] {spec[0]} call 1: plain join 65,536 x 1,048,576", flush=True)
    big = synth.plain_dense(seed=42, device=gpu)
    ref, got, c = both(big, spec)
    assert_same(ref, got, c)
    assert_exact(big, got)
    print(f"[noalloc] {spec[0]} call 2: plain join 3,000 x 50,001", flush=True)
    small = synth.plain_dense(seed=9, n_build=3000, n_probe=50001, probe_range=4000, device=gpu)
    ref, got, c = both(small, spec)
    assert_same(ref, got, c)


def test_noalloc_duplicates_twice(gpu):
    """Duplicated build keys (multi-match emission) through the hash and radix
    plans, larger then smaller."""
    for n_r, n_s in ((60000, 500000), (7000, 40001)):
        inp = synth.random_small(13, n_r, n_s, -3000, 3000, device=gpu)
        for spec in SPECS[1:3]:
            print(f"[noalloc] duplicates {spec[0]} {n_r} x {n_s}", flush=True)
            ref, got, c = both(inp, spec)
            assert_same(ref, got, c)


def test_noalloc_capacity_error(gpu):
    inp = synth.plain_dense(seed=5, n_build=2000, n_probe=30000, probe_range=2500, device=gpu)
    plan = forced_plan(inp, SPECS[1])
    args = (inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan)
    ref = eg.join(*args)
    assert ref.count > 10
    ob = torch.empty(10, dtype=torch.int32, device=gpu)
    op = torch.empty(10, dtype=torch.int32, device=gpu)
    with pytest.raises(eg.EigerError) as e:
        eg.join_noalloc(*args, outputs=(ob, op))
    assert e.value.code == eg.EIGER_ERR_CAPACITY and e.value.count == ref.count
