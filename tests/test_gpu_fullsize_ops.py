"""Parity of the group-by and the multi-key sort at their benchmark sizes (2^28 rows).

Group-by (Section 5.3 shape: two sums; 2^10 groups -> HASH, 2^20 groups ->
PARTITION by the rule, and the other variant forced): the group count, the
total count and the per-column total sums (mod 2^64) equal the column's; every
group key is a key of the column and occurs once; and a seeded sample of 256
groups has exactly the oracle's count and sums (oracle.group_by over the rows of
the sampled keys).

Multi-key sort (Section 5.6 shape: 4 int32 keys, half narrow, half of 256
values): the stable sorting permutation is unique, and three properties at full
size pin it: it is a permutation, consecutive rows are in lexicographic key
order, and equal key tuples keep ascending row ids. At 4,096 seeded positions
the sorted fused key equals the oracle's fused key of the row placed there
(oracle plan from oracle statistics; dictionary codes = ranks among the
column's distinct values).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from oracle import skf

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N = 1 << 28


@pytest.mark.parametrize("groups_log2", [10, 20])
@pytest.mark.parametrize("variant", ["rule", "other"])
def test_groupby_full_size(gpu, groups_log2, variant):
    keys, vals = synth.groupby_input(42, N, 1 << groups_log2, torch.int32, 2, torch.int32, device=gpu)
    st = eg.stats(keys)
    plan = eg.groupby_plan(st)
    if variant == "other":
        other = eg.GB_PARTITION if plan.variant == eg.GB_HASH else eg.GB_HASH
        plan = eg.groupby_plan(st, eg.SEL_FORCED, eg.make_groupby_plan(other))
    print(f"[groupby-full] 2^{groups_log2} groups, {eg.GB_NAMES[plan.variant]}", flush=True)
    r = eg.groupby(keys, vals, plan)
    distinct = torch.unique(keys)
    assert r.groups == distinct.numel()
    assert int(r.counts.sum()) == N
    for c in range(2):  # total of each sum column = column total, mod 2^64 (torch int64 wraps)
        assert int(r.sums[c].sum()) == int(vals[c].to(torch.int64).sum())
    gk = torch.sort(r.keys.to(torch.int64)).values
    assert torch.equal(gk, distinct.to(torch.int64))  # every key once, nothing else
    rng = np.random.default_rng(groups_log2)
    sample = np.sort(rng.choice(distinct.cpu().numpy(), 256, replace=False)).astype(np.int64)
    s_t = torch.from_numpy(sample).to(gpu)
    rows = torch.isin(keys.to(torch.int64), s_t)
    ok, oc, osums = oracle.group_by(keys[rows], [v[rows] for v in vals])
    assert np.array_equal(ok, sample)
    pos = torch.searchsorted(gk, s_t)
    order = torch.argsort(r.keys.to(torch.int64))
    idx = order[pos]
    assert np.array_equal(r.counts[idx].cpu().numpy(), oc)
    for c in range(2):
        assert np.array_equal(r.sums[c][idx].cpu().numpy(), osums[c])


def test_multikey_sort_full_size(gpu):
    cols = synth.multikey_table(42, N, 4, torch.int32, narrow_bits=8, sparse_ndv=256, device=gpu)
    perm, srt, fin = eg.sort_multikey(cols, with_sorted=True)
    print(f"[sort-full] fused {fin.total_bits} bits", flush=True)
    p = perm.to(torch.int64)
    assert torch.bincount(p, minlength=N).eq(1).all()
    s = [c[p] for c in cols]
    # lexicographic order of consecutive rows; ties keep ascending row ids
    state = torch.zeros(N - 1, dtype=torch.int8, device=gpu)  # 1 greater, -1 smaller, 0 equal so far
    for c in s:
        und = state == 0
        state = torch.where(und & (c[1:] > c[:-1]), torch.ones_like(state), state)
        state = torch.where(und & (c[1:] < c[:-1]), -torch.ones_like(state), state)
    assert bool((state >= 0).all())
    ties = state == 0
    assert bool((p[1:][ties] > p[:-1][ties]).all())
    del s, state, ties
    # the sorted fused keys are the oracle's fuse of the rows in that order, on a sample
    hc = [c.cpu().numpy() for c in cols]
    st = [oracle.column_stats(c) for c in hc]
    uniq = [np.unique(c) for c in hc]
    op = skf.skf_plan(st, [False] * 4, [u.size for u in uniq])
    assert op.total_bits == fin.total_bits
    rng = np.random.default_rng(5)
    at = np.sort(rng.choice(N, 4096, replace=False))
    rows = p[torch.from_numpy(at).to(gpu)].cpu().numpy()
    # a dictionary code is the value's rank among the column's distinct values
    codes = [np.searchsorted(u, c[rows]) if k.kind == skf.DICT else None for c, u, k in zip(hc, uniq, op.keys)]
    want = skf.fuse([c[rows] for c in hc], op, codes)
    got = srt.cpu().numpy().view(np.uint32)[at]
    assert np.array_equal(got, want)
