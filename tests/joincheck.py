"""Helpers shared by the GPU parity tests: run the library through its C ABI
and compare with the oracle."""
import numpy as np
import torch

import oracle
import paper_2607_04489_amd as eg

# (name, variant, radix_bits, radix_passes, load_factor)
SPECS = [
    ("direct", eg.DIRECT, 0, 0, 0.0),
    ("hash_lf50", eg.GLOBAL_HASH, 0, 0, 0.5),
    ("hash_lf85", eg.GLOBAL_HASH, 0, 0, 0.85),
    ("radix_b1", eg.RADIX, 1, 1, 0.5),
    ("radix_b6", eg.RADIX, 6, 1, 0.5),
    ("radix_b9", eg.RADIX, 9, 1, 0.75),
    ("radix_b10p2", eg.RADIX, 10, 2, 0.5),
    ("radix_b15p2", eg.RADIX, 15, 2, 0.6),
    # the plan the rule picks for large duplicated int32 builds: two 8-bit
    # passes (256-bucket write-combining scatter in pass 2) into 65,536
    # grouped LDS tables at load factor 0.25
    ("radix_b16p2_lf25", eg.RADIX, 16, 2, 0.25),
    # load factor 0.9: the LDS table's largest row capacity (grouped tables for
    # 32-bit keys fill their LDS almost exactly) and, at 4 bits, partitions
    # larger than one table, so several chunks per partition
    ("radix_b4_lf90", eg.RADIX, 4, 1, 0.9),
    ("cache_b1", eg.RADIX_CACHE, 1, 1, 0.5),
    ("cache_b6", eg.RADIX_CACHE, 6, 1, 0.75),
    ("cache_b10", eg.RADIX_CACHE, 10, 1, 0.5),
    ("sort_merge", eg.SORT_MERGE, 0, 0, 0.0),
]
SPEC_IDS = [s[0] for s in SPECS]


def forced_plan(inp, spec):
    _, variant, bits, passes, lf = spec
    sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
    return eg.join_plan(sb, sp, eg.SEL_FORCED, eg.make_plan(variant, bits, passes, lf))


def gpu_canonical(res) -> np.ndarray:
    b = res.build_rowid.cpu().numpy().view(np.uint32)
    p = res.probe_rowid.cpu().numpy().view(np.uint32)
    return oracle.canonical_pairs(b, p)


def assert_exact(inp, res):
    """Canonical pair list, count and checksum equal to the sort-merge oracle."""
    pairs, cnt, cs = oracle.join_sortmerge(inp.build_keys, inp.build_payload,
                                           inp.probe_keys, inp.probe_payload)
    assert res.count == cnt, (res.count, cnt)
    assert res.checksum == cs, (res.checksum, cs)
    got = gpu_canonical(res)
    assert got.shape == pairs.shape
    assert np.array_equal(got, pairs)


def host_threads() -> int:
    """Threads for the oracle's sorts and totals: this process's CPUs, at most 16."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


class FullSizeRef:
    """Oracle facts of one instance too large for a full sort-merge pair list,
    computed once and reused for every plan run on it:
      * count and checksum from the oracle's per-key aggregates (join_totals);
      * for `sample` seeded probe rows, their matching build rows one by one
        (probe_matches)."""

    def __init__(self, inp, sample=20000, seed=0, threads=None):
        threads = threads or host_threads()
        self.count, self.checksum = oracle.join_totals(inp.build_keys, inp.build_payload, inp.probe_keys,
                                                       inp.probe_payload, threads=threads)
        g = torch.Generator().manual_seed(seed)
        self.rows = torch.randint(0, inp.n_probe, (sample,), generator=g)
        self.offs, self.ids = oracle.probe_matches(inp.build_keys, inp.probe_keys, self.rows.numpy(),
                                                   threads=threads)


def assert_full_size(inp, res, ref: FullSizeRef):
    """Checks of a full-size result against the oracle, all on the same seeded
    inputs:
      * count and checksum equal the oracle's per-key-aggregate totals;
      * every output pair joins equal keys (checked on the GPU with torch);
      * no pair appears twice.
    A set of valid, distinct pairs as large as the true result is the result.
    Sampled probe rows are also compared one by one with the oracle's matches."""
    assert res.count == ref.count, (res.count, ref.count)
    assert res.checksum == ref.checksum, (res.checksum, ref.checksum)
    if ref.count == 0:
        return
    b = res.build_rowid.to(torch.int64) & 0xFFFFFFFF
    p = res.probe_rowid.to(torch.int64) & 0xFFFFFFFF
    assert int(b.max()) < inp.n_build and int(p.max()) < inp.n_probe
    step = 1 << 26
    for lo in range(0, res.count, step):
        hi = min(res.count, lo + step)
        assert torch.equal(inp.build_keys[b[lo:hi]], inp.probe_keys[p[lo:hi]])
    packed = torch.sort((b << 32) | p).values
    assert not bool((packed[1:] == packed[:-1]).any())
    del packed
    # sampled probe rows: (sample index, build row) of every output pair of a
    # sampled row, sorted, against the same list from the oracle
    order = torch.argsort(p)
    ps, bs = p[order], b[order]
    del order, b, p
    rows_d = ref.rows.to(ps.device)
    lo = torch.searchsorted(ps, rows_d, right=False)
    hi = torch.searchsorted(ps, rows_d, right=True)
    n = (hi - lo).cpu().numpy()
    want_n = np.diff(ref.offs)
    bad = np.nonzero(n != want_n)[0]
    assert bad.size == 0, [(int(ref.rows[t]), int(n[t]), int(want_n[t])) for t in bad[:5]]
    if int(n.sum()) == 0:
        return
    t_idx = torch.repeat_interleave(torch.arange(len(n), device=ps.device), hi - lo)
    starts = torch.repeat_interleave(lo, hi - lo)
    within = torch.arange(t_idx.numel(), device=ps.device) - torch.repeat_interleave(
        torch.cumsum(hi - lo, 0) - (hi - lo), hi - lo)
    got = torch.sort((t_idx << 32) | bs[starts + within]).values.cpu().numpy().astype(np.uint64)
    want = (np.repeat(np.arange(len(n), dtype=np.uint64), want_n.astype(np.int64)) << np.uint64(32)) | \
        ref.ids.astype(np.uint64)
    assert np.array_equal(got, np.sort(want))
