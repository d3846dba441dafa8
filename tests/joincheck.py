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
    # load factor 0.9: the LDS table's largest row capacity (grouped tables for
    # 32-bit keys fill their LDS almost exactly) and, at 4 bits, partitions
    # larger than one table, so several chunks per partition
    ("radix_b4_lf90", eg.RADIX, 4, 1, 0.9),
    ("cache_b1", eg.RADIX_CACHE, 1, 1, 0.5),
    ("cache_b6", eg.RADIX_CACHE, 6, 1, 0.75),
    ("cache_b10", eg.RADIX_CACHE, 10, 1, 0.5),
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


def assert_full_size(inp, res, threads=16, sample=20000, seed=0):
    """Checks for results too large for the sort-merge oracle, all on the same
    seeded inputs:
      * count and checksum equal the oracle's per-key-aggregate totals;
      * every output pair joins equal keys (checked on the GPU with torch);
      * no pair appears twice.
    A set of valid, distinct pairs as large as the true result is the result.
    Sampled probe rows are also compared one by one with the oracle."""
    cnt, cs = oracle.join_totals(inp.build_keys, inp.build_payload, inp.probe_keys,
                                 inp.probe_payload, threads=threads)
    assert res.count == cnt, (res.count, cnt)
    assert res.checksum == cs, (res.checksum, cs)
    b = res.build_rowid.to(torch.int64) & 0xFFFFFFFF
    p = res.probe_rowid.to(torch.int64) & 0xFFFFFFFF
    assert int(b.max()) < inp.n_build and int(p.max()) < inp.n_probe
    step = 1 << 26
    for lo in range(0, res.count, step):
        hi = min(res.count, lo + step)
        assert torch.equal(inp.build_keys[b[lo:hi]], inp.probe_keys[p[lo:hi]])
    packed = torch.sort((b << 32) | p).values
    assert not bool((packed[1:] == packed[:-1]).any())
    del b, packed
    # sampled probe rows, one at a time against the oracle
    g = torch.Generator().manual_seed(seed)
    rows = torch.randint(0, inp.n_probe, (sample,), generator=g)
    offs, ids = oracle.probe_matches(inp.build_keys, inp.probe_keys, rows.numpy())
    order = torch.argsort(p)
    ps = p[order]
    bs = (res.build_rowid.to(torch.int64) & 0xFFFFFFFF)[order]
    rows_d = rows.to(p.device)
    lo = torch.searchsorted(ps, rows_d, right=False).cpu().numpy()
    hi = torch.searchsorted(ps, rows_d, right=True).cpu().numpy()
    bs_h = None
    for t in range(sample):
        want = ids[offs[t]:offs[t + 1]]
        n = hi[t] - lo[t]
        assert n == len(want), (int(rows[t]), n, len(want))
        if n:
            got = np.sort(bs[lo[t]:hi[t]].cpu().numpy())
            assert np.array_equal(got, want)
    del bs_h
