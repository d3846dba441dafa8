"""Batched joins in one graph launch against the oracle and the single-join
path: per-join canonical pairs, counts and checksums; replays of the graph
with other GPU work in between; flags for duplicated build keys."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth

pytestmark = pytest.mark.gpu


def as_tuple(inp):
    return (inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)


def check_batch(b, inputs, flags_expected=None):
    counts, sums, variants, flags = b.results()
    for j, inp in enumerate(inputs):
        if flags_expected is not None and j in flags_expected:
            assert flags[j] & eg.BATCH_DUPLICATE_BUILD, j
            continue
        assert flags[j] == 0, j
        pairs, cnt, cs = oracle.join_sortmerge(*as_tuple(inp))
        assert (counts[j], sums[j]) == (cnt, cs), j
        ob, op = b.pairs(j, cnt)
        got = oracle.canonical_pairs(ob.cpu().numpy().view(np.uint32), op.cpu().numpy().view(np.uint32))
        assert np.array_equal(got, pairs), j
    return counts, sums, variants, flags


def small_batch(gpu, n=120, seed=3):
    inputs = synth.batched_joins(seed, n, log2_lo=2.0, log2_hi=12.0, device=gpu)
    # edge cases: an empty build, an empty probe, a one-row build
    inputs[5] = synth.JoinInput("empty_build", inputs[5].build_keys[:0], inputs[5].build_payload[:0],
                                inputs[5].probe_keys, inputs[5].probe_payload)
    inputs[6] = synth.JoinInput("empty_probe", inputs[6].build_keys, inputs[6].build_payload,
                                inputs[6].probe_keys[:0], inputs[6].probe_payload[:0])
    inputs[7] = synth.JoinInput("one_row", inputs[7].build_keys[:1], inputs[7].build_payload[:1],
                                inputs[7].probe_keys, inputs[7].probe_payload)
    return inputs


def test_batch_matches_oracle(gpu):
    inputs = small_batch(gpu)
    b = eg.Batch([as_tuple(i) for i in inputs])
    b.launch()
    _, _, variants, _ = check_batch(b, inputs)
    assert set(variants.tolist()) == {eg.DIRECT, eg.GLOBAL_HASH}  # dense and sparse joins both seen


def test_batch_replays_with_other_work_between(gpu):
    inputs = small_batch(gpu, n=60, seed=4)
    b = eg.Batch([as_tuple(i) for i in inputs], tune={b: (0.25, 4096) for b in range(33)})
    first = None
    for r in range(3):
        b.launch()
        res = b.results()
        x = torch.randn(1 << 20, device=gpu)
        torch.cuda.synchronize()
        assert float(x.abs().sum()) > 0  # eager work between replays
        if first is None:
            first = res
            check_batch(b, inputs)
        else:
            for a, c in zip(first, res):
                assert np.array_equal(a, c)


def test_batch_flags_duplicated_builds(gpu):
    inputs = small_batch(gpu, n=20, seed=5)
    for j in (2, 3):  # one dense, one sparse join with a repeated build key
        bk = inputs[j].build_keys.clone()
        bk[-1] = bk[0]
        inputs[j] = synth.JoinInput("dup", bk, inputs[j].build_payload, inputs[j].probe_keys,
                                    inputs[j].probe_payload)
    b = eg.Batch([as_tuple(i) for i in inputs])
    b.launch()
    check_batch(b, inputs, flags_expected={2, 3})


def test_batch_agrees_with_single_joins(gpu):
    inputs = synth.batched_joins(6, 40, log2_lo=8.0, log2_hi=15.0, device=gpu)
    b = eg.Batch([as_tuple(i) for i in inputs])
    b.launch()
    counts, sums, _, flags = b.results()
    for j, inp in enumerate(inputs):
        sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
        r = eg.join(*as_tuple(inp), eg.join_plan(sb, sp), count_only=True)
        assert (r.count, r.checksum) == (counts[j], sums[j])
    assert not flags.any()


def test_batch_rejects_bad_descriptors(gpu):
    inp = synth.batched_joins(7, 2, device=gpu)
    with pytest.raises(eg.EigerError):
        eg.Batch([(inp[0].build_keys, inp[0].build_payload, inp[0].probe_keys.to(torch.int64),
                   inp[0].probe_payload)])


def test_batch_flagged_joins_resolve_through_eiger_join(gpu):
    """Joins with repeated build keys are flagged by the graph and joined again
    through eiger_join; their results equal the oracle's."""
    inputs = small_batch(gpu, n=12, seed=8)
    for j in (1, 4):
        bk = inputs[j].build_keys.clone()
        bk[1::3] = bk[0]  # many copies of one key
        inputs[j] = synth.JoinInput("dups", bk, inputs[j].build_payload, inputs[j].probe_keys,
                                    inputs[j].probe_payload)
    b = eg.Batch([as_tuple(i) for i in inputs])
    b.launch()
    _, _, _, flags = check_batch(b, inputs, flags_expected={1, 4})
    fixed = b.resolve_flagged(flags)
    assert sorted(fixed) == [1, 4]
    for j, res in fixed.items():
        pairs, cnt, cs = oracle.join_sortmerge(*as_tuple(inputs[j]))
        assert (res.count, res.checksum) == (cnt, cs)
        got = oracle.canonical_pairs(res.build_rowid.cpu().numpy().view(np.uint32),
                                     res.probe_rowid.cpu().numpy().view(np.uint32))
        assert np.array_equal(got, pairs)


def test_batch_spec_shape_in_waves(gpu):
    """Joins of the batched workload's full size range (build rows 2^U(8,22),
    probe rows 4-16x) run in two graph waves; 64 joins -- the 8 largest and 56
    more drawn with a seed -- are compared pair for pair with the oracle, and
    every join's count and checksum with the single-join path."""
    from joincheck import host_threads
    n, seed = 192, 11
    sizes = [synth.batched_join_params(seed, j, 8.0, 22.0)[:2] for j in range(n)]
    assert max(nb for nb, _ in sizes) > (1 << 21)
    largest = sorted(range(n), key=lambda j: -sizes[j][1])[:8]
    rng = np.random.default_rng(seed)
    rest = [j for j in range(n) if j not in largest]
    sample = set(largest) | set(int(j) for j in rng.choice(rest, 56, replace=False))
    checked = 0
    for wave in (range(0, n // 2), range(n // 2, n)):
        inputs = {j: synth.batched_join(seed, j, 8.0, 22.0, device=gpu) for j in wave}
        order = list(wave)
        b = eg.Batch([as_tuple(inputs[j]) for j in order])
        b.launch()
        counts, sums, _, flags = b.results()
        assert not flags.any()
        for t, j in enumerate(order):
            inp = inputs[j]
            if j in sample:
                print(f"[batch-spec] join {j}: {inp.n_build} x {inp.n_probe}", flush=True)
                pairs, cnt, cs = oracle.join_sortmerge(*as_tuple(inp), threads=host_threads())
                assert (counts[t], sums[t]) == (cnt, cs), j
                ob, op = b.pairs(t, cnt)
                got = oracle.canonical_pairs(ob.cpu().numpy().view(np.uint32), op.cpu().numpy().view(np.uint32))
                assert np.array_equal(got, pairs), j
                checked += 1
            else:
                r = eg.join(*as_tuple(inp), eg.join_plan(eg.stats(inp.build_keys), eg.stats(inp.probe_keys)),
                            count_only=True)
                assert (r.count, r.checksum) == (counts[t], sums[t]), j
        b.destroy()
        del inputs
        torch.cuda.empty_cache()
    assert checked == 64


def test_batch_partitioned_buckets_match_oracle(gpu):
    """Size buckets tuned to the partitioned join run RADIX inside the graph
    (next to hash and direct joins of other buckets): pairs, counts and
    checksums equal the oracle's, duplicated build keys included (RADIX joins
    them natively, no flag), and a join with more pairs than probe rows is
    flagged for capacity and resolved through eiger_join."""
    inputs = synth.batched_joins(12, 48, log2_lo=6.0, log2_hi=16.0, device=gpu)
    dup = 3 if inputs[3].n_build >= 1024 else max(range(48), key=lambda j: inputs[j].n_build)
    bk = inputs[dup].build_keys.clone()
    bk[1::7] = bk[0]
    inputs[dup] = synth.JoinInput("dups", bk, inputs[dup].build_payload, inputs[dup].probe_keys,
                                  inputs[dup].probe_payload)
    # all probe rows of one join carry the repeated key: more pairs than probe rows
    over = max((j for j in range(48) if j != dup), key=lambda j: inputs[j].n_build)
    obk = inputs[over].build_keys.clone()
    obk[:4] = obk[0]
    opk = torch.full_like(inputs[over].probe_keys, int(obk[0]))
    inputs[over] = synth.JoinInput("over", obk, inputs[over].build_payload, opk, inputs[over].probe_payload)
    tune = {b: (0.25, 4096, max(1, b - 10)) for b in range(10, 33)}
    b = eg.Batch([as_tuple(i) for i in inputs], tune)
    b.launch()
    counts, sums, variants, flags = b.results()
    radix = [j for j, i in enumerate(inputs) if i.n_build >= 1024 and i.n_probe > 0]
    assert len(radix) >= 8 and all(variants[j] == eg.RADIX for j in radix)
    assert dup in radix and over in radix
    for j, inp in enumerate(inputs):
        pairs, cnt, cs = oracle.join_sortmerge(*as_tuple(inp))
        assert (counts[j], sums[j]) == (cnt, cs), j
        if j == over:
            assert flags[j] == eg.BATCH_CAPACITY
            continue
        assert flags[j] == 0, j
        ob, op = b.pairs(j, cnt)
        got = oracle.canonical_pairs(ob.cpu().numpy().view(np.uint32), op.cpu().numpy().view(np.uint32))
        assert np.array_equal(got, pairs), j
    fixed = b.resolve_flagged(flags)
    assert sorted(fixed) == [over]
    pairs, cnt, cs = oracle.join_sortmerge(*as_tuple(inputs[over]))
    got = oracle.canonical_pairs(fixed[over].build_rowid.cpu().numpy().view(np.uint32),
                                 fixed[over].probe_rowid.cpu().numpy().view(np.uint32))
    assert np.array_equal(got, pairs)
    # replays give the same results
    b.launch()
    again = b.results()
    assert all(np.array_equal(a, c) for a, c in zip((counts, sums, variants, flags), again))
