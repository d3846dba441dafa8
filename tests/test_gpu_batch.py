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
