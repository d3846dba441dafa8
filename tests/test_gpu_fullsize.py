"""Oracle parity of the benchmarked workloads at their full sizes.

The large sparse join (16,777,216 unique int64 build keys x 536,870,912 probe
rows, ~4.8e8 pairs) and the skewed many-to-many join (16,777,216 distinct int32
keys with geometric duplicates, ~6.7e7 build rows x 268,435,456 Zipf probe rows,
~1.1e9 pairs, s = 0.5 / 1.0 / 1.5) are run through eiger_join with the plans the
benchmark uses (learned selector with its rule fallback, the rule) and the other
variants that can run them, and each result is checked against the oracle with
joincheck.assert_full_size: count and checksum from the oracle's per-key
aggregates, key equality of every pair, no duplicate pair, and 20,000 sampled
probe rows matched one by one (Section 5.2 defines R, S and the match ratio;
Section 3.2 the hash and partitioned hash joins).
"""
import os

import pytest
import torch

import paper_2607_04489_amd as eg
import synth
from joincheck import FullSizeRef, assert_full_size

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

MODEL = os.path.join(os.path.dirname(eg.__file__), "selector_model.json")


def _plans(inp, extra):
    """(name, plan) pairs: learned (when a model file exists), rule, then `extra`
    forced (variant, bits, passes, lf) specs."""
    from paper_2607_04489_amd import selector as selmod
    sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
    out = []
    if os.path.exists(MODEL):
        selmod.load_model()
        out.append(("learned", eg.join_plan(sb, sp, eg.SEL_LEARNED)))
    out.append(("rule", eg.join_plan(sb, sp, eg.SEL_RULE)))
    for name, v, bits, passes, lf in extra:
        out.append((name, eg.join_plan(sb, sp, eg.SEL_FORCED, eg.make_plan(v, bits, passes, lf))))
    seen, uniq = set(), []
    for name, pl in out:
        key = (pl.variant, pl.radix_bits, pl.radix_passes, round(float(pl.load_factor), 3))
        if key not in seen:
            seen.add(key)
            uniq.append((name, pl))
    return uniq


def _run_all(inp, plans):
    ref = FullSizeRef(inp)
    for name, pl in plans:
        print(f"[fullsize] {inp.name} plan {name} {pl.describe()}", flush=True)
        res = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, pl)
        assert_full_size(inp, res, ref)
        del res
        torch.cuda.empty_cache()


def test_sparse_unique64_full(gpu):
    inp = synth.sparse_unique64(seed=42, device=gpu)
    inp.meta.pop("source_row", None)
    plans = _plans(inp, [("hash_lf25", eg.GLOBAL_HASH, 0, 0, 0.25),
                         ("hash_lf50", eg.GLOBAL_HASH, 0, 0, 0.5),
                         ("cache_b10", eg.RADIX_CACHE, 10, 1, 0.5)])
    _run_all(inp, plans)


@pytest.mark.parametrize("s", [0.5, 1.0, 1.5])
def test_skewed_dup32_full(gpu, s):
    inp = synth.skewed_dup32(seed=42, zipf_s=s, device=gpu)
    plans = _plans(inp, [("radix_b16p2_lf25", eg.RADIX, 16, 2, 0.25)])
    _run_all(inp, plans)
