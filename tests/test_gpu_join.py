"""eiger_join on the GPU against the join oracle, for every variant and a spread
of knobs: canonical pair lists, counts and checksums must be identical."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from joincheck import SPECS, SPEC_IDS, assert_exact, forced_plan

pytestmark = pytest.mark.gpu


def run(inp, spec, **kw):
    plan = forced_plan(inp, spec)
    return eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan, **kw)


@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_plain_dense_small(gpu, spec):
    inp = synth.plain_dense(seed=3, n_build=4096, n_probe=100003, probe_range=5000, device=gpu)
    assert_exact(inp, run(inp, spec))


@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_plain_dense_full(gpu, spec):
    """The 65,536 x 1,048,576 plain join at full size, every variant."""
    inp = synth.plain_dense(seed=42, device=gpu)
    assert_exact(inp, run(inp, spec))


@pytest.mark.parametrize("spec", [s for s in SPECS if s[1] != eg.DIRECT], ids=[s[0] for s in SPECS if s[1] != eg.DIRECT])
def test_sparse_unique64(gpu, spec):
    inp = synth.sparse_unique64(seed=4, n_build=100000, n_probe=1000003, device=gpu)
    assert_exact(inp, run(inp, spec))


def test_direct_refuses_sparse_range(gpu):
    inp = synth.sparse_unique64(seed=4, n_build=1000, n_probe=1000, device=gpu)
    with pytest.raises(eg.EigerError) as e:
        run(inp, SPECS[0])
    assert e.value.code == eg.EIGER_ERR_UNSUPPORTED


@pytest.mark.parametrize("s", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("spec", [s for s in SPECS if s[1] != eg.DIRECT], ids=[s[0] for s in SPECS if s[1] != eg.DIRECT])
def test_skewed_dup32(gpu, spec, s):
    inp = synth.skewed_dup32(seed=5, n_distinct=20000, n_probe=300001, zipf_s=s, device=gpu)
    assert_exact(inp, run(inp, spec))


def test_skewed_dense_direct(gpu):
    """Duplicated build keys in a dense range: DIRECT's CSR runs."""
    inp = synth.random_small(11, 50000, 400000, -20000, 20000, device=gpu)
    assert_exact(inp, run(inp, SPECS[0]))


ADVERSARIAL = {
    "all_equal": lambda d: synth.JoinInput("all_equal", torch.full((1500,), 7, dtype=torch.int32, device=d),
                                           torch.arange(1500, dtype=torch.int32, device=d),
                                           torch.full((3000,), 7, dtype=torch.int32, device=d),
                                           torch.arange(3000, dtype=torch.int32, device=d) - 1500),
    "empty_build": lambda d: synth.random_small(1, 0, 1000, 0, 100, device=d),
    "empty_probe": lambda d: synth.random_small(1, 1000, 0, 0, 100, device=d),
    "one_build_row": lambda d: synth.random_small(2, 1, 5000, 0, 3, device=d),
    "narrow_dups": lambda d: synth.random_small(3, 3000, 20000, -5, 5, device=d),
    "int32_full_range": lambda d: synth.random_small(4, 20000, 50000, -(1 << 31), (1 << 31) - 1, device=d),
    "int64_full_range": lambda d: synth.random_small(5, 20000, 50000, -(1 << 63), (1 << 63) - 1,
                                                     dtype=torch.int64, payload_dtype=torch.int64, device=d),
    "mixed_payloads": lambda d: synth.random_small(6, 7000, 30000, 0, 9000, dtype=torch.int32,
                                                   payload_dtype=torch.int64, device=d),
}


def with_extremes(inp, dtype):
    info = torch.iinfo(dtype)
    ext = torch.tensor([info.min, info.max, info.min, 0, -1], dtype=dtype, device=inp.build_keys.device)
    return synth.JoinInput(inp.name + "+ext", torch.cat([inp.build_keys, ext]),
                           torch.cat([inp.build_payload, inp.build_payload[:5]]),
                           torch.cat([ext, inp.probe_keys, ext]),
                           torch.cat([inp.probe_payload[:5], inp.probe_payload, inp.probe_payload[:5]]))


@pytest.mark.parametrize("case", list(ADVERSARIAL))
@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_adversarial(gpu, case, spec):
    inp = ADVERSARIAL[case](gpu)
    if case.endswith("full_range"):
        inp = with_extremes(inp, inp.build_keys.dtype)
    if spec[1] == eg.DIRECT:
        st = eg.stats(inp.build_keys)
        if st.n and st.max - st.min + 1 > (1 << 30):
            pytest.skip("DIRECT needs a dense key range")
    assert_exact(inp, run(inp, spec))


@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_payload_dtype_mix(gpu, spec):
    inp = synth.random_small(8, 5000, 40000, 0, 7000, dtype=torch.int64, payload_dtype=torch.int32, device=gpu)
    inp.probe_payload = synth.rand64(8, 99, torch.arange(inp.n_probe, device=gpu))
    assert_exact(inp, run(inp, spec))


def test_misaligned_probe_view(gpu):
    inp = synth.random_small(9, 5000, 40001, 0, 6000, device=gpu)
    inp.probe_keys = inp.probe_keys[1:]
    inp.probe_payload = inp.probe_payload[1:]
    for spec in SPECS:
        assert_exact(inp, run(inp, spec))


@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_capacity_and_count_only(gpu, spec):
    inp = synth.random_small(10, 3000, 30000, 0, 2000, device=gpu)
    _, cnt, cs = oracle.join_sortmerge(inp.build_keys, inp.build_payload, inp.probe_keys,
                                       inp.probe_payload, with_pairs=False)
    plan = forced_plan(inp, spec)
    r = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan, count_only=True)
    assert (r.count, r.checksum) == (cnt, cs)
    small = (torch.empty(cnt // 2, dtype=torch.int32, device=gpu), torch.empty(cnt // 2, dtype=torch.int32, device=gpu))
    with pytest.raises(eg.EigerError) as e:
        eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan, outputs=small)
    assert e.value.code == eg.EIGER_ERR_CAPACITY and e.value.count == cnt
    # the binding's retry path: a too-small capacity grows to the exact count
    r = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan, capacity=10)
    assert_exact(inp, r)


def test_rule_plan_end_to_end(gpu):
    for inp in (synth.plain_dense(seed=1, device=gpu),
                synth.sparse_unique64(seed=2, n_build=300000, n_probe=2000000, device=gpu),
                synth.skewed_dup32(seed=3, n_distinct=30000, n_probe=400000, zipf_s=1.0, device=gpu)):
        plan = eg.join_plan(eg.stats(inp.build_keys), eg.stats(inp.probe_keys))
        assert_exact(inp, eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan))


def test_repeatable(gpu):
    inp = synth.skewed_dup32(seed=6, n_distinct=20000, n_probe=200000, zipf_s=1.5, device=gpu)
    for spec in SPECS[1:]:
        a, b = run(inp, spec), run(inp, spec)
        assert (a.count, a.checksum) == (b.count, b.checksum)
        from joincheck import gpu_canonical
        assert np.array_equal(gpu_canonical(a), gpu_canonical(b))
