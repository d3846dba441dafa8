"""Wide joins on the GPU against the wide-join oracle: every materialized
payload column of both sides, the row ids and the row count, for GFUR under
every variant and GFTR under one- and two-pass RADIX plans, with int32 and
int64 keys and columns, duplicates on both sides and empty sides."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from joincheck import forced_plan

pytestmark = pytest.mark.gpu

PLANS = [
    ("direct", eg.DIRECT, 0, 0, 0.0, (eg.MAT_GFUR,)),
    ("hash", eg.GLOBAL_HASH, 0, 0, 0.5, (eg.MAT_GFUR,)),
    ("radix_b6", eg.RADIX, 6, 1, 0.5, (eg.MAT_GFUR, eg.MAT_GFTR)),
    ("radix_b12p2", eg.RADIX, 12, 2, 0.25, (eg.MAT_GFUR, eg.MAT_GFTR)),
    ("cache_b6", eg.RADIX_CACHE, 6, 1, 0.5, (eg.MAT_GFUR,)),
    ("sort_merge", eg.SORT_MERGE, 0, 0, 0.0, (eg.MAT_GFUR,)),
]


def check_wide(inp, bcols, pcols, res):
    pairs, outR, outS = oracle.join_wide(inp.build_keys, bcols, inp.probe_keys, pcols)
    assert res.count == len(pairs)
    b = res.build_rowid.cpu().numpy().view(np.uint32).astype(np.uint64)
    p = res.probe_rowid.cpu().numpy().view(np.uint32).astype(np.uint64)
    packed = (b << np.uint64(32)) | p
    order = np.argsort(packed, kind="stable")
    assert np.array_equal(packed[order], pairs)
    for got, want in zip(res.build_cols, outR):
        assert np.array_equal(got.cpu().numpy()[order], want)
    for got, want in zip(res.probe_cols, outS):
        assert np.array_equal(got.cpu().numpy()[order], want)


def mixed_cols(inp, gen):
    """Three payload columns a side, int32 and int64 mixed."""
    nb, ns = inp.n_build, inp.n_probe
    b = [torch.randint(-2**31, 2**31, (nb,), generator=gen, dtype=torch.int64).to(torch.int32),
         torch.randint(-2**62, 2**62, (nb,), generator=gen, dtype=torch.int64),
         torch.arange(nb, dtype=torch.int32)]
    s = [torch.randint(-2**62, 2**62, (ns,), generator=gen, dtype=torch.int64),
         torch.randint(-2**31, 2**31, (ns,), generator=gen, dtype=torch.int64).to(torch.int32),
         torch.arange(ns, dtype=torch.int64)]
    return b, s


@pytest.mark.parametrize("plan_spec", PLANS, ids=[p[0] for p in PLANS])
@pytest.mark.parametrize("match", [300, 1000])
def test_wide_paper_shape(gpu, plan_spec, match):
    """Unique int32 build keys, three int32 payload columns a side (the paper's
    four-column tables), match ratio 0.3 and 1.0; several tiles and a ragged tail."""
    inp = synth.wide_join(seed=5, n_build=30011, n_probe=400009, match_per_mille=match, device=gpu)
    name, v, bits, passes, lf, mats = plan_spec
    plan = forced_plan(inp, (name, v, bits, passes, lf))
    for mat in mats:
        res = eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], plan, mat)
        assert res.materialized == mat
        check_wide(inp, inp.meta["build_cols"], inp.meta["probe_cols"], res)


@pytest.mark.parametrize("plan_spec", [p for p in PLANS if p[1] != eg.DIRECT], ids=[p[0] for p in PLANS if p[1] != eg.DIRECT])
def test_wide_int64_keys_mixed_columns_duplicates(gpu, plan_spec):
    """int64 keys over a narrow range (duplicates on both sides), mixed
    int32/int64 payload columns, through every strategy the plan allows."""
    inp = synth.random_small(21, 20000, 150000, -3000, 3000, dtype=torch.int64, device=gpu)
    g = torch.Generator().manual_seed(4)
    bcols, pcols = mixed_cols(inp, g)
    bcols, pcols = [c.to(gpu) for c in bcols], [c.to(gpu) for c in pcols]
    name, v, bits, passes, lf, mats = plan_spec
    plan = forced_plan(inp, (name, v, bits, passes, lf))
    for mat in mats:
        res = eg.join_wide(inp.build_keys, bcols, inp.probe_keys, pcols, plan, mat)
        check_wide(inp, bcols, pcols, res)


def test_wide_auto_and_edges(gpu):
    inp = synth.wide_join(seed=6, n_build=5000, n_probe=60000, match_per_mille=900, device=gpu)
    radix = forced_plan(inp, ("r", eg.RADIX, 8, 1, 0.5))
    res = eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], radix)
    assert res.materialized == eg.MAT_GFTR  # estimated match ratio 0.9
    check_wide(inp, inp.meta["build_cols"], inp.meta["probe_cols"], res)
    hashp = forced_plan(inp, ("h", eg.GLOBAL_HASH, 0, 0, 0.5))
    res = eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], hashp)
    assert res.materialized == eg.MAT_GFUR
    with pytest.raises(eg.EigerError) as e:
        eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], hashp,
                     eg.MAT_GFTR)
    assert e.value.code == eg.EIGER_ERR_UNSUPPORTED
    # no payload columns: the narrow pair list
    res = eg.join_wide(inp.build_keys, [], inp.probe_keys, [], radix, eg.MAT_GFTR)
    assert res.materialized == eg.MAT_GFUR
    check_wide(inp, [], [], res)
    # count-only, a too-small capacity, empty sides
    c = eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], radix,
                     eg.MAT_GFTR, count_only=True)
    assert c.count == res.count
    small = eg.join_wide(inp.build_keys, inp.meta["build_cols"], inp.probe_keys, inp.meta["probe_cols"], radix,
                         eg.MAT_GFTR, capacity=10)
    check_wide(inp, inp.meta["build_cols"], inp.meta["probe_cols"], small)
    for nb, ns in ((0, 1000), (1000, 0)):
        e_inp = synth.wide_join(seed=7, n_build=nb, n_probe=ns, device=gpu)
        for mat in (eg.MAT_GFUR, eg.MAT_GFTR):
            r = eg.join_wide(e_inp.build_keys, e_inp.meta["build_cols"], e_inp.probe_keys, e_inp.meta["probe_cols"],
                             forced_plan(e_inp, ("r", eg.RADIX, 4, 1, 0.5)), mat)
            assert r.count == 0
