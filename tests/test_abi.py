"""The C-ABI library: it loads without a GPU, exports every symbol the header
declares, and its host-only logic (planning, argument checks that precede any
HIP call) behaves as documented in include/eiger.h."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

import paper_2607_04489_amd as eg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "eiger.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eiger_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not eg.available():
        import __graft_entry__
        __graft_entry__.build()
    return eg.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_version(lib):
    assert eg.version() >= 100


def stats(n, lo, hi, ndv, dtype=eg.INT32):
    s = eg.StatsT()
    s.n, s.min, s.max, s.ndv, s.dtype, s.hll_p = n, lo, hi, ndv, dtype, 14
    return eg.Stats(s, None)


def plan(b, p, sel=eg.SEL_RULE, forced=None):
    return eg.join_plan(b, p, sel, forced)


def test_rule_plan_dense_range(lib):
    # distinct keys in a dense range: the hash table (one line per probe) beats CSR runs
    p = plan(stats(65536, 0, 65535, 65536.0), stats(1 << 20, 0, 81919, 81920.0))
    assert p.variant == eg.GLOBAL_HASH
    assert (p.build_min, p.build_max) == (0, 65535)
    assert p.predicted_out == (65536 * (1 << 20)) // 81920
    # duplicated keys in a dense range: DIRECT's CSR runs
    p = plan(stats(65536, 0, 16383, 16384.0), stats(1 << 20, 0, 16383, 16384.0))
    assert p.variant == eg.DIRECT


def test_rule_plan_int32_table_budget(lib):
    # 2^24 distinct int32 keys: a 1 GiB table is probed in place; 2^25 (2 GiB): partitioned
    p = plan(stats(1 << 24, 0, 1 << 30, float(1 << 24)), stats(1 << 28, 0, 1 << 30, float(1 << 24)))
    assert p.variant == eg.GLOBAL_HASH
    p = plan(stats(1 << 25, 0, 1 << 30, float(1 << 25)), stats(1 << 28, 0, 1 << 30, float(1 << 25)))
    assert p.variant in (eg.RADIX, eg.RADIX_CACHE)


def test_rule_plan_sparse_small_is_global_hash(lib):
    p = plan(stats(100000, -(1 << 62), 1 << 62, 1e5, eg.INT64), stats(1 << 24, -(1 << 62), 1 << 62, 1e7, eg.INT64))
    assert p.variant == eg.GLOBAL_HASH and 0 < p.load_factor <= 0.9


def test_rule_plan_sparse_large(lib):
    # a 1 GiB table is still probed faster in place than partitioned
    p = plan(stats(1 << 24, -(1 << 63), (1 << 63) - 1, 1.6e7, eg.INT64),
             stats(1 << 29, -(1 << 63), (1 << 63) - 1, 1.6e7, eg.INT64))
    assert p.variant == eg.GLOBAL_HASH
    # beyond the table budget the join partitions
    p = plan(stats(1 << 28, -(1 << 63), (1 << 63) - 1, 2.6e8, eg.INT64),
             stats(1 << 29, -(1 << 63), (1 << 63) - 1, 2.6e8, eg.INT64))
    assert p.variant in (eg.RADIX, eg.RADIX_CACHE)
    assert 1 <= p.radix_bits <= 18 and p.radix_passes in (1, 2)


def test_fixed_hash_and_forced(lib):
    b, s = stats(1000, 0, 999, 1000.0), stats(5000, 0, 5000, 5000.0)
    p = plan(b, s, eg.SEL_FIXED_HASH)
    assert p.variant == eg.GLOBAL_HASH and abs(p.load_factor - 0.5) < 1e-6
    p = plan(b, s, eg.SEL_FORCED, eg.make_plan(eg.RADIX, 6, 1, 0.6))
    assert (p.variant, p.radix_bits, p.radix_passes) == (eg.RADIX, 6, 1)
    assert abs(p.load_factor - 0.6) < 1e-6


def test_plan_errors(lib):
    b, s = stats(1000, 0, 999, 1000.0), stats(5000, 0, 5000, 5000.0, eg.INT64)
    with pytest.raises(eg.EigerError) as e:
        plan(b, s)
    assert e.value.code == eg.EIGER_ERR_DTYPE
    s = stats(5000, 0, 5000, 5000.0)
    with pytest.raises(eg.EigerError) as e:
        plan(b, s, eg.SEL_FORCED, None)
    assert e.value.code == eg.EIGER_ERR_INVALID_ARG
    with pytest.raises(eg.EigerError) as e:
        plan(b, s, 99)
    assert e.value.code == eg.EIGER_ERR_INVALID_ARG
    wide = stats(1000, 0, 1 << 40, 1000.0, eg.INT64)
    with pytest.raises(eg.EigerError) as e:
        plan(wide, stats(10, 0, 5, 5.0, eg.INT64), eg.SEL_FORCED, eg.make_plan(eg.DIRECT))
    assert e.value.code == eg.EIGER_ERR_UNSUPPORTED


def col(ptr, n, dtype):
    return eg.Column(ptr, n, dtype, 0)


def test_join_argument_checks_before_any_gpu_work(lib):
    p = plan(stats(10, 0, 9, 10.0), stats(10, 0, 9, 10.0))
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()
    good = col(4096, 10, eg.INT32)

    def call(bk, bp, pk, pp, pl=p, ob=None, op=None, cap=0, ws=None, nws=0):
        return lib.eiger_join(bk, bp, pk, pp, ctypes.byref(pl), ob, op, cap, ctypes.byref(cnt),
                              ctypes.byref(cs), ws, nws, None)

    assert call(good, good, col(4096, 10, eg.INT64), col(4096, 10, eg.INT64)) == eg.EIGER_ERR_DTYPE
    assert call(col(4096, 10, 7), good, good, good) == eg.EIGER_ERR_DTYPE
    assert call(col(None, 10, eg.INT32), good, good, good) == eg.EIGER_ERR_INVALID_ARG
    assert call(col(4098, 10, eg.INT32), good, good, good) == eg.EIGER_ERR_INVALID_ARG  # misaligned
    assert call(col(4096, 1 << 32, eg.INT32), col(4096, 1 << 32, eg.INT32), good, good) == eg.EIGER_ERR_TOO_LARGE
    assert call(good, col(4096, 9, eg.INT32), good, good) == eg.EIGER_ERR_INVALID_ARG
    assert call(good, good, good, good, ob=4096, op=None, cap=10) == eg.EIGER_ERR_INVALID_ARG
    assert call(good, good, good, good, cap=10) == eg.EIGER_ERR_INVALID_ARG
    bad = eg.PlanT()
    ctypes.memmove(ctypes.byref(bad), ctypes.byref(p), ctypes.sizeof(p))
    bad.variant = 9
    assert call(good, good, good, good, pl=bad) == eg.EIGER_ERR_INVALID_ARG
    bad.variant = eg.RADIX
    bad.load_factor = 0.5
    bad.radix_bits = 30
    assert call(good, good, good, good, pl=bad) == eg.EIGER_ERR_INVALID_ARG
    assert call(good, good, good, good, ws=None, nws=0) == eg.EIGER_ERR_WORKSPACE
    assert "workspace" in eg.lib().eiger_last_error().decode()


def test_workspace_sizes_grow_with_inputs(lib):
    b = stats(1 << 20, -(1 << 40), 1 << 40, 1e6, eg.INT64)
    s = stats(1 << 24, -(1 << 40), 1 << 40, 1e6, eg.INT64)
    sizes = []
    for v, bits, passes in [(eg.GLOBAL_HASH, 0, 0), (eg.RADIX, 8, 1), (eg.RADIX, 12, 2), (eg.RADIX_CACHE, 8, 1)]:
        p = plan(b, s, eg.SEL_FORCED, eg.make_plan(v, bits, passes, 0.5))
        small = ctypes.c_size_t()
        big = ctypes.c_size_t()
        assert lib.eiger_join_workspace_size(ctypes.byref(p), col(0, 1000, 1), col(0, 1000, 1),
                                             col(0, 5000, 1), col(0, 5000, 1), ctypes.byref(small)) == 0
        assert lib.eiger_join_workspace_size(ctypes.byref(p), col(0, 1 << 20, 1), col(0, 1 << 20, 1),
                                             col(0, 1 << 24, 1), col(0, 1 << 24, 1), ctypes.byref(big)) == 0
        assert 0 < small.value < big.value
        sizes.append(big.value)
    # a two-pass radix join keeps two partitioned copies of each side
    assert sizes[2] > sizes[1] > sizes[0]
    assert sizes[3] > sizes[0]


def test_stats_empty_column_needs_no_gpu(lib):
    out = eg.StatsT()
    regs = (ctypes.c_uint8 * (1 << 14))()
    assert lib.eiger_stats(col(None, 0, eg.INT64), ctypes.byref(out), regs, None, 0, None) == 0
    assert (out.n, out.min, out.max, out.ndv, out.flags) == (0, 0, 0, 0.0, 1)
    assert lib.eiger_stats(col(None, 0, 5), ctypes.byref(out), None, None, 0, None) == eg.EIGER_ERR_DTYPE
    assert lib.eiger_stats(col(4096, 100, eg.INT32), ctypes.byref(out), None, None, 0, None) == eg.EIGER_ERR_WORKSPACE
    assert lib.eiger_stats_workspace_size(100, eg.INT32) > 0


def test_profile_table_without_gpu(lib):
    eg.profile_enable(True)
    assert eg.profile_read() == {}
    eg.profile_enable(False)


def test_selector_host_functions(lib):
    b, s = stats(10000, 0, 9999, 10000.0), stats(50000, 0, 20000, 20000.0)
    f = eg.selector_features(b, s)
    assert f.shape == (16,) and bool(torch.isfinite(f).all())
    assert abs(float(f[0]) - np.log2(10001)) < 1e-5 and float(f[6]) == 0.0
    assert eg.mlp_param_count() == 6288
    for c in range(16):
        p = eg.selector_class_plan(c, b, s)
        assert p is not None and 0 <= p.variant <= 3
    wide = stats(1000, -(1 << 40), 1 << 40, 1000.0, eg.INT64)
    assert eg.selector_class_plan(0, wide, stats(10, 0, 5, 5.0, eg.INT64)) is None
    with pytest.raises(eg.EigerError):
        eg.selector_class_plan(16, b, s)


def test_selector_load_rejects_bad_models(lib):
    import torch as T
    with pytest.raises(eg.EigerError) as e:
        eg.selector_load(T.zeros(6288), np.zeros(16), np.zeros(16))
    assert e.value.code == eg.EIGER_ERR_MODEL
    bad = T.zeros(6288)
    bad[5] = float("nan")
    with pytest.raises(eg.EigerError):
        eg.selector_load(bad, np.zeros(16), np.ones(16))


def test_selector_load_factor_near_tie(lib):
    """A GLOBAL_HASH choice moves to the largest load factor predicted within
    1% (log2(1.01) in log2 ms) of it; other variants keep the plain argmin."""
    import torch as T
    from paper_2607_04489_amd import selector
    b, s = stats(1 << 20, -(1 << 40), 1 << 40, float(1 << 20), eg.INT64), \
        stats(1 << 22, -(1 << 40), 1 << 40, float(1 << 20), eg.INT64)
    cases = [  # output biases of classes 1, 2, 3 (GLOBAL_HASH 0.25 / 0.5 / 0.75), 8 -> load factor / variant
        ((3.0, 3.01, 3.02, 5.0), (eg.GLOBAL_HASH, 0.5)),
        ((3.0, 3.02, 3.03, 5.0), (eg.GLOBAL_HASH, 0.25)),
        ((3.0, 3.01, 3.005, 5.0), (eg.GLOBAL_HASH, 0.75)),
        ((3.01, 3.0, 3.02, 5.0), (eg.GLOBAL_HASH, 0.5)),
        ((3.005, 5.0, 5.0, 3.0), (eg.RADIX, 0.25)),
    ]
    for (b1, b2, b3, b8), want in cases:
        params = T.zeros(6288)
        params[6272:] = 6.0
        params[6272 + 1], params[6272 + 2], params[6272 + 3], params[6272 + 8] = b1, b2, b3, b8
        eg.selector_load(params, np.zeros(16), np.ones(16))
        got = plan(b, s, eg.SEL_LEARNED)
        assert (got.variant, round(got.load_factor, 3)) == want, ((b1, b2, b3, b8), got.describe())
        y = params[6272:].numpy().astype(np.float32)
        y[0] = np.inf  # DIRECT is infeasible over this key range
        ref = eg.selector_class_plan(selector.choose(y), b, s)
        assert (ref.variant, round(ref.load_factor, 3)) == want


def test_selector_domain_guard_falls_back_to_rule(lib):
    """Outside the installed model's training box EIGER_SEL_LEARNED returns the
    rule plan with EIGER_PLAN_RULE_FALLBACK; inside it returns the model's class."""
    import torch as T
    params = T.zeros(6288)
    params[6272:] = 5.0
    params[6272 + 1] = -1.0  # the output bias alone ranks class 1 (GLOBAL_HASH lf 0.25) first
    b, s = stats(1 << 20, -(1 << 40), 1 << 40, float(1 << 20), eg.INT64), \
        stats(1 << 22, -(1 << 40), 1 << 40, float(1 << 20), eg.INT64)
    f = eg.selector_features(b, s).numpy()
    eg.selector_load(params, np.zeros(16), np.ones(16), f - 0.5, f + 0.5)
    inside = plan(b, s, eg.SEL_LEARNED)
    assert (inside.variant, round(inside.load_factor, 3), inside.flags) == (eg.GLOBAL_HASH, 0.25, 0)
    big = stats(1 << 26, -(1 << 40), 1 << 40, float(1 << 26), eg.INT64)
    out = plan(big, s, eg.SEL_LEARNED)
    rule = plan(big, s, eg.SEL_RULE)
    assert out.flags == eg.PLAN_RULE_FALLBACK and rule.flags == 0
    assert out.describe() == dict(rule.describe(), rule_fallback=True)
    # no box: the model decides everywhere
    eg.selector_load(params, np.zeros(16), np.ones(16))
    assert plan(big, s, eg.SEL_LEARNED).flags == 0
    with pytest.raises(eg.EigerError) as e:
        eg.selector_load(params, np.zeros(16), np.ones(16), f + 1.0, f)
    assert e.value.code == eg.EIGER_ERR_MODEL
    lo = T.as_tensor(f).contiguous()
    assert lib.eiger_selector_load(eg._fptr(params), eg._fptr(T.zeros(16)), eg._fptr(T.ones(16)),
                                   eg._fptr(lo), None) == eg.EIGER_ERR_INVALID_ARG


def batch_arr(specs):
    arr = (eg.BatchJoinT * len(specs))()
    for i, (ptr, nb, npr) in enumerate(specs):
        arr[i] = eg.BatchJoinT(ptr, ptr, ptr, ptr, nb, npr)
    return arr


def test_batch_host_checks(lib):
    size = ctypes.c_size_t()
    ok = batch_arr([(4096, 1000, 8000), (8192, 5, 40), (4096, 0, 10)])
    assert lib.eiger_join_batch_workspace_size(ok, 3, eg.INT32, eg.INT32, None, ctypes.byref(size)) == 0
    small = size.value
    big = batch_arr([(4096, 1 << 20, 1 << 22), (8192, 5, 40), (4096, 0, 10)])
    assert lib.eiger_join_batch_workspace_size(big, 3, eg.INT32, eg.INT32, None, ctypes.byref(size)) == 0
    assert size.value > small > 0
    tune = (eg.BatchTuneT * eg.BATCH_BUCKETS)(*[eg.BatchTuneT(0.25, 4096)] * eg.BATCH_BUCKETS)
    assert lib.eiger_join_batch_workspace_size(ok, 3, eg.INT32, eg.INT32, ctypes.byref(tune),
                                               ctypes.byref(size)) == 0
    assert size.value > small  # a lower load factor needs larger tables
    assert lib.eiger_join_batch_workspace_size(ok, 0, eg.INT32, eg.INT32, None, ctypes.byref(size)) == eg.EIGER_ERR_INVALID_ARG
    assert lib.eiger_join_batch_workspace_size(ok, 3, 7, eg.INT32, None, ctypes.byref(size)) == eg.EIGER_ERR_DTYPE
    assert lib.eiger_join_batch_workspace_size(batch_arr([(None, 10, 10)]), 1, eg.INT32, eg.INT32, None,
                                               ctypes.byref(size)) == eg.EIGER_ERR_INVALID_ARG
    assert lib.eiger_join_batch_workspace_size(batch_arr([(4098, 10, 10)]), 1, eg.INT64, eg.INT32, None,
                                               ctypes.byref(size)) == eg.EIGER_ERR_INVALID_ARG
    assert lib.eiger_join_batch_workspace_size(batch_arr([(4096, 1 << 33, 10)]), 1, eg.INT32, eg.INT32, None,
                                               ctypes.byref(size)) == eg.EIGER_ERR_TOO_LARGE
    h = ctypes.c_void_p()
    assert lib.eiger_join_batch_create(ok, 3, eg.INT32, eg.INT32, None, None, None, None, 0, None,
                                       ctypes.byref(h)) == eg.EIGER_ERR_INVALID_ARG  # NULL outputs
    assert lib.eiger_join_batch_create(ok, 3, eg.INT32, eg.INT32, None, 4096, 4096, None, 0, None,
                                       ctypes.byref(h)) == eg.EIGER_ERR_WORKSPACE
    assert lib.eiger_join_batch_launch(None, None) == eg.EIGER_ERR_INVALID_ARG
    assert lib.eiger_join_batch_destroy(None) == 0


def test_batch_bucket():
    assert [eg.batch_bucket(n) for n in (0, 1, 2, 3, 4, 255, 256, 1 << 20)] == [0, 0, 1, 1, 2, 7, 8, 20]


MAX_ROWS = (1 << 32) - (1 << 16)


def test_row_limit_is_eiger_max_rows(lib):
    """A column may hold EIGER_MAX_ROWS = 2^32 - 2^16 rows; one more is
    EIGER_ERR_TOO_LARGE (the join's sizing, the join and the statistics)."""
    b = stats(MAX_ROWS, -(1 << 40), 1 << 40, float(MAX_ROWS), eg.INT64)
    ok = col(4096, MAX_ROWS, eg.INT64)
    over = col(4096, MAX_ROWS + 1, eg.INT64)
    half = col(4096, 1 << 31, eg.INT64)  # RADIX_CACHE's one table stays below 2^32 slots
    size = ctypes.c_size_t()
    for v, bits, passes, r in [(eg.GLOBAL_HASH, 0, 0, ok), (eg.RADIX, 16, 2, ok), (eg.RADIX_CACHE, 10, 1, half)]:
        p = plan(b, b, eg.SEL_FORCED, eg.make_plan(v, bits, passes, 0.9 if v == eg.RADIX_CACHE else 0.5))
        assert lib.eiger_join_workspace_size(ctypes.byref(p), r, r, ok, ok, ctypes.byref(size)) == 0, \
            eg.lib().eiger_last_error()
        assert size.value > 16 * MAX_ROWS
        assert lib.eiger_join_workspace_size(ctypes.byref(p), over, over, ok, ok,
                                             ctypes.byref(size)) == eg.EIGER_ERR_TOO_LARGE
        assert lib.eiger_join_workspace_size(ctypes.byref(p), r, r, over, over,
                                             ctypes.byref(size)) == eg.EIGER_ERR_TOO_LARGE
    out = eg.StatsT()
    assert lib.eiger_stats(col(4096, MAX_ROWS + 1, eg.INT32), ctypes.byref(out), None, None, 0,
                           None) == eg.EIGER_ERR_TOO_LARGE


def test_noalloc_checks_before_any_gpu_work(lib):
    """eiger_join_noalloc refuses, on the host, plans whose workspace exceeds its
    fixed scratch array, and shares eiger_join's argument checks."""
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()
    b = stats(10_000_000, -(1 << 40), 1 << 40, 1e7, eg.INT64)
    p = plan(b, b, eg.SEL_FORCED, eg.make_plan(eg.GLOBAL_HASH, 0, 0, 0.5))
    big = col(4096, 10_000_000, eg.INT64)
    size = ctypes.c_size_t()
    assert lib.eiger_join_workspace_size(ctypes.byref(p), big, big, big, big, ctypes.byref(size)) == 0
    assert size.value > eg.NOALLOC_SCRATCH_BYTES
    rc = lib.eiger_join_noalloc(big, big, big, big, ctypes.byref(p), None, None, 0, ctypes.byref(cnt),
                                ctypes.byref(cs), None)
    assert rc == eg.EIGER_ERR_TOO_LARGE
    assert "scratch" in eg.lib().eiger_last_error().decode()
    small = stats(10, 0, 9, 10.0)
    ps = plan(small, small)
    good = col(4096, 10, eg.INT32)
    assert lib.eiger_join_noalloc(good, good, col(4096, 10, eg.INT64), col(4096, 10, eg.INT64), ctypes.byref(ps),
                                  None, None, 0, ctypes.byref(cnt), ctypes.byref(cs), None) == eg.EIGER_ERR_DTYPE
    assert lib.eiger_join_noalloc(good, good, good, good, ctypes.byref(ps), 4096, None, 10, ctypes.byref(cnt),
                                  ctypes.byref(cs), None) == eg.EIGER_ERR_INVALID_ARG
    assert lib.eiger_join_noalloc(good, good, good, good, ctypes.byref(ps), None, None, 0, None,
                                  ctypes.byref(cs), None) == eg.EIGER_ERR_INVALID_ARG
