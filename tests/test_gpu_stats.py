"""eiger_stats on the GPU against the statistics oracle: registers byte-exact,
min/max exact, the distinct estimate within fp64 rounding of the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth

pytestmark = pytest.mark.gpu


def check(col):
    st = eg.stats(col)
    ref = oracle.column_stats(col)
    assert st.n == ref["n"]
    assert (st.min, st.max) == (ref["min"], ref["max"])
    assert np.array_equal(st.regs.numpy(), ref["regs"])
    assert st.ndv == pytest.approx(ref["ndv"], rel=1e-12, abs=1e-12)
    return st


# 1048576 / 1081344 int32 rows: 32 / 33 partial sketches, the two sides of the
# switch to the two-stage register merge (int64: 64 / 66)
@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 4099, 65536, 1000003, 1048576, 1081344])
@pytest.mark.parametrize("dtype", [torch.int32, torch.int64])
def test_stats_sizes(gpu, n, dtype):
    lo, hi = (-(1 << 31), (1 << 31) - 1) if dtype == torch.int32 else (-(1 << 63), (1 << 63) - 1)
    col = synth.random_small(n, n, 1, lo, hi, dtype=dtype, device=gpu).build_keys
    check(col)


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_stats_misaligned_views(gpu, offset):
    base = synth.random_small(5, 100000, 1, -1000, 1000000, device=gpu).build_keys
    check(base[offset:])
    base64 = synth.random_small(6, 100000, 1, -(1 << 40), 1 << 40, dtype=torch.int64, device=gpu).build_keys
    check(base64[offset:])


def test_stats_extremes_and_empty(gpu):
    check(torch.tensor([-(1 << 63), (1 << 63) - 1, 0], dtype=torch.int64, device=gpu))
    check(torch.tensor([-(1 << 31), (1 << 31) - 1], dtype=torch.int32, device=gpu))
    st = eg.stats(torch.zeros(0, dtype=torch.int32, device=gpu))
    assert (st.n, st.ndv, st.raw.flags) == (0, 0.0, 1)


def test_stats_workload_columns(gpu):
    inp = synth.plain_dense(seed=42, device=gpu)
    st = check(inp.build_keys)
    assert (st.min, st.max) == (0, 65535)
    check(inp.probe_keys)
    inp = synth.sparse_unique64(seed=1, n_build=1 << 20, n_probe=1 << 22, device=gpu)
    st = check(inp.build_keys)
    assert abs(st.ndv / (1 << 20) - 1) < 3 * 1.04 / 128
    check(inp.probe_keys)


def test_stats_int32_equals_sign_extended_int64(gpu):
    col = synth.random_small(3, 50000, 1, -(1 << 31), (1 << 31) - 1, device=gpu).build_keys
    a, b = eg.stats(col), eg.stats(col.to(torch.int64))
    assert np.array_equal(a.regs.numpy(), b.regs.numpy()) and (a.min, a.max) == (b.min, b.max)
