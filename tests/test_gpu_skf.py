"""Radix sort, order-preserving dictionary encoding, smart key fusion and the
multi-key sort / join on the GPU against oracle.skf, bit for bit: sorted keys
and the stable permutation, dictionary codes and values, fused keys under the
same plan, the multi-key sort's permutation and the multi-key join's pairs.
Sizes span several tiles with a ragged tail; edge cases: empty and single-row
inputs, constant keys, INT64_MIN / INT64_MAX keys, descending keys, a table too
small for the distinct values (retry), and codes too wide to fuse."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from oracle import skf

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def host(t):
    return t.detach().cpu().numpy()


def rand_keys(seed, n, key_bytes, key_bits, dev):
    g = np.random.default_rng(seed)
    k = g.integers(0, 1 << 63, n, dtype=np.int64).view(np.uint64) | (g.integers(0, 2, n).astype(np.uint64) << 63)
    if key_bits < 64:
        k &= np.uint64((1 << key_bits) - 1)
    if key_bytes == 4:
        k = k.astype(np.uint32).view(np.int32)
    else:
        k = k.view(np.int64)
    return torch.from_numpy(k.copy()).to(dev)


@pytest.mark.parametrize("key_bytes,key_bits", [(4, 0), (4, 1), (4, 7), (4, 8), (4, 13), (4, 24), (4, 32),
                                                (8, 33), (8, 47), (8, 64)])
@pytest.mark.parametrize("n", [1, 4095, 4097, 1_000_003])
def test_sort_pairs(gpu, key_bytes, key_bits, n):
    keys = rand_keys(key_bits * 7 + n, n, key_bytes, key_bits, gpu)
    ko, vo = eg.sort_pairs(keys, key_bits)
    want_k, want_p = skf.sort_pairs(host(keys), key_bits)
    got_k = host(ko).view(np.uint32 if key_bytes == 4 else np.uint64).astype(np.uint64)
    assert np.array_equal(got_k, want_k)
    assert np.array_equal(host(vo).astype(np.int64), want_p)


def test_sort_pairs_values_and_empty(gpu):
    keys = rand_keys(3, 70001, 4, 20, gpu)
    vals = torch.arange(70001, dtype=torch.int32, device=gpu).flip(0)
    _, vo = eg.sort_pairs(keys, 20, vals)
    _, p = skf.sort_pairs(host(keys), 20)
    assert np.array_equal(host(vo), host(vals)[p])
    ko, vo = eg.sort_pairs(torch.empty(0, dtype=torch.int64, device=gpu), 64)
    assert ko.numel() == 0 and vo.numel() == 0


@pytest.mark.parametrize("dtype,ndv", [(torch.int32, 1), (torch.int32, 7), (torch.int32, 1000),
                                       (torch.int64, 100_000), (torch.int64, 3)])
def test_dict_encode(gpu, dtype, ndv):
    n = 1_000_003
    col = synth.distinct_values(ndv, ndv, n, device=gpu)
    if dtype == torch.int32:
        col = (col >> 32).to(torch.int32)
    else:
        col[:2] = torch.tensor([I64_MIN, I64_MAX], device=gpu)
    codes, dic, got_ndv = eg.dict_encode(col)
    want_codes, want_ndv, want_dict = skf.dict_encode(host(col))
    assert got_ndv == want_ndv
    assert np.array_equal(host(codes).astype(np.int64), want_codes)
    assert np.array_equal(host(dic).astype(np.int64), want_dict)


def test_dict_encode_small_table_retry_and_edges(gpu):
    col = synth.distinct_values(5, 5000, 100_000, device=gpu)
    codes, dic, ndv = eg.dict_encode(col, slots=1024)   # 5000 values: retried with more slots
    want, wndv, wdict = skf.dict_encode(host(col))
    assert ndv == wndv and np.array_equal(host(codes).astype(np.int64), want)
    one = torch.tensor([I64_MIN], dtype=torch.int64, device=gpu)
    codes, dic, ndv = eg.dict_encode(one)
    assert ndv == 1 and host(codes).tolist() == [0] and host(dic).tolist() == [I64_MIN]
    codes, dic, ndv = eg.dict_encode(torch.empty(0, dtype=torch.int32, device=gpu))
    assert ndv == 0 and codes.numel() == 0


def oracle_plan(cols, desc, for_max_bits=eg.SKF_FOR_MAX_BITS, dict_max_ndv=eg.SKF_DICT_MAX_NDV):
    hc = [host(c) for c in cols]
    st = [oracle.column_stats(c) for c in hc]
    exact = [len(np.unique(c)) for c in hc]
    p = skf.skf_plan(st, desc, exact, for_max_bits, dict_max_ndv)
    codes = [skf.dict_encode(c)[0] if k.kind == skf.DICT else None for c, k in zip(hc, p.keys)]
    return p, hc, codes


def same_plan(got, want):
    assert got.total_bits == want.total_bits and got.fused_bytes == want.fused_bytes
    for g, w in zip(got.key[: got.n_keys], want.keys):
        assert (g.code, g.bits, g.shift, g.descending) == (w.kind, w.bits, w.shift, int(w.descending))
        if w.kind == skf.FOR:
            assert g.base == w.base
        else:
            assert g.ndv == w.ndv


TABLES = {
    "4xi32_8b": dict(n_keys=4, dtype=torch.int32, narrow_bits=8, sparse_ndv=256),
    "2xi32_12b": dict(n_keys=2, dtype=torch.int32, narrow_bits=12, sparse_ndv=3000),
    "4xi64_12b": dict(n_keys=4, dtype=torch.int64, narrow_bits=12, sparse_ndv=4096),
    "3xi64_20b": dict(n_keys=3, dtype=torch.int64, narrow_bits=20, sparse_ndv=50_000),
}


@pytest.mark.parametrize("name", list(TABLES))
@pytest.mark.parametrize("desc_mask", [0, 0b0101, 0b1010])
def test_fuse_and_sort_multikey(gpu, name, desc_mask):
    kw = TABLES[name]
    n = 1_000_003
    cols = synth.multikey_table(11, n, device=gpu, **kw)
    desc = [bool((desc_mask >> c) & 1) for c in range(kw["n_keys"])]
    want_plan, hc, codes = oracle_plan(cols, desc)
    want_fused = skf.fuse(hc, want_plan, codes)
    fa, _, fin = eg.skf_fuse(cols, plan=eg.skf_plan([eg.stats(c) for c in cols], desc))
    same_plan(fin, want_plan)
    got = host(fa).view(np.uint32 if fin.fused_bytes == 4 else np.uint64)
    assert np.array_equal(got, want_fused)
    perm, srt, fin2 = eg.sort_multikey(cols, desc, with_sorted=True)
    same_plan(fin2, want_plan)
    _, want_perm = skf.sort_multikey(hc, desc)
    assert np.array_equal(host(perm).astype(np.int64), want_perm)      # stable: one permutation
    assert np.array_equal(host(srt).view(got.dtype), want_fused[want_perm])


def test_sort_multikey_edges(gpu):
    # constant key: zero bits, the permutation is the identity
    c = torch.full((5000,), -7, dtype=torch.int32, device=gpu)
    perm, _, fin = eg.sort_multikey([c])
    assert fin.total_bits == 0 and np.array_equal(host(perm), np.arange(5000))
    # one row, and no rows
    perm, _, _ = eg.sort_multikey([torch.tensor([5], dtype=torch.int64, device=gpu)])
    assert host(perm).tolist() == [0]
    perm, _, _ = eg.sort_multikey([torch.empty(0, dtype=torch.int32, device=gpu)])
    assert perm.numel() == 0
    # a full-range int64 key alone: a 64-bit frame of reference, descending
    a = torch.tensor([I64_MIN, I64_MAX, 0, -1, I64_MIN], dtype=torch.int64, device=gpu)
    perm, srt, fin = eg.sort_multikey([a], [True], plan=eg.skf_plan([eg.stats(a)], [True], dict_max_ndv=0),
                                      with_sorted=True)
    assert fin.fused_bytes == 8 and fin.key[0].bits == 64
    assert host(perm).tolist() == [1, 2, 3, 0, 4]
    # two full-range keys need 128 bits: refused
    b = a.clone()
    p = eg.skf_plan([eg.stats(a), eg.stats(b)], dict_max_ndv=0)
    with pytest.raises(eg.EigerError) as e:
        eg.sort_multikey([a, b], plan=p)
    assert e.value.code == eg.EIGER_ERR_UNSUPPORTED


@pytest.mark.parametrize("n_keys,dtype", [(2, torch.int32), (3, torch.int64)])
def test_join_multikey(gpu, n_keys, dtype):
    R, S = synth.multikey_join(21, 30_000, 400_001, n_keys, dtype, narrow_bits=6, sparse_ndv=40, device=gpu)
    res, fin, _ = eg.join_multikey(R, S)
    want = skf.join_multikey([host(r) for r in R], [host(s) for s in S])
    got = oracle.canonical_pairs(host(res.build_rowid).astype(np.uint32), host(res.probe_rowid).astype(np.uint32))
    assert res.count == want.size and np.array_equal(got, want)


def test_fuse_vector_and_scalar_forms(gpu):
    # aligned columns take the 16-byte fusion form, a view one row in takes the
    # per-row form; both must give the oracle's fused keys (ragged tails too)
    cols = synth.multikey_table(17, 300_007, device=gpu, **TABLES["4xi32_8b"])
    for view in (cols, [c[1:] for c in cols], [c[:299_999] for c in cols]):
        want_plan, hc, codes = oracle_plan(view, [False, True, False, False])
        fa, _, fin = eg.skf_fuse(view, plan=eg.skf_plan([eg.stats(c) for c in view], [False, True, False, False]))
        same_plan(fin, want_plan)
        assert np.array_equal(host(fa).view(np.uint32), skf.fuse(hc, want_plan, codes))
