"""Pins of the smart-key-fusion oracle (oracle.skf) against what the paper and
the mathematics fix: the dictionary code's definition by brute force, order and
equality preservation of the fused key over every pair of rows, the plan's width
arithmetic at its thresholds, the multi-key sort against Python's tuple sort and
the multi-key join against a double loop."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import skf

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def brute_codes(col):
    vals = set(int(x) for x in col)
    return [sum(1 for v in vals if v < int(x)) for x in col]


def test_dict_encode_small_example():
    # distinct values 10 < 20 < 30 take codes 0, 1, 2 (Algorithm 1: the position of
    # each distinct key after the argsort becomes every row's code)
    codes, ndv, dic = skf.dict_encode(np.array([30, 10, 30, 20, 10]))
    assert codes.tolist() == [2, 0, 2, 1, 0]
    assert ndv == 3 and dic.tolist() == [10, 20, 30]


@pytest.mark.parametrize("seed", range(6))
def test_dict_encode_brute_force(seed):
    rng = np.random.default_rng(seed)
    pool = rng.choice(np.array([I64_MIN, I64_MAX, -1, 0, 1, 7, 1 << 40, -(1 << 33)], dtype=np.int64), 5)
    col = np.concatenate([pool, rng.integers(-50, 50, 30)])[rng.permutation(35)]
    codes, ndv, dic = skf.dict_encode(col)
    assert codes.tolist() == brute_codes(col)
    assert ndv == len(set(col.tolist()))
    assert (dic[codes] == col).all()


def test_dict_encode_dense_column_is_identity():
    col = np.random.default_rng(3).permutation(1000)
    codes, ndv, _ = skf.dict_encode(col)
    assert ndv == 1000 and (codes == col).all()


def _stats(cols):
    return [oracle.column_stats(c) for c in cols]


def _exact(cols):
    return [len(set(np.asarray(c).tolist())) for c in cols]


def test_plan_widths_and_thresholds():
    # range 255 needs 8 bits, 256 needs 9; a constant key needs none
    cols = [np.array([5, 260]), np.array([5, 261]), np.array([9, 9])]
    p = skf.skf_plan(_stats(cols), [False] * 3, _exact(cols))
    assert [k.kind for k in p.keys] == [skf.FOR] * 3
    assert [k.bits for k in p.keys] == [8, 9, 0]
    assert [k.shift for k in p.keys] == [9, 0, 0] and p.total_bits == 17 and p.fused_bytes == 4
    assert [k.base for k in p.keys] == [5, 5, 9]
    # a wide key of few distinct values takes the dictionary; width of ndv - 1
    wide = np.array([I64_MIN, 0, I64_MAX, 0, 12345] * 4)
    p = skf.skf_plan(_stats([wide]), [False], _exact([wide]))
    assert p.keys[0].kind == skf.DICT and p.keys[0].ndv == 4 and p.keys[0].bits == 2
    # wide and many distinct values: full frame-of-reference width
    many = np.arange(5000, dtype=np.int64) * (1 << 30)
    p = skf.skf_plan(_stats([many]), [False], _exact([many]), dict_max_ndv=1000)
    assert p.keys[0].kind == skf.FOR and p.keys[0].bits == (4999 << 30).bit_length()


@pytest.mark.parametrize("bits,expect", [((16, 16), 4), ((16, 17), 8), ((32, 32), 8), ((32, 33), 0),
                                         ((20, 20, 24), 8), ((20, 20, 25), 0)])
def test_fused_bytes_at_the_boundaries(bits, expect):
    cols = [np.array([0, (1 << b) - 1], dtype=np.int64) for b in bits]
    p = skf.skf_plan(_stats(cols), [False] * len(bits), _exact(cols), for_max_bits=64)
    assert p.total_bits == sum(bits) and p.fused_bytes == expect


def _cmp_key(row, desc):
    return tuple(-v if d else v for v, d in zip(row, desc))


@pytest.mark.parametrize("seed", range(8))
def test_fused_key_orders_and_separates_like_the_tuples(seed):
    rng = np.random.default_rng(seed)
    n = 40
    narrow = rng.integers(-3, 4, n)                                        # FOR
    sparse = rng.choice(np.array([I64_MIN, -10 ** 15, 3, 10 ** 17, I64_MAX]), n)  # dictionary
    mid = rng.integers(1000, 1000 + 64, n)                                 # FOR with an offset base
    cols = [narrow, sparse, mid]
    desc = [bool(seed & 1), bool(seed & 2), bool(seed & 4)]
    p = skf.skf_plan(_stats(cols), desc, _exact(cols))
    assert [k.kind for k in p.keys] == [skf.FOR, skf.DICT, skf.FOR]
    codes = [None, skf.dict_encode(sparse)[0], None]
    f = skf.fuse(cols, p, codes)
    assert f.dtype == np.uint32 and int(f.max()) < (1 << p.total_bits)
    rows = list(zip(*(c.tolist() for c in cols)))
    for i, j in itertools.product(range(n), repeat=2):
        a, b = _cmp_key(rows[i], desc), _cmp_key(rows[j], desc)
        assert (a < b) == (int(f[i]) < int(f[j])), (i, j)
        assert (a == b) == (f[i] == f[j]), (i, j)


def test_fuse_single_ascending_key_is_key_minus_min():
    col = np.array([-7, 3, -7, 100], dtype=np.int64)
    p = skf.skf_plan(_stats([col]), [False], _exact([col]))
    assert skf.fuse([col], p).tolist() == [0, 10, 0, 107]
    p = skf.skf_plan(_stats([col]), [True], _exact([col]))
    assert skf.fuse([col], p).tolist() == [127, 117, 127, 20]   # 7-bit complement


def test_fuse_eight_bytes_with_extremes():
    a = np.array([I64_MIN, I64_MAX, 0], dtype=np.int64)        # 64-bit range alone
    p = skf.skf_plan(_stats([a]), [False], _exact([a]), dict_max_ndv=0)
    assert p.fused_bytes == 8 and p.keys[0].bits == 64
    assert skf.fuse([a], p).tolist() == [0, (1 << 64) - 1, 1 << 63]


@pytest.mark.parametrize("seed", range(5))
def test_sort_multikey_against_python_sort(seed):
    rng = np.random.default_rng(seed)
    n = 200
    cols = [rng.integers(0, 4, n), rng.choice(np.array([I64_MIN, -5, 9, I64_MAX]), n), rng.integers(-9, 9, n)]
    desc = [bool(seed & 1), bool(seed & 2), False]
    got, perm = skf.sort_multikey(cols, desc)
    rows = list(zip(*(c.tolist() for c in cols)))
    want = sorted(rows, key=lambda r: _cmp_key(r, desc))
    assert [tuple(r) for r in got.tolist()] == want
    assert sorted(perm.tolist()) == list(range(n))
    assert [rows[i] for i in perm] == want


@pytest.mark.parametrize("seed", range(5))
def test_join_multikey_against_double_loop(seed):
    rng = np.random.default_rng(seed)
    R = [rng.integers(0, 3, 30), rng.choice(np.array([I64_MIN, 5, I64_MAX]), 30)]
    S = [rng.integers(0, 4, 50), rng.choice(np.array([I64_MIN, 5, 6, I64_MAX]), 50)]
    want = sorted((i << 32) | j for i in range(30) for j in range(50)
                  if R[0][i] == S[0][j] and R[1][i] == S[1][j])
    assert skf.join_multikey(R, S).tolist() == want


def test_join_multikey_empty_side():
    assert skf.join_multikey([np.zeros(0, np.int64)], [np.arange(3)]).size == 0


def test_sort_pairs_is_stable_and_masks():
    keys = np.array([5, 3, 5 + 16, 3, 0, 15], dtype=np.uint32)
    k, perm = skf.sort_pairs(keys, 4)        # 5 + 16 has low 4 bits 5
    assert k.tolist() == [0, 3, 3, 5, 5, 15]
    assert perm.tolist() == [4, 1, 3, 0, 2, 5]
    k, perm = skf.sort_pairs(np.array([-1, 0, 1], dtype=np.int64), 64)   # unsigned order
    assert perm.tolist() == [1, 2, 0]
