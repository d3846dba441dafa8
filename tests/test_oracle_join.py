"""Pins of the join oracle against brute force, closed forms and invariants.

The join result is the plain definition of an inner equi-join (Section 5.2:
build side R, probe side S; Section 2.2: tuple ids as the delegate of the
payload columns): all (i, j) with kR[i] == kS[j], their count, and the sum of
pR[i] * pS[j] mod 2^64. None of these checks reuses the oracle's code.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def wrap64(x: int) -> int:
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


def brute_force(kR, pR, kS, pS):
    """Nested loops in (i, j) order: already canonical."""
    pairs, total = [], 0
    for i, (k, a) in enumerate(zip(kR, pR)):
        for j, (l, b) in enumerate(zip(kS, pS)):
            if k == l:
                pairs.append((i << 32) | j)
                total += a * b
    return np.array(pairs, dtype=np.uint64), len(pairs), wrap64(total)


def check_all(kR, pR, kS, pS):
    kR, pR, kS, pS = (list(map(int, x)) for x in (kR, pR, kS, pS))
    bp, bc, bs = brute_force(kR, pR, kS, pS)
    pairs, cnt, cs = oracle.join_sortmerge(kR, pR, kS, pS)
    assert cnt == bc and cs == bs
    assert np.array_equal(pairs, bp)
    tc, ts = oracle.join_totals(kR, pR, kS, pS)
    assert (tc, ts) == (bc, bs)
    tc, ts = oracle.join_totals(kR, pR, kS, pS, threads=3)
    assert (tc, ts) == (bc, bs)


def test_hand_example():
    # R = keys 5, 7, 5 with payloads 10, 20, 30; S = keys 5, 9, 7, 5 with 2, 4, -1, 3.
    # Matches: (0,0) (0,3) (1,2) (2,0) (2,3); checksum 20 + 30 - 20 + 60 + 90 = 180.
    pairs, cnt, cs = oracle.join_sortmerge([5, 7, 5], [10, 20, 30], [5, 9, 7, 5], [2, 4, -1, 3])
    assert cnt == 5 and cs == 180
    assert [(int(x) >> 32, int(x) & 0xFFFFFFFF) for x in pairs] == [(0, 0), (0, 3), (1, 2), (2, 0), (2, 3)]


def test_checksum_wraps_mod_2_64():
    # INT64_MIN * -1 = 2^63 = INT64_MIN mod 2^64; (2^63 - 1) * 2 = -2 mod 2^64.
    _, cnt, cs = oracle.join_sortmerge([1], [I64_MIN], [1], [-1])
    assert (cnt, cs) == (1, I64_MIN)
    _, cnt, cs = oracle.join_sortmerge([1, 1], [I64_MAX, I64_MAX], [1], [2])
    assert (cnt, cs) == (2, wrap64(4 * I64_MAX))


@pytest.mark.parametrize("case", [
    "empty_build", "empty_probe", "both_empty", "one_build_row", "all_equal", "disjoint",
    "negative", "int32_extremes", "int64_extremes", "narrow_dups", "wide_unique"])
def test_adversarial_vs_brute_force(case):
    rng = np.random.default_rng(7)
    if case == "empty_build":
        kR, kS = [], [1, 2, 3]
    elif case == "empty_probe":
        kR, kS = [1, 2, 3], []
    elif case == "both_empty":
        kR, kS = [], []
    elif case == "one_build_row":
        kR, kS = [4], list(rng.integers(0, 8, 50))
    elif case == "all_equal":
        kR, kS = [3] * 17, [3] * 23
    elif case == "disjoint":
        kR, kS = list(range(0, 40)), list(range(40, 90))
    elif case == "negative":
        kR, kS = list(rng.integers(-20, 0, 60)), list(rng.integers(-25, 5, 80))
    elif case == "int32_extremes":
        kR = [I32_MIN, I32_MAX, 0, -1, I32_MIN, 7]
        kS = [I32_MAX, I32_MIN, I32_MIN, 1, -1, 0, 7, 7]
    elif case == "int64_extremes":
        kR = [I64_MIN, I64_MAX, 0, -1, I64_MAX]
        kS = [I64_MAX, I64_MIN, 5, -1, I64_MIN, I64_MAX]
    elif case == "narrow_dups":
        kR, kS = list(rng.integers(0, 6, 70)), list(rng.integers(0, 9, 90))
    else:
        kR = list(rng.permutation(200)[:120])
        kS = list(rng.integers(-10, 230, 150))
    pR = list(rng.integers(I64_MIN, I64_MAX, len(kR), dtype=np.int64, endpoint=True))
    pS = list(rng.integers(I64_MIN, I64_MAX, len(kS), dtype=np.int64, endpoint=True))
    check_all(kR, pR, kS, pS)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_random_small_vs_brute_force(seed):
    for lo, hi, nb, npr in [(0, 15, 64, 200), (-50, 50, 300, 300), (I32_MIN, I32_MAX, 100, 100)]:
        inp = synth.random_small(seed, nb, npr, lo, hi)
        check_all(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)


def test_plain_dense_closed_form():
    """Build keys are a permutation of [0, n_build): probe row j matches exactly
    build row inv[kS[j]] when kS[j] < n_build, so P needs no join code at all."""
    inp = synth.plain_dense(seed=3, n_build=4096, n_probe=50000, probe_range=5000)
    kR = inp.build_keys.numpy().astype(np.int64)
    kS = inp.probe_keys.numpy().astype(np.int64)
    pR = inp.build_payload.numpy().astype(np.int64)
    pS = inp.probe_payload.numpy().astype(np.int64)
    assert np.array_equal(np.sort(kR), np.arange(4096))
    inv = np.empty(4096, dtype=np.int64)
    inv[kR] = np.arange(4096)
    j = np.nonzero(kS < 4096)[0]
    i = inv[kS[j]]
    expect = np.sort((i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64))
    checksum = wrap64(int(np.sum(pR[i] * pS[j])))  # products < 10^6, sum < 2^63
    pairs, cnt, cs = oracle.join_sortmerge(kR, pR, kS, pS)
    assert cnt == len(j) and cs == checksum
    assert np.array_equal(pairs, expect)


def test_sparse_unique64_recorded_sources():
    """Each matching probe row records the build row its key was copied from;
    build keys are unique, so that row is its only partner."""
    inp = synth.sparse_unique64(seed=5, n_build=20000, n_probe=100000)
    src = inp.meta["source_row"].numpy()
    j = np.nonzero(src >= 0)[0]
    expect = np.sort((src[j].astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64))
    pR = inp.build_payload.numpy().astype(np.uint64)
    pS = inp.probe_payload.numpy().astype(np.uint64)
    with np.errstate(over="ignore"):
        checksum = wrap64(int(np.sum(pR[src[j]] * pS[j], dtype=np.uint64)))
    pairs, cnt, cs = oracle.join_sortmerge(inp.build_keys, inp.build_payload,
                                           inp.probe_keys, inp.probe_payload)
    assert cnt == len(j) and cs == checksum
    assert np.array_equal(pairs, expect)
    assert abs(len(j) / 100000 - 0.9) < 0.01


def test_count_is_sum_of_key_count_products():
    """count = sum_k cR(k) cS(k) and checksum = sum_k (sum pR)(sum pS) mod 2^64,
    computed here with Python dicts over the whole skewed instance."""
    inp = synth.skewed_dup32(seed=2, n_distinct=3000, n_probe=40000, zipf_s=1.0)
    kR, pR = inp.build_keys.tolist(), inp.build_payload.tolist()
    kS, pS = inp.probe_keys.tolist(), inp.probe_payload.tolist()
    cR, sR, cS, sS = {}, {}, {}, {}
    for k, p in zip(kR, pR):
        cR[k] = cR.get(k, 0) + 1
        sR[k] = sR.get(k, 0) + p
    for k, p in zip(kS, pS):
        cS[k] = cS.get(k, 0) + 1
        sS[k] = sS.get(k, 0) + p
    count = sum(cR[k] * cS[k] for k in cR if k in cS)
    checksum = wrap64(sum(sR[k] * sS[k] for k in sR if k in sS))
    _, cnt, cs = oracle.join_sortmerge(kR, pR, kS, pS, with_pairs=False)
    assert (cnt, cs) == (count, checksum)
    assert oracle.join_totals(kR, pR, kS, pS, threads=4) == (count, checksum)


def test_probe_matches_agree_with_pairs():
    inp = synth.random_small(9, 500, 2000, 0, 300)
    pairs, _, _ = oracle.join_sortmerge(inp.build_keys, inp.build_payload,
                                        inp.probe_keys, inp.probe_payload)
    rows = np.array([0, 5, 17, 1999, 640, 640], dtype=np.int64)
    offs, ids = oracle.probe_matches(inp.build_keys, inp.probe_keys, rows)
    kR, kS = inp.build_keys.numpy(), inp.probe_keys.numpy()
    for t, j in enumerate(rows):
        got = ids[offs[t]:offs[t + 1]].tolist()
        assert got == sorted(np.nonzero(kR == kS[j])[0].tolist())
        from_pairs = sorted(int(x) >> 32 for x in pairs if (int(x) & 0xFFFFFFFF) == j)
        assert got == from_pairs


def test_planted_mistake_is_caught():
    """A mistake planted in a copy of the result (one pair dropped, one probe id
    shifted) must fail the pair comparison used by the parity tests."""
    inp = synth.random_small(4, 100, 300, 0, 40)
    pairs, _, _ = oracle.join_sortmerge(inp.build_keys, inp.build_payload,
                                        inp.probe_keys, inp.probe_payload)
    bp, _, _ = brute_force(*(list(map(int, x)) for x in (
        inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)))
    assert np.array_equal(pairs, bp)
    assert not np.array_equal(pairs[1:], bp[:-1])
    bad = pairs.copy()
    bad[3] += np.uint64(1)
    assert not np.array_equal(np.sort(bad), bp)


@pytest.mark.parametrize("threads", [2, 5, 16])
def test_threaded_sorts_match_one_thread(threads):
    """The threaded slice sort + pairwise merges (an odd slice count leaves one
    run to copy through) give the same pairs, count and checksum as one thread,
    on inputs large enough to take the threaded path (>= 2^16 rows per side),
    with heavy duplicates so that equal keys cross slice boundaries; the pairs
    are also checked against numpy's own canonical order of the same set."""
    inp = synth.random_small(21, 70000, 90000, 0, 3000)
    one = oracle.join_sortmerge(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)
    many = oracle.join_sortmerge(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload,
                                 threads=threads)
    assert one[1:] == many[1:]
    assert np.array_equal(one[0], many[0])
    assert np.array_equal(many[0], np.sort(many[0]))
    rows = np.arange(0, 90000, 997, dtype=np.int64)
    o1, i1 = oracle.probe_matches(inp.build_keys, inp.probe_keys, rows)
    o2, i2 = oracle.probe_matches(inp.build_keys, inp.probe_keys, rows, threads=threads)
    assert np.array_equal(o1, o2) and np.array_equal(i1, i2)
    kR, kS = inp.build_keys.numpy(), inp.probe_keys.numpy()
    for t, j in enumerate(rows[:20]):
        assert i2[o2[t]:o2[t + 1]].tolist() == np.nonzero(kR == kS[j])[0].tolist()


def wide_brute_force(kR, colsR, kS, colsS):
    """Nested loops in (i, j) order: the result rows of the wide join."""
    rows = []
    for i in range(len(kR)):
        for j in range(len(kS)):
            if kR[i] == kS[j]:
                rows.append((i, j, [int(c[i]) for c in colsR], [int(c[j]) for c in colsS]))
    return rows


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_wide_join_vs_brute_force(seed):
    """Wide join: canonical pairs and every materialized column equal the
    nested-loop result (duplicates on both sides, int32 and int64 columns,
    extreme values)."""
    rng = np.random.default_rng(seed)
    nR, nS = int(rng.integers(0, 60)), int(rng.integers(0, 200))
    kR = rng.integers(-6, 6, nR).astype(np.int32)
    kS = rng.integers(-8, 8, nS).astype(np.int32)
    colsR = [rng.integers(-2**31, 2**31, nR, dtype=np.int64).astype(np.int32),
             rng.integers(-2**63, 2**63 - 1, nR, dtype=np.int64), np.arange(nR, dtype=np.int32)]
    colsS = [rng.integers(-2**63, 2**63 - 1, nS, dtype=np.int64), np.arange(nS, dtype=np.int64) * 3]
    pairs, outR, outS = oracle.join_wide(kR, colsR, kS, colsS)
    want = wide_brute_force(kR, colsR, kS, colsS)
    assert len(pairs) == len(want)
    assert [((int(p) >> 32), int(p) & 0xFFFFFFFF) for p in pairs] == [(i, j) for i, j, _, _ in want]
    for c in range(len(colsR)):
        assert outR[c].dtype == colsR[c].dtype
        assert [int(v) for v in outR[c]] == [r[2][c] for r in want]
    for c in range(len(colsS)):
        assert outS[c].dtype == colsS[c].dtype
        assert [int(v) for v in outS[c]] == [r[3][c] for r in want]


def test_wide_join_row_id_columns_reproduce_the_pairs():
    """Materializing a column holding each row's own index gives back the pair
    list (a transposed or shifted gather would not)."""
    rng = np.random.default_rng(9)
    kR = rng.integers(0, 300, 2000).astype(np.int64)
    kS = rng.integers(0, 400, 5000).astype(np.int64)
    pairs, outR, outS = oracle.join_wide(kR, [np.arange(2000, dtype=np.int64)], kS, [np.arange(5000, dtype=np.int32)])
    assert np.array_equal(outR[0].astype(np.uint64), pairs >> np.uint64(32))
    assert np.array_equal(outS[0].astype(np.uint64), pairs & np.uint64(0xFFFFFFFF))
    assert np.array_equal(kR[outR[0]], kS[outS[0]])
