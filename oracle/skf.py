"""Smart key fusion and order-preserving dictionary encoding -- TEST INFRASTRUCTURE ONLY.

Same rule as the rest of ``oracle``: only ``tests/``, the smoke check and the
benchmark's CPU baseline may import this module; it imports nothing from the GPU
library. Plain numpy, written from the paper:

  * dict_encode    -- order-preserving dictionary encoding (Algorithm 1)
  * skf_plan       -- smart key fusion: per key, frame-of-reference or dictionary
                      code and its bit width; fused key width (Section 4.3)
  * fuse           -- the fused 4- or 8-byte key of each row (Section 4.3)
  * sort_pairs     -- the stable order of (key, row) pairs by a key's low bits
  * sort_multikey  -- rows ordered by several keys, each ascending or descending
                      (Section 3.6, cases 1 and 2)
  * join_multikey  -- the inner equi-join on several key columns (Section 4.3:
                      multiple keys in joins)

Readings where the paper leaves a choice open (each is also stated in the
function's docstring): the range test compares the bit width of max - min with a
threshold in bits; a key that is neither narrow nor of low NDV still enters the
fusion at its full frame-of-reference width; the first key takes the most
significant bits; a descending key is complemented within its width; a dictionary
code's width is that of the exact distinct count, which the encoding returns.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import _as_i64, canonical_pairs, join_sortmerge

FOR, DICT = 0, 1
DEFAULT_FOR_MAX_BITS = 16
DEFAULT_DICT_MAX_NDV = 1 << 20


def dict_encode(col):
    """Order-preserving dictionary encoding (Algorithm 1; Section 4.3). The five
    steps (leader election in a hash table, retrieval of the distinct keys with
    their group ids, argsort of the distinct keys, scatter of each position to its
    group, gather by every row) end at one result with a plain definition: the
    dictionary is the ascending list of the column's distinct values and a row's
    code is the position of its value in that list, i.e. the number of distinct
    values smaller than it. Returns (codes int64, ndv, dictionary int64)."""
    k = _as_i64(col)
    uniq, inv = np.unique(k, return_inverse=True)
    return inv.reshape(-1).astype(np.int64), int(uniq.size), uniq


def bit_width(x: int) -> int:
    """Bits needed to hold the non-negative integer x (0 for x == 0)."""
    return int(x).bit_length()


@dataclass
class KeyCode:
    kind: int          # FOR or DICT
    bits: int          # width of the code
    shift: int         # position of the code's lowest bit in the fused key
    descending: bool
    base: int          # FOR: the key's minimum; DICT: 0
    ndv: int = 0       # DICT: exact distinct count


@dataclass
class SkfPlan:
    keys: list = field(default_factory=list)
    total_bits: int = 0
    fused_bytes: int = 0   # 4, 8, or 0 when the codes need more than 64 bits


def skf_plan(stats, descending, ndv_exact=None, for_max_bits: int = DEFAULT_FOR_MAX_BITS,
             dict_max_ndv: int = DEFAULT_DICT_MAX_NDV) -> SkfPlan:
    """Smart key fusion (Section 4.3), one decision per key in the paper's order:
    the key's range max - min is found first; a range whose bit width is at most
    `for_max_bits` takes frame-of-reference encoding (code = key - min) packed in
    that width. Otherwise the HLL++ distinct estimate decides: at most
    `dict_max_ndv` takes the order-preserving dictionary (code = rank among the
    distinct values, width of ndv - 1 for the exact ndv in `ndv_exact`); above it
    the key keeps its full frame-of-reference width. Codes are then laid side by
    side, the first key in the most significant bits; the fused key is 4 bytes
    when they fit 32 bits, 8 bytes when they fit 64, else fusion is impossible.

    `stats`: per key a dict with 'n', 'min', 'max', 'ndv' (as column_stats
    returns); `descending`: per key bool; `ndv_exact`: per key exact distinct
    count (needed for dictionary keys)."""
    plan = SkfPlan()
    for c, st in enumerate(stats):
        empty = st["n"] == 0
        rng = 0 if empty else int(st["max"]) - int(st["min"])
        w = bit_width(rng)
        if w <= for_max_bits or empty:
            kc = KeyCode(FOR, w, 0, bool(descending[c]), 0 if empty else int(st["min"]))
        elif st["ndv"] <= dict_max_ndv:
            ndv = int(ndv_exact[c])
            kc = KeyCode(DICT, bit_width(max(ndv - 1, 0)), 0, bool(descending[c]), 0, ndv)
        else:
            kc = KeyCode(FOR, w, 0, bool(descending[c]), int(st["min"]))
        plan.keys.append(kc)
    total = sum(k.bits for k in plan.keys)
    plan.total_bits = total
    plan.fused_bytes = 4 if total <= 32 else (8 if total <= 64 else 0)
    pos = total
    for k in plan.keys:
        pos -= k.bits
        k.shift = pos
    return plan


def fuse(cols, plan: SkfPlan, dict_codes=None) -> np.ndarray:
    """The fused key of every row (Section 4.3): each key's code -- key - base
    for frame-of-reference (an exact non-negative integer below 2^bits), the
    dictionary code for a dictionary key -- complemented within its width when the
    key sorts descending, shifted to its position and OR-ed in. Comparing fused
    keys as unsigned integers compares the rows lexicographically by the keys,
    and equal fused keys mean equal keys. Returns uint32 or uint64."""
    if plan.fused_bytes == 0:
        raise ValueError("the key codes need more than 64 bits")
    n = len(_as_i64(cols[0])) if cols else 0
    out = np.zeros(n, dtype=np.uint64)
    for c, k in enumerate(plan.keys):
        if k.bits == 0:
            continue
        if k.kind == FOR:
            # key - base lies in [0, 2^64): the difference of the two's-complement
            # patterns mod 2^64 is that exact value
            v = _as_i64(cols[c]).view(np.uint64) - np.uint64(k.base & 0xFFFFFFFFFFFFFFFF)
        else:
            v = np.asarray(dict_codes[c]).astype(np.uint64)
        assert v.size == 0 or int(v.max()) < (1 << k.bits)
        if k.descending:
            v = v ^ np.uint64((1 << k.bits) - 1)
        out |= v << np.uint64(k.shift)
    return out.astype(np.uint32) if plan.fused_bytes == 4 else out


def sort_pairs(keys, key_bits: int):
    """Radix sort's result (Section 3.6, case 1): the keys ordered ascending by
    the unsigned value of their low key_bits bits, and the stable permutation
    that orders them (equal keys keep their input order, as every LSD radix pass
    does). Plain definition: numpy's stable argsort of the masked keys. Returns
    (masked keys sorted as uint64, permutation int64)."""
    k = np.asarray(keys)
    k = k.view(np.uint32 if k.dtype.itemsize == 4 else np.uint64).astype(np.uint64)
    if key_bits < 64:
        k = k & np.uint64((1 << key_bits) - 1)
    perm = np.argsort(k, kind="stable")
    return k[perm], perm


def sort_multikey(cols, descending):
    """Rows ordered lexicographically by the key columns, each ascending or
    descending (Section 3.6). Plain definition: Python's sort of the key tuples,
    with a descending key compared reversed. Equal tuples may come in any order,
    so the unique result is the sorted key table: returns (keys sorted as an
    (n, n_keys) int64 array, one ordering permutation)."""
    ks = [_as_i64(c) for c in cols]
    n = len(ks[0]) if ks else 0
    if n == 0:
        return np.zeros((0, len(ks)), np.int64), np.zeros(0, np.int64)
    # np.lexsort sorts by its last row first; a descending key sorts by its negated rank
    ranks = []
    for c, k in enumerate(ks):
        _, r = np.unique(k, return_inverse=True)
        r = r.reshape(-1).astype(np.int64)
        ranks.append(-r if descending[c] else r)
    perm = np.lexsort(ranks[::-1])
    return np.stack([k[perm] for k in ks], axis=1), perm


def join_multikey(colsR, colsS, threads: int = 1) -> np.ndarray:
    """Inner equi-join on several key columns: the pairs (i, j) with
    colsR[c][i] == colsS[c][j] for every key c. Each distinct key tuple of R and
    S together gets one integer id (np.unique over the stacked tuples), and the
    pairs are those of the single-key join on the ids. Returns canonical pairs
    (build_row << 32 | probe_row, ascending)."""
    kR = [_as_i64(c) for c in colsR]
    kS = [_as_i64(c) for c in colsS]
    nR, nS = len(kR[0]), len(kS[0])
    if nR == 0 or nS == 0:
        return np.zeros(0, np.uint64)
    both = np.stack([np.concatenate([a, b]) for a, b in zip(kR, kS)], axis=1)
    _, ids = np.unique(both, axis=0, return_inverse=True)
    ids = ids.reshape(-1).astype(np.int64)
    pairs, _, _ = join_sortmerge(ids[:nR], ids[:nR], ids[nR:], ids[nR:], threads=threads)
    return pairs


__all__ = ["FOR", "DICT", "DEFAULT_FOR_MAX_BITS", "DEFAULT_DICT_MAX_NDV", "dict_encode", "bit_width",
           "KeyCode", "SkfPlan", "skf_plan", "fuse", "sort_pairs", "sort_multikey", "join_multikey",
           "canonical_pairs"]
