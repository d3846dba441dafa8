"""CPU oracle for the equi-join path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the benchmark's
``cpu_baseline`` leg may import this package. The GPU library never imports,
links or calls it, and it imports nothing from the GPU library.

Contents (each function cites the passage of the paper it follows):
  * join_sortmerge  -- the join result (pairs, count, checksum) by sort-merge
  * join_totals     -- count and checksum from per-key aggregates of R
  * probe_matches   -- matching build rows of sampled probe rows
  * join_wide       -- the join result with both sides' payload columns materialized
  * group_by        -- groups of a key column with a count and per-column sums
  * column_stats    -- count, min, max, HLL registers and distinct estimate
  * fmix64          -- the 64-bit hash used by the sketch
The C part lives in ``eiger_oracle.c`` and is compiled with gcc on first use.
The MLP reference for the learned selector lives in ``oracle.mlp``; smart key
fusion, the order-preserving dictionary encoding and the multi-key sort and
join live in ``oracle.skf``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eiger_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None

HLL_P = 14  # 2^14 registers; the paper does not fix the precision, this is the library's choice


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O3, OpenMP for the sorts and the totals
    loop; no -march=native: the library may run on another host's CPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, pi64, pu64 = ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
            vp = ctypes.c_void_p
            lib.oracle_join_sortmerge.argtypes = [i64, vp, vp, i64, vp, vp, vp, i64, ctypes.c_int, pi64, pi64]
            lib.oracle_join_sortmerge.restype = ctypes.c_int
            lib.oracle_join_totals.argtypes = [i64, vp, vp, i64, vp, vp, ctypes.c_int, pi64, pi64]
            lib.oracle_join_totals.restype = ctypes.c_int
            lib.oracle_probe_matches.argtypes = [i64, vp, vp, i64, vp, vp, vp, i64, ctypes.c_int]
            lib.oracle_probe_matches.restype = ctypes.c_int
            lib.oracle_fmix64.argtypes = [ctypes.c_uint64]
            lib.oracle_fmix64.restype = ctypes.c_uint64
            lib.oracle_hll_registers.argtypes = [i64, vp, ctypes.c_int, vp]
            lib.oracle_hll_registers.restype = None
            del pu64
            _lib = lib
    return _lib


def _as_i64(a) -> np.ndarray:
    """Host int64 copy of a column (torch tensor or array), sign-extending 4-byte ints."""
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    a = np.asarray(a)
    if a.dtype != np.int64:
        a = a.astype(np.int64)
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def join_sortmerge(kR, pR, kS, pS, with_pairs: bool = True, threads: int = 1):
    """Inner equi-join by sort-merge (Section 3.2, Table 1; result definition in
    the module docstring of eiger_oracle.c). Returns (pairs, count, checksum);
    pairs is the canonical ascending u64 array of (build_row << 32 | probe_row),
    or None when with_pairs is False. `threads` only speeds up the sorts."""
    lib = _load()
    kR, pR, kS, pS = map(_as_i64, (kR, pR, kS, pS))
    assert kR.shape == pR.shape and kS.shape == pS.shape
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.oracle_join_sortmerge(len(kR), _ptr(kR), _ptr(pR), len(kS), _ptr(kS), _ptr(pS),
                                   None, 0, int(threads), ctypes.byref(cnt), ctypes.byref(cs))
    if rc < 0:
        raise MemoryError("oracle_join_sortmerge")
    if not with_pairs:
        return None, cnt.value, cs.value
    pairs = np.empty(max(cnt.value, 1), dtype=np.uint64)
    rc = lib.oracle_join_sortmerge(len(kR), _ptr(kR), _ptr(pR), len(kS), _ptr(kS), _ptr(pS),
                                   _ptr(pairs), cnt.value, int(threads), ctypes.byref(cnt), ctypes.byref(cs))
    if rc != 0:
        raise RuntimeError(f"oracle_join_sortmerge rc={rc}")
    return pairs[: cnt.value], cnt.value, cs.value


def join_totals(kR, pR, kS, pS, threads: int = 1):
    """(count, checksum) from per-key aggregates of the build side; equal to the
    pair sums by distributivity mod 2^64."""
    lib = _load()
    kR, pR, kS, pS = map(_as_i64, (kR, pR, kS, pS))
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.oracle_join_totals(len(kR), _ptr(kR), _ptr(pR), len(kS), _ptr(kS), _ptr(pS),
                                int(threads), ctypes.byref(cnt), ctypes.byref(cs))
    if rc != 0:
        raise MemoryError("oracle_join_totals")
    return cnt.value, cs.value


def probe_matches(kR, kS, rows, threads: int = 1):
    """For each queried probe row, the ascending build row ids with the same key.
    Returns (offsets[len(rows)+1], ids)."""
    lib = _load()
    kR, kS = _as_i64(kR), _as_i64(kS)
    q = _as_i64(rows)
    assert q.size == 0 or (q.min() >= 0 and q.max() < len(kS))
    offs = np.zeros(len(q) + 1, dtype=np.int64)
    rc = lib.oracle_probe_matches(len(kR), _ptr(kR), _ptr(kS), len(q), _ptr(q), _ptr(offs), None, 0,
                                  int(threads))
    if rc < 0:
        raise MemoryError("oracle_probe_matches")
    ids = np.zeros(max(int(offs[-1]), 1), dtype=np.uint32)
    rc = lib.oracle_probe_matches(len(kR), _ptr(kR), _ptr(kS), len(q), _ptr(q), _ptr(offs),
                                  _ptr(ids), int(offs[-1]), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_probe_matches rc={rc}")
    return offs, ids[: int(offs[-1])]


def fmix64(x: int) -> int:
    """MurmurHash3's 64-bit finalizer (Appleby), the sketch's key hash."""
    return int(_load().oracle_fmix64(ctypes.c_uint64(x & ((1 << 64) - 1))))


def hll_registers(keys, p: int = HLL_P) -> np.ndarray:
    """Dense HyperLogLog registers of a key column (Section 4.1 cites HLL++ for
    distinct counts); see oracle_hll_registers for the per-key update."""
    lib = _load()
    k = _as_i64(keys)
    regs = np.zeros(1 << p, dtype=np.uint8)
    lib.oracle_hll_registers(len(k), _ptr(k), int(p), _ptr(regs))
    return regs


def _sigma(x: float) -> float:
    """sigma(x) = x + sum_{k>=1} x^(2^k) 2^(k-1), summed until the terms vanish."""
    if x == 1.0:
        return math.inf
    total, power, weight = x, x, 1.0
    while True:
        power = power * power
        nxt = total + power * weight
        weight *= 2.0
        if nxt == total:
            return total
        total = nxt


def _tau(x: float) -> float:
    """tau(x) = (1 - x - sum_{k>=1} (1 - x^(2^-k))^2 2^-k) / 3, summed until the terms vanish."""
    if x == 0.0 or x == 1.0:
        return 0.0
    total, root, weight = 1.0 - x, x, 1.0
    while True:
        root = math.sqrt(root)
        weight *= 0.5
        nxt = total - (1.0 - root) ** 2 * weight
        if nxt == total:
            return total / 3.0
        total = nxt


def hll_estimate(regs) -> float:
    """Distinct-count estimate from dense registers, fp64.

    The paper relies on HLL++ (Section 4.1) without fixing its details. HLL++'s
    small-range bias correction is an empirical table that is not part of the
    paper; this reading uses instead O. Ertl's table-free improved estimator
    ("New cardinality estimation algorithms for HyperLogLog sketches", 2017),
    which keeps the 1.04/sqrt(m) error over the whole range. With
    C_k = #{j : M[j] = k}, q = 64 - p (ranks run 0..q+1):

        n = alpha_inf m^2 / ( m sigma(C_0/m) + sum_{k=1..q} C_k 2^-k
                              + m tau(1 - C_{q+1}/m) 2^-q ),
        alpha_inf = 1 / (2 ln 2).

    All-empty registers give 0.
    """
    regs = np.asarray(regs, dtype=np.int64)
    m = regs.size
    p = int(round(math.log2(m)))
    q = 64 - p
    counts = [int(np.count_nonzero(regs == k)) for k in range(q + 2)]
    if counts[0] == m:
        return 0.0
    denom = m * _sigma(counts[0] / m)
    for k in range(1, q + 1):
        denom += counts[k] * 2.0 ** (-k)
    denom += m * _tau(1.0 - counts[q + 1] / m) * 2.0 ** (-q)
    return m * m / (2.0 * math.log(2.0)) / denom


def column_stats(keys, p: int = HLL_P) -> dict:
    """Statistics of a key column (Section 4: min, max and an HLL++ sketch of
    intermediate data). Empty columns give n = 0, min = max = 0, ndv = 0."""
    k = _as_i64(keys)
    regs = hll_registers(k, p)
    if k.size == 0:
        return {"n": 0, "min": 0, "max": 0, "regs": regs, "ndv": 0.0}
    return {"n": int(k.size), "min": int(k.min()), "max": int(k.max()), "regs": regs,
            "ndv": hll_estimate(regs)}


def _host(a) -> np.ndarray:
    """Host copy of a column (torch tensor or array), dtype kept."""
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a))


def join_wide(kR, colsR, kS, colsS, threads: int = 1):
    """Wide inner equi-join: the join result with every payload column of both
    relations materialized for each result pair (Section 5.2.1: the wide join,
    tables of a key and several payload columns whose payloads must be
    materialized; Section 3.2: GFUR and GFTR are two ways of producing this same
    result, from the untransformed or from the transformed relations).

    Plain definition: take the canonical pair list P of the inner equi-join
    (join_sortmerge), then output column c of R at result row t is colsR[c][i_t]
    and of S is colsS[c][j_t] for the t-th pair (i_t, j_t) of P, in the input
    column's dtype. Returns (pairs, outR, outS)."""
    pairs, _, _ = join_sortmerge(kR, kR, kS, kS, threads=threads)
    i = (pairs >> np.uint64(32)).astype(np.int64)
    j = (pairs & np.uint64(0xFFFFFFFF)).astype(np.int64)
    return pairs, [_host(c)[i] for c in colsR], [_host(c)[j] for c in colsS]


def group_by(keys, vals):
    """Group-by with a count and a sum per value column (Section 3.3 group-by
    operators; Section 4.1 / 5.3: the number of groups decides between the
    hash-based and the partition-based algorithm, both of which produce this
    result). Plain definition: the groups are the distinct key values; group k
    has count = #{i : keys[i] == k} and, for value column c,
    sum_c = sum over those rows of vals[c][i] (sign-extended, mod 2^64, as
    int64). Returns (group keys ascending as int64, counts int64, [sums int64])."""
    k = _as_i64(keys)
    if k.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), [np.zeros(0, np.int64) for _ in vals]
    uniq, inv = np.unique(k, return_inverse=True)
    counts = np.bincount(inv, minlength=uniq.size).astype(np.int64)
    sums = []
    for v in vals:
        acc = np.zeros(uniq.size, dtype=np.uint64)
        np.add.at(acc, inv, _as_i64(v).view(np.uint64))
        sums.append(acc.view(np.int64))
    return uniq, counts, sums


def canonical_pairs(build_rows, probe_rows) -> np.ndarray:
    """Pack (build_row, probe_row) into u64 (b << 32 | p) and sort ascending."""
    b = np.asarray(build_rows).astype(np.uint64)
    q = np.asarray(probe_rows).astype(np.uint64)
    return np.sort((b << np.uint64(32)) | q)
