"""Seeded synthetic inputs for the equi-join path (shared by tests, bench and smoke).

This module only draws input columns. It holds none of the join or statistics
arithmetic: no hashing of keys for tables or sketches, no matching, no
aggregation. Everything is integer-exact torch code that runs on whichever
device the caller names, and gives bit-identical columns on the CPU and on
the GPU (integer ops are exact; the one floating-point step, the Zipf CDF, is
built on the CPU and only compared against).

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style: value
number ``i`` of stream ``(seed, stream)`` is ``mix(base + (i + 1) * gamma)``.
The SplitMix64 output function ``mix`` is a bijection on 64-bit words, which
is also how unique keys are made without a uniqueness check.

The workload shapes follow the paper's join microbenchmarks (Section 5.2:
a smaller build side R, a larger probe side S, a match ratio = share of S
rows with a partner in R), and stand in for star-schema joins: a
dimension-like build side with unique or duplicated keys and a fact-like
probe side whose keys follow a uniform, sampled or Zipf distribution.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Reinterpret a Python int in [0, 2^64) as a signed 64-bit value."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


def _srl(z: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 words (torch's >> is arithmetic)."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function; a bijection of 64-bit words (wrapping int64)."""
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def _mix64_int(x: int) -> int:
    x &= (1 << 64) - 1
    x = ((x ^ (x >> 30)) * _M1) & ((1 << 64) - 1)
    x = ((x ^ (x >> 27)) * _M2) & ((1 << 64) - 1)
    return x ^ (x >> 31)


def _stream_base(seed: int, stream: int) -> int:
    return _mix64_int(_mix64_int(seed * 0x632BE59BD9B4E019 + 0x1234567) + stream * _GAMMA)


def rand64(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """64 random bits (as int64) for counters ``idx`` of stream ``(seed, stream)``."""
    base = _s64(_stream_base(seed, stream))
    return mix64(base + (idx + 1) * _s64(_GAMMA))


def uniform_below(r: torch.Tensor, n: int) -> torch.Tensor:
    """Map random words to [0, n) using their top 30 bits (n < 2^33)."""
    assert 0 < n < (1 << 33)
    return (_srl(r, 34) * n) >> 30


def uniform01(r: torch.Tensor) -> torch.Tensor:
    """Map random words to fp64 in [0, 1) using their top 53 bits (exact)."""
    return _srl(r, 11).to(torch.float64) * (2.0 ** -53)


def bij31(x: torch.Tensor, seed: int) -> torch.Tensor:
    """A keyed bijection of [0, 2^31): odd multiplies and xor-shifts mod 2^31."""
    m = (1 << 31) - 1
    k = _stream_base(seed, 7)
    x = (x + (k & m)) & m
    x = (x * (((k >> 31) & m) | 1)) & m
    x = x ^ (x >> 15)
    x = (x * 0x2C1B3C6D) & m
    x = x ^ (x >> 13)
    x = (x * 0x297A2D39) & m
    x = x ^ (x >> 16)
    return x


def permutation(seed: int, stream: int, n: int, device) -> torch.Tensor:
    """A seeded permutation of [0, n): argsort of n distinct random words."""
    idx = torch.arange(n, dtype=torch.int64, device=device)
    return torch.argsort(rand64(seed, stream, idx))


def geometric_table(q_num: int = 3, q_den: int = 4, kmax: int = 128) -> torch.Tensor:
    """T[k-1] = floor(q^k * 2^53), k = 1..kmax, with q = q_num/q_den, exact integers."""
    return torch.tensor([(q_num ** k << 53) // q_den ** k for k in range(1, kmax + 1)],
                        dtype=torch.int64)


def geometric(r: torch.Tensor, table: torch.Tensor) -> torch.Tensor:
    """Geometric draw on {1, 2, ...} with P(d > k) = q^k (truncated at len(table)+1).

    d = 1 + #{k : u53 < floor(q^k 2^53)}; the table is decreasing, so this is a
    count of thresholds above u53 done with searchsorted on the reversed table.
    """
    u = _srl(r, 11)
    asc = torch.flip(table, [0]).to(u.device)
    return 1 + (asc.numel() - torch.searchsorted(asc, u, right=True))


def zipf_cdf(n: int, s: float) -> torch.Tensor:
    """CDF over ranks 1..n with weights r^-s, fp64, summed in rank order on the CPU."""
    w = torch.arange(1, n + 1, dtype=torch.float64).pow(-s)
    c = torch.cumsum(w, 0)
    return c / c[-1]


def zipf_ranks(r: torch.Tensor, cdf: torch.Tensor) -> torch.Tensor:
    """0-based ranks: the first index whose CDF value exceeds a uniform draw."""
    u = uniform01(r)
    idx = torch.searchsorted(cdf.to(u.device), u, right=True)
    return torch.clamp(idx, max=cdf.numel() - 1)


@dataclass
class JoinInput:
    """One equi-join instance: build side R and probe side S, as device tensors."""
    name: str
    build_keys: torch.Tensor
    build_payload: torch.Tensor
    probe_keys: torch.Tensor
    probe_payload: torch.Tensor
    meta: dict = field(default_factory=dict)

    @property
    def n_build(self) -> int:
        return int(self.build_keys.numel())

    @property
    def n_probe(self) -> int:
        return int(self.probe_keys.numel())


def plain_dense(seed: int = 42, n_build: int = 65536, n_probe: int = 1 << 20,
                probe_range: int = 81920, device="cpu") -> JoinInput:
    """Plain join: unique int32 build keys = a shuffle of [0, n_build), payload
    U[0, 1000); probe keys U[0, probe_range) (about n_build/probe_range match),
    payload U[0, 1000). Defaults are the 65,536 x 1,048,576 instance."""
    dev = torch.device(device)
    perm = permutation(seed, 1, n_build, dev)
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)
    return JoinInput(
        name=f"plain_dense_{n_build}x{n_probe}",
        build_keys=perm.to(torch.int32),
        build_payload=uniform_below(rand64(seed, 2, ib), 1000).to(torch.int32),
        probe_keys=uniform_below(rand64(seed, 3, ip), probe_range).to(torch.int32),
        probe_payload=uniform_below(rand64(seed, 4, ip), 1000).to(torch.int32),
        meta={"seed": seed, "probe_range": probe_range},
    )


def wide_join(seed: int = 42, n_build: int = 1 << 16, n_probe: int = 1 << 28, match_per_mille: int = 1000,
              n_cols: int = 3, key_dtype=torch.int32, col_dtype=torch.int32, device="cpu") -> JoinInput:
    """Wide join (the paper's Section 5.2 wide-join and match-ratio workloads:
    tables of a key and three payload columns, a smaller build side R with
    unique keys and a larger probe side S). Build keys = a shuffle of
    [0, n_build) spread by a factor 2 (key = 2 * index, so odd keys never
    match); a probe row matches with probability match_per_mille / 1000 and then
    copies a uniformly drawn build key, otherwise it takes an odd key. Payload
    columns: n_cols per side, uniform over the column dtype's full range.
    meta["build_cols"] / meta["probe_cols"] hold the payload columns
    (build_payload / probe_payload are the first of them)."""
    dev = torch.device(device)
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)
    bk = 2 * permutation(seed, 1, n_build, dev)
    hit = uniform_below(rand64(seed, 2, ip), 1000) < match_per_mille
    src = uniform_below(rand64(seed, 3, ip), max(n_build, 1))
    miss = 2 * uniform_below(rand64(seed, 4, ip), 1 << 30) + 1
    pk = torch.where(hit, bk[src] if n_build else miss, miss)

    def col(stream, idx):
        r = rand64(seed, stream, idx)
        return r if col_dtype == torch.int64 else (r >> 32).to(torch.int32)

    bcols = [col(10 + c, ib) for c in range(n_cols)]
    pcols = [col(20 + c, ip) for c in range(n_cols)]
    return JoinInput(name=f"wide_{n_build}x{n_probe}_m{match_per_mille}", build_keys=bk.to(key_dtype),
                     build_payload=bcols[0] if n_cols else bk.to(col_dtype), probe_keys=pk.to(key_dtype),
                     probe_payload=pcols[0] if n_cols else pk.to(col_dtype),
                     meta={"build_cols": bcols, "probe_cols": pcols, "match_per_mille": match_per_mille})


def groupby_input(seed: int = 42, n: int = 1 << 28, groups: int = 1 << 10, key_dtype=torch.int32,
                  n_vals: int = 2, val_dtype=torch.int32, device="cpu"):
    """Group-by input (the paper's group-by microbenchmarks, Section 5.3: a key
    column with g groups and two aggregated columns): each row's key is one of
    `groups` distinct values, drawn uniformly; the distinct values are spread
    over the key type's positive range (a keyed bijection of [0, groups) for
    int32, SplitMix64 outputs for int64). Value columns uniform over the value
    type's full range. Returns (keys, [value columns])."""
    dev = torch.device(device)
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    gid = uniform_below(rand64(seed, 1, idx), max(groups, 1))
    if key_dtype == torch.int32:
        bits = max(1, min(31, (max(groups, 2) - 1).bit_length()))
        keys = (bij_bits(gid, bits, seed) << (31 - bits)).to(torch.int32)
    else:
        keys = mix64(gid + _stream_base(seed, 2))
    vals = []
    for c in range(n_vals):
        r = rand64(seed, 10 + c, idx)
        vals.append(r if val_dtype == torch.int64 else (r >> 32).to(torch.int32))
    return keys, vals


def sparse_unique64(seed: int = 42, n_build: int = 1 << 24, n_probe: int = 1 << 29,
                    match_per_mille: int = 900, device="cpu") -> JoinInput:
    """Large sparse join: unique int64 build keys spread over the full 64-bit range,
    int64 payloads over the full range; each probe row takes, with probability
    match_per_mille/1000, the key of a uniformly drawn build row (recorded in
    meta['source_row'], -1 for no partner), else a key that no build row has.

    Build keys are mix64(i + offset) for i < n_build and non-matching probe keys
    are mix64(offset + n_build + j): distinct arguments of a bijection, so build
    keys are unique and non-matching keys are absent from the build side.
    """
    dev = torch.device(device)
    off = _s64(_stream_base(seed, 10))
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)
    bk = mix64(ib + off)
    bp = rand64(seed, 11, ib)
    r_sel = rand64(seed, 12, ip)
    hit = uniform_below(r_sel, 1000) < match_per_mille
    src = uniform_below(rand64(seed, 13, ip), n_build)
    miss_keys = mix64(ip + (off + n_build))
    pk = torch.where(hit, bk[src], miss_keys)
    src = torch.where(hit, src, torch.full_like(src, -1))
    del miss_keys, r_sel
    pp = rand64(seed, 14, ip)
    return JoinInput(
        name=f"sparse_unique64_{n_build}x{n_probe}",
        build_keys=bk, build_payload=bp, probe_keys=pk, probe_payload=pp,
        meta={"seed": seed, "source_row": src, "match_per_mille": match_per_mille},
    )


def skewed_dup32(seed: int = 42, n_distinct: int = 1 << 24, n_probe: int = 1 << 28,
                 zipf_s: float = 1.0, device="cpu") -> JoinInput:
    """Skewed many-to-many join: n_distinct int32 keys drawn without replacement
    from [0, 2^31) (a keyed bijection of 0..n_distinct-1); each key repeated a
    Geometric(mean 4) number of times (P(d > k) = (3/4)^k), rows shuffled;
    probe keys = key[perm[rank]] with rank ~ Zipf(zipf_s) over 1..n_distinct;
    payloads U[0, 1000) int32 on both sides."""
    dev = torch.device(device)
    iv = torch.arange(n_distinct, dtype=torch.int64, device=dev)
    distinct = bij31(iv, seed)
    dup = geometric(rand64(seed, 20, iv), geometric_table())
    keys = torch.repeat_interleave(distinct, dup)
    n_build = int(keys.numel())
    keys = keys[permutation(seed, 21, n_build, dev)]
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)
    cdf = zipf_cdf(n_distinct, zipf_s)
    rank = zipf_ranks(rand64(seed, 22, ip), cdf)
    rank_to_key = permutation(seed, 23, n_distinct, dev)
    pk = distinct[rank_to_key[rank]]
    return JoinInput(
        name=f"skewed_dup32_s{zipf_s}_{n_build}x{n_probe}",
        build_keys=keys.to(torch.int32),
        build_payload=uniform_below(rand64(seed, 24, ib), 1000).to(torch.int32),
        probe_keys=pk.to(torch.int32),
        probe_payload=uniform_below(rand64(seed, 25, ip), 1000).to(torch.int32),
        meta={"seed": seed, "zipf_s": zipf_s, "n_distinct": n_distinct},
    )


def random_small(seed: int, n_build: int, n_probe: int, key_lo: int, key_hi: int,
                 dtype=torch.int32, payload_dtype=torch.int32, device="cpu") -> JoinInput:
    """Small adversarial instance: keys uniform over [key_lo, key_hi] (inclusive,
    so duplicates appear when the range is narrow), payloads over the payload
    type's full range."""
    dev = torch.device(device)
    span = key_hi - key_lo + 1
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)

    def keys(stream, idx):
        r = rand64(seed, stream, idx)
        if span >= (1 << 64):
            return r
        if span < (1 << 33):
            return key_lo + uniform_below(r, span)
        # wide spans: modulo is fine for adversarial tests (slight bias only)
        return key_lo + torch.remainder(_srl(r, 1), span)

    def pay(stream, idx):
        r = rand64(seed, stream, idx)
        if payload_dtype == torch.int32:
            return (r >> 32).to(torch.int32)
        return r

    return JoinInput(
        name=f"random_small_{n_build}x{n_probe}_[{key_lo},{key_hi}]",
        build_keys=keys(30, ib).to(dtype), build_payload=pay(31, ib),
        probe_keys=keys(32, ip).to(dtype), probe_payload=pay(33, ip),
        meta={"seed": seed},
    )


def distinct_values(seed: int, n_distinct: int, n_rows: int, device="cpu") -> torch.Tensor:
    """int64 column of n_rows whose values are exactly n_distinct distinct words
    (every value appears at least once when n_rows >= n_distinct); used for
    sketch accuracy tests where the true distinct count must be known."""
    dev = torch.device(device)
    off = _s64(_stream_base(seed, 40))
    vals = mix64(torch.arange(n_distinct, dtype=torch.int64, device=dev) + off)
    if n_rows <= n_distinct:
        return vals[:n_rows]
    extra = uniform_below(rand64(seed, 41, torch.arange(n_rows - n_distinct, dtype=torch.int64,
                                                             device=dev)), n_distinct)
    return torch.cat([vals, vals[extra]])


def config_names():
    return ["plain_dense", "sparse_unique64", "skewed_dup32"]


__all__ = [
    "JoinInput", "mix64", "rand64", "uniform_below", "uniform01", "bij31", "permutation",
    "geometric", "geometric_table", "zipf_cdf", "zipf_ranks", "plain_dense",
    "sparse_unique64", "skewed_dup32", "random_small", "distinct_values",
]

# sanity: the 2^53 scaling of the geometric table matches uniform01's resolution
assert math.isclose(2.0 ** -53 * (1 << 53), 1.0)


# ---------------------------------------------------------------------------
# Instances for the learned variant selector: a spread of build sizes, key
# widths, key densities, duplicate factors, probe skew and selectivity.

def _u01(seed, stream, idx):
    return float(uniform01(rand64(seed, stream, torch.tensor([idx], dtype=torch.int64)))[0])


def selector_params(seed: int, idx: int, max_build_log2: float = 22.0, max_probe_log2: float = 25.0,
                    family: int = 1, min_build_log2: float = 10.0) -> dict:
    """Draw the shape of instance `idx`.

    Family 1: build rows 2^U(min_build_log2, max_build_log2), key width
    int32/int64, density (distinct/range) 10^U(-6, 0), duplicate factor 1 (40%)
    or U{2..16}, probe Zipf exponent U[0, 1.5], selectivity U[0.01, 1], probe
    rows = build rows * 2^U(0, 4) capped at 2^max_probe_log2; rows that miss take
    keys above the build range.

    Family 2 widens what family 1 leaves out: probe rows = build rows * 2^U(0, 5);
    half of the instances put missing keys into the gaps between build keys (so
    the probe range equals the build range) instead of above it; and 40% of the
    int64 instances spread their keys over the whole 64-bit range.

    Family 3 is family 2 with probe rows = build rows * 2^U(0, 6), meant for the
    largest builds (the caller passes the size bounds)."""
    u = [_u01(seed, 200 + k, idx) for k in range(8)]
    n_build = int(round(2.0 ** (min_build_log2 + u[0] * (max_build_log2 - min_build_log2))))
    wide = u[1] < 0.5
    density = 10.0 ** (-6.0 * u[2])
    dup = 1 if u[3] < 0.4 else 2 + int(u[3] * 1e6) % 15
    zipf_s = 1.5 * u[4]
    selectivity = 0.01 + 0.99 * u[5]
    mult_log2 = {1: 4.0, 2: 5.0, 3: 6.0}[family]
    n_probe = int(min(round(n_build * 2.0 ** (mult_log2 * u[6])), 2 ** max_probe_log2))
    pr = {"n_build": n_build, "wide": wide, "density": density, "dup": dup, "zipf_s": zipf_s,
          "selectivity": selectivity, "n_probe": n_probe}
    if family != 1:
        u8 = _u01(seed, 208, idx)
        pr["family"] = family
        pr["layout"] = "full64" if (wide and u8 < 0.4) else "spread"
        pr["miss"] = "inside" if (pr["layout"] == "full64" or u[7] >= 0.5) else "above"
    return pr


def selector_instance(seed: int, idx: int, device="cpu", **kw) -> JoinInput:
    """Build instance `idx` of the selector workload (see selector_params).

    Layout "spread" (family 1 always): distinct build keys are
    base + i*step + jitter_i with jitter_i in [0, step) (strictly increasing, so
    distinct, spread over the chosen range). Layout "full64": distinct build
    keys are mix64(c + i), a bijection, so they are distinct and spread over
    all 64-bit values. Each distinct key is repeated U{1..2*dup-1} times. Probe
    rows take a build key with probability `selectivity` (rank drawn Zipf(s)
    over the distinct keys through a random rank->key map), else a key that no
    build row holds: above the build range ("above"), inside one of its gaps
    (offset != jitter_i in the i-th step, "inside"), or mix64(c + n_distinct + j)
    for the full64 layout."""
    pr = selector_params(seed, idx, **kw)
    dev = torch.device(device)
    dtype = torch.int64 if pr["wide"] else torch.int32
    n_distinct = max(1, pr["n_build"] // pr["dup"])
    sid = seed * 7919 + idx
    iv = torch.arange(n_distinct, dtype=torch.int64, device=dev)
    layout = pr.get("layout", "spread")
    if layout == "full64":
        c = _s64(_stream_base(sid, 10))
        distinct = mix64(iv + c)
        step, base, rng_len = 0, 0, 0
    else:
        max_range = (1 << 61) if pr["wide"] else (1 << 30)
        rng_len = int(min(max_range, max(n_distinct, round(n_distinct / pr["density"]))))
        step = max(1, rng_len // n_distinct)
        rng_len = step * n_distinct
        base = -(rng_len // 2)
        jitter = torch.remainder(_srl(rand64(sid, 1, iv), 1), step) if step > 1 else torch.zeros_like(iv)
        distinct = base + iv * step + jitter
    if pr["dup"] > 1:
        counts = 1 + uniform_below(rand64(sid, 2, iv), 2 * pr["dup"] - 1)
        keys = torch.repeat_interleave(distinct, counts)
    else:
        keys = distinct
    n_build = int(keys.numel())
    keys = keys[permutation(sid, 3, n_build, dev)]
    ib = torch.arange(n_build, dtype=torch.int64, device=dev)
    ip = torch.arange(pr["n_probe"], dtype=torch.int64, device=dev)
    hit = uniform01(rand64(sid, 4, ip)) < pr["selectivity"]
    if pr["zipf_s"] > 0.05 and n_distinct > 1:
        rank = zipf_ranks(rand64(sid, 5, ip), zipf_cdf(n_distinct, pr["zipf_s"]))
    else:
        rank = uniform_below(rand64(sid, 5, ip), n_distinct)
    rank_to_key = permutation(sid, 6, n_distinct, dev)
    r7 = rand64(sid, 7, ip)
    miss_mode = pr.get("miss", "above")
    if layout == "full64":
        miss = mix64(c + n_distinct + _srl(r7, 24))
    elif miss_mode == "inside" and step > 1:
        slot = uniform_below(r7, n_distinct)
        jit = jitter[slot]
        off = torch.remainder(jit + 1 + torch.remainder(_srl(rand64(sid, 11, ip), 1), step - 1), step)
        miss = base + slot * step + off
    else:
        miss = base + rng_len + torch.remainder(_srl(r7, 1), rng_len)
    pk = torch.where(hit, distinct[rank_to_key[rank]], miss)
    pay_b = rand64(sid, 8, ib)
    pay_p = rand64(sid, 9, ip)
    if dtype == torch.int32:
        pay_b, pay_p = (pay_b >> 40).to(torch.int32), (pay_p >> 40).to(torch.int32)
    return JoinInput(name=f"selector_{seed}_{idx}", build_keys=keys.to(dtype), build_payload=pay_b,
                     probe_keys=pk.to(dtype), probe_payload=pay_p, meta={"params": pr})


def bij_bits(x: torch.Tensor, bits: int, seed: int) -> torch.Tensor:
    """A keyed bijection of [0, 2^bits) (bits <= 31): add, odd multiply and
    xor-shift steps, each invertible mod 2^bits."""
    m = (1 << bits) - 1
    k = _stream_base(seed, 8)
    x = (x + (k & m)) & m
    x = (x * (((k >> 32) & m) | 1)) & m
    x = x ^ (x >> (bits // 2))
    x = (x * 0x2C1B3C6D) & m
    x = x ^ (x >> (bits // 3 + 1))
    return x


def batched_join_params(seed: int, j: int, log2_lo: float = 8.0, log2_hi: float = 18.0):
    """Sizes of join j of a batch without drawing it: (build rows, probe rows,
    match rate, dense). Build rows round(2^U(log2_lo, log2_hi)); probe rows =
    build rows * U[4, 16]; match rate U[0.1, 1]; even joins dense."""
    u = [_u01(seed, 500 + k, j) for k in range(4)]
    nb = int(round(2.0 ** (log2_lo + u[0] * (log2_hi - log2_lo))))
    npr = int(round(nb * (4.0 + 12.0 * u[1])))
    m = 0.1 + 0.9 * u[2]
    return nb, npr, m, j % 2 == 0


def batched_join(seed: int, j: int, log2_lo: float = 8.0, log2_hi: float = 18.0, device="cpu") -> JoinInput:
    """Join j of a batch of independent unique-key int32 joins of uneven sizes
    (sizes from batched_join_params). Dense joins: build keys = a shuffle of
    [b, b + n) and probe keys U[b, b + n/m). Sparse joins: build keys =
    2 * (a keyed bijection of their indices on [0, 2^30)), matching probe rows
    copy a uniformly drawn build key, the others take odd keys 2v + 1. Payloads
    U[0, 1000). Each join depends only on (seed, j), so a batch can be drawn
    in any order or in parts."""
    dev = torch.device(device)
    nb, npr, m, dense = batched_join_params(seed, j, log2_lo, log2_hi)
    u3 = _u01(seed, 503, j)
    js = seed * 1000003 + j
    ib = torch.arange(nb, dtype=torch.int64, device=dev)
    ip = torch.arange(npr, dtype=torch.int64, device=dev)
    if dense:
        b = int(u3 * (1 << 29))
        bk = b + permutation(js, 1, nb, dev)
        span = max(1, int(round(nb / m)))
        pk = b + uniform_below(rand64(js, 2, ip), span)
    else:
        bk = 2 * bij_bits(ib, 30, js)
        hit = uniform01(rand64(js, 3, ip)) < m
        src = uniform_below(rand64(js, 4, ip), nb)
        miss = 2 * uniform_below(rand64(js, 5, ip), 1 << 30) + 1
        pk = torch.where(hit, bk[src], miss)
    return JoinInput(name=f"batch_{j}", build_keys=bk.to(torch.int32),
                     build_payload=uniform_below(rand64(js, 6, ib), 1000).to(torch.int32),
                     probe_keys=pk.to(torch.int32),
                     probe_payload=uniform_below(rand64(js, 7, ip), 1000).to(torch.int32),
                     meta={"dense": dense, "match": m})


def batched_joins(seed: int, n_joins: int, log2_lo: float = 8.0, log2_hi: float = 18.0, device="cpu"):
    """Joins 0 .. n_joins-1 of a batch (batched_join). Returns a list of JoinInput."""
    return [batched_join(seed, j, log2_lo, log2_hi, device) for j in range(n_joins)]


def multikey_table(seed: int = 42, n: int = 1 << 28, n_keys: int = 4, dtype=torch.int32, narrow_bits: int = 8,
                   sparse_ndv: int = 256, device="cpu", stream0: int = 60):
    """Key columns of the paper's multi-key sort (Section 5.6): half of the keys
    have a narrow value range (even positions: base + uniform [0, 2^narrow_bits),
    base drawn per key), the other half a sparse spread of few distinct values
    (odd positions: one of `sparse_ndv` distinct values spread over the type's
    whole range, drawn uniformly per row). Returns a list of `n_keys` columns."""
    dev = torch.device(device)
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    top = 31 if dtype == torch.int32 else 62
    cols = []
    for c in range(n_keys):
        r = rand64(seed, stream0 + c, idx)
        if c % 2 == 0:
            base = (_stream_base(seed, stream0 + 20 + c) >> 8) % ((1 << top) - (1 << narrow_bits))
            base -= 1 << (top - 1)
            col = base + uniform_below(r, 1 << narrow_bits)
        else:
            d = torch.arange(sparse_ndv, dtype=torch.int64, device=dev)
            if dtype == torch.int32:
                vals = bij31(d, seed + c) * 2 - (1 << 31)
            else:
                vals = mix64(d + _s64(_stream_base(seed, stream0 + 40 + c)))
            col = vals[uniform_below(r, sparse_ndv)]
        cols.append(col.to(dtype))
    return cols


def multikey_join(seed: int = 42, n_build: int = 1 << 16, n_probe: int = 1 << 20, n_keys: int = 2,
                  dtype=torch.int32, narrow_bits: int = 8, sparse_ndv: int = 256, match_per_mille: int = 500,
                  device="cpu"):
    """Two relations joined on `n_keys` key columns drawn like multikey_table:
    each probe row copies the key tuple of a uniformly drawn build row with
    probability match_per_mille/1000, else draws a fresh tuple from the same
    distribution (which may or may not occur in the build side). Returns
    (build key columns, probe key columns)."""
    dev = torch.device(device)
    R = multikey_table(seed, n_build, n_keys, dtype, narrow_bits, sparse_ndv, device, stream0=60)
    fresh = multikey_table(seed, n_probe, n_keys, dtype, narrow_bits, sparse_ndv, device, stream0=90)
    ip = torch.arange(n_probe, dtype=torch.int64, device=dev)
    take = uniform_below(rand64(seed, 120, ip), 1000) < match_per_mille
    src = uniform_below(rand64(seed, 121, ip), max(n_build, 1))
    S = [torch.where(take, r[src] if n_build else f, f) for r, f in zip(R, fresh)]
    return R, S
