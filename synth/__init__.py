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
rows with a partner in R) and the star-schema stand-ins listed in the design doc.
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
