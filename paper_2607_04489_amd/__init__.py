"""Python binding of the gfx950 equi-join library (libeiger.so).

Argument marshalling only: every step of the join path runs in the library's
HIP kernels. Torch supplies device memory (inputs, outputs, workspace) and the
stream. The names follow the C ABI in include/eiger.h:

    stats(keys)                          -> Stats        (eiger_stats)
    join_plan(build_stats, probe_stats)  -> Plan         (eiger_join_plan)
    join(bk, bp, pk, pp, plan)           -> JoinResult   (eiger_join)

There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeiger.so")

EIGER_OK = 0
EIGER_ERR_INVALID_ARG = -1
EIGER_ERR_DTYPE = -2
EIGER_ERR_TOO_LARGE = -3
EIGER_ERR_CAPACITY = -4
EIGER_ERR_WORKSPACE = -5
EIGER_ERR_HIP = -6
EIGER_ERR_UNSUPPORTED = -7
EIGER_ERR_MODEL = -8

INT32, INT64 = 0, 1
DIRECT, GLOBAL_HASH, RADIX, RADIX_CACHE = 0, 1, 2, 3
VARIANT_NAMES = {DIRECT: "direct", GLOBAL_HASH: "global_hash", RADIX: "radix", RADIX_CACHE: "radix_cache"}
SEL_RULE, SEL_LEARNED, SEL_FIXED_HASH, SEL_FORCED = 0, 1, 2, 3
HLL_P = 14


class EigerError(RuntimeError):
    def __init__(self, code: int, msg: str, count: Optional[int] = None):
        super().__init__(f"eiger error {code}: {msg}")
        self.code = code
        self.count = count


class Column(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class StatsT(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("min", ctypes.c_int64), ("max", ctypes.c_int64),
                ("ndv", ctypes.c_double), ("dtype", ctypes.c_int32), ("hll_p", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class PlanT(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("radix_bits", ctypes.c_int32),
                ("radix_passes", ctypes.c_int32), ("key_dtype", ctypes.c_int32),
                ("load_factor", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("build_min", ctypes.c_int64), ("build_max", ctypes.c_int64),
                ("predicted_out", ctypes.c_int64), ("reserved", ctypes.c_int64 * 4)]

    def describe(self) -> dict:
        d = {"variant": VARIANT_NAMES.get(self.variant, str(self.variant)),
             "predicted_out": int(self.predicted_out)}
        if self.variant != DIRECT:
            d["load_factor"] = round(float(self.load_factor), 3)
        if self.variant in (RADIX, RADIX_CACHE):
            d["radix_bits"] = int(self.radix_bits)
        if self.variant == RADIX:
            d["radix_passes"] = int(self.radix_passes)
        return d


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = None


def available() -> bool:
    return os.path.exists(LIB_PATH)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2607_04489_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.eiger_stats_workspace_size.argtypes = [i64, i32]
        L.eiger_stats_workspace_size.restype = sz
        L.eiger_stats.argtypes = [Column, ctypes.POINTER(StatsT), vp, vp, sz, vp]
        L.eiger_stats.restype = ctypes.c_int
        L.eiger_join_plan.argtypes = [ctypes.POINTER(StatsT), ctypes.POINTER(StatsT), i32,
                                      ctypes.POINTER(PlanT), ctypes.POINTER(PlanT)]
        L.eiger_join_plan.restype = ctypes.c_int
        L.eiger_join_workspace_size.argtypes = [ctypes.POINTER(PlanT), Column, Column, Column, Column,
                                                ctypes.POINTER(sz)]
        L.eiger_join_workspace_size.restype = ctypes.c_int
        L.eiger_join.argtypes = [Column, Column, Column, Column, ctypes.POINTER(PlanT), vp, vp, i64,
                                 ctypes.POINTER(i64), ctypes.POINTER(i64), vp, sz, vp]
        L.eiger_join.restype = ctypes.c_int
        L.eiger_last_error.argtypes = []
        L.eiger_last_error.restype = ctypes.c_char_p
        L.eiger_version.restype = ctypes.c_int
        L.eiger_profile_enable.argtypes = [ctypes.c_int]
        L.eiger_profile_enable.restype = ctypes.c_int
        L.eiger_profile_read.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
        L.eiger_profile_read.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, count: Optional[int] = None):
    if rc != EIGER_OK:
        raise EigerError(rc, lib().eiger_last_error().decode(), count)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.int32:
        return INT32
    if t.dtype == torch.int64:
        return INT64
    raise EigerError(EIGER_ERR_DTYPE, f"unsupported dtype {t.dtype}")


def column(t) -> Column:
    """Describe a contiguous 1-D int32/int64 torch tensor (device memory) as an eiger_column."""
    if t.dim() != 1 or not t.is_contiguous():
        raise EigerError(EIGER_ERR_INVALID_ARG, "columns must be contiguous 1-D tensors")
    return Column(t.data_ptr() if t.numel() else None, t.numel(), _dtype_code(t), 0)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Stats:
    raw: StatsT
    regs: object  # torch.uint8 tensor on the host, 2^14 registers

    @property
    def n(self):
        return int(self.raw.n)

    @property
    def min(self):
        return int(self.raw.min)

    @property
    def max(self):
        return int(self.raw.max)

    @property
    def ndv(self):
        return float(self.raw.ndv)


def stats(keys, stream=None, workspace=None) -> Stats:
    """eiger_stats: count, min, max and distinct estimate of a device key column."""
    import torch
    col = column(keys)
    need = lib().eiger_stats_workspace_size(col.n, col.dtype)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, keys.device)
    out = StatsT()
    regs = torch.zeros(1 << HLL_P, dtype=torch.uint8)
    _check(lib().eiger_stats(col, ctypes.byref(out), ctypes.c_void_p(regs.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return Stats(out, regs)


def join_plan(build: Stats, probe: Stats, selector: int = SEL_RULE,
              forced: Optional[PlanT] = None) -> PlanT:
    """eiger_join_plan: variant and knobs from the two sides' statistics."""
    out = PlanT()
    _check(lib().eiger_join_plan(ctypes.byref(build.raw), ctypes.byref(probe.raw), selector,
                                 ctypes.byref(forced) if forced is not None else None,
                                 ctypes.byref(out)))
    return out


def make_plan(variant: int, radix_bits: int = 0, radix_passes: int = 0,
              load_factor: float = 0.5) -> PlanT:
    """A `forced` plan for join_plan(..., SEL_FORCED, forced)."""
    p = PlanT()
    p.variant, p.radix_bits, p.radix_passes, p.load_factor = variant, radix_bits, radix_passes, load_factor
    return p


def join_workspace_size(plan: PlanT, bk, bp, pk, pp) -> int:
    n = ctypes.c_size_t()
    _check(lib().eiger_join_workspace_size(ctypes.byref(plan), column(bk), column(bp), column(pk),
                                           column(pp), ctypes.byref(n)))
    return int(n.value)


@dataclass
class JoinResult:
    build_rowid: object  # torch.int32 tensor holding uint32 row ids, length count
    probe_rowid: object
    count: int
    checksum: int


def join(bk, bp, pk, pp, plan: PlanT, capacity: Optional[int] = None, stream=None,
         workspace=None, outputs=None, count_only: bool = False) -> JoinResult:
    """eiger_join. Output arrays are allocated here (capacity defaults to the plan's
    predicted size with headroom, at least the probe row count) unless `outputs`
    = (out_b, out_p) is given. When the result does not fit, the call is repeated
    once with the exact count the library reports."""
    import torch
    cols = [column(t) for t in (bk, bp, pk, pp)]
    need = ctypes.c_size_t()
    _check(lib().eiger_join_workspace_size(ctypes.byref(plan), *cols, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, pk.device)
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()

    def run(ob, op, cap):
        return lib().eiger_join(*cols, ctypes.byref(plan),
                                ctypes.c_void_p(ob.data_ptr()) if ob is not None else None,
                                ctypes.c_void_p(op.data_ptr()) if op is not None else None,
                                cap, ctypes.byref(cnt), ctypes.byref(cs),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))

    if count_only:
        _check(run(None, None, 0))
        return JoinResult(None, None, cnt.value, cs.value)
    if outputs is not None:
        ob, op = outputs
        rc = run(ob, op, min(ob.numel(), op.numel()))
        _check(rc, cnt.value)
        return JoinResult(ob[: cnt.value], op[: cnt.value], cnt.value, cs.value)
    if capacity is None:
        capacity = max(int(plan.predicted_out * 1.25) + 1024, pk.numel())
    ob = torch.empty(capacity, dtype=torch.int32, device=pk.device)
    op = torch.empty(capacity, dtype=torch.int32, device=pk.device)
    rc = run(ob, op, capacity)
    if rc == EIGER_ERR_CAPACITY:
        capacity = cnt.value
        del ob, op
        ob = torch.empty(capacity, dtype=torch.int32, device=pk.device)
        op = torch.empty(capacity, dtype=torch.int32, device=pk.device)
        rc = run(ob, op, capacity)
    _check(rc, cnt.value)
    return JoinResult(ob[: cnt.value], op[: cnt.value], cnt.value, cs.value)


def profile_enable(on: bool = True):
    _check(lib().eiger_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel name: (launches, total_ms)} since profiling was enabled."""
    rows = (KernelTime * 256)()
    n = ctypes.c_int()
    _check(lib().eiger_profile_read(rows, 256, ctypes.byref(n)))
    return {rows[i].name.decode(): (int(rows[i].launches), float(rows[i].total_ms))
            for i in range(min(n.value, 256))}


def version() -> int:
    return int(lib().eiger_version())
