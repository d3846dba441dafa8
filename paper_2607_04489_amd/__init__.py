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
DIRECT, GLOBAL_HASH, RADIX, RADIX_CACHE, SORT_MERGE = 0, 1, 2, 3, 4
VARIANT_NAMES = {DIRECT: "direct", GLOBAL_HASH: "global_hash", RADIX: "radix", RADIX_CACHE: "radix_cache",
                 SORT_MERGE: "sort_merge"}
SEL_RULE, SEL_LEARNED, SEL_FIXED_HASH, SEL_FORCED = 0, 1, 2, 3
PLAN_RULE_FALLBACK = 1
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
        if self.flags & PLAN_RULE_FALLBACK:
            d["rule_fallback"] = True
        return d


class GroupByPlanT(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("radix_bits", ctypes.c_int32), ("key_dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("slots", ctypes.c_int64), ("predicted_groups", ctypes.c_int64),
                ("sentinel", ctypes.c_int64), ("reserved", ctypes.c_int64 * 2)]

    def describe(self) -> dict:
        d = {"variant": GB_NAMES.get(self.variant, str(self.variant)), "slots": int(self.slots),
             "predicted_groups": int(self.predicted_groups)}
        if self.variant == GB_PARTITION:
            d["radix_bits"] = int(self.radix_bits)
        return d


GB_HASH, GB_PARTITION = 0, 1


class SkfKeyT(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("bits", ctypes.c_int32), ("shift", ctypes.c_int32),
                ("descending", ctypes.c_int32), ("base", ctypes.c_int64), ("ndv", ctypes.c_int64),
                ("slots", ctypes.c_int64), ("dtype", ctypes.c_int32), ("range_bits", ctypes.c_int32)]


SKF_MAX_KEYS = 8
SKF_FOR, SKF_DICT = 0, 1
SKF_FOR_MAX_BITS = 16
SKF_DICT_MAX_NDV = 1 << 20


class SkfPlanT(ctypes.Structure):
    _fields_ = [("n_keys", ctypes.c_int32), ("total_bits", ctypes.c_int32), ("fused_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("key", SkfKeyT * SKF_MAX_KEYS)]

    def describe(self) -> dict:
        return {"total_bits": int(self.total_bits), "fused_bytes": int(self.fused_bytes),
                "keys": [{"code": "dict" if k.code == SKF_DICT else "for", "bits": int(k.bits),
                          "shift": int(k.shift), "descending": bool(k.descending), "base": int(k.base),
                          "ndv": int(k.ndv), "slots": int(k.slots)}
                         for k in self.key[: self.n_keys]]}
GB_NAMES = {GB_HASH: "hash", GB_PARTITION: "partition"}


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
        L.eiger_join_wide_workspace_size.argtypes = [ctypes.POINTER(PlanT), i32, Column, vp, i32, Column, vp, i32,
                                                     ctypes.POINTER(sz)]
        L.eiger_join_wide_workspace_size.restype = ctypes.c_int
        L.eiger_join_wide.argtypes = [Column, vp, i32, Column, vp, i32, ctypes.POINTER(PlanT), i32, vp, vp, vp, vp,
                                      i64, ctypes.POINTER(i64), ctypes.POINTER(i32), vp, sz, vp]
        L.eiger_join_wide.restype = ctypes.c_int
        L.eiger_calibrate.argtypes = [i32, vp, vp, i64, i64, ctypes.POINTER(ctypes.c_double), vp]
        L.eiger_calibrate.restype = ctypes.c_int
        L.eiger_groupby_plan.argtypes = [ctypes.POINTER(StatsT), i32, ctypes.POINTER(GroupByPlanT),
                                         ctypes.POINTER(GroupByPlanT)]
        L.eiger_groupby_plan.restype = ctypes.c_int
        L.eiger_groupby_workspace_size.argtypes = [ctypes.POINTER(GroupByPlanT), Column, vp, i32, ctypes.POINTER(sz)]
        L.eiger_groupby_workspace_size.restype = ctypes.c_int
        L.eiger_groupby.argtypes = [Column, vp, i32, ctypes.POINTER(GroupByPlanT), vp, vp, vp, i64,
                                    ctypes.POINTER(i64), vp, sz, vp]
        L.eiger_groupby.restype = ctypes.c_int
        L.eiger_join_noalloc.argtypes = [Column, Column, Column, Column, ctypes.POINTER(PlanT), vp, vp, i64,
                                         ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
        L.eiger_join_noalloc.restype = ctypes.c_int
        psk = ctypes.POINTER(SkfPlanT)
        L.eiger_sort_pairs_workspace_size.argtypes = [i32, i64, i32, ctypes.POINTER(sz)]
        L.eiger_sort_pairs_workspace_size.restype = ctypes.c_int
        L.eiger_sort_pairs.argtypes = [i32, vp, vp, i64, i32, vp, vp, vp, sz, vp]
        L.eiger_sort_pairs.restype = ctypes.c_int
        L.eiger_skf_plan.argtypes = [ctypes.POINTER(StatsT), vp, i32, i32, i64, psk]
        L.eiger_skf_plan.restype = ctypes.c_int
        L.eiger_skf_plan_join.argtypes = [ctypes.POINTER(StatsT), ctypes.POINTER(StatsT), i32, i32, i64, psk]
        L.eiger_skf_plan_join.restype = ctypes.c_int
        L.eiger_skf_workspace_size.argtypes = [psk, i64, i64, i32, ctypes.POINTER(sz)]
        L.eiger_skf_workspace_size.restype = ctypes.c_int
        L.eiger_skf_fuse.argtypes = [vp, vp, i32, psk, vp, vp, psk, vp, sz, vp]
        L.eiger_skf_fuse.restype = ctypes.c_int
        L.eiger_sort_multikey.argtypes = [vp, i32, psk, vp, vp, psk, vp, sz, vp]
        L.eiger_sort_multikey.restype = ctypes.c_int
        L.eiger_dict_encode_workspace_size.argtypes = [Column, i64, ctypes.POINTER(sz)]
        L.eiger_dict_encode_workspace_size.restype = ctypes.c_int
        L.eiger_dict_encode.argtypes = [Column, i64, vp, vp, i64, ctypes.POINTER(i64), vp, sz, vp]
        L.eiger_dict_encode.restype = ctypes.c_int
        L.eiger_last_error.argtypes = []
        L.eiger_last_error.restype = ctypes.c_char_p
        L.eiger_version.restype = ctypes.c_int
        L.eiger_profile_enable.argtypes = [ctypes.c_int]
        L.eiger_profile_enable.restype = ctypes.c_int
        L.eiger_profile_read.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
        L.eiger_profile_read.restype = ctypes.c_int
        L.eiger_mlp_param_count.restype = ctypes.c_int64
        L.eiger_selector_features.argtypes = [ctypes.POINTER(StatsT), ctypes.POINTER(StatsT), vp]
        L.eiger_selector_features.restype = ctypes.c_int
        L.eiger_selector_class_plan.argtypes = [i32, ctypes.POINTER(StatsT), ctypes.POINTER(StatsT),
                                                ctypes.POINTER(PlanT)]
        L.eiger_selector_class_plan.restype = ctypes.c_int
        L.eiger_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.eiger_mlp_forward.restype = ctypes.c_int
        L.eiger_mlp_train_workspace_size.argtypes = [i32]
        L.eiger_mlp_train_workspace_size.restype = sz
        L.eiger_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, ctypes.c_float, i32, vp, vp, sz, vp]
        L.eiger_mlp_train_step.restype = ctypes.c_int
        L.eiger_selector_load.argtypes = [vp, vp, vp, vp, vp]
        L.eiger_selector_load.restype = ctypes.c_int
        L.eiger_selector_loaded.restype = ctypes.c_int
        L.eiger_join_batch_workspace_size.argtypes = [vp, i32, i32, i32, vp, ctypes.POINTER(sz)]
        L.eiger_join_batch_workspace_size.restype = ctypes.c_int
        L.eiger_join_batch_create.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
        L.eiger_join_batch_create.restype = ctypes.c_int
        L.eiger_join_batch_launch.argtypes = [vp, vp]
        L.eiger_join_batch_launch.restype = ctypes.c_int
        L.eiger_join_batch_results.argtypes = [vp, vp, vp, vp, vp, vp]
        L.eiger_join_batch_results.restype = ctypes.c_int
        L.eiger_join_batch_destroy.argtypes = [vp]
        L.eiger_join_batch_destroy.restype = ctypes.c_int
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


def groupby_plan(key_stats: Stats, selector: int = SEL_RULE, forced: Optional[GroupByPlanT] = None) -> GroupByPlanT:
    """eiger_groupby_plan: HASH or PARTITION from the keys' statistics (HLL estimate)."""
    out = GroupByPlanT()
    _check(lib().eiger_groupby_plan(ctypes.byref(key_stats.raw), selector,
                                    ctypes.byref(forced) if forced is not None else None, ctypes.byref(out)))
    return out


def make_groupby_plan(variant: int, radix_bits: int = 0) -> GroupByPlanT:
    p = GroupByPlanT()
    p.variant, p.radix_bits = variant, radix_bits
    return p


@dataclass
class GroupByResult:
    keys: object     # group keys (key dtype), length groups
    counts: object   # torch.int64
    sums: list       # torch.int64 per value column
    groups: int
    plan: GroupByPlanT


def groupby(keys, vals, plan: Optional[GroupByPlanT] = None, capacity: Optional[int] = None, stream=None,
            workspace=None) -> GroupByResult:
    """eiger_groupby: groups of `keys` with counts and sums of the value columns.
    Without a plan, the keys' statistics are computed and the rule planner picks
    one. A plan whose table turns out too small (the estimate was low) is run
    again with eight times the slots (on a copy of the plan); a result above
    `capacity` is run again at its exact size."""
    import torch
    if plan is None:
        plan = groupby_plan(stats(keys, stream))
    kc = column(keys)
    arr = (Column * max(len(vals), 1))()
    for i, t in enumerate(vals):
        arr[i] = column(t)
    groups = ctypes.c_int64()

    def run(pl, cap):
        need = ctypes.c_size_t()
        _check(lib().eiger_groupby_workspace_size(ctypes.byref(pl), kc, arr, len(vals), ctypes.byref(need)))
        ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value,
                                                                                                     keys.device)
        ok = torch.empty(max(cap, 1), dtype=keys.dtype, device=keys.device)
        oc = torch.empty(max(cap, 1), dtype=torch.int64, device=keys.device)
        osum = [torch.empty(max(cap, 1), dtype=torch.int64, device=keys.device) for _ in vals]
        ptrs = (ctypes.c_void_p * max(len(vals), 1))(*[t.data_ptr() for t in osum])
        rc = lib().eiger_groupby(kc, arr, len(vals), ctypes.byref(pl), ctypes.c_void_p(ok.data_ptr()),
                                 ctypes.c_void_p(oc.data_ptr()), ptrs, cap, ctypes.byref(groups),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
        return rc, ok, oc, osum

    plan = GroupByPlanT.from_buffer_copy(plan)
    if capacity is None:
        capacity = min(keys.numel(), int(plan.predicted_groups * 1.25) + 1024)
    rc, ok, oc, osum = run(plan, capacity)
    while rc == EIGER_ERR_TOO_LARGE and plan.slots < 2 * keys.numel() + 1:
        plan.slots *= 8
        rc, ok, oc, osum = run(plan, capacity)
    if rc == EIGER_ERR_CAPACITY:
        rc, ok, oc, osum = run(plan, groups.value)
    _check(rc)
    g = groups.value
    return GroupByResult(ok[:g], oc[:g], [t[:g] for t in osum], g, plan)



def sort_pairs(keys, key_bits: int, vals=None, stream=None, workspace=None):
    """eiger_sort_pairs: stable LSD radix sort of (key, value) pairs by the low
    key_bits bits of the key. keys: a device int32 or int64 tensor holding the
    unsigned key bits; vals: int32 tensor (row ids 0..n-1 when None). Returns
    (sorted keys, values in sorted order)."""
    import torch
    n = keys.numel()
    kb = keys.element_size()
    need = ctypes.c_size_t()
    _check(lib().eiger_sort_pairs_workspace_size(kb, n, key_bits, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value,
                                                                                             keys.device)
    ko = torch.empty_like(keys)
    vo = torch.empty(n, dtype=torch.int32, device=keys.device)
    _check(lib().eiger_sort_pairs(kb, ctypes.c_void_p(keys.data_ptr()),
                                  ctypes.c_void_p(vals.data_ptr()) if vals is not None else None, n, key_bits,
                                  ctypes.c_void_p(ko.data_ptr()), ctypes.c_void_p(vo.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return ko, vo


def _stats_array(items):
    arr = (StatsT * len(items))()
    for i, st in enumerate(items):
        arr[i] = st.raw
    return arr


def skf_plan(key_stats, descending=None, for_max_bits: int = SKF_FOR_MAX_BITS,
             dict_max_ndv: int = SKF_DICT_MAX_NDV) -> SkfPlanT:
    """eiger_skf_plan: frame-of-reference or dictionary code per key from its statistics."""
    out = SkfPlanT()
    desc = (ctypes.c_int32 * len(key_stats))(*[int(bool(d)) for d in (descending or [0] * len(key_stats))])
    _check(lib().eiger_skf_plan(_stats_array(key_stats), desc, len(key_stats), for_max_bits, dict_max_ndv,
                                ctypes.byref(out)))
    return out


def skf_plan_join(build_stats, probe_stats, for_max_bits: int = SKF_FOR_MAX_BITS,
                  dict_max_ndv: int = SKF_DICT_MAX_NDV) -> SkfPlanT:
    """eiger_skf_plan_join: one fusion plan valid for both relations of a join."""
    out = SkfPlanT()
    _check(lib().eiger_skf_plan_join(_stats_array(build_stats), _stats_array(probe_stats), len(build_stats),
                                     for_max_bits, dict_max_ndv, ctypes.byref(out)))
    return out


def _grow_dict_slots(plan: SkfPlanT) -> None:
    for k in plan.key[: plan.n_keys]:
        if k.code == SKF_DICT:
            k.slots *= 8


def _skf_call(fn, plan: SkfPlanT, n_rows: int, sort: int, device):
    """Runs fn(plan, ws) -> rc, retrying with larger dictionary tables while the
    library reports more distinct values than a table holds."""
    while True:
        need = ctypes.c_size_t()
        _check(lib().eiger_skf_workspace_size(ctypes.byref(plan), n_rows, 0, sort, ctypes.byref(need)))
        ws = _workspace(need.value, device)
        rc = fn(plan, ws)
        if rc == EIGER_ERR_TOO_LARGE and any(k.code == SKF_DICT and k.slots < (1 << 31)
                                             for k in plan.key[: plan.n_keys]):
            _grow_dict_slots(plan)
            continue
        _check(rc)
        return


def _fused_view(buf, plan: SkfPlanT, n: int):
    import torch
    return buf.view(torch.int32)[:n] if plan.fused_bytes == 4 else buf.view(torch.int64)[:n]


def skf_fuse(keys_a, keys_b=None, plan: Optional[SkfPlanT] = None, stream=None):
    """eiger_skf_fuse: one fused 4- or 8-byte key per row of one relation (or of
    two, with one shared encoding). Without a plan, the keys' statistics are
    computed and eiger_skf_plan (eiger_skf_plan_join for two relations) decides.
    Returns (fused_a, fused_b or None, final plan); fused keys are int32/int64
    tensors holding the unsigned fused bits."""
    import torch
    if plan is None:
        if keys_b is None:
            plan = skf_plan([stats(k, stream) for k in keys_a])
        else:
            plan = skf_plan_join([stats(k, stream) for k in keys_a], [stats(k, stream) for k in keys_b])
    plan = SkfPlanT.from_buffer_copy(plan)
    na = keys_a[0].numel()
    nb = keys_b[0].numel() if keys_b is not None else 0
    dev = keys_a[0].device
    ca = (Column * len(keys_a))(*[column(t) for t in keys_a])
    cb = (Column * len(keys_b))(*[column(t) for t in keys_b]) if keys_b is not None else None
    oa = torch.empty(max(na, 1), dtype=torch.int64, device=dev)
    ob = torch.empty(max(nb, 1), dtype=torch.int64, device=dev)
    fin = SkfPlanT()

    def run(pl, ws):
        need = ctypes.c_size_t()
        _check(lib().eiger_skf_workspace_size(ctypes.byref(pl), na, nb, 0, ctypes.byref(need)))
        if ws.numel() < need.value:
            ws = _workspace(need.value, dev)
        return lib().eiger_skf_fuse(ca, cb, len(keys_a), ctypes.byref(pl), ctypes.c_void_p(oa.data_ptr()),
                                    ctypes.c_void_p(ob.data_ptr()), ctypes.byref(fin),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))

    _skf_call(run, plan, na + nb, 0, dev)
    return _fused_view(oa, fin, na), (_fused_view(ob, fin, nb) if keys_b is not None else None), fin


def sort_multikey(keys, descending=None, plan: Optional[SkfPlanT] = None, with_sorted: bool = False, stream=None):
    """eiger_sort_multikey: the stable sorting permutation of the rows by several
    keys (each ascending or descending) through smart key fusion and one radix
    sort. Returns (perm int32, sorted fused keys or None, final plan)."""
    import torch
    if plan is None:
        plan = skf_plan([stats(k, stream) for k in keys], descending)
    plan = SkfPlanT.from_buffer_copy(plan)
    n = keys[0].numel()
    dev = keys[0].device
    ck = (Column * len(keys))(*[column(t) for t in keys])
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    srt = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if with_sorted else None
    fin = SkfPlanT()

    def run(pl, ws):
        return lib().eiger_sort_multikey(ck, len(keys), ctypes.byref(pl), ctypes.c_void_p(perm.data_ptr()),
                                         ctypes.c_void_p(srt.data_ptr()) if srt is not None else None,
                                         ctypes.byref(fin), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_ptr(stream))

    _skf_call(run, plan, n, 1, dev)
    return perm[:n], (_fused_view(srt, fin, n) if srt is not None else None), fin


def dict_encode(col, slots: Optional[int] = None, stream=None):
    """eiger_dict_encode: order-preserving dictionary codes of one column.
    Returns (codes int32, dictionary in the column's dtype, ndv)."""
    import torch
    if slots is None:
        est = stats(col, stream).ndv
        slots = 1024
        while slots < 2 * (1.05 * est + 16):
            slots <<= 1
    n = col.numel()
    c = column(col)
    codes = torch.empty(max(n, 1), dtype=torch.int32, device=col.device)
    ndv = ctypes.c_int64()
    while True:
        need = ctypes.c_size_t()
        _check(lib().eiger_dict_encode_workspace_size(c, slots, ctypes.byref(need)))
        ws = _workspace(need.value, col.device)
        cap = min(n, slots // 2) if n else 0
        dic = torch.empty(max(cap, 1), dtype=col.dtype, device=col.device)
        rc = lib().eiger_dict_encode(c, slots, ctypes.c_void_p(codes.data_ptr()), ctypes.c_void_p(dic.data_ptr()),
                                     max(cap, 1), ctypes.byref(ndv), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream_ptr(stream))
        if rc == EIGER_ERR_TOO_LARGE and slots < (1 << 31):
            slots *= 8
            continue
        _check(rc)
        return codes[:n], dic[: ndv.value], ndv.value


def join_multikey(build_keys, probe_keys, build_payload=None, probe_payload=None, selector: int = SEL_RULE,
                  stream=None):
    """Equi-join on several key columns: smart key fusion of both relations with
    one shared encoding, then the single-key join path (statistics, plan, join)
    on the fused keys. Payloads default to the build / probe row ids' zeros.
    Returns (JoinResult, fusion plan, join plan)."""
    import torch
    fa, fb, fin = skf_fuse(build_keys, probe_keys, stream=stream)
    bp = build_payload if build_payload is not None else torch.zeros_like(fa)
    pp = probe_payload if probe_payload is not None else torch.zeros_like(fb)
    jp = join_plan(stats(fa, stream), stats(fb, stream), selector)
    return join(fa, bp, fb, pp, jp, stream=stream), fin, jp


MAT_GFUR, MAT_GFTR, MAT_AUTO = 0, 1, 2
MAT_NAMES = {MAT_GFUR: "gfur", MAT_GFTR: "gftr"}


@dataclass
class WideResult:
    build_rowid: object   # torch.int32 tensors holding uint32 row ids, length count
    probe_rowid: object
    build_cols: list      # materialized payload columns, each in its input column's dtype
    probe_cols: list
    count: int
    materialized: int     # MAT_GFUR or MAT_GFTR


def _col_array(cols):
    arr = (Column * max(len(cols), 1))()
    for i, t in enumerate(cols):
        arr[i] = column(t)
    return arr


def join_wide(bk, bcols, pk, pcols, plan: PlanT, materialize: int = MAT_AUTO, capacity: Optional[int] = None,
              stream=None, workspace=None, count_only: bool = False) -> WideResult:
    """eiger_join_wide: the join with every payload column of both sides
    materialized (GFUR, GFTR or AUTO). Outputs are allocated here (capacity
    defaults to the plan's prediction with headroom, at least the probe rows);
    a result that does not fit is run again once at its exact size."""
    import torch
    ca, cb = _col_array(bcols), _col_array(pcols)
    kb, kp = column(bk), column(pk)
    need = ctypes.c_size_t()
    _check(lib().eiger_join_wide_workspace_size(ctypes.byref(plan), int(materialize), kb, ca, len(bcols), kp, cb,
                                                len(pcols), ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, pk.device)
    cnt, used = ctypes.c_int64(), ctypes.c_int32()

    def run(cap):
        if cap == 0:
            outs = (None, None, [], [])
            ptr_b = ptr_p = None
        else:
            outs = (torch.empty(cap, dtype=torch.int32, device=pk.device),
                    torch.empty(cap, dtype=torch.int32, device=pk.device),
                    [torch.empty(cap, dtype=t.dtype, device=pk.device) for t in bcols],
                    [torch.empty(cap, dtype=t.dtype, device=pk.device) for t in pcols])
            ptr_b = (ctypes.c_void_p * max(len(bcols), 1))(*[t.data_ptr() for t in outs[2]])
            ptr_p = (ctypes.c_void_p * max(len(pcols), 1))(*[t.data_ptr() for t in outs[3]])
        rc = lib().eiger_join_wide(kb, ca, len(bcols), kp, cb, len(pcols), ctypes.byref(plan), int(materialize),
                                   ctypes.c_void_p(outs[0].data_ptr()) if cap else None,
                                   ctypes.c_void_p(outs[1].data_ptr()) if cap else None,
                                   ptr_b, ptr_p, cap, ctypes.byref(cnt), ctypes.byref(used),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
        return rc, outs

    if count_only:
        rc, _ = run(0)
        _check(rc, cnt.value)
        return WideResult(None, None, [], [], cnt.value, used.value)
    if capacity is None:
        capacity = max(int(plan.predicted_out * 1.25) + 1024, pk.numel())
    rc, outs = run(capacity)
    if rc == EIGER_ERR_CAPACITY:
        del outs
        rc, outs = run(cnt.value)
    _check(rc, cnt.value)
    n = cnt.value
    return WideResult(outs[0][:n], outs[1][:n], [t[:n] for t in outs[2]], [t[:n] for t in outs[3]], n, used.value)


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def join_noalloc(bk, bp, pk, pp, plan: PlanT, outputs=None, stream=None) -> JoinResult:
    """eiger_join_noalloc: the join with the library's fixed scratch array as its
    workspace. `outputs` = (out_b, out_p) device int32 tensors, or None for
    count-only mode. Raises EigerError (code EIGER_ERR_CAPACITY with .count set
    when the outputs are too small)."""
    cols = [column(t) for t in (bk, bp, pk, pp)]
    cnt, cs = ctypes.c_int64(), ctypes.c_int64()
    if outputs is None:
        ob = op = None
        cap = 0
    else:
        ob, op = outputs
        cap = min(ob.numel(), op.numel())
    rc = lib().eiger_join_noalloc(*cols, ctypes.byref(plan),
                                  ctypes.c_void_p(ob.data_ptr()) if ob is not None else None,
                                  ctypes.c_void_p(op.data_ptr()) if op is not None else None,
                                  cap, ctypes.byref(cnt), ctypes.byref(cs), _stream_ptr(stream))
    _check(rc, cnt.value)
    if ob is None:
        return JoinResult(None, None, cnt.value, cs.value)
    return JoinResult(ob[: cnt.value], op[: cnt.value], cnt.value, cs.value)


# ---- learned selector -------------------------------------------------------------

SEL_FEATURES, SEL_CLASSES, MLP_HIDDEN = 16, 16, 64


def mlp_param_count() -> int:
    return int(lib().eiger_mlp_param_count())


def _fptr(t):
    return ctypes.c_void_p(t.data_ptr())


def selector_features(build: Stats, probe: Stats):
    """eiger_selector_features: the 16 raw features (torch float32, host)."""
    import torch
    out = torch.zeros(SEL_FEATURES, dtype=torch.float32)
    _check(lib().eiger_selector_features(ctypes.byref(build.raw), ctypes.byref(probe.raw), _fptr(out)))
    return out


def selector_class_plan(cls: int, build: Stats, probe: Stats) -> Optional[PlanT]:
    """The plan of selector class `cls`, or None when the class cannot run these inputs."""
    out = PlanT()
    rc = lib().eiger_selector_class_plan(int(cls), ctypes.byref(build.raw), ctypes.byref(probe.raw),
                                         ctypes.byref(out))
    if rc == EIGER_ERR_UNSUPPORTED:
        return None
    _check(rc)
    return out


def mlp_forward(params, x, stream=None):
    """eiger_mlp_forward on device tensors: params [6288], x [B, 16] -> y [B, 16]."""
    import torch
    y = torch.empty(x.shape[0], SEL_CLASSES, dtype=torch.float32, device=x.device)
    _check(lib().eiger_mlp_forward(_fptr(params), _fptr(x), int(x.shape[0]), _fptr(y), _stream_ptr(stream)))
    return y


class MlpTrainer:
    """Device state of full-batch Adam training through eiger_mlp_train_step."""

    def __init__(self, params, batch: int):
        import torch
        self.params = params.detach().clone().float().contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.ws = _workspace(lib().eiger_mlp_train_workspace_size(int(batch)), params.device)
        self.batch = int(batch)
        self.t = 0

    def step(self, x, target, mask, lr: float, stream=None) -> None:
        assert x.shape[0] == self.batch
        self.t += 1
        _check(lib().eiger_mlp_train_step(_fptr(self.params), _fptr(self.m), _fptr(self.v), _fptr(self.grads),
                                          _fptr(x), _fptr(target), _fptr(mask), self.batch, float(lr), self.t,
                                          _fptr(self.loss), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                          _stream_ptr(stream)))


def selector_load(params, feat_mean, feat_std, feat_lo=None, feat_hi=None) -> None:
    """eiger_selector_load from host float32 tensors; feat_lo/feat_hi (raw
    feature bounds of the training data) turn on the domain check."""
    import torch
    p = params.detach().cpu().float().contiguous()
    m = torch.as_tensor(feat_mean, dtype=torch.float32).contiguous()
    sd = torch.as_tensor(feat_std, dtype=torch.float32).contiguous()
    lo = None if feat_lo is None else torch.as_tensor(feat_lo, dtype=torch.float32).contiguous()
    hi = None if feat_hi is None else torch.as_tensor(feat_hi, dtype=torch.float32).contiguous()
    _check(lib().eiger_selector_load(_fptr(p), _fptr(m), _fptr(sd), None if lo is None else _fptr(lo),
                                     None if hi is None else _fptr(hi)))


def selector_loaded() -> bool:
    return bool(lib().eiger_selector_loaded())


# ---- batched joins -----------------------------------------------------------------

BATCH_BUCKETS = 33
BATCH_DUPLICATE_BUILD = 1
BATCH_CAPACITY = 2


class BatchJoinT(ctypes.Structure):
    _fields_ = [("build_keys", ctypes.c_void_p), ("build_payload", ctypes.c_void_p),
                ("probe_keys", ctypes.c_void_p), ("probe_payload", ctypes.c_void_p),
                ("n_build", ctypes.c_int64), ("n_probe", ctypes.c_int64)]


class BatchTuneT(ctypes.Structure):
    _fields_ = [("load_factor", ctypes.c_float), ("probe_tile", ctypes.c_int32), ("radix_bits", ctypes.c_int32)]


def batch_bucket(n_build: int) -> int:
    """Tuning bucket of a join: floor(log2(n_build)) (0 for n_build <= 1)."""
    return max(0, int(n_build).bit_length() - 1)


class Batch:
    """A captured batch of joins (eiger_join_batch_*). `joins` is a list of
    (build_keys, build_payload, probe_keys, probe_payload) device tensors; `tune`
    maps bucket -> (load_factor, probe_tile[, radix_bits]); radix_bits > 0 runs
    the bucket's joins through the partitioned join inside the graph. The
    tensors must outlive the batch."""

    def __init__(self, joins, tune=None, stream=None):
        import torch
        self.joins = joins
        k0, p0 = joins[0][0], joins[0][1]
        self.kdt, self.pdt = _dtype_code(k0), _dtype_code(p0)
        arr = (BatchJoinT * len(joins))()
        for i, (bk, bp, pk, pp) in enumerate(joins):
            for t in (bk, pk):
                if _dtype_code(t) != self.kdt:
                    raise EigerError(EIGER_ERR_DTYPE, "batch: key dtypes differ")
            for t in (bp, pp):
                if _dtype_code(t) != self.pdt:
                    raise EigerError(EIGER_ERR_DTYPE, "batch: payload dtypes differ")
            arr[i] = BatchJoinT(bk.data_ptr() if bk.numel() else None, bp.data_ptr() if bp.numel() else None,
                                pk.data_ptr() if pk.numel() else None, pp.data_ptr() if pp.numel() else None,
                                bk.numel(), pk.numel())
        self._arr = arr
        self._tune = None
        if tune:
            t = (BatchTuneT * BATCH_BUCKETS)()
            for b in range(BATCH_BUCKETS):
                v = tuple(tune.get(b, (0.5, 16384)))
                lf, tile, bits = (v + (0,))[:3]
                t[b] = BatchTuneT(float(lf), int(tile), int(bits))
            self._tune = t
        need = ctypes.c_size_t()
        _check(lib().eiger_join_batch_workspace_size(ctypes.byref(arr), len(joins), self.kdt, self.pdt,
                                                     ctypes.byref(self._tune) if self._tune else None,
                                                     ctypes.byref(need)))
        dev = joins[0][2].device
        self.offsets = [0]
        for (_, _, pk, _) in joins:
            self.offsets.append(self.offsets[-1] + pk.numel())
        total = max(self.offsets[-1], 1)
        self.out_b = torch.empty(total, dtype=torch.int32, device=dev)
        self.out_p = torch.empty(total, dtype=torch.int32, device=dev)
        self.ws = _workspace(need.value, dev)
        h = ctypes.c_void_p()
        _check(lib().eiger_join_batch_create(ctypes.byref(arr), len(joins), self.kdt, self.pdt,
                                             ctypes.byref(self._tune) if self._tune else None,
                                             ctypes.c_void_p(self.out_b.data_ptr()),
                                             ctypes.c_void_p(self.out_p.data_ptr()),
                                             ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                             _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().eiger_join_batch_launch(self.handle, _stream_ptr(stream)))

    def results(self, stream=None):
        """(counts, checksums, variants, flags) as numpy arrays (waits for the stream)."""
        import numpy as np
        n = len(self.joins)
        c, s = np.zeros(n, np.int64), np.zeros(n, np.int64)
        v, f = np.zeros(n, np.int32), np.zeros(n, np.uint32)
        _check(lib().eiger_join_batch_results(self.handle, c.ctypes.data_as(ctypes.c_void_p),
                                              s.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p),
                                              f.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
        return c, s, v, f

    def pairs(self, j, count):
        lo = self.offsets[j]
        return self.out_b[lo:lo + count], self.out_p[lo:lo + count]

    def resolve_flagged(self, flags, selector: int = SEL_RULE, stream=None) -> dict:
        """Joins the batch flagged (repeated build keys: the graph's first-match
        probes do not hold for them; or a partitioned join with more pairs than
        its output range) run again one by one through eiger_join with the
        `selector` plan, which handles duplicates. Returns {join index:
        JoinResult}; the batch's own output ranges of those joins are not used."""
        out = {}
        for j in (int(x) for x in (flags != 0).nonzero()[0]):
            bk, bp, pk, pp = self.joins[j]
            plan = join_plan(stats(bk, stream), stats(pk, stream), selector)
            out[j] = join(bk, bp, pk, pp, plan, stream=stream)
        return out

    def destroy(self):
        if self.handle:
            lib().eiger_join_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


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
