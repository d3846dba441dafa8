// join_direct.hip -- DIRECT variant: a table indexed by key - min for dense build key ranges.
//
// Build: count rows per key value, exclusive scan into offsets, scatter row ids
// and payloads into CSR order (the scatter advances each key's offset to its end,
// so the offsets array ends up holding end offsets). Duplicate build keys are
// handled by the CSR layout. Probe: one bounds check and two offset reads per
// probe row, then the key's CSR run.
#include "join_common.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr int kNT = 256;
constexpr int kIPT = 8;
constexpr int kSCAP = 4096;

template <typename K, typename PB>
struct DirectTab {
  static constexpr bool kHashed = false;
  static constexpr bool kRuns = true;
  uint64_t min;  // as two's-complement bits
  uint64_t range;
  const uint32_t *__restrict__ end;  // end offset of each key value's run
  const uint32_t *__restrict__ rowid;
  const PB *__restrict__ pay;

  __device__ __forceinline__ bool run(K key, uint32_t &s, uint32_t &e) const {
    const uint64_t d = static_cast<uint64_t>(sext(key)) - min;
    if (d >= range) return false;
    s = d ? end[d - 1] : 0u;
    e = end[d];
    return true;
  }
  // `first` receives the start of the key value's run (kRuns)
  __device__ __forceinline__ uint32_t lookup(K key, uint32_t &first, uint64_t &psum) const {
    uint32_t s, e;
    if (!run(key, s, e) || s == e) return 0;
    first = s;
    for (uint32_t t = s; t < e; ++t) psum += static_cast<uint64_t>(sext(pay[t]));
    return e - s;
  }
  __device__ __forceinline__ uint32_t row_at(uint32_t i) const { return rowid[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint32_t s, e;
    if (!run(key, s, e)) return;
    for (uint32_t t = s; t < e; ++t) f(rowid[t]);
  }
};

template <typename K>
__global__ void k_direct_count(const K *__restrict__ keys, uint64_t n, uint64_t min, uint64_t range,
                               uint32_t *__restrict__ cnt, uint64_t *__restrict__ flags) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t d = static_cast<uint64_t>(sext(keys[i])) - min;
    if (d < range)
      atomicAdd(&cnt[d], 1u);
    else
      atomicOr(reinterpret_cast<unsigned long long *>(flags), kFlagBuildOutOfRange);
  }
}

template <typename K, typename PB>
__global__ void k_direct_fill(const K *__restrict__ keys, const PB *__restrict__ pay, uint64_t n,
                              uint64_t min, uint64_t range, uint32_t *__restrict__ off,
                              uint32_t *__restrict__ rowid, PB *__restrict__ cpay) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t d = static_cast<uint64_t>(sext(keys[i])) - min;
    if (d < range) {
      const uint32_t pos = atomicAdd(&off[d], 1u);
      rowid[pos] = static_cast<uint32_t>(i);
      cpay[pos] = pay[i];
    }
  }
}

// Each workgroup streams a contiguous range of probe rows (an equal share of
// whole sub-tiles).
template <class Tab, typename K, typename PS>
__global__ void __launch_bounds__(kNT) k_probe(Tab tab, const K *__restrict__ pk,
                                               const PS *__restrict__ pp, uint64_t n, EmitOut o) {
  __shared__ EmitLds<kNT, kSCAP> L;
  uint64_t fill = 0;
  uint64_t cs = 0;
  constexpr uint64_t sub = uint64_t(kNT) * kIPT;
  const uint64_t nsub = (n + sub - 1) / sub;
  const uint64_t per = (nsub + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = blockIdx.x * per * sub;
  const uint64_t hi = lo + per * sub < n ? lo + per * sub : n;
  probe_range<kNT, kIPT, kSCAP>(tab, pk, pp, static_cast<const uint32_t *>(nullptr), lo, hi, L, fill,
                                o, cs);
  finish(L, o, fill, cs);
}

unsigned grid_for(uint64_t work, uint64_t per_block, int per_cu) {
  uint64_t g = (work + per_block - 1) / per_block;
  const uint64_t cap = uint64_t(device_cu_count()) * per_cu;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g ? g : 1);
}

template <typename K, typename PB, typename PS>
int direct_impl(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const uint64_t min = static_cast<uint64_t>(a.plan.build_min);
  const uint64_t range = static_cast<uint64_t>(a.plan.build_max) - min + 1;  // checked by caller
  JoinCounters *c = ws.take<JoinCounters>(1);
  uint32_t *off = ws.take<uint32_t>(range);
  uint32_t *rowid = ws.take<uint32_t>(a.nR ? a.nR : 1);
  PB *cpay = ws.take<PB>(a.nR ? a.nR : 1);
  uint64_t *tmp = ws.take<uint64_t>(scan_tmp_elems(range));
  uint64_t *total = ws.take<uint64_t>(1);
  *ctr = c;
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if ((rc = fill_u32(off, range, 0, s))) return rc;
  const K *bk = static_cast<const K *>(a.bk);
  if (a.nR) {
    EIGER_LAUNCH("direct_count", k_direct_count<K>, dim3(grid_for(a.nR, 256 * 4, 8)), dim3(256), 0, s,
                 bk, a.nR, min, range, off, &c->flags);
  }
  if ((rc = exclusive_scan_u32(off, off, range, tmp, total, s))) return rc;
  if (a.nR) {
    EIGER_LAUNCH("direct_fill", (k_direct_fill<K, PB>), dim3(grid_for(a.nR, 256 * 4, 8)), dim3(256), 0,
                 s, bk, static_cast<const PB *>(a.bp), a.nR, min, range, off, rowid, cpay);
  }
  if (a.nS && a.nR) {
    DirectTab<K, PB> tab{min, range, off, rowid, cpay};
    EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
    EIGER_LAUNCH("direct_probe", (k_probe<DirectTab<K, PB>, K, PS>),
                 dim3(grid_for(a.nS, uint64_t(kNT) * kIPT, 4)), dim3(kNT), 0, s, tab,
                 static_cast<const K *>(a.pk), static_cast<const PS *>(a.pp), a.nS, o);
  }
  return EIGER_OK;
}

}  // namespace

int run_direct(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const bool k64 = a.kdt == EIGER_INT64, b64 = a.bpdt == EIGER_INT64, p64 = a.ppdt == EIGER_INT64;
#define EIGER_DISPATCH(KT, BT, PT) return direct_impl<KT, BT, PT>(a, ws, ctr)
  if (!k64 && !b64 && !p64) EIGER_DISPATCH(int32_t, int32_t, int32_t);
  if (!k64 && !b64 && p64) EIGER_DISPATCH(int32_t, int32_t, int64_t);
  if (!k64 && b64 && !p64) EIGER_DISPATCH(int32_t, int64_t, int32_t);
  if (!k64 && b64 && p64) EIGER_DISPATCH(int32_t, int64_t, int64_t);
  if (k64 && !b64 && !p64) EIGER_DISPATCH(int64_t, int32_t, int32_t);
  if (k64 && !b64 && p64) EIGER_DISPATCH(int64_t, int32_t, int64_t);
  if (k64 && b64 && !p64) EIGER_DISPATCH(int64_t, int64_t, int32_t);
  EIGER_DISPATCH(int64_t, int64_t, int64_t);
#undef EIGER_DISPATCH
}

}  // namespace eiger
