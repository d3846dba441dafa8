// join_smj.hip -- SORT_MERGE variant: both relations radix-sorted on their keys,
// then merged (Section 3.2 and Table 1: the sort-merge join next to the hash and
// partitioned hash joins; Section 5.2.2: it wins for medium probe sides).
//
//  1. encode: every key becomes an order-preserving unsigned code of the build
//     range, key - build_min; a probe key outside the build range becomes
//     max - min + 1, which no build key has. The code width (bits of max - min + 1)
//     sets the number of radix passes and the 4- or 8-byte code type.
//  2. sort: (code, row id) pairs of each side by the stable LSD radix sort.
//  3. gather: payloads into sorted order (build payloads for the checksum's
//     per-key sums, probe payloads for its products).
//  4. merge: each workgroup takes consecutive sorted probe rows; for each
//     sub-tile it finds the build window [lower bound of its first code, upper
//     bound of its last code) once, and every probe row binary-searches only
//     that window; a key's build rows are one contiguous run of the sorted build
//     side, emitted straight from it.
#include "join_common.hpp"
#include "sort.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr int kMNT = 256;
constexpr int kMIPT = 8;
constexpr int kMSCAP = 4096;

template <typename K, typename U>
__global__ void __launch_bounds__(256) k_smj_encode(const K *__restrict__ keys, uint64_t n, uint64_t min,
                                                    uint64_t span, bool build, U *__restrict__ out,
                                                    uint64_t *__restrict__ flags) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t d = static_cast<uint64_t>(sext(keys[i])) - min;
    if (d > span) {
      if (build) atomicOr(reinterpret_cast<unsigned long long *>(flags), kFlagBuildOutOfRange);
      d = span + 1;
    }
    out[i] = static_cast<U>(d);
  }
}

template <typename P>
__global__ void __launch_bounds__(256) k_smj_gather(const uint32_t *__restrict__ rid, uint64_t n,
                                                    const P *__restrict__ pay, P *__restrict__ out) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = pay[rid[i]];
}

// The sorted build side seen through one sub-tile's window [lo, hi).
template <typename U, typename PB>
struct SortTab {
  static constexpr bool kHashed = false;
  static constexpr bool kRuns = true;
  const U *__restrict__ code;      // sorted build codes
  const uint32_t *__restrict__ rid;  // build row ids in that order
  const PB *__restrict__ pay;      // build payloads in that order
  uint32_t lo, hi;

  __device__ __forceinline__ uint32_t lower(U k) const {
    uint32_t a = lo, b = hi;
    while (a < b) {
      const uint32_t m = a + (b - a) / 2;
      if (code[m] < k)
        a = m + 1;
      else
        b = m;
    }
    return a;
  }
  __device__ __forceinline__ uint32_t upper(U k, uint32_t from) const {
    uint32_t a = from, b = hi;
    while (a < b) {
      const uint32_t m = a + (b - a) / 2;
      if (code[m] <= k)
        a = m + 1;
      else
        b = m;
    }
    return a;
  }
  __device__ __forceinline__ uint32_t lookup(U k, uint32_t &first, uint64_t &psum) const {
    const uint32_t s = lower(k);
    if (s >= hi || code[s] != k) return 0;
    const uint32_t e = upper(k, s + 1);
    first = s;
    for (uint32_t t = s; t < e; ++t) psum += static_cast<uint64_t>(sext(pay[t]));
    return e - s;
  }
  __device__ __forceinline__ uint32_t row_at(uint32_t i) const { return rid[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(U, F) const {}
};

// Bound of the whole sorted build side (thread-local, no window).
template <typename U>
__device__ __forceinline__ uint32_t bound(const U *__restrict__ code, uint32_t n, U k, bool upper_bound) {
  uint32_t a = 0, b = n;
  while (a < b) {
    const uint32_t m = a + (b - a) / 2;
    if (code[m] < k || (upper_bound && code[m] == k))
      a = m + 1;
    else
      b = m;
  }
  return a;
}

template <typename U, typename PB, typename PS>
__global__ void __launch_bounds__(kMNT) k_smj_merge(SortTab<U, PB> tab, uint32_t nR, const U *__restrict__ sk,
                                                    const PS *__restrict__ sp, const uint32_t *__restrict__ srid,
                                                    uint64_t nS, EmitOut o) {
  __shared__ EmitLds<kMNT, kMSCAP> L;
  __shared__ uint32_t win[2];
  uint64_t fill = 0, cs = 0;
  constexpr uint64_t sub = uint64_t(kMNT) * kMIPT;
  const uint64_t nsub = (nS + sub - 1) / sub;
  const uint64_t per = (nsub + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = blockIdx.x * per * sub;
  const uint64_t hi = lo + per * sub < nS ? lo + per * sub : nS;
  ProbeRegs<kMIPT, U, PS> cur;
  for (uint64_t t = lo; t < hi; t += sub) {
    const uint64_t te = t + sub < hi ? t + sub : hi;
    if (threadIdx.x == 0) win[0] = bound(tab.code, nR, sk[t], false);
    if (threadIdx.x == 64) win[1] = bound(tab.code, nR, sk[te - 1], true);
    __syncthreads();
    SortTab<U, PB> w = tab;
    w.lo = win[0];
    w.hi = win[1];
    __syncthreads();
    probe_load<kMNT, kMIPT>(cur, sk, sp, srid, t, te);
    probe_process<kMNT, kMIPT, kMSCAP>(w, cur, L, fill, o, cs);
  }
  finish(L, o, fill, cs);
}

unsigned smj_grid(uint64_t work, uint64_t per_block, int per_cu) {
  uint64_t g = (work + per_block - 1) / per_block;
  const uint64_t cap = uint64_t(device_cu_count()) * per_cu;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g ? g : 1);
}

template <typename K, typename U, typename PB, typename PS>
int smj_impl(const JoinArgs &a, Workspace &ws, JoinCounters **ctr, uint64_t span, int bits) {
  JoinCounters *c = ws.take<JoinCounters>(1);
  U *uR = ws.take<U>(a.nR), *uRs = ws.take<U>(a.nR);
  uint32_t *ridR = ws.take<uint32_t>(a.nR);
  PB *payR = ws.take<PB>(a.nR);
  U *uS = ws.take<U>(a.nS), *uSs = ws.take<U>(a.nS);
  uint32_t *ridS = ws.take<uint32_t>(a.nS);
  PS *payS = ws.take<PS>(a.nS);
  // one region for both sorts (they run one after the other on the stream)
  Workspace probe_size(nullptr, 0);
  radix_sort_pairs(sizeof(U), nullptr, nullptr, std::max(a.nR, a.nS), bits, nullptr, nullptr, probe_size, nullptr);
  char *sort_ws = ws.take<char>(probe_size.used + 256);
  *ctr = c;
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if (a.nR == 0 || a.nS == 0) return EIGER_OK;
  const uint64_t min = static_cast<uint64_t>(a.plan.build_min);
  EIGER_LAUNCH("smj_encode", (k_smj_encode<K, U>), dim3(smj_grid(a.nR, 256 * 4, 8)), dim3(256), 0, s,
               static_cast<const K *>(a.bk), a.nR, min, span, true, uR, &c->flags);
  EIGER_LAUNCH("smj_encode", (k_smj_encode<K, U>), dim3(smj_grid(a.nS, 256 * 4, 8)), dim3(256), 0, s,
               static_cast<const K *>(a.pk), a.nS, min, span, false, uS, &c->flags);
  {
    Workspace sw(sort_ws, probe_size.used + 256);
    if ((rc = radix_sort_pairs(sizeof(U), uR, nullptr, a.nR, bits, uRs, ridR, sw, s))) return rc;
  }
  {
    Workspace sw(sort_ws, probe_size.used + 256);
    if ((rc = radix_sort_pairs(sizeof(U), uS, nullptr, a.nS, bits, uSs, ridS, sw, s))) return rc;
  }
  EIGER_LAUNCH("smj_gather", (k_smj_gather<PB>), dim3(smj_grid(a.nR, 256 * 4, 8)), dim3(256), 0, s, ridR, a.nR,
               static_cast<const PB *>(a.bp), payR);
  EIGER_LAUNCH("smj_gather", (k_smj_gather<PS>), dim3(smj_grid(a.nS, 256 * 4, 8)), dim3(256), 0, s, ridS, a.nS,
               static_cast<const PS *>(a.pp), payS);
  SortTab<U, PB> tab{uRs, ridR, payR, 0, static_cast<uint32_t>(a.nR)};
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  EIGER_LAUNCH("smj_merge", (k_smj_merge<U, PB, PS>), dim3(smj_grid(a.nS, uint64_t(kMNT) * kMIPT, 4)), dim3(kMNT), 0,
               s, tab, static_cast<uint32_t>(a.nR), uSs, payS, ridS, a.nS, o);
  return EIGER_OK;
}

template <typename K, typename U>
int smj_pay(const JoinArgs &a, Workspace &ws, JoinCounters **ctr, uint64_t span, int bits) {
  const bool b64 = a.bpdt == EIGER_INT64, p64 = a.ppdt == EIGER_INT64;
  if (!b64 && !p64) return smj_impl<K, U, int32_t, int32_t>(a, ws, ctr, span, bits);
  if (!b64 && p64) return smj_impl<K, U, int32_t, int64_t>(a, ws, ctr, span, bits);
  if (b64 && !p64) return smj_impl<K, U, int64_t, int32_t>(a, ws, ctr, span, bits);
  return smj_impl<K, U, int64_t, int64_t>(a, ws, ctr, span, bits);
}

int bit_width64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

}  // namespace

int run_sort_merge(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  // span of the build codes; the probe's "no such key" code is span + 1
  const uint64_t span = a.nR ? static_cast<uint64_t>(a.plan.build_max) - static_cast<uint64_t>(a.plan.build_min) : 0;
  const int bits = span == UINT64_MAX ? 64 : bit_width64(span + 1);
  const bool k64 = a.kdt == EIGER_INT64;
  if (bits <= 32) return k64 ? smj_pay<int64_t, uint32_t>(a, ws, ctr, span, bits)
                             : smj_pay<int32_t, uint32_t>(a, ws, ctr, span, bits);
  return k64 ? smj_pay<int64_t, uint64_t>(a, ws, ctr, span, bits) : smj_pay<int32_t, uint64_t>(a, ws, ctr, span, bits);
}

}  // namespace eiger
