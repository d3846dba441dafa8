// groupby.hip -- group-by with a count and per-column sums, hash-based or
// partition-based, chosen from the HLL distinct-count estimate of the key
// column (Section 3.3: group-by algorithms; Section 4.1: the number of groups,
// estimated with HLL++ before the operator runs, picks the algorithm and sizes
// the hash table; Section 5.3.2: the "Auto" series).
//
//  HASH       one open-addressing table of groups in HBM, sized from the
//             estimate. Every workgroup first aggregates its rows in an LDS
//             table (so a few hot groups cost one global update per workgroup,
//             not one per row); rows whose group does not fit in LDS go to the
//             global table; at the end each workgroup merges its LDS groups
//             into the global table, which is then compacted into the output.
//  PARTITION  rows partitioned on the top bits of the key hash (values
//             carried along), then one workgroup per partition aggregates it in
//             LDS and writes its groups straight out (partitions own disjoint
//             keys). A partition with more groups than its LDS table spills
//             into the global table, and its LDS groups are merged there too.
// Group keys live in the tables as sign-extended 64-bit words; a value that is
// not a key (the plan's sentinel) marks empty slots, so a key is claimed with
// one 64-bit CAS.
#include <algorithm>
#include <cmath>
#include <string>

#include "sort.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr int kGNT = 256;
constexpr uint32_t kGLds = 2048;            // LDS table slots (power of two)
constexpr uint32_t kGLdsOpen = kGLds / 2;   // new groups an LDS table accepts
constexpr int kGMaxVals = 2;
constexpr uint32_t kGChunk = 1u << 16;      // rows per workgroup chunk (HASH)
constexpr int kGBatch = 8;                  // rows a thread loads before aggregating them
constexpr uint64_t kGMaxProbe = 4096;       // longest walk in the global table
// rule: HASH while the estimated groups fit one LDS table (beyond it, rows that
// miss the LDS table cost global atomics per row, and PARTITION measured faster
// from 2^14 groups up at 2^28 rows)
constexpr double kGbHashMaxGroups = kGLdsOpen;
constexpr double kGbGroupsPerPartition = 512.0;

struct GbGlobal {
  unsigned long long *key;
  unsigned long long *cnt;
  unsigned long long *sum[kGMaxVals];
  uint64_t mask;
  unsigned long long sentinel;
  uint32_t *overflow;
};

// Value columns as 32-bit words: lo and hi word arrays (for a 4-byte column hi
// points at lo, so every load is unconditional), the word stride, and which
// columns are 8 bytes wide.
struct GbVals {
  const uint32_t *lo[kGMaxVals];
  const uint32_t *hi[kGMaxVals];
  uint32_t stride[kGMaxVals];
  uint32_t wide[kGMaxVals];
  int n;
};

struct GbLds {
  unsigned long long key[kGLds];
  unsigned long long cnt[kGLds];
  unsigned long long sum[kGMaxVals][kGLds];
  uint32_t used;
  uint32_t spilled;
  unsigned long long scan[kGNT / 64 + 1];
};

// A value from its two loaded words: 64-bit, or the low word sign-extended.
__device__ __forceinline__ uint64_t combine(const GbVals &v, int c, uint32_t lo, uint32_t hi) {
  return v.wide[c] ? (uint64_t(hi) << 32) | lo
                   : static_cast<uint64_t>(static_cast<int64_t>(static_cast<int32_t>(lo)));
}

// Slot of key k in the global table, claiming an empty one if needed; -1 when
// the whole table was walked (more groups than slots: *overflow is set).
__device__ __forceinline__ int64_t global_slot(const GbGlobal &t, unsigned long long k) {
  uint64_t s = fmix64(k) & t.mask;
  // a table at most half full never needs a walk this long; stopping here keeps
  // an overfull table (a far too low estimate) from costing a whole-table walk
  // per row before the caller plans again with more slots
  const uint64_t limit = t.mask < kGMaxProbe ? t.mask + 1 : kGMaxProbe;
  for (uint64_t step = 0; step < limit; ++step) {
    // a slot changes once, from the sentinel to a key: any other value read is final
    const unsigned long long cur = __atomic_load_n(&t.key[s], __ATOMIC_RELAXED);
    if (cur == k) return static_cast<int64_t>(s);
    if (cur == t.sentinel) {
      const unsigned long long old = atomicCAS(&t.key[s], t.sentinel, k);
      if (old == t.sentinel || old == k) return static_cast<int64_t>(s);
    }
    s = (s + 1) & t.mask;
  }
  atomicOr(t.overflow, 1u);
  return -1;
}

__device__ __forceinline__ void global_add(const GbGlobal &t, unsigned long long k, unsigned long long c,
                                           const unsigned long long *sums, int nv) {
  const int64_t s = global_slot(t, k);
  if (s < 0) return;
  atomicAdd(&t.cnt[s], c);
  for (int v = 0; v < nv; ++v) atomicAdd(&t.sum[v][s], sums[v]);
}

// LDS slot of key k, claiming an empty slot while the table takes new groups;
// -1: not in the table and the table is closed (the row goes global).
__device__ __forceinline__ int lds_slot(GbLds &L, unsigned long long k, unsigned long long sentinel) {
  uint32_t s = static_cast<uint32_t>(fmix64(k)) & (kGLds - 1);
  for (uint32_t step = 0; step < kGLds; ++step) {
    const unsigned long long cur = L.key[s];
    if (cur == k) return static_cast<int>(s);
    if (cur == sentinel) {
      // closed for new groups once kGLdsOpen were claimed; claims racing with the
      // last one can add at most one per thread of the workgroup
      if (__atomic_load_n(&L.used, __ATOMIC_RELAXED) >= kGLdsOpen) return -1;
      const unsigned long long old = atomicCAS(&L.key[s], sentinel, k);
      if (old == sentinel) {
        atomicAdd(&L.used, 1u);
        return static_cast<int>(s);
      }
      if (old == k) return static_cast<int>(s);
    }
    s = (s + 1) & (kGLds - 1);
  }
  return -1;
}

__device__ __forceinline__ void lds_clear(GbLds &L, unsigned long long sentinel, int nv) {
  for (uint32_t i = threadIdx.x; i < kGLds; i += kGNT) {
    L.key[i] = sentinel;
    L.cnt[i] = 0;
    for (int v = 0; v < nv; ++v) L.sum[v][i] = 0;
  }
  if (threadIdx.x == 0) {
    L.used = 0;
    L.spilled = 0;
  }
  __syncthreads();
}

// One row's contribution to the LDS table (or, when it is closed, to the global one).
__device__ __forceinline__ void lds_add(GbLds &L, const GbGlobal &g, unsigned long long k, unsigned long long c,
                                        const unsigned long long *sv, int nv) {
  const int s = lds_slot(L, k, g.sentinel);
  if (s >= 0) {
    atomicAdd(&L.cnt[s], c);
    for (int v = 0; v < nv; ++v) atomicAdd(&L.sum[v][s], sv[v]);
  } else {
    L.spilled = 1;
    global_add(g, k, c, sv, nv);
  }
}

// Groups a thread keeps in registers before its rows reach the LDS table: with
// a handful of groups every row of a workgroup would otherwise hit the same few
// LDS words, and same-address LDS atomics serialize.
constexpr int kGRegGroups = 4;

// Aggregate rows [lo, hi) into the LDS table (rows that do not fit go global).
// kReg: first into per-thread register groups (HASH, few groups).
template <typename K, bool kReg>
__device__ __forceinline__ void aggregate_rows(GbLds &L, const GbGlobal &g, const K *__restrict__ keys,
                                               const GbVals &vals, uint64_t lo, uint64_t hi) {
  unsigned long long rk[kGRegGroups], rc[kGRegGroups], rs[kGMaxVals][kGRegGroups];
#pragma unroll
  for (int j = 0; j < kGRegGroups; ++j) {
    rk[j] = g.sentinel;
    rc[j] = 0;
#pragma unroll
    for (int v = 0; v < kGMaxVals; ++v) rs[v][j] = 0;
  }
  // kGBatch rows per thread are loaded before any is aggregated, so each
  // thread keeps several loads in flight; loaded words are only combined
  // (sign extension, 64-bit values) after the whole batch was issued
  constexpr uint64_t step = uint64_t(kGNT) * kGBatch;
  for (uint64_t base = lo; base < hi; base += step) {
    K rk_[kGBatch];
    uint32_t wlo[kGBatch][kGMaxVals], whi[kGBatch][kGMaxVals];
#pragma unroll
    for (int b = 0; b < kGBatch; ++b) {
      const uint64_t i = base + uint64_t(b) * kGNT + threadIdx.x;
      if (i < hi) {
        rk_[b] = keys[i];
#pragma unroll
        for (int v = 0; v < kGMaxVals; ++v) {
          if (v < vals.n) {
            const uint64_t at = i * vals.stride[v];
            wlo[b][v] = vals.lo[v][at];
            whi[b][v] = vals.hi[v][at];
          }
        }
      }
    }
    unsigned long long bk[kGBatch], bv[kGBatch][kGMaxVals];
#pragma unroll
    for (int b = 0; b < kGBatch; ++b) {
      const bool in = base + uint64_t(b) * kGNT + threadIdx.x < hi;
      bk[b] = in ? static_cast<unsigned long long>(sext(rk_[b])) : g.sentinel;
#pragma unroll
      for (int v = 0; v < kGMaxVals; ++v)
        bv[b][v] = v < vals.n && in ? combine(vals, v, wlo[b][v], whi[b][v]) : 0ull;
    }
#pragma unroll
    for (int b = 0; b < kGBatch; ++b) {
      const unsigned long long k = bk[b];
      if (k == g.sentinel) continue;  // past the end (no key equals the sentinel)
      const unsigned long long *sv = bv[b];
      if (kReg) {
        bool done = false;
#pragma unroll
        for (int j = 0; j < kGRegGroups; ++j) {
          // a free register group takes the key if no earlier one holds it
          if (!done && (rk[j] == k || rk[j] == g.sentinel)) {
            rk[j] = k;
            rc[j] += 1;
#pragma unroll
            for (int v = 0; v < kGMaxVals; ++v) rs[v][j] += sv[v];
            done = true;
          }
        }
        if (done) continue;
      }
      lds_add(L, g, k, 1ull, sv, vals.n);
    }
  }
  if (kReg) {
#pragma unroll
    for (int j = 0; j < kGRegGroups; ++j) {
      if (rk[j] != g.sentinel) {
        unsigned long long sv[kGMaxVals];
#pragma unroll
        for (int v = 0; v < kGMaxVals; ++v) sv[v] = rs[v][j];
        lds_add(L, g, rk[j], rc[j], sv, vals.n);
      }
    }
  }
  __syncthreads();
}

// Merge the LDS groups into the global table.
__device__ __forceinline__ void lds_merge(GbLds &L, const GbGlobal &g, int nv) {
  for (uint32_t i = threadIdx.x; i < kGLds; i += kGNT) {
    const unsigned long long k = L.key[i];
    if (k == g.sentinel) continue;
    unsigned long long sv[kGMaxVals];
    for (int v = 0; v < nv; ++v) sv[v] = L.sum[v][i];
    global_add(g, k, L.cnt[i], sv, nv);
  }
}

struct GbOut {
  void *keys;  // key dtype
  unsigned long long *cnt;
  unsigned long long *sum[kGMaxVals];
  uint64_t cap;
  unsigned long long *cursor;
  int kwide;
};

__device__ __forceinline__ void put_group(const GbOut &o, uint64_t pos, unsigned long long k, unsigned long long c,
                                          const unsigned long long *sv, int nv) {
  if (pos >= o.cap || !o.keys) return;
  if (o.kwide)
    static_cast<unsigned long long *>(o.keys)[pos] = k;
  else
    static_cast<uint32_t *>(o.keys)[pos] = static_cast<uint32_t>(k);
  o.cnt[pos] = c;
  for (int v = 0; v < nv; ++v) o.sum[v][pos] = sv[v];
}

// Emit the occupied slots of one table range [lo, hi) of (key, cnt, sums)
// arrays. The whole workgroup walks the range in rounds of kGEmitPer slots per
// thread (each thread a contiguous run), and each round reserves its output
// with ONE atomic: a device-wide counter that every wave hit separately cost
// more than the rest of a group-by with millions of groups. Uniform across
// the workgroup (contains barriers); `scan` holds kGNT / 64 + 1 words of LDS.
constexpr int kGEmitPer = 8;
__device__ __forceinline__ void emit_range(const unsigned long long *key, const unsigned long long *cnt,
                                           const unsigned long long *sum0, const unsigned long long *sum1,
                                           uint64_t lo, uint64_t hi, unsigned long long sentinel, int nv,
                                           const GbOut &o, unsigned long long *scan) {
  constexpr uint64_t round = uint64_t(kGNT) * kGEmitPer;
  for (uint64_t base = lo; base < hi; base += round) {
    const uint64_t mine = base + uint64_t(threadIdx.x) * kGEmitPer;
    uint32_t live = 0;
#pragma unroll
    for (int j = 0; j < kGEmitPer; ++j) {
      const uint64_t i = mine + j;
      if (i < hi && key[i] != sentinel) live |= 1u << j;
    }
    unsigned long long total;
    const unsigned long long off =
        block_exclusive_scan<kGNT, unsigned long long>(static_cast<unsigned long long>(__popc(live)), scan, &total);
    if (total == 0) continue;
    if (threadIdx.x == 0) scan[kGNT / 64] = atomicAdd(o.cursor, total);
    __syncthreads();
    unsigned long long at = scan[kGNT / 64] + off;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kGEmitPer; ++j) {
      if (!((live >> j) & 1u)) continue;
      const uint64_t i = mine + j;
      unsigned long long sv[kGMaxVals] = {0, 0};
      if (nv > 0) sv[0] = sum0[i];
      if (nv > 1) sv[1] = sum1[i];
      put_group(o, at++, key[i], cnt[i], sv, nv);
    }
  }
}

__global__ void __launch_bounds__(kGNT) k_gb_clear(GbGlobal g, int nv) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i <= g.mask; i += stride) {
    g.key[i] = g.sentinel;
    g.cnt[i] = 0;
    for (int v = 0; v < nv; ++v) g.sum[v][i] = 0;
  }
}

// HASH: chunks of kGChunk rows per workgroup, LDS pre-aggregation, merge.
template <typename K>
__global__ void __launch_bounds__(kGNT) k_gb_hash(const K *__restrict__ keys, uint64_t n, GbVals vals, GbGlobal g) {
  __shared__ GbLds L;
  for (uint64_t lo = uint64_t(blockIdx.x) * kGChunk; lo < n; lo += uint64_t(gridDim.x) * kGChunk) {
    lds_clear(L, g.sentinel, vals.n);
    aggregate_rows<K, true>(L, g, keys, vals, lo, min(n, lo + kGChunk));
    lds_merge(L, g, vals.n);
    __syncthreads();
  }
}

// PARTITION: work item = one of the S equal slices of a partition (S = 1 when
// partitions are small). A whole partition that did not spill writes its groups
// out directly; slices and spilled partitions merge into the global table.
template <typename K>
__global__ void __launch_bounds__(kGNT)
    k_gb_partition(const K *__restrict__ keys, GbVals vals, const uint32_t *__restrict__ off, uint32_t F, uint32_t S,
                   GbGlobal g, GbOut o) {
  __shared__ GbLds L;
  const uint64_t items = uint64_t(F) * S;
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const uint32_t p = static_cast<uint32_t>(it / S), sl = static_cast<uint32_t>(it % S);
    const uint64_t plo = off[p], len = off[p + 1] - plo;
    const uint64_t lo = plo + len * sl / S, hi = plo + len * (sl + 1) / S;
    if (lo == hi) continue;
    lds_clear(L, g.sentinel, vals.n);
    aggregate_rows<K, false>(L, g, keys, vals, lo, hi);
    if (L.spilled || S > 1) {
      lds_merge(L, g, vals.n);
    } else {
      emit_range(L.key, L.cnt, L.sum[0], L.sum[1], 0, kGLds, g.sentinel, vals.n, o, L.scan);
    }
    __syncthreads();
  }
}

// Compaction of the global table into the output.
__global__ void __launch_bounds__(kGNT) k_gb_emit(GbGlobal g, int nv, GbOut o) {
  const uint64_t slots = g.mask + 1;
  const uint64_t per = (slots + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = uint64_t(blockIdx.x) * per, hi = min(slots, lo + per);
  __shared__ unsigned long long scan[kGNT / 64 + 1];
  emit_range(g.key, g.cnt, g.sum[0], g.sum[1], lo, hi, g.sentinel, nv, o, scan);
}

int gb_sentinel(const eiger_groupby_plan_t &p, unsigned long long *out) {
  *out = static_cast<unsigned long long>(p.sentinel);
  return EIGER_OK;
}

// Slices per partition: few partitions (few groups) are cut into slices so the
// grid still has about four work items per CU of the 256; slices keep at least
// 2^14 rows. With more than one slice every group reaches the global table.
constexpr uint64_t kGTargetItems = 1024;
uint32_t gb_slices(uint64_t n, int bits) {
  const uint64_t F = uint64_t(1) << bits;
  uint32_t S = 1;
  while (uint64_t(S) * F < kGTargetItems && n / (uint64_t(S) * 2 * F) >= (uint64_t(1) << 14)) S <<= 1;
  return S;
}

uint64_t gb_slots(double groups) {
  uint64_t s = 1024;
  while (static_cast<double>(s) < 2.0 * groups + 1.0) s <<= 1;
  return s;
}

struct GbLayout {
  GbGlobal g;
  unsigned long long *cursor;
  uint32_t *overflow;
};

GbLayout gb_layout(Workspace &ws, uint64_t slots, int nv, unsigned long long sentinel) {
  GbLayout L{};
  L.g.key = ws.take<unsigned long long>(slots);
  L.g.cnt = ws.take<unsigned long long>(slots);
  for (int v = 0; v < kGMaxVals; ++v) L.g.sum[v] = v < nv ? ws.take<unsigned long long>(slots) : nullptr;
  L.g.mask = slots - 1;
  L.g.sentinel = sentinel;
  L.cursor = ws.take<unsigned long long>(1);
  L.overflow = ws.take<uint32_t>(1);
  L.g.overflow = L.overflow;
  return L;
}

GbVals gb_vals(const eiger_column *vals, int32_t nv) {
  GbVals v{};
  v.n = nv;
  for (int32_t c = 0; c < nv; ++c) {
    const uint32_t *base = static_cast<const uint32_t *>(vals[c].data);
    const bool wide = vals[c].dtype == EIGER_INT64;
    v.lo[c] = base;
    v.hi[c] = wide && base ? base + 1 : base;
    v.wide[c] = wide ? 1u : 0u;
    v.stride[c] = wide ? 2 : 1;
  }
  return v;
}

// Lays out and (with a workspace base) enqueues the group-by.
template <typename K>
int gb_impl(const eiger_column &keys, const eiger_column *vals, int32_t nv, const eiger_groupby_plan_t &plan,
            const GbOut &out_in, Workspace &ws, GbLayout *lay, hipStream_t s) {
  const uint64_t n = static_cast<uint64_t>(keys.n);
  unsigned long long sentinel;
  gb_sentinel(plan, &sentinel);
  *lay = gb_layout(ws, static_cast<uint64_t>(plan.slots), nv, sentinel);
  PartitionOut part{};
  PartLanes wc{};
  if (plan.variant == EIGER_GB_PARTITION) {
    for (int32_t c = 0; c < nv; ++c) {
      const uint32_t *base = static_cast<const uint32_t *>(vals[c].data);
      if (vals[c].dtype == EIGER_INT64) {
        wc.src[wc.n] = base;
        wc.stride[wc.n++] = 2;
        wc.src[wc.n] = base ? base + 1 : nullptr;
        wc.stride[wc.n++] = 2;
      } else {
        wc.src[wc.n] = base;
        wc.stride[wc.n++] = 1;
      }
    }
    int rc = radix_partition_lanes(static_cast<int>(dtype_size(keys.dtype)), keys.data, n, wc, plan.radix_bits, ws,
                                   &part, n > 0 ? s : nullptr, n > 0);
    if (rc) return rc;
  }
  if (!ws.base) return EIGER_OK;
  const GbGlobal &g = lay->g;
  GbOut o = out_in;
  o.cursor = lay->cursor;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(lay->cursor), 1, 0, s))) return rc;
  if ((rc = fill_u32(lay->overflow, 1, 0, s))) return rc;
  const unsigned cus = static_cast<unsigned>(device_cu_count());
  EIGER_LAUNCH("groupby_clear", k_gb_clear, dim3(std::min<uint64_t>((plan.slots + kGNT - 1) / kGNT, cus * 8)),
               dim3(kGNT), 0, s, g, nv);
  if (n == 0) return EIGER_OK;
  if (plan.variant == EIGER_GB_HASH) {
    const GbVals v = gb_vals(vals, nv);
    const uint64_t chunks = (n + kGChunk - 1) / kGChunk;
    EIGER_LAUNCH("groupby_hash", k_gb_hash<K>, dim3(static_cast<unsigned>(std::min<uint64_t>(chunks, cus * 2))),
                 dim3(kGNT), 0, s, static_cast<const K *>(keys.data), n, v, g);
  } else {
    // partitioned values: one word array per lane (stride 1)
    GbVals v{};
    v.n = nv;
    int w = 0;
    for (int32_t c = 0; c < nv; ++c) {
      const bool wide = vals[c].dtype == EIGER_INT64;
      v.lo[c] = part.words[w];
      v.hi[c] = wide ? part.words[w + 1] : part.words[w];
      v.wide[c] = wide ? 1u : 0u;
      v.stride[c] = 1;
      w += wide ? 2 : 1;
    }
    const uint32_t F = 1u << plan.radix_bits;
    const uint32_t S = gb_slices(n, plan.radix_bits);
    EIGER_LAUNCH("groupby_partition", k_gb_partition<K>,
                 dim3(static_cast<unsigned>(std::min<uint64_t>(uint64_t(F) * S, cus * 2))), dim3(kGNT), 0, s,
                 static_cast<const K *>(part.keys), v, part.off, F, S, g, o);
  }
  EIGER_LAUNCH("groupby_emit", k_gb_emit, dim3(static_cast<unsigned>(std::min<uint64_t>(
                                              (plan.slots + 4095) / 4096, cus * 4))),
               dim3(kGNT), 0, s, g, nv, o);
  return EIGER_OK;
}

int gb_run(const eiger_column &keys, const eiger_column *vals, int32_t nv, const eiger_groupby_plan_t &plan,
           const GbOut &o, Workspace &ws, GbLayout *lay, hipStream_t s) {
  if (keys.dtype == EIGER_INT64) return gb_impl<int64_t>(keys, vals, nv, plan, o, ws, lay, s);
  return gb_impl<int32_t>(keys, vals, nv, plan, o, ws, lay, s);
}

int gb_check(const eiger_column &keys, const eiger_column *vals, int32_t nv, const eiger_groupby_plan_t *plan) {
  if (!plan) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: plan is NULL");
  if (keys.dtype != EIGER_INT32 && keys.dtype != EIGER_INT64)
    return fail(EIGER_ERR_DTYPE, "eiger_groupby: key dtype must be EIGER_INT32 or EIGER_INT64");
  if (keys.dtype != plan->key_dtype) return fail(EIGER_ERR_DTYPE, "eiger_groupby: plan.key_dtype differs from the keys");
  if (keys.n < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: negative row count");
  if (keys.n > EIGER_MAX_ROWS) return fail(EIGER_ERR_TOO_LARGE, "eiger_groupby: more than EIGER_MAX_ROWS rows");
  if (keys.n > 0 && (!keys.data || reinterpret_cast<uintptr_t>(keys.data) % dtype_size(keys.dtype)))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: keys NULL or misaligned");
  if (nv < 0 || nv > kGMaxVals) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: 0 to 2 value columns");
  if (nv > 0 && !vals) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: NULL value column array");
  for (int32_t c = 0; c < nv; ++c) {
    if (vals[c].dtype != EIGER_INT32 && vals[c].dtype != EIGER_INT64)
      return fail(EIGER_ERR_DTYPE, "eiger_groupby: value dtype must be EIGER_INT32 or EIGER_INT64");
    if (vals[c].n != keys.n) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: value column length differs");
    if (keys.n > 0 && (!vals[c].data || reinterpret_cast<uintptr_t>(vals[c].data) % dtype_size(vals[c].dtype)))
      return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: value column NULL or misaligned");
  }
  if (plan->variant != EIGER_GB_HASH && plan->variant != EIGER_GB_PARTITION)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: plan.variant is not an eiger_groupby_variant");
  if (plan->slots < 1024 || (plan->slots & (plan->slots - 1)))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: plan.slots must be a power of two >= 1024");
  if (plan->variant == EIGER_GB_PARTITION && (plan->radix_bits < 1 || plan->radix_bits > 18))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: plan.radix_bits must be in [1, 18]");
  if (plan->flags & EIGER_GB_NO_SENTINEL)
    return fail(EIGER_ERR_UNSUPPORTED, "eiger_groupby: the keys span the whole int64 domain (no free value marks "
                                       "empty slots)");
  return EIGER_OK;
}

}  // namespace
}  // namespace eiger

using namespace eiger;

extern "C" int eiger_groupby_plan(const eiger_stats_t *keys, int32_t selector, const eiger_groupby_plan_t *forced,
                                  eiger_groupby_plan_t *out) {
  if (!keys || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby_plan: NULL argument");
  if (keys->dtype != EIGER_INT32 && keys->dtype != EIGER_INT64)
    return fail(EIGER_ERR_DTYPE, "eiger_groupby_plan: unsupported key dtype");
  eiger_groupby_plan_t p{};
  p.key_dtype = keys->dtype;
  // a value outside [min, max] marks empty slots; int32 keys never reach INT64_MIN
  if (keys->dtype == EIGER_INT32 || keys->n == 0 || keys->min > INT64_MIN) {
    p.sentinel = INT64_MIN;
  } else if (keys->max < INT64_MAX) {
    p.sentinel = INT64_MAX;
  } else {
    p.flags |= EIGER_GB_NO_SENTINEL;
  }
  const double est = std::max(1.0, std::min(keys->ndv, static_cast<double>(std::max<int64_t>(keys->n, 1))));
  p.predicted_groups = static_cast<int64_t>(std::llround(est));
  if (selector == EIGER_SEL_FORCED) {
    if (!forced) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby_plan: EIGER_SEL_FORCED needs `forced`");
    p.variant = forced->variant;
    p.radix_bits = forced->radix_bits;
  } else if (selector == EIGER_SEL_RULE || selector == EIGER_SEL_LEARNED) {
    p.variant = est <= kGbHashMaxGroups ? EIGER_GB_HASH : EIGER_GB_PARTITION;
    p.radix_bits = 0;
  } else {
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby_plan: selector must be EIGER_SEL_RULE or EIGER_SEL_FORCED");
  }
  if (p.variant == EIGER_GB_PARTITION && (p.radix_bits < 1 || p.radix_bits > 18)) {
    int bits = 1;
    while (bits < 18 && est / std::ldexp(1.0, bits) > kGbGroupsPerPartition) ++bits;
    p.radix_bits = bits;
  }
  // the global table: NDV-sized (twice the estimate) when every group reaches
  // it (HASH, or sliced partitions); unsliced partitions only spill into it
  const bool all_global = p.variant == EIGER_GB_HASH || gb_slices(static_cast<uint64_t>(keys->n), p.radix_bits) > 1;
  p.slots = static_cast<int64_t>(gb_slots(all_global ? est : est / 8.0));
  *out = p;
  return EIGER_OK;
}

extern "C" int eiger_groupby_workspace_size(const eiger_groupby_plan_t *plan, eiger_column keys,
                                            const eiger_column *vals, int32_t n_vals, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby_workspace_size: bytes is NULL");
  static const int64_t dummy[1] = {0};
  eiger_column k = keys, v[kGMaxVals];
  if (k.n > 0) k.data = dummy;
  if (n_vals < 0 || n_vals > kGMaxVals) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: 0 to 2 value columns");
  for (int32_t c = 0; c < n_vals; ++c) {
    if (!vals) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: NULL value column array");
    v[c] = vals[c];
    if (v[c].n > 0) v[c].data = dummy;
  }
  int rc = gb_check(k, v, n_vals, plan);
  if (rc) return rc;
  Workspace ws(nullptr, 0);
  GbLayout lay{};
  if ((rc = gb_run(k, v, n_vals, *plan, GbOut{}, ws, &lay, nullptr))) return rc;
  *bytes = ws.used;
  return EIGER_OK;
}

extern "C" int eiger_groupby(eiger_column keys, const eiger_column *vals, int32_t n_vals,
                             const eiger_groupby_plan_t *plan, void *out_keys, int64_t *out_counts,
                             int64_t *const *out_sums, int64_t out_capacity, int64_t *out_groups, void *ws_ptr,
                             size_t ws_bytes, void *stream) {
  int rc = gb_check(keys, vals, n_vals, plan);
  if (rc) return rc;
  if (!out_groups) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: out_groups is NULL");
  if (out_capacity < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: negative out_capacity");
  if (out_capacity > 0 && (!out_keys || !out_counts || (n_vals > 0 && !out_sums)))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: NULL output arrays");
  for (int32_t c = 0; out_capacity > 0 && c < n_vals; ++c)
    if (!out_sums[c]) return fail(EIGER_ERR_INVALID_ARG, "eiger_groupby: NULL sum output");
  {
    Workspace dry(nullptr, 0);
    GbLayout lay{};
    if ((rc = gb_run(keys, vals, n_vals, *plan, GbOut{}, dry, &lay, nullptr))) return rc;
    if (!ws_ptr || dry.used > ws_bytes)
      return fail(EIGER_ERR_WORKSPACE, "eiger_groupby: workspace too small (need " + std::to_string(dry.used) +
                                           " bytes)");
  }
  GbOut o{};
  o.keys = out_capacity > 0 ? out_keys : nullptr;
  o.cnt = reinterpret_cast<unsigned long long *>(out_counts);
  for (int32_t c = 0; c < n_vals; ++c)
    o.sum[c] = out_capacity > 0 ? reinterpret_cast<unsigned long long *>(out_sums[c]) : nullptr;
  o.cap = static_cast<uint64_t>(out_capacity);
  o.kwide = keys.dtype == EIGER_INT64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws(ws_ptr, ws_bytes);
  GbLayout lay{};
  if ((rc = gb_run(keys, vals, n_vals, *plan, o, ws, &lay, s))) return rc;
  struct {
    unsigned long long groups;
    uint32_t overflow;
  } host{};
  EIGER_HIP(hipMemcpyAsync(&host.groups, lay.cursor, sizeof(host.groups), hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipMemcpyAsync(&host.overflow, lay.overflow, sizeof(host.overflow), hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipStreamSynchronize(s));
  if (host.overflow)
    return fail(EIGER_ERR_TOO_LARGE, "eiger_groupby: more groups than the plan's table slots (the distinct-count "
                                     "estimate was low); raise plan.slots");
  *out_groups = static_cast<int64_t>(host.groups);
  if (host.groups > static_cast<uint64_t>(out_capacity))
    return fail(EIGER_ERR_CAPACITY, "eiger_groupby: " + std::to_string(host.groups) + " groups exceed out_capacity " +
                                        std::to_string(out_capacity));
  return EIGER_OK;
}
