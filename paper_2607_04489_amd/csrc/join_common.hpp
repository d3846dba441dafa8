// join_common.hpp -- output materialization shared by the join variants.
//
// Every variant probes tiles of NT * IPT probe rows. A probe row may match any
// number of build rows. Matches are compacted per workgroup with a block-wide
// exclusive scan of per-thread match counts and staged in LDS; a full stage is
// flushed with ONE atomic add on the global output cursor and written out with
// consecutive threads on consecutive addresses. The payload aggregate uses
// distributivity mod 2^64: a probe row adds probe_payload * (sum of the payloads
// of its matching build rows).
#pragma once

#include "common.hpp"

namespace eiger {

// Where pairs go. ob/op may be null (count-only); positions >= cap are dropped.
struct EmitOut {
  uint32_t *ob;
  uint32_t *op;
  uint64_t cap;
  uint64_t *cursor;    // device u64, zero before the first launch
  uint64_t *checksum;  // device u64, zero before the first launch
};

template <int NT, int SCAP>
struct EmitLds {
  uint32_t b[SCAP];
  uint32_t p[SCAP];
  uint32_t scan[NT / 64 + 1];
  uint64_t base;
  uint64_t red[NT / 64];
};

__device__ __forceinline__ void put_pair(const EmitOut &o, uint64_t pos, uint32_t b, uint32_t p) {
  if (o.ob && pos < o.cap) {
    o.ob[pos] = b;
    o.op[pos] = p;
  }
}

// Reserve `count` output slots for the whole workgroup; all threads get the base.
template <int NT, int SCAP>
__device__ __forceinline__ uint64_t reserve(EmitLds<NT, SCAP> &L, const EmitOut &o, uint32_t count) {
  if (threadIdx.x == 0) L.base = atomicAdd(reinterpret_cast<unsigned long long *>(o.cursor),
                                           static_cast<unsigned long long>(count));
  __syncthreads();
  const uint64_t base = L.base;
  __syncthreads();
  return base;
}

// Write the staged pairs [0, fill) to the output. Uniform across the workgroup.
template <int NT, int SCAP>
__device__ __forceinline__ void flush(EmitLds<NT, SCAP> &L, const EmitOut &o, uint32_t fill) {
  if (fill == 0) return;
  const uint64_t base = reserve(L, o, fill);
  if (o.ob) {
    for (uint32_t i = threadIdx.x; i < fill; i += NT) put_pair(o, base + i, L.b[i], L.p[i]);
  }
  __syncthreads();
}

// Finish a workgroup's share: flush the stage and add its checksum part.
template <int NT, int SCAP>
__device__ __forceinline__ void finish(EmitLds<NT, SCAP> &L, const EmitOut &o, uint32_t fill,
                                       uint64_t cs) {
  flush(L, o, fill);
  const uint64_t s = block_sum_u64<NT>(cs, L.red);
  if (threadIdx.x == 0 && s != 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(o.checksum), static_cast<unsigned long long>(s));
}

// Probe rows [lo, hi) (at most NT * IPT of them) against `tab` and materialize
// the matches. Tab provides
//   uint32_t lookup(K key, uint32_t &first_rowid, uint64_t &payload_sum) const
//   template <class F> void for_each(K key, F f) const   // f(build_rowid)
// Probe row ids are `prow[i]` when prow is non-null, else the index i itself.
// Uniform across the workgroup (contains barriers).
template <int NT, int IPT, int SCAP, class Tab, typename K, typename PS>
__device__ __forceinline__ void probe_tile(const Tab &tab, const K *__restrict__ pk,
                                           const PS *__restrict__ pp,
                                           const uint32_t *__restrict__ prow, uint64_t lo,
                                           uint64_t hi, EmitLds<NT, SCAP> &L, uint32_t &fill,
                                           const EmitOut &o, uint64_t &cs) {
  K key[IPT];
  uint32_t cnt[IPT], first[IPT], rid[IPT];
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const uint64_t i = lo + uint64_t(k) * NT + threadIdx.x;
    cnt[k] = 0;
    if (i < hi) {
      key[k] = pk[i];
      rid[k] = prow ? prow[i] : static_cast<uint32_t>(i);
    }
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const uint64_t i = lo + uint64_t(k) * NT + threadIdx.x;
    if (i < hi) {
      uint64_t psum = 0;
      cnt[k] = tab.lookup(key[k], first[k], psum);
      if (cnt[k]) cs += psum * static_cast<uint64_t>(sext(pp[i]));
      mine += cnt[k];
    }
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan<NT>(mine, L.scan, &total);
  if (total == 0) return;
  if (fill + total > SCAP) {
    flush(L, o, fill);
    fill = 0;
  }
  if (total > SCAP) {
    // A tile with more matches than the stage holds (heavy duplicates): write
    // straight to the output range reserved for the whole tile.
    const uint64_t base = reserve(L, o, total);
    uint64_t pos = base + off;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (cnt[k] == 1) {
        put_pair(o, pos++, first[k], rid[k]);
      } else if (cnt[k] > 1) {
        const uint32_t r = rid[k];
        tab.for_each(key[k], [&](uint32_t b) { put_pair(o, pos++, b, r); });
      }
    }
    return;
  }
  uint32_t pos = fill + off;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (cnt[k] == 1) {
      L.b[pos] = first[k];
      L.p[pos] = rid[k];
      ++pos;
    } else if (cnt[k] > 1) {
      const uint32_t r = rid[k];
      tab.for_each(key[k], [&](uint32_t b) {
        L.b[pos] = b;
        L.p[pos] = r;
        ++pos;
      });
    }
  }
  __syncthreads();
  fill += total;
}

}  // namespace eiger
