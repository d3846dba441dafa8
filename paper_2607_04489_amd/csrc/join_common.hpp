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

// Slot of a hash table in device memory: key, build row id and build payload
// side by side, 16 bytes (32 when key and payload are both 8 bytes), so one
// probe step is one aligned vector load. rowid == kEmpty marks an empty slot.
template <typename K, typename P>
struct alignas((sizeof(K) + sizeof(P) + 4 <= 16) ? 16 : 32) Slot {
  K key;
  uint32_t rowid;
  P pay;
};

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
  uint64_t scan[NT / 64 + 1];
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
__device__ __forceinline__ uint64_t reserve(EmitLds<NT, SCAP> &L, const EmitOut &o, uint64_t count) {
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

// Finish a workgroup's share: flush the stage and add its checksum part. In
// count-only mode `fill` is instead the workgroup's whole pair count (uniform).
template <int NT, int SCAP>
__device__ __forceinline__ void finish(EmitLds<NT, SCAP> &L, const EmitOut &o, uint64_t fill,
                                       uint64_t cs) {
  if (o.ob) {
    flush(L, o, static_cast<uint32_t>(fill));
  } else if (threadIdx.x == 0 && fill) {
    atomicAdd(reinterpret_cast<unsigned long long *>(o.cursor), static_cast<unsigned long long>(fill));
  }
  const uint64_t s = block_sum_u64<NT>(cs, L.red);
  if (threadIdx.x == 0 && s != 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(o.checksum), static_cast<unsigned long long>(s));
}

// Registers of one probe sub-tile: up to IPT rows per thread, rows
// lo + k * NT + threadIdx.x. (Holding the next sub-tile in registers as well
// was measured slower on gfx950: the extra registers cost more occupancy than
// the overlap gained.)
template <int IPT, typename K, typename PS>
struct ProbeRegs {
  K key[IPT];
  PS pay[IPT];
  uint32_t rid[IPT];
  uint64_t lo, hi;
};

template <int NT, int IPT, typename K, typename PS>
__device__ __forceinline__ void probe_load(ProbeRegs<IPT, K, PS> &r, const K *__restrict__ pk,
                                           const PS *__restrict__ pp,
                                           const uint32_t *__restrict__ prow, uint64_t lo,
                                           uint64_t hi) {
  r.lo = lo;
  r.hi = hi;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const uint64_t i = lo + uint64_t(k) * NT + threadIdx.x;
    if (i < hi) {
      r.key[k] = pk[i];
      r.pay[k] = pp[i];
      r.rid[k] = prow ? prow[i] : static_cast<uint32_t>(i);
    }
  }
}

// Count the matches of every loaded row. Tables of two kinds:
//  * hashed tables (Tab::kHashed) expose an index type Index, home(key),
//    next(i), load(i) -> slot and a `unique` flag (build keys known to be
//    distinct). The first slot of
//    every row is loaded before any is inspected, so a thread keeps IPT random
//    loads in flight; only rows whose walk is not finished load again, and a
//    unique table stops a walk at its first match.
//  * other tables expose lookup(key, first, payload_sum) -> count, where
//    `first` is the first match's row id, or with Tab::kRuns the start of the
//    key's contiguous run of rows (emit_matches).
template <int NT, int IPT, class Tab, typename K, typename PS>
__device__ __forceinline__ void count_matches(const Tab &tab, const ProbeRegs<IPT, K, PS> &r,
                                              uint32_t (&cnt)[IPT], uint32_t (&first)[IPT],
                                              uint64_t (&psum)[IPT]) {
  bool valid[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    valid[k] = r.lo + uint64_t(k) * NT + threadIdx.x < r.hi;
    cnt[k] = 0;
    psum[k] = 0;
  }
  if constexpr (Tab::kHashed) {
    typename Tab::Index idx[IPT];
    typename Tab::SlotT sl[IPT];
    bool live[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (valid[k]) idx[k] = tab.home(r.key[k]);
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (valid[k]) sl[k] = tab.load(idx[k]);
    bool any = false;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      live[k] = valid[k];
      if (!live[k]) continue;
      if (sl[k].rowid == kEmpty) {
        live[k] = false;
      } else {
        if (sl[k].key == r.key[k]) {
          ++cnt[k];
          first[k] = sl[k].rowid;
          psum[k] += static_cast<uint64_t>(sext(sl[k].pay));
          if (tab.unique) live[k] = false;
        }
        if (live[k]) {
          idx[k] = tab.next(idx[k]);
          any = true;
        }
      }
    }
    while (any) {
      any = false;
#pragma unroll
      for (int k = 0; k < IPT; ++k)
        if (live[k]) sl[k] = tab.load(idx[k]);
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        if (!live[k]) continue;
        if (sl[k].rowid == kEmpty) {
          live[k] = false;
        } else {
          if (sl[k].key == r.key[k]) {
            ++cnt[k];
            first[k] = sl[k].rowid;
            psum[k] += static_cast<uint64_t>(sext(sl[k].pay));
            if (tab.unique) live[k] = false;
          }
          if (live[k]) {
            idx[k] = tab.next(idx[k]);
            any = true;
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (valid[k]) cnt[k] = tab.lookup(r.key[k], first[k], psum[k]);
  }
}

// Calls f(build_rowid) for each of the `cnt` matches of a probe row whose
// lookup gave `first`. Tables that keep a key's rows contiguous (Tab::kRuns)
// return the start of the run in `first` and expose row_at(i), so the matches
// are read straight from the run; other tables return the first match's row
// id and walk again (for_each) when there are more.
template <class Tab, typename K, class F>
__device__ __forceinline__ void emit_matches(const Tab &tab, K key, uint32_t cnt, uint32_t first, F f) {
  if constexpr (Tab::kRuns) {
    for (uint32_t j = 0; j < cnt; ++j) f(tab.row_at(first + j));
  } else {
    if (cnt == 1)
      f(first);
    else if (cnt > 1)
      tab.for_each(key, f);
  }
}

// Probe the loaded rows against `tab` and materialize the matches. Tables also
// provide  template <class F> void for_each(K key, F f) const  (f(build_rowid)
// for every match) for rows with more than one match. Match totals are 64-bit:
// a sub-tile of rows that each meet billions of build rows does not wrap.
// Uniform across the workgroup (contains barriers).
template <int NT, int IPT, int SCAP, class Tab, typename K, typename PS>
__device__ __forceinline__ void probe_process(const Tab &tab, const ProbeRegs<IPT, K, PS> &r,
                                              EmitLds<NT, SCAP> &L, uint64_t &fill,
                                              const EmitOut &o, uint64_t &cs) {
  uint32_t cnt[IPT], first[IPT];
  uint64_t psum[IPT];
  count_matches<NT, IPT>(tab, r, cnt, first, psum);
  uint64_t mine = 0;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (cnt[k]) cs += psum[k] * static_cast<uint64_t>(sext(r.pay[k]));
    mine += cnt[k];
  }
  uint64_t total;
  const uint64_t off = block_exclusive_scan<NT, uint64_t>(mine, L.scan, &total);
  if (total == 0) return;
  if (!o.ob) {  // count-only: no positions are needed, so nothing is reserved
    fill += total;
    return;
  }
  if (fill + total > SCAP) {
    flush(L, o, static_cast<uint32_t>(fill));
    fill = 0;
  }
  // (probes of 8 rows per thread keep the per-row path below: the row table's
  // registers would cost them occupancy)
  if constexpr (Tab::kRuns && IPT <= 4) {
    static_assert(SCAP >= 2 * NT && NT <= 65536, "the stage holds a round's row table");
    if (total > SCAP) {
      // More matches than the stage holds (duplicated build keys; the stage is
      // empty here). Reserve the sub-tile's output range, then expand one row
      // slot k at a time (NT rows per round): the round's row table goes into
      // the stage arrays, and the pairs are written by consecutive threads at
      // consecutive positions, each reading its build row by index from the
      // key's run.
      const uint64_t base = reserve(L, o, total);
      uint64_t done = 0;  // pairs of this sub-tile placed so far (uniform)
      // row table: rd[i] = run start of row i minus the index of its first
      // pair (mod 2^32), so pair g of row i is build row tab.row_at(rd[i] + g);
      // rq[i] = its probe row id; row_of: the row of each pair of a chunk
      uint32_t *rd = L.b, *rq = L.b + NT;
      uint16_t *row_of = reinterpret_cast<uint16_t *>(L.p);
      constexpr uint32_t CH = 2 * SCAP;
      // every round's offsets from one scan of 16-bit fields when the whole
      // sub-tile has fewer than 2^16 pairs (no field can carry into the next)
      const bool packed = total < (uint64_t(1) << 16);
      uint64_t pk_ok = 0, pk_tot = 0;
      if (packed) {
        uint64_t v = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) v |= static_cast<uint64_t>(cnt[k]) << (16 * k);
        pk_ok = block_exclusive_scan<NT, uint64_t>(v, L.scan, &pk_tot);
      }
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        uint64_t tk, ok;
        if (packed) {
          ok = (pk_ok >> (16 * k)) & 0xFFFFu;
          tk = (pk_tot >> (16 * k)) & 0xFFFFu;
        } else {
          ok = block_exclusive_scan<NT, uint64_t>(cnt[k], L.scan, &tk);
        }
        if (tk == 0) continue;
        if (tk >= (uint64_t(1) << 32)) {  // offsets do not fit the row table: per row
          uint64_t pos = base + done + ok;
          const uint32_t rr = r.rid[k];
          emit_matches(tab, r.key[k], cnt[k], first[k], [&](uint32_t b) { put_pair(o, pos++, b, rr); });
          done += tk;
          continue;
        }
        rd[threadIdx.x] = first[k] - static_cast<uint32_t>(ok);
        rq[threadIdx.x] = r.rid[k];
        // pairs of the round in chunks of CH: each thread marks its row on its
        // pairs' entries of `row_of`, then consecutive threads take consecutive
        // pairs, so the stores are coalesced
        for (uint64_t c0 = 0; c0 < tk; c0 += CH) {
          const uint64_t c1 = c0 + CH < tk ? c0 + CH : tk;
          const uint64_t a = ok > c0 ? ok : c0;
          const uint64_t e = ok + cnt[k] < c1 ? ok + cnt[k] : c1;
          for (uint64_t g = a; g < e; ++g) row_of[g - c0] = static_cast<uint16_t>(threadIdx.x);
          __syncthreads();
          uint64_t g = c0 + threadIdx.x;
          for (; g + NT < c1; g += 2 * NT) {  // two pairs per step: two lookup chains in flight
            const uint32_t i0 = row_of[g - c0], i1 = row_of[g + NT - c0];
            const uint32_t b0 = tab.row_at(rd[i0] + static_cast<uint32_t>(g));
            const uint32_t b1 = tab.row_at(rd[i1] + static_cast<uint32_t>(g + NT));
            put_pair(o, base + done + g, b0, rq[i0]);
            put_pair(o, base + done + g + NT, b1, rq[i1]);
          }
          if (g < c1) {
            const uint32_t i = row_of[g - c0];
            put_pair(o, base + done + g, tab.row_at(rd[i] + static_cast<uint32_t>(g)), rq[i]);
          }
          __syncthreads();
        }
        done += tk;
      }
      return;
    }
  }
  if (total > SCAP) {
    // More matches than the stage holds (duplicated build keys; the stage is
    // empty here): reserve the sub-tile's whole output range with one atomic,
    // then stage it one row slot k at a time (NT rows per round) and copy each
    // round to its place in the range, so these pairs are also written
    // contiguously; a round that alone overflows the stage writes straight
    // into the range.
    const uint64_t base = reserve(L, o, total);
    uint64_t done = 0;  // pairs of this sub-tile placed so far (uniform)
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      uint64_t tk;
      const uint64_t ok = block_exclusive_scan<NT, uint64_t>(cnt[k], L.scan, &tk);
      if (tk == 0) continue;
      if (tk > SCAP) {
        uint64_t pos = base + done + ok;
        const uint32_t rr = r.rid[k];
        emit_matches(tab, r.key[k], cnt[k], first[k], [&](uint32_t b) { put_pair(o, pos++, b, rr); });
        done += tk;
        continue;
      }
      uint32_t pos = static_cast<uint32_t>(ok);
      const uint32_t rr = r.rid[k];
      emit_matches(tab, r.key[k], cnt[k], first[k], [&](uint32_t b) {
        L.b[pos] = b;
        L.p[pos] = rr;
        ++pos;
      });
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < tk; i += NT) put_pair(o, base + done + i, L.b[i], L.p[i]);
      __syncthreads();
      done += tk;
    }
    return;
  }
  uint32_t pos = static_cast<uint32_t>(fill + off);
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const uint32_t rr = r.rid[k];
    emit_matches(tab, r.key[k], cnt[k], first[k], [&](uint32_t b) {
      L.b[pos] = b;
      L.p[pos] = rr;
      ++pos;
    });
  }
  __syncthreads();
  fill += total;
}

// Probe the rows [lo, hi) in sub-tiles of NT * IPT rows. Uniform across the
// workgroup.
template <int NT, int IPT, int SCAP, class Tab, typename K, typename PS>
__device__ __forceinline__ void probe_range(const Tab &tab, const K *__restrict__ pk,
                                            const PS *__restrict__ pp,
                                            const uint32_t *__restrict__ prow, uint64_t lo,
                                            uint64_t hi, EmitLds<NT, SCAP> &L, uint64_t &fill,
                                            const EmitOut &o, uint64_t &cs) {
  constexpr uint64_t sub = uint64_t(NT) * IPT;
  if (lo >= hi) return;
  ProbeRegs<IPT, K, PS> cur;
  for (uint64_t t = lo; t < hi; t += sub) {
    probe_load<NT, IPT>(cur, pk, pp, prow, t, t + sub < hi ? t + sub : hi);
    probe_process<NT, IPT, SCAP>(tab, cur, L, fill, o, cs);
  }
}

}  // namespace eiger
