// join_radix.hip -- RADIX variant: hash-radix partitioning, then one LDS-resident
// hash table per partition.
//
// The paper's partitioned hash join (Section 3.2, Table 1; its internals are
// those of Wu et al., which the paper cites rather than prints) is re-derived
// here for gfx950:
//  * Both sides are partitioned on the top bits of fmix64(key) (hashing before
//    partitioning evens out partition sizes, as the paper does for its
//    partitioned group-by, Section 3.3), in one or two passes of at most 9 bits.
//  * A pass is histogram -> exclusive scan -> scatter. The scatter sorts a tile
//    of 2048 tuples by partition in LDS first, so consecutive threads write
//    consecutive addresses of one partition. Key, payload and row id travel
//    together (the GFTR idea, Section 3.2: payloads follow the keys' transform),
//    so the join phase reads only partitioned, contiguous data.
//  * Pass 2 partitions every pass-1 partition on the next bits ("segments"); a
//    workgroup handles a chunk of one segment.
//  * Join: one work item per (partition, probe tile). The workgroup builds an
//    LDS open-addressing table (multiset, CAS on the row-id word) from the
//    partition's build rows -- in several chunks when they do not fit -- and
//    streams the probe tile against it.
#include <algorithm>

#include "join_common.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr int kPNT = 512;       // partition workgroup
constexpr int kPIPT = 4;        // tuples per thread per tile
constexpr int kPTile = kPNT * kPIPT;
constexpr uint32_t kChunk = 16384;  // tuples per partitioning workgroup (one histogram)
constexpr int kMaxPassBits = 9;     // buckets per pass <= kPNT

constexpr int kJNT = 512;       // join workgroup
constexpr int kJIPT = 4;
constexpr int kJSCAP = 2048;    // staged output pairs
constexpr int kTableBytes = 48 * 1024;
constexpr uint32_t kJTile = 32768;  // probe rows per work item

__device__ __forceinline__ uint32_t bucket_of(uint64_t key_bits, int shift, uint32_t mask) {
  return static_cast<uint32_t>(fmix64(key_bits) >> shift) & mask;
}

// Largest s with cpre[s] <= c, over s in [0, nseg).
__device__ __forceinline__ uint32_t find_segment(const uint32_t *cpre, uint32_t nseg, uint32_t c) {
  uint32_t lo = 0, hi = nseg;  // invariant: cpre[lo] <= c < cpre[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (cpre[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

// Chunks per segment, written as counts for an exclusive scan (entry nseg = 0).
__global__ void k_chunk_counts(const uint32_t *__restrict__ seg_off, uint32_t nseg,
                               uint32_t *__restrict__ cnt) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) cnt[s] = (seg_off[s + 1] - seg_off[s] + kChunk - 1) / kChunk;
  if (s == nseg) cnt[s] = 0;
}

__global__ void k_single_segment(uint32_t *seg_off, uint32_t *cpre, uint32_t n) {
  if (threadIdx.x == 0) {
    seg_off[0] = 0;
    seg_off[1] = n;
    cpre[0] = 0;
    cpre[1] = (n + kChunk - 1) / kChunk;
  }
}

template <typename K>
__global__ void __launch_bounds__(kPNT)
    k_part_hist(const K *__restrict__ keys, const uint32_t *__restrict__ seg_off,
                const uint32_t *__restrict__ cpre, uint32_t nseg, int shift, int bits,
                uint32_t *__restrict__ C) {
  __shared__ uint32_t hist[1 << kMaxPassBits];
  const uint32_t c = blockIdx.x;
  if (c >= cpre[nseg]) return;
  const uint32_t B = 1u << bits;
  for (uint32_t b = threadIdx.x; b < B; b += kPNT) hist[b] = 0;
  __syncthreads();
  const uint32_t s = find_segment(cpre, nseg, c);
  const uint32_t lc = c - cpre[s], nch = cpre[s + 1] - cpre[s];
  const uint32_t lo = seg_off[s] + lc * kChunk;
  const uint32_t hi = min(seg_off[s + 1], lo + kChunk);
  for (uint32_t i = lo + threadIdx.x; i < hi; i += kPNT)
    atomicAdd(&hist[bucket_of(static_cast<uint64_t>(sext(keys[i])), shift, B - 1)], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < B; b += kPNT) C[uint64_t(cpre[s]) * B + uint64_t(b) * nch + lc] = hist[b];
}

template <typename K, typename P, bool kRows>
__global__ void __launch_bounds__(kPNT)
    k_part_scatter(const K *__restrict__ keys, const P *__restrict__ pays,
                   const uint32_t *__restrict__ rows, const uint32_t *__restrict__ seg_off,
                   const uint32_t *__restrict__ cpre, uint32_t nseg, int shift, int bits,
                   const uint32_t *__restrict__ C, K *__restrict__ okeys, P *__restrict__ opays,
                   uint32_t *__restrict__ orows) {
  __shared__ K lk[kPTile];
  __shared__ P lp[kPTile];
  __shared__ uint32_t lr[kPTile];
  __shared__ uint16_t lb[kPTile];
  __shared__ uint32_t hist[1 << kMaxPassBits], loff[1 << kMaxPassBits], gcur[1 << kMaxPassBits];
  __shared__ uint32_t scan_tmp[kPNT / 64 + 1];
  const uint32_t c = blockIdx.x;
  if (c >= cpre[nseg]) return;
  const uint32_t B = 1u << bits;
  const uint32_t s = find_segment(cpre, nseg, c);
  const uint32_t lc = c - cpre[s], nch = cpre[s + 1] - cpre[s];
  const uint32_t lo = seg_off[s] + lc * kChunk;
  const uint32_t hi = min(seg_off[s + 1], lo + kChunk);
  for (uint32_t b = threadIdx.x; b < B; b += kPNT) {
    hist[b] = 0;
    gcur[b] = C[uint64_t(cpre[s]) * B + uint64_t(b) * nch + lc];
  }
  __syncthreads();
  for (uint32_t t0 = lo; t0 < hi; t0 += kPTile) {
    const uint32_t t1 = min(hi, t0 + kPTile);
    K key[kPIPT];
    P pay[kPIPT];
    uint32_t row[kPIPT], bk[kPIPT], rk[kPIPT];
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        key[k] = keys[i];
        pay[k] = pays[i];
        row[k] = kRows ? rows[i] : i;
        bk[k] = bucket_of(static_cast<uint64_t>(sext(key[k])), shift, B - 1);
        rk[k] = atomicAdd(&hist[bk[k]], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of the tile histogram (B <= kPNT: one bucket per thread)
    uint32_t total;
    const uint32_t h = threadIdx.x < B ? hist[threadIdx.x] : 0u;
    const uint32_t ex = block_exclusive_scan<kPNT>(h, scan_tmp, &total);
    if (threadIdx.x < B) loff[threadIdx.x] = ex;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        const uint32_t pos = loff[bk[k]] + rk[k];
        lk[pos] = key[k];
        lp[pos] = pay[k];
        lr[pos] = row[k];
        lb[pos] = static_cast<uint16_t>(bk[k]);
      }
    }
    __syncthreads();
    const uint32_t n = t1 - t0;
    for (uint32_t e = threadIdx.x; e < n; e += kPNT) {
      const uint32_t b = lb[e];
      const uint32_t dst = gcur[b] + (e - loff[b]);
      okeys[dst] = lk[e];
      opays[dst] = lp[e];
      orows[dst] = lr[e];
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += kPNT) {
      gcur[b] += hist[b];
      hist[b] = 0;
    }
    __syncthreads();
  }
}

// Final partition offsets: partition (s, b) starts at the first chunk's scanned
// counter of bucket b in segment s (or at the segment start when it has no chunks).
__global__ void k_part_offsets(const uint32_t *__restrict__ seg_off, const uint32_t *__restrict__ cpre,
                               uint32_t nseg, int bits, const uint32_t *__restrict__ C,
                               uint32_t *__restrict__ part_off, uint32_t n) {
  const uint32_t B = 1u << bits;
  const uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < uint64_t(nseg) * B) {
    const uint32_t s = static_cast<uint32_t>(q >> bits), b = static_cast<uint32_t>(q & (B - 1));
    const uint32_t nch = cpre[s + 1] - cpre[s];
    part_off[q] = nch ? C[uint64_t(cpre[s]) * B + uint64_t(b) * nch] : seg_off[s];
  }
  if (q == uint64_t(nseg) * B) part_off[q] = n;
}

// Work items per partition: probe tiles when both sides are non-empty.
__global__ void k_items(const uint32_t *__restrict__ offR, const uint32_t *__restrict__ offS,
                        uint32_t F, uint32_t *__restrict__ cnt) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < F) {
    const uint32_t nr = offR[p + 1] - offR[p], ns = offS[p + 1] - offS[p];
    cnt[p] = (nr && ns) ? (ns + kJTile - 1) / kJTile : 0u;
  }
  if (p == F) cnt[p] = 0;
}

template <typename K, typename PB>
struct LdsTab {
  K *tk;
  uint32_t *tr;
  PB *tp;
  uint32_t nslots;

  __device__ __forceinline__ uint32_t home(K key) const {
    const uint32_t h = static_cast<uint32_t>(fmix64(static_cast<uint64_t>(sext(key))));
    return static_cast<uint32_t>((uint64_t(h) * nslots) >> 32);
  }
  __device__ __forceinline__ uint32_t lookup(K key, uint32_t &first, uint64_t &psum) const {
    uint32_t i = home(key), c = 0;
    for (;;) {
      const uint32_t r = tr[i];
      if (r == kEmpty) break;
      if (tk[i] == key) {
        first = r;
        psum += static_cast<uint64_t>(sext(tp[i]));
        ++c;
      }
      i = (i + 1 == nslots) ? 0 : i + 1;
    }
    return c;
  }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint32_t i = home(key);
    for (;;) {
      const uint32_t r = tr[i];
      if (r == kEmpty) break;
      if (tk[i] == key) f(r);
      i = (i + 1 == nslots) ? 0 : i + 1;
    }
  }
};

template <typename K, typename PB>
__host__ __device__ constexpr uint32_t lds_max_slots() {
  return kTableBytes / (sizeof(K) + sizeof(PB) + sizeof(uint32_t));
}

template <typename K, typename PB, typename PS>
__global__ void __launch_bounds__(kJNT)
    k_radix_join(const K *__restrict__ rk, const PB *__restrict__ rp, const uint32_t *__restrict__ rr,
                 const uint32_t *__restrict__ offR, const K *__restrict__ sk,
                 const PS *__restrict__ sp, const uint32_t *__restrict__ sr,
                 const uint32_t *__restrict__ offS, const uint32_t *__restrict__ item_off, uint32_t F,
                 uint32_t max_build, float lf, EmitOut o) {
  constexpr uint32_t MAXS = lds_max_slots<K, PB>();
  __shared__ K tk[MAXS];
  __shared__ uint32_t tr[MAXS];
  __shared__ PB tp[MAXS];
  __shared__ EmitLds<kJNT, kJSCAP> L;
  uint32_t fill = 0;
  uint64_t cs = 0;
  const uint32_t nitems = item_off[F];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    // partition p: item_off[p] <= it < item_off[p+1]
    uint32_t lo = 0, hi = F;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (item_off[mid] <= it) lo = mid; else hi = mid;
    }
    const uint32_t p = lo;
    const uint32_t tile = it - item_off[p];
    const uint32_t r0 = offR[p], r1 = offR[p + 1];
    const uint32_t s0 = offS[p] + tile * kJTile;
    const uint32_t s1 = min(offS[p + 1], s0 + kJTile);
    for (uint32_t c0 = r0; c0 < r1; c0 += max_build) {
      const uint32_t c1 = min(r1, c0 + max_build);
      const uint32_t nb = c1 - c0;
      uint32_t ns = static_cast<uint32_t>(static_cast<float>(nb) / lf) + 1;
      ns = ns < 64 ? 64 : (ns > MAXS ? MAXS : ns);
      for (uint32_t i = threadIdx.x; i < ns; i += kJNT) tr[i] = kEmpty;
      __syncthreads();
      LdsTab<K, PB> tab{tk, tr, tp, ns};
      for (uint32_t j = c0 + threadIdx.x; j < c1; j += kJNT) {
        const K key = rk[j];
        uint32_t i = tab.home(key);
        for (;;) {
          if (atomicCAS(&tr[i], kEmpty, rr[j]) == kEmpty) {
            tk[i] = key;
            tp[i] = rp[j];
            break;
          }
          i = (i + 1 == ns) ? 0 : i + 1;
        }
      }
      __syncthreads();
      for (uint32_t t = s0; t < s1; t += kJNT * kJIPT)
        probe_tile<kJNT, kJIPT, kJSCAP>(tab, sk, sp, sr, t, min(s1, t + kJNT * kJIPT), L, fill, o, cs);
      __syncthreads();
    }
  }
  finish(L, o, fill, cs);
}

template <typename K, typename P>
struct Side {
  K *k;
  P *p;
  uint32_t *r;
};

struct PassPlan {
  int bits[2];
  int passes;
};

PassPlan split_bits(int bits, int passes) {
  PassPlan pp{};
  if (bits > 2 * kMaxPassBits) bits = 2 * kMaxPassBits;
  if (passes < 1) passes = 1;
  if (passes > 2) passes = 2;
  if (bits > kMaxPassBits) passes = 2;
  if (bits < 2) passes = 1;
  pp.passes = passes;
  if (passes == 1) {
    pp.bits[0] = bits;
    pp.bits[1] = 0;
  } else {
    pp.bits[0] = (bits + 1) / 2;
    pp.bits[1] = bits - pp.bits[0];
  }
  return pp;
}

uint64_t ub_chunks(uint64_t n, uint32_t nseg) { return (n + kChunk - 1) / kChunk + nseg; }

// One partitioning pass of n tuples from `in` into `out`. Segments are given by
// seg_off/cpre (device, nseg + 1 entries each); on return part_off (device,
// nseg * 2^bits + 1 entries) holds the partition boundaries.
template <typename K, typename P, bool kRows>
int part_pass(const K *ik, const P *ip, const uint32_t *ir, Side<K, P> out, uint64_t n,
              const uint32_t *seg_off, const uint32_t *cpre, uint32_t nseg, int shift, int bits,
              uint32_t *C, uint64_t *tmp, uint64_t *total, uint32_t *part_off, hipStream_t s) {
  const uint64_t ub = ub_chunks(n, nseg);
  const uint64_t nC = ub << bits;
  int rc;
  if ((rc = fill_u32(C, nC, 0, s))) return rc;
  EIGER_LAUNCH("radix_hist", k_part_hist<K>, dim3(unsigned(ub)), dim3(kPNT), 0, s, ik, seg_off, cpre,
               nseg, shift, bits, C);
  if ((rc = exclusive_scan_u32(C, C, nC, tmp, total, s))) return rc;
  EIGER_LAUNCH("radix_scatter", (k_part_scatter<K, P, kRows>), dim3(unsigned(ub)), dim3(kPNT), 0, s,
               ik, ip, ir, seg_off, cpre, nseg, shift, bits, C, out.k, out.p, out.r);
  const uint64_t nq = (uint64_t(nseg) << bits) + 1;
  EIGER_LAUNCH("radix_offsets", k_part_offsets, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, s,
               seg_off, cpre, nseg, bits, C, part_off, static_cast<uint32_t>(n));
  return EIGER_OK;
}

template <typename K, typename P>
struct SideBufs {
  Side<K, P> a, b;            // pass-1 output, pass-2 output
  uint32_t *seg1, *cpre1;     // single segment descriptors
  uint32_t *off1;             // pass-1 partition offsets (2^b1 + 1)
  uint32_t *cpre2;            // pass-2 chunk prefix (2^b1 + 1)
  uint32_t *off;              // final partition offsets
};

template <typename K, typename P>
SideBufs<K, P> side_layout(Workspace &ws, uint64_t n, const PassPlan &pp) {
  SideBufs<K, P> S{};
  const uint64_t m = n ? n : 1;
  S.a = Side<K, P>{ws.take<K>(m), ws.take<P>(m), ws.take<uint32_t>(m)};
  if (pp.passes == 2) S.b = Side<K, P>{ws.take<K>(m), ws.take<P>(m), ws.take<uint32_t>(m)};
  S.seg1 = ws.take<uint32_t>(2);
  S.cpre1 = ws.take<uint32_t>(2);
  S.off1 = ws.take<uint32_t>((uint64_t(1) << pp.bits[0]) + 1);
  S.cpre2 = ws.take<uint32_t>((uint64_t(1) << pp.bits[0]) + 1);
  S.off = pp.passes == 2 ? ws.take<uint32_t>((uint64_t(1) << (pp.bits[0] + pp.bits[1])) + 1) : S.off1;
  return S;
}

// Partition one side completely; returns the side holding the final partitions.
template <typename K, typename P>
int partition_side(const K *keys, const P *pays, uint64_t n, SideBufs<K, P> &S, const PassPlan &pp,
                   uint32_t *C, uint64_t *tmp, uint64_t *total, hipStream_t s, Side<K, P> *final_side) {
  EIGER_LAUNCH("radix_seg", k_single_segment, dim3(1), dim3(64), 0, s, S.seg1, S.cpre1,
               static_cast<uint32_t>(n));
  int rc;
  const int b1 = pp.bits[0];
  if ((rc = part_pass<K, P, false>(keys, pays, nullptr, S.a, n, S.seg1, S.cpre1, 1, 64 - b1, b1, C, tmp,
                                   total, S.off1, s)))
    return rc;
  if (pp.passes == 1) {
    *final_side = S.a;
    return EIGER_OK;
  }
  const uint32_t nseg = 1u << b1;
  EIGER_LAUNCH("radix_chunks", k_chunk_counts, dim3((nseg + 1 + 255) / 256), dim3(256), 0, s, S.off1,
               nseg, S.cpre2);
  if ((rc = exclusive_scan_u32(S.cpre2, S.cpre2, nseg + 1, tmp, total, s))) return rc;
  const int b2 = pp.bits[1];
  if ((rc = part_pass<K, P, true>(S.a.k, S.a.p, S.a.r, S.b, n, S.off1, S.cpre2, nseg, 64 - b1 - b2, b2,
                                  C, tmp, total, S.off, s)))
    return rc;
  *final_side = S.b;
  return EIGER_OK;
}

uint64_t counters_len(uint64_t n, const PassPlan &pp) {
  uint64_t m = ub_chunks(n, 1) << pp.bits[0];
  if (pp.passes == 2) {
    uint64_t m2 = ub_chunks(n, 1u << pp.bits[0]) << pp.bits[1];
    if (m2 > m) m = m2;
  }
  return m;
}

template <typename K, typename PB, typename PS>
int radix_impl(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const PassPlan pp = split_bits(a.plan.radix_bits, a.plan.radix_passes);
  const int bits = pp.bits[0] + pp.bits[1];
  const uint32_t F = 1u << bits;
  float lf = a.plan.load_factor;
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  const RadixLimits lim = radix_limits(a.kdt, a.bpdt, lf);

  JoinCounters *c = ws.take<JoinCounters>(1);
  SideBufs<K, PB> R = side_layout<K, PB>(ws, a.nR, pp);
  SideBufs<K, PS> S = side_layout<K, PS>(ws, a.nS, pp);
  const uint64_t nC = std::max(counters_len(a.nR, pp), counters_len(a.nS, pp));
  uint32_t *C = ws.take<uint32_t>(nC);
  uint64_t *tmp = ws.take<uint64_t>(scan_tmp_elems(std::max<uint64_t>(nC, F + 1)));
  uint64_t *total = ws.take<uint64_t>(1);
  uint32_t *items = ws.take<uint32_t>(F + 1);
  *ctr = c;
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if (a.nR == 0 || a.nS == 0) return EIGER_OK;
  Side<K, PB> fr;
  Side<K, PS> fs;
  if ((rc = partition_side<K, PB>(static_cast<const K *>(a.bk), static_cast<const PB *>(a.bp), a.nR, R,
                                  pp, C, tmp, total, s, &fr)))
    return rc;
  if ((rc = partition_side<K, PS>(static_cast<const K *>(a.pk), static_cast<const PS *>(a.pp), a.nS, S,
                                  pp, C, tmp, total, s, &fs)))
    return rc;
  EIGER_LAUNCH("radix_items", k_items, dim3((F + 1 + 255) / 256), dim3(256), 0, s, R.off, S.off, F,
               items);
  if ((rc = exclusive_scan_u32(items, items, F + 1, tmp, total, s))) return rc;
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  const unsigned grid = static_cast<unsigned>(device_cu_count()) * 2;
  EIGER_LAUNCH("radix_join", (k_radix_join<K, PB, PS>), dim3(grid), dim3(kJNT), 0, s, fr.k, fr.p, fr.r,
               R.off, fs.k, fs.p, fs.r, S.off, items, F, lim.max_build, lf, o);
  return EIGER_OK;
}

}  // namespace

RadixLimits radix_limits(int32_t kdt, int32_t bpdt, float lf) {
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  RadixLimits r{};
  const uint32_t slot = static_cast<uint32_t>(dtype_size(kdt) + dtype_size(bpdt) + 4);
  r.max_slots = kTableBytes / slot;
  r.max_build = static_cast<uint32_t>(static_cast<float>(r.max_slots) * lf);
  if (r.max_build < 1) r.max_build = 1;
  if (r.max_build >= r.max_slots) r.max_build = r.max_slots - 1;
  return r;
}

int run_radix(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const bool k64 = a.kdt == EIGER_INT64, b64 = a.bpdt == EIGER_INT64, p64 = a.ppdt == EIGER_INT64;
#define EIGER_DISPATCH(KT, BT, PT) return radix_impl<KT, BT, PT>(a, ws, ctr)
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
