// join_radix.hip -- RADIX variant: hash-radix partitioning, then one LDS-resident
// hash table per partition.
//
// The paper's partitioned hash join (Section 3.2, Table 1; its internals are
// those of Wu et al., which the paper cites rather than prints) is re-derived
// here for gfx950:
//  * Both sides are partitioned on the top bits of part_hash(key) (hashing before
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
constexpr int kMaxPassBits = 10;    // at most 1024 buckets per pass
constexpr int kMaxB = 1 << kMaxPassBits;
constexpr int kBPT = kMaxB / kPNT;  // buckets owned by each thread in the tile scan

constexpr int kJNT = 512;       // join workgroup
constexpr int kJIPT = 4;
constexpr int kJSCAP = 2048;    // staged output pairs
constexpr int kTableBytes = 48 * 1024;
constexpr uint32_t kJTile = 32768;  // probe rows per work item

// Bucket of a partition hash (part_hash) in a pass of `mask + 1` buckets.
__device__ __forceinline__ uint32_t bucket_of(uint64_t h, int shift, uint32_t mask) {
  return static_cast<uint32_t>(h >> shift) & mask;
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
  // 8 keys per thread are loaded before any is counted, so the loads overlap
  constexpr int U = 8;
  for (uint32_t i0 = lo; i0 < hi; i0 += kPNT * U) {
    K kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = i0 + u * kPNT + threadIdx.x;
      if (i < hi) kk[u] = keys[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = i0 + u * kPNT + threadIdx.x;
      if (i < hi) atomicAdd(&hist[bucket_of(part_hash(kk[u]), shift, B - 1)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < B; b += kPNT) C[uint64_t(cpre[s]) * B + uint64_t(b) * nch + lc] = hist[b];
}

template <typename K, typename P, bool kRows>
__device__ __forceinline__ void load_part_tile(K (&key)[kPIPT], P (&pay)[kPIPT], uint32_t (&row)[kPIPT],
                                               const K *__restrict__ keys, const P *__restrict__ pays,
                                               const uint32_t *__restrict__ rows, uint32_t t0,
                                               uint32_t hi) {
#pragma unroll
  for (int k = 0; k < kPIPT; ++k) {
    const uint32_t i = t0 + k * kPNT + threadIdx.x;
    if (i < hi) {
      key[k] = keys[i];
      pay[k] = pays[i];
      row[k] = kRows ? rows[i] : i;
    }
  }
}

// Scatter one chunk into its partitions. Per tile of kPTile tuples: rank each
// tuple within its bucket (LDS atomics), scan the tile histogram, sort the tile
// by bucket in LDS, then write each bucket's run to its output position, so
// consecutive threads store consecutive addresses. The next tile's loads are
// issued before the current tile's LDS phases.
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
  __shared__ uint32_t hist[kMaxB], gcur[kMaxB], gdst[kMaxB], loff[kMaxB];
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
  K key[kPIPT], nkey[kPIPT];
  P pay[kPIPT], npay[kPIPT];
  uint32_t row[kPIPT], nrow[kPIPT];
  load_part_tile<K, P, kRows>(key, pay, row, keys, pays, rows, lo, hi);
  __syncthreads();
  for (uint32_t t0 = lo; t0 < hi; t0 += kPTile) {
    const uint32_t t1 = min(hi, t0 + kPTile);
    uint32_t bk[kPIPT], rk[kPIPT];
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        bk[k] = bucket_of(part_hash(key[k]), shift, B - 1);
        rk[k] = atomicAdd(&hist[bk[k]], 1u);
      }
    }
    if (t0 + kPTile < hi) load_part_tile<K, P, kRows>(nkey, npay, nrow, keys, pays, rows, t0 + kPTile, hi);
    __syncthreads();
    // scan of the tile histogram; each thread owns kBPT consecutive buckets
    uint32_t v[kBPT], sum = 0;
#pragma unroll
    for (int j = 0; j < kBPT; ++j) {
      const uint32_t b = threadIdx.x * kBPT + j;
      v[j] = b < B ? hist[b] : 0u;
      sum += v[j];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan<kPNT>(sum, scan_tmp, &total);
#pragma unroll
    for (int j = 0; j < kBPT; ++j) {
      const uint32_t b = threadIdx.x * kBPT + j;
      if (b < B) {
        loff[b] = ex;
        gdst[b] = gcur[b] - ex;  // output position of tile slot e of bucket b: gdst[b] + e
        gcur[b] += v[j];
        hist[b] = 0;
        ex += v[j];
      }
    }
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
      const uint32_t dst = gdst[lb[e]] + e;
      okeys[dst] = lk[e];
      opays[dst] = lp[e];
      orows[dst] = lr[e];
    }
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      key[k] = nkey[k];
      pay[k] = npay[k];
      row[k] = nrow[k];
    }
    // The next tile's first LDS writes are its hist atomics (hist was cleared
    // above); gdst/loff/lk are rewritten only after the next barrier.
  }
}

// Write-combining scatter for up to MAXB buckets, used for 4-byte keys and
// payloads. Same tile sort as k_part_scatter, but a bucket's tuples are
// written only in whole groups of kWcGroup tuples that end on a
// kWcGroup-aligned output index (64 bytes of each 4-byte column); the
// remainder waits in a per-bucket LDS buffer for the next tile, so a chunk's
// run in a bucket reaches memory in aligned pieces except at its two ends.
constexpr int kWcGroup = 16;

template <typename K, typename P, bool kRows, int MAXB>
__global__ void __launch_bounds__(kPNT)
    k_part_scatter_wc(const K *__restrict__ keys, const P *__restrict__ pays,
                      const uint32_t *__restrict__ rows, const uint32_t *__restrict__ seg_off,
                      const uint32_t *__restrict__ cpre, uint32_t nseg, int shift, int bits,
                      const uint32_t *__restrict__ C, K *__restrict__ okeys, P *__restrict__ opays,
                      uint32_t *__restrict__ orows) {
  constexpr int G = kWcGroup;
  static_assert(MAXB <= 256, "bucket ids of tile positions are kept in one byte");
  __shared__ K lk[kPTile];
  __shared__ P lp[kPTile];
  __shared__ uint32_t lr[kPTile];
  __shared__ uint8_t lb[kPTile];
  __shared__ K qk[MAXB * G];
  __shared__ P qp[MAXB * G];
  __shared__ uint32_t qr[MAXB * G];
  __shared__ uint32_t hist[MAXB], loff[MAXB], gcur[MAXB], pend[MAXB], emit[MAXB];
  const uint32_t c = blockIdx.x;
  if (c >= cpre[nseg]) return;
  const uint32_t B = 1u << bits;
  const uint32_t s = find_segment(cpre, nseg, c);
  const uint32_t lc = c - cpre[s], nch = cpre[s + 1] - cpre[s];
  const uint32_t lo = seg_off[s] + lc * kChunk;
  const uint32_t hi = min(seg_off[s + 1], lo + kChunk);
  for (uint32_t b = threadIdx.x; b < B; b += kPNT) {
    hist[b] = 0;
    pend[b] = 0;
    gcur[b] = C[uint64_t(cpre[s]) * B + uint64_t(b) * nch + lc];
  }
  K key[kPIPT], nkey[kPIPT];
  P pay[kPIPT], npay[kPIPT];
  uint32_t row[kPIPT], nrow[kPIPT];
  load_part_tile<K, P, kRows>(key, pay, row, keys, pays, rows, lo, hi);
  __syncthreads();
  for (uint32_t t0 = lo; t0 < hi; t0 += kPTile) {
    const uint32_t t1 = min(hi, t0 + kPTile);
    uint32_t bk[kPIPT], rk[kPIPT];
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        bk[k] = bucket_of(part_hash(key[k]), shift, B - 1);
        rk[k] = atomicAdd(&hist[bk[k]], 1u);
      }
    }
    if (t0 + kPTile < hi) load_part_tile<K, P, kRows>(nkey, npay, nrow, keys, pays, rows, t0 + kPTile, hi);
    __syncthreads();
    // wave 0: exclusive scan of the tile histogram (-> loff) and, per bucket,
    // how many tuples leave this tile: pending ones first, then the head of the
    // tile run, up to the last kWcGroup-aligned output index (-> emit)
    if (threadIdx.x < 64) {
      constexpr int PER = MAXB / 64;
      uint32_t h[PER], hs = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t b = threadIdx.x * PER + j;
        h[j] = b < B ? hist[b] : 0u;
        hs += h[j];
      }
      uint32_t hr = wave_inclusive_scan(hs) - hs;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t b = threadIdx.x * PER + j;
        if (b < B) {
          const uint32_t end = (gcur[b] + pend[b] + h[j]) & ~uint32_t(G - 1);
          loff[b] = hr;
          emit[b] = end > gcur[b] ? end - gcur[b] : 0u;
        }
        hr += h[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        const uint32_t pos = loff[bk[k]] + rk[k];
        lk[pos] = key[k];
        lp[pos] = pay[k];
        lr[pos] = row[k];
        lb[pos] = static_cast<uint8_t>(bk[k]);
      }
    }
    __syncthreads();
    // Out: tuple j of bucket b's emitted run (pending tuples are j < pend[b],
    // tile position p is j = pend[b] + p - loff[b]) goes to gcur[b] + j.
    const uint32_t n = t1 - t0;
    for (uint32_t q = threadIdx.x; q < B * G; q += kPNT) {
      const uint32_t b = q / G, j = q % G;
      if (j < pend[b] && emit[b]) {
        okeys[gcur[b] + j] = qk[q];
        opays[gcur[b] + j] = qp[q];
        orows[gcur[b] + j] = qr[q];
      }
    }
    for (uint32_t p = threadIdx.x; p < n; p += kPNT) {
      const uint32_t b = lb[p], j = pend[b] + p - loff[b];
      if (j < emit[b]) {
        okeys[gcur[b] + j] = lk[p];
        opays[gcur[b] + j] = lp[p];
        orows[gcur[b] + j] = lr[p];
      }
    }
    __syncthreads();
    // Kept: the rest of each bucket's run (fewer than kWcGroup tuples) moves to
    // the front of its pending buffer, in order.
    for (uint32_t p = threadIdx.x; p < n; p += kPNT) {
      const uint32_t b = lb[p], j = pend[b] + p - loff[b];
      if (j >= emit[b]) {
        const uint32_t q = b * G + (j - emit[b]);
        qk[q] = lk[p];
        qp[q] = lp[p];
        qr[q] = lr[p];
      }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += kPNT) {
      pend[b] = pend[b] + hist[b] - emit[b];
      gcur[b] += emit[b];
      hist[b] = 0;
    }
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      key[k] = nkey[k];
      pay[k] = npay[k];
      row[k] = nrow[k];
    }
    __syncthreads();
  }
  // chunk end: the remaining tuples of every bucket
  for (uint32_t q = threadIdx.x; q < B * G; q += kPNT) {
    const uint32_t b = q / G, j = q % G;
    if (j < pend[b]) {
      okeys[gcur[b] + j] = qk[q];
      opays[gcur[b] + j] = qp[q];
      orows[gcur[b] + j] = qr[q];
    }
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
struct LdsSlot {
  K key;
  uint32_t rowid;
  PB pay;
};

// LDS latency is short, so LDS tables walk one row at a time (kHashed = false)
// and keep registers for occupancy.
template <typename K, typename PB>
struct LdsTab {
  static constexpr bool kHashed = false;
  static constexpr bool kRuns = false;
  using SlotT = LdsSlot<K, PB>;
  K *tk;
  uint32_t *tr;
  PB *tp;
  uint32_t nslots;
  bool unique;

  __device__ __forceinline__ uint32_t home(K key) const {
    const uint32_t h = static_cast<uint32_t>(fmix64(static_cast<uint64_t>(sext(key))));
    return static_cast<uint32_t>((uint64_t(h) * nslots) >> 32);
  }
  __device__ __forceinline__ uint32_t next(uint32_t i) const { return (i + 1 == nslots) ? 0 : i + 1; }
  __device__ __forceinline__ SlotT load(uint32_t i) const { return SlotT{tk[i], tr[i], tp[i]}; }
  __device__ __forceinline__ uint32_t lookup(K key, uint32_t &first, uint64_t &psum) const {
    uint32_t i = home(key), c = 0;
    for (;;) {
      const uint32_t r = tr[i];
      if (r == kEmpty) break;
      if (tk[i] == key) {
        first = r;
        psum += static_cast<uint64_t>(sext(tp[i]));
        ++c;
        if (unique) break;
      }
      i = next(i);
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
      i = next(i);
    }
  }
};

template <typename K, typename PB>
__host__ __device__ constexpr uint32_t lds_max_slots() {
  return kTableBytes / (sizeof(K) + sizeof(PB) + sizeof(uint32_t));
}

// LDS table of one chunk of 32-bit build keys, grouped by key. Each distinct
// key owns one 64-bit slot word  key << 32 | cursor << 16 | count  (count 0 =
// empty; linear probing over distinct keys only); its build rows sit together
// in rid[start, start + count) with start = cursor - count once placed, and the
// key's payload sum (sign-extended, mod 2^64) is kept at psum[start]. A probe
// stops at its key's slot, and its matches are one contiguous run.
struct GrpTab {
  static constexpr bool kHashed = false;
  static constexpr bool kRuns = true;
  const unsigned long long *w;
  const uint32_t *rid;
  const uint64_t *psum;
  uint32_t nslots;

  __device__ __forceinline__ uint32_t home(int32_t key) const {
    const uint32_t h = static_cast<uint32_t>(fmix64(static_cast<uint64_t>(sext(key))));
    return static_cast<uint32_t>((uint64_t(h) * nslots) >> 32);
  }
  __device__ __forceinline__ uint32_t next(uint32_t i) const { return (i + 1 == nslots) ? 0 : i + 1; }
  __device__ __forceinline__ uint32_t find(int32_t key, uint32_t &start) const {
    for (uint32_t i = home(key);; i = next(i)) {
      const unsigned long long v = w[i];
      const uint32_t c = static_cast<uint32_t>(v & 0xFFFFu);
      if (c == 0) return 0;
      if (static_cast<uint32_t>(v >> 32) == static_cast<uint32_t>(key)) {
        start = static_cast<uint32_t>((v >> 16) & 0xFFFFu) - c;
        return c;
      }
    }
  }
  // `first` receives the start of the key's run of rows (kRuns)
  __device__ __forceinline__ uint32_t lookup(int32_t key, uint32_t &first, uint64_t &ps) const {
    uint32_t st = 0;
    const uint32_t c = find(key, st);
    if (c) {
      first = st;
      ps += psum[st];
    }
    return c;
  }
  __device__ __forceinline__ uint32_t row_at(uint32_t i) const { return rid[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(int32_t key, F f) const {
    uint32_t st = 0;
    const uint32_t c = find(key, st);
    for (uint32_t j = 0; j < c; ++j) f(rid[st + j]);
  }
};

// Build rows one grouped table holds at load factor lf: ns >= n / lf slots of
// 8 bytes plus 12 bytes (row id, payload sum word) per row in kTableBytes.
__host__ __device__ inline uint32_t grouped_max_build(float lf) {
  return static_cast<uint32_t>(static_cast<float>(kTableBytes) / (8.0f / lf + 12.0f));
}

// Join one chunk [c0, c1) of a partition's 32-bit build rows with probe rows
// [s0, s1) through a grouped table. Uniform across the workgroup.
template <typename PB, typename PS>
__device__ __forceinline__ void join_chunk_grouped(const int32_t *__restrict__ rk, const PB *__restrict__ rp,
                                                   const uint32_t *__restrict__ rr, uint32_t c0, uint32_t c1,
                                                   const int32_t *__restrict__ sk, const PS *__restrict__ sp,
                                                   const uint32_t *__restrict__ sr, uint32_t s0, uint32_t s1,
                                                   float lf, EmitLds<kJNT, kJSCAP> &L, uint64_t &fill,
                                                   const EmitOut &o, uint64_t &cs) {
  __shared__ __align__(16) unsigned char lds[kTableBytes];
  const uint32_t nb = c1 - c0;
  // slots: nb / lf + 1, at least 64, at most what fits beside the rows (> nb
  // because nb <= grouped_max_build), so every walk reaches an empty slot
  const uint32_t cap = (kTableBytes - nb * 12u) / 8u;
  uint32_t ns = static_cast<uint32_t>(static_cast<float>(nb) / lf) + 1;
  ns = ns < 64 ? 64 : ns;
  ns = ns > cap ? cap : ns;
  unsigned long long *W = reinterpret_cast<unsigned long long *>(lds);
  uint64_t *ps = reinterpret_cast<uint64_t *>(lds + size_t(ns) * 8);
  uint32_t *rid = reinterpret_cast<uint32_t *>(lds + size_t(ns) * 8 + size_t(nb) * 8);
  GrpTab tab{W, rid, ps, ns};
  for (uint32_t i = threadIdx.x; i < ns; i += kJNT) W[i] = 0;
  __syncthreads();
  // 1. one slot per distinct key, with its row count
  for (uint32_t j = c0 + threadIdx.x; j < c1; j += kJNT) {
    const uint32_t key = static_cast<uint32_t>(rk[j]);
    uint32_t i = tab.home(rk[j]);
    for (;;) {
      unsigned long long v = W[i];
      if ((v & 0xFFFFu) == 0) {
        v = atomicCAS(&W[i], 0ull, (static_cast<unsigned long long>(key) << 32) | 1ull);
        if (v == 0) break;  // claimed with count 1
      }
      if (static_cast<uint32_t>(v >> 32) == key) {
        atomicAdd(&W[i], 1ull);
        break;
      }
      i = tab.next(i);
    }
  }
  __syncthreads();
  // 2. group starts: exclusive scan of the counts in slot order (each thread a
  //    contiguous run of slots), written into the cursor field
  {
    const uint32_t per = (ns + kJNT - 1) / kJNT;
    const uint32_t lo = min(ns, threadIdx.x * per), hi = min(ns, lo + per);
    uint32_t local = 0;
    for (uint32_t i = lo; i < hi; ++i) local += static_cast<uint32_t>(W[i] & 0xFFFFu);
    uint64_t tot;
    uint32_t run = static_cast<uint32_t>(block_exclusive_scan<kJNT, uint64_t>(local, L.scan, &tot));
    for (uint32_t i = lo; i < hi; ++i) {
      const unsigned long long v = W[i];
      W[i] = (v & 0xFFFFFFFF0000FFFFull) | (static_cast<unsigned long long>(run) << 16);
      run += static_cast<uint32_t>(v & 0xFFFFu);
    }
  }
  __syncthreads();
  // 3. place every row in its key's group (the cursor field advances to the end)
  for (uint32_t j = c0 + threadIdx.x; j < c1; j += kJNT) {
    const uint32_t key = static_cast<uint32_t>(rk[j]);
    uint32_t i = tab.home(rk[j]);
    while (static_cast<uint32_t>(W[i] >> 32) != key || (W[i] & 0xFFFFu) == 0) i = tab.next(i);
    const uint32_t pos = static_cast<uint32_t>((atomicAdd(&W[i], 1ull << 16) >> 16) & 0xFFFFu);
    rid[pos] = rr ? rr[j] : j;  // no row-id array: the row's position (wide joins)
    ps[pos] = static_cast<uint64_t>(sext(rp[j]));
  }
  __syncthreads();
  // 4. payload sum of each group, kept at its start
  for (uint32_t i = threadIdx.x; i < ns; i += kJNT) {
    const unsigned long long v = W[i];
    const uint32_t c = static_cast<uint32_t>(v & 0xFFFFu);
    if (c) {
      const uint32_t st = static_cast<uint32_t>((v >> 16) & 0xFFFFu) - c;
      uint64_t sum = 0;
      for (uint32_t q = 0; q < c; ++q) sum += ps[st + q];
      ps[st] = sum;
    }
  }
  __syncthreads();
  probe_range<kJNT, kJIPT, kJSCAP>(tab, sk, sp, sr, s0, s1, L, fill, o, cs);
}

// Join one chunk of a partition through a multiset table (one slot per build
// row; used for 64-bit keys). Uniform across the workgroup.
template <typename K, typename PB, typename PS>
__device__ __forceinline__ void join_chunk_multiset(const K *__restrict__ rk, const PB *__restrict__ rp,
                                                    const uint32_t *__restrict__ rr, uint32_t c0, uint32_t c1,
                                                    const K *__restrict__ sk, const PS *__restrict__ sp,
                                                    const uint32_t *__restrict__ sr, uint32_t s0, uint32_t s1,
                                                    float lf, EmitLds<kJNT, kJSCAP> &L, uint64_t &fill,
                                                    const EmitOut &o, uint64_t &cs) {
  constexpr uint32_t MAXS = lds_max_slots<K, PB>();
  __shared__ K tk[MAXS];
  __shared__ uint32_t tr[MAXS];
  __shared__ PB tp[MAXS];
  __shared__ uint32_t dup;
  const uint32_t nb = c1 - c0;
  uint32_t ns = static_cast<uint32_t>(static_cast<float>(nb) / lf) + 1;
  ns = ns < 64 ? 64 : (ns > MAXS ? MAXS : ns);
  for (uint32_t i = threadIdx.x; i < ns; i += kJNT) tr[i] = kEmpty;
  if (threadIdx.x == 0) dup = 0;
  __syncthreads();
  LdsTab<K, PB> tab{tk, tr, tp, ns, false};
  for (uint32_t j = c0 + threadIdx.x; j < c1; j += kJNT) {
    const K key = rk[j];
    uint32_t i = tab.home(key);
    for (;;) {
      if (atomicCAS(&tr[i], kEmpty, rr ? rr[j] : j) == kEmpty) {
        tk[i] = key;
        tp[i] = rp[j];
        break;
      }
      i = (i + 1 == ns) ? 0 : i + 1;
    }
  }
  __syncthreads();
  // distinct build keys in this table let probes stop at their first match
  for (uint32_t j = c0 + threadIdx.x; j < c1; j += kJNT) {
    uint32_t cnt = 0;
    tab.for_each(rk[j], [&](uint32_t) { ++cnt; });
    if (cnt > 1) dup = 1;
  }
  __syncthreads();
  tab.unique = dup == 0;
  probe_range<kJNT, kJIPT, kJSCAP>(tab, sk, sp, sr, s0, s1, L, fill, o, cs);
}

template <typename K, typename PB, typename PS>
__global__ void __launch_bounds__(kJNT)
    k_radix_join(const K *__restrict__ rk, const PB *__restrict__ rp, const uint32_t *__restrict__ rr,
                 const uint32_t *__restrict__ offR, const K *__restrict__ sk,
                 const PS *__restrict__ sp, const uint32_t *__restrict__ sr,
                 const uint32_t *__restrict__ offS, const uint32_t *__restrict__ item_off,
                 const uint32_t *__restrict__ item_part, uint32_t F, uint32_t max_build, float lf,
                 EmitOut o) {
  __shared__ EmitLds<kJNT, kJSCAP> L;
  uint64_t fill = 0;
  uint64_t cs = 0;
  const uint32_t nitems = item_off[F];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const uint32_t p = item_part[it];
    const uint32_t tile = it - item_off[p];
    const uint32_t r0 = offR[p], r1 = offR[p + 1];
    const uint32_t s0 = offS[p] + tile * kJTile;
    const uint32_t s1 = min(offS[p + 1], s0 + kJTile);
    for (uint32_t c0 = r0; c0 < r1; c0 += max_build) {
      const uint32_t c1 = min(r1, c0 + max_build);
      if constexpr (sizeof(K) == 4)
        join_chunk_grouped<PB, PS>(rk, rp, rr, c0, c1, sk, sp, sr, s0, s1, lf, L, fill, o, cs);
      else
        join_chunk_multiset<K, PB, PS>(rk, rp, rr, c0, c1, sk, sp, sr, s0, s1, lf, L, fill, o, cs);
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

unsigned grid_for_rows(uint64_t n) {
  uint64_t g = (n + 511) / 512;
  const uint64_t cap = uint64_t(device_cu_count()) * 8;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g ? g : 1);
}

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
  // Write-combining pays off when keys and payloads are 4-byte columns (the
  // skewed int32 join: 6.8 vs 8.3 ms for two 8-bit passes of both sides); with
  // 8-byte columns the plain tile scatter is faster (10.0 vs 8.3 ms for one
  // 8-bit pass of 512M int64 rows).
  bool done = false;
  if constexpr (sizeof(K) == 4 && sizeof(P) == 4) {
    if (bits <= 7) {
      EIGER_LAUNCH("radix_scatter", (k_part_scatter_wc<K, P, kRows, 128>), dim3(unsigned(ub)), dim3(kPNT), 0,
                   s, ik, ip, ir, seg_off, cpre, nseg, shift, bits, C, out.k, out.p, out.r);
      done = true;
    } else if (bits <= 8) {
      EIGER_LAUNCH("radix_scatter", (k_part_scatter_wc<K, P, kRows, 256>), dim3(unsigned(ub)), dim3(kPNT), 0,
                   s, ik, ip, ir, seg_off, cpre, nseg, shift, bits, C, out.k, out.p, out.r);
      done = true;
    }
  }
  if (!done) {
    EIGER_LAUNCH("radix_scatter", (k_part_scatter<K, P, kRows>), dim3(unsigned(ub)), dim3(kPNT), 0, s,
                 ik, ip, ir, seg_off, cpre, nseg, shift, bits, C, out.k, out.p, out.r);
  }
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

// Partition of every work item: part[t] = p for off[p] <= t < off[p+1] (off is
// the exclusive scan of the per-partition item counts), so a workgroup finds its
// item's partition with one load.
__global__ void k_item_part(const uint32_t *__restrict__ off, uint32_t F, uint32_t *__restrict__ part) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < F)
    for (uint32_t t = off[p], e = off[p + 1]; t < e; ++t) part[t] = p;
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
  // each partition has at most ceil(its probe rows / kJTile) items
  uint32_t *item_part = ws.take<uint32_t>(uint64_t(F) + (a.nS + kJTile - 1) / kJTile + 1);
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
  EIGER_LAUNCH("radix_items", k_item_part, dim3((F + 255) / 256), dim3(256), 0, s, items, F, item_part);
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  const unsigned grid = static_cast<unsigned>(device_cu_count()) * 2;
  EIGER_LAUNCH("radix_join", (k_radix_join<K, PB, PS>), dim3(grid), dim3(kJNT), 0, s, fr.k, fr.p, fr.r,
               R.off, fs.k, fs.p, fs.r, S.off, items, item_part, F, lim.max_build, lf, o);
  return EIGER_OK;
}

// ---------------------------------------------------------------------------
// Wide joins, GFTR materialization (Section 3.2: the payload columns go
// through the same partitioning as the keys): the scatter carries up to
// kMaxWords 32-bit payload words per tuple along with the key and row id, and
// the join emits positions in the partitioned arrays, from which the payload
// words are later gathered partition by partition.

// Up to kMaxWords 32-bit word lanes. Lane w of row i is src[w][i * src_stride[w]]
// (an 8-byte column is two lanes, its low and high words, with stride 2); the
// scatter writes it to dst[w][position] (stride 1).
struct Lanes {
  const uint32_t *src[kMaxWords];
  uint32_t src_stride[kMaxWords];
  uint32_t *dst[kMaxWords];
  int n;
};

// k_part_scatter's tile sort, moving key, row id and the word lanes.
template <typename K, bool kRows>
__global__ void __launch_bounds__(kPNT)
    k_part_scatter_carry(const K *__restrict__ keys, const uint32_t *__restrict__ rows, Lanes lanes,
                         const uint32_t *__restrict__ seg_off, const uint32_t *__restrict__ cpre, uint32_t nseg,
                         int shift, int bits, const uint32_t *__restrict__ C, K *__restrict__ okeys,
                         uint32_t *__restrict__ orows) {
  __shared__ K lk[kPTile];
  __shared__ uint32_t lr[kPTile];
  __shared__ uint32_t lw[kMaxWords][kPTile];
  __shared__ uint16_t lb[kPTile];
  __shared__ uint32_t hist[kMaxB], gcur[kMaxB], gdst[kMaxB], loff[kMaxB];
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
    uint32_t row[kPIPT], bk[kPIPT], rk[kPIPT];
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        key[k] = keys[i];
        row[k] = kRows ? rows[i] : i;
        bk[k] = bucket_of(part_hash(key[k]), shift, B - 1);
        rk[k] = atomicAdd(&hist[bk[k]], 1u);
      }
    }
    __syncthreads();
    uint32_t v[kBPT], sum = 0;
#pragma unroll
    for (int j = 0; j < kBPT; ++j) {
      const uint32_t b = threadIdx.x * kBPT + j;
      v[j] = b < B ? hist[b] : 0u;
      sum += v[j];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan<kPNT>(sum, scan_tmp, &total);
#pragma unroll
    for (int j = 0; j < kBPT; ++j) {
      const uint32_t b = threadIdx.x * kBPT + j;
      if (b < B) {
        loff[b] = ex;
        gdst[b] = gcur[b] - ex;
        gcur[b] += v[j];
        hist[b] = 0;
        ex += v[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPIPT; ++k) {
      const uint32_t i = t0 + k * kPNT + threadIdx.x;
      if (i < t1) {
        const uint32_t pos = loff[bk[k]] + rk[k];
        lk[pos] = key[k];
        lr[pos] = row[k];
        lb[pos] = static_cast<uint16_t>(bk[k]);
        for (int w = 0; w < lanes.n; ++w) lw[w][pos] = lanes.src[w][uint64_t(i) * lanes.src_stride[w]];
      }
    }
    __syncthreads();
    const uint32_t n = t1 - t0;
    for (uint32_t e = threadIdx.x; e < n; e += kPNT) {
      const uint32_t dst = gdst[lb[e]] + e;
      okeys[dst] = lk[e];
      orows[dst] = lr[e];
      for (int w = 0; w < lanes.n; ++w) lanes.dst[w][dst] = lw[w][e];
    }
    __syncthreads();
  }
}

template <typename K, bool kRows>
int part_pass_carry(const K *ik, const uint32_t *ir, const Lanes &lanes, K *ok, uint32_t *orow, uint64_t n,
                    const uint32_t *seg_off, const uint32_t *cpre, uint32_t nseg, int shift, int bits,
                    uint32_t *C, uint64_t *tmp, uint64_t *total, uint32_t *part_off, hipStream_t s) {
  const uint64_t ub = ub_chunks(n, nseg);
  const uint64_t nC = ub << bits;
  int rc;
  if ((rc = fill_u32(C, nC, 0, s))) return rc;
  EIGER_LAUNCH("radix_hist", k_part_hist<K>, dim3(unsigned(ub)), dim3(kPNT), 0, s, ik, seg_off, cpre, nseg, shift,
               bits, C);
  if ((rc = exclusive_scan_u32(C, C, nC, tmp, total, s))) return rc;
  EIGER_LAUNCH("radix_scatter", (k_part_scatter_carry<K, kRows>), dim3(unsigned(ub)), dim3(kPNT), 0, s, ik, ir,
               lanes, seg_off, cpre, nseg, shift, bits, C, ok, orow);
  const uint64_t nq = (uint64_t(nseg) << bits) + 1;
  EIGER_LAUNCH("radix_offsets", k_part_offsets, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, s, seg_off, cpre,
               nseg, bits, C, part_off, static_cast<uint32_t>(n));
  return EIGER_OK;
}

// One side of a wide radix join: keys, row ids and nw word lanes per pass.
template <typename K>
struct WideSide {
  K *k[2];
  uint32_t *r[2];
  uint32_t *w[2][kMaxWords];
  uint32_t *seg1, *cpre1, *off1, *cpre2, *off;
};

template <typename K>
WideSide<K> wide_side_layout(Workspace &ws, uint64_t n, int nw, const PassPlan &pp) {
  WideSide<K> S{};
  const uint64_t m = n ? n : 1;
  for (int q = 0; q < pp.passes; ++q) {
    S.k[q] = ws.take<K>(m);
    S.r[q] = ws.take<uint32_t>(m);
    for (int w = 0; w < nw; ++w) S.w[q][w] = ws.take<uint32_t>(m);
  }
  S.seg1 = ws.take<uint32_t>(2);
  S.cpre1 = ws.take<uint32_t>(2);
  S.off1 = ws.take<uint32_t>((uint64_t(1) << pp.bits[0]) + 1);
  S.cpre2 = ws.take<uint32_t>((uint64_t(1) << pp.bits[0]) + 1);
  S.off = pp.passes == 2 ? ws.take<uint32_t>((uint64_t(1) << (pp.bits[0] + pp.bits[1])) + 1) : S.off1;
  return S;
}

// Partition a side carrying its word lanes (src); the final pass's arrays are
// S.k[last], S.r[last], S.w[last][*].
template <typename K>
int partition_side_carry(const K *keys, const Lanes &src, uint64_t n, WideSide<K> &S, const PassPlan &pp,
                         uint32_t *C, uint64_t *tmp, uint64_t *total, hipStream_t s) {
  EIGER_LAUNCH("radix_seg", k_single_segment, dim3(1), dim3(64), 0, s, S.seg1, S.cpre1, static_cast<uint32_t>(n));
  Lanes l1 = src;
  for (int w = 0; w < src.n; ++w) l1.dst[w] = S.w[0][w];
  int rc;
  const int b1 = pp.bits[0];
  if ((rc = part_pass_carry<K, false>(keys, nullptr, l1, S.k[0], S.r[0], n, S.seg1, S.cpre1, 1, 64 - b1, b1, C, tmp,
                                      total, S.off1, s)))
    return rc;
  if (pp.passes == 1) return EIGER_OK;
  const uint32_t nseg = 1u << b1;
  EIGER_LAUNCH("radix_chunks", k_chunk_counts, dim3((nseg + 1 + 255) / 256), dim3(256), 0, s, S.off1, nseg, S.cpre2);
  if ((rc = exclusive_scan_u32(S.cpre2, S.cpre2, nseg + 1, tmp, total, s))) return rc;
  Lanes l2{};
  l2.n = src.n;
  for (int w = 0; w < src.n; ++w) {
    l2.src[w] = S.w[0][w];
    l2.src_stride[w] = 1;
    l2.dst[w] = S.w[1][w];
  }
  const int b2 = pp.bits[1];
  return part_pass_carry<K, true>(S.k[0], S.r[0], l2, S.k[1], S.r[1], n, S.off1, S.cpre2, nseg, 64 - b1 - b2, b2, C,
                                  tmp, total, S.off, s);
}

template <typename K>
int radix_wide_impl(const JoinArgs &a, const WordCols &colsR, const WordCols &colsS, Workspace &ws,
                    JoinCounters **ctr, WideSource *outR, WideSource *outS) {
  const PassPlan pp = split_bits(a.plan.radix_bits, a.plan.radix_passes);
  const int bits = pp.bits[0] + pp.bits[1];
  const uint32_t F = 1u << bits;
  float lf = a.plan.load_factor;
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  const RadixLimits lim = radix_limits(a.kdt, a.kdt, lf);
  JoinCounters *c = ws.take<JoinCounters>(1);
  WideSide<K> R = wide_side_layout<K>(ws, a.nR, colsR.n, pp);
  WideSide<K> S = wide_side_layout<K>(ws, a.nS, colsS.n, pp);
  const uint64_t nC = std::max(counters_len(a.nR, pp), counters_len(a.nS, pp));
  uint32_t *C = ws.take<uint32_t>(nC);
  uint64_t *tmp = ws.take<uint64_t>(scan_tmp_elems(std::max<uint64_t>(nC, F + 1)));
  uint64_t *total = ws.take<uint64_t>(1);
  uint32_t *items = ws.take<uint32_t>(F + 1);
  uint32_t *item_part = ws.take<uint32_t>(uint64_t(F) + (a.nS + kJTile - 1) / kJTile + 1);
  *ctr = c;
  const int last = pp.passes - 1;
  outR->rows = R.r[last];
  outS->rows = S.r[last];
  for (int w = 0; w < kMaxWords; ++w) {
    outR->words[w] = w < colsR.n ? R.w[last][w] : nullptr;
    outS->words[w] = w < colsS.n ? S.w[last][w] : nullptr;
  }
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if (a.nR == 0 || a.nS == 0) return EIGER_OK;
  Lanes lr{}, ls{};
  lr.n = colsR.n;
  ls.n = colsS.n;
  for (int w = 0; w < colsR.n; ++w) {
    lr.src[w] = colsR.src[w];
    lr.src_stride[w] = colsR.stride[w];
  }
  for (int w = 0; w < colsS.n; ++w) {
    ls.src[w] = colsS.src[w];
    ls.src_stride[w] = colsS.stride[w];
  }
  if ((rc = partition_side_carry<K>(static_cast<const K *>(a.bk), lr, a.nR, R, pp, C, tmp, total, s))) return rc;
  if ((rc = partition_side_carry<K>(static_cast<const K *>(a.pk), ls, a.nS, S, pp, C, tmp, total, s))) return rc;
  EIGER_LAUNCH("radix_items", k_items, dim3((F + 1 + 255) / 256), dim3(256), 0, s, R.off, S.off, F, items);
  if ((rc = exclusive_scan_u32(items, items, F + 1, tmp, total, s))) return rc;
  EIGER_LAUNCH("radix_items", k_item_part, dim3((F + 255) / 256), dim3(256), 0, s, items, F, item_part);
  // positions, not row ids: no row-id arrays go in, and the keys stand in for
  // the payloads (the wide join reports no payload aggregate)
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  const unsigned grid = static_cast<unsigned>(device_cu_count()) * 2;
  const K *rk = R.k[last], *sk = S.k[last];
  EIGER_LAUNCH("radix_join", (k_radix_join<K, K, K>), dim3(grid), dim3(kJNT), 0, s, rk, rk,
               static_cast<const uint32_t *>(nullptr), R.off, sk, sk, static_cast<const uint32_t *>(nullptr), S.off,
               items, item_part, F, lim.max_build, lf, o);
  return EIGER_OK;
}

}  // namespace

RadixLimits radix_limits(int32_t kdt, int32_t bpdt, float lf) {
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  RadixLimits r{};
  if (kdt == EIGER_INT32) {  // grouped tables (join_chunk_grouped)
    r.max_build = grouped_max_build(lf);
    r.max_slots = static_cast<uint32_t>(kTableBytes / 8);
    return r;
  }
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

int run_radix_wide(const JoinArgs &a, const WordCols &colsR, const WordCols &colsS, Workspace &ws, JoinCounters **ctr,
                   WideSource *outR, WideSource *outS) {
  if (a.kdt == EIGER_INT64) return radix_wide_impl<int64_t>(a, colsR, colsS, ws, ctr, outR, outS);
  return radix_wide_impl<int32_t>(a, colsR, colsS, ws, ctr, outR, outS);
}

}  // namespace eiger

// ============================================================================
// RADIX_CACHE: one partitioning pass over the probe side; the build side goes
// into ONE table laid out partition-major (partition p owns slots
// [table_off[p], table_off[p+1])), each region sized to stay in an XCD's L2.
// Probe tiles are taken in partition order and split into eight contiguous
// ranges, one per XCD (workgroup w runs on XCD w % 8 under round-robin
// dispatch), so the workgroups of an XCD work on one partition at a time and
// its table region is read from that XCD's L2.
// ============================================================================
namespace eiger {
namespace {

constexpr int kCNT = 256;
constexpr int kCIPT = 4;
constexpr int kCSCAP = 4096;
constexpr uint32_t kCTileMax = 16384;  // probe rows per work item (upper bound)
constexpr int kXcds = 8;
constexpr double kL2RegionMax = 3.0 * 1024 * 1024;  // larger regions use the shared schedule

__device__ __forceinline__ uint32_t fastrange32(uint64_t h, uint32_t n) {
  return static_cast<uint32_t>((uint64_t(static_cast<uint32_t>(h)) * n) >> 32);
}

template <typename K, typename PB>
struct CacheTab {
  static constexpr bool kHashed = true;
  static constexpr bool kRuns = false;
  using SlotT = Slot<K, PB>;
  using Index = uint32_t;  // regions hold fewer than 2^32 slots
  const Slot<K, PB> *__restrict__ slots;
  uint32_t n;
  bool unique;

  __device__ __forceinline__ uint32_t home(K key) const {
    return fastrange32(fmix64(static_cast<uint64_t>(sext(key))), n);
  }
  __device__ __forceinline__ uint32_t next(uint32_t i) const { return (i + 1 == n) ? 0 : i + 1; }
  __device__ __forceinline__ SlotT load(uint32_t i) const { return slots[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint32_t i = home(key);
    for (;;) {
      const Slot<K, PB> s = slots[i];
      if (s.rowid == kEmpty) break;
      if (s.key == key) f(s.rowid);
      i = next(i);
    }
  }
};

// Sets *dup when some build key occurs twice (each build row counts its key in
// its partition's region).
template <typename K, typename PB>
__global__ void k_cache_unique(const K *__restrict__ keys, uint64_t n, int bits,
                               const uint32_t *__restrict__ table_off,
                               const Slot<K, PB> *__restrict__ table, uint32_t *dup) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    if (*static_cast<volatile uint32_t *>(dup)) return;
    const K key = keys[r];
    const uint32_t p = static_cast<uint32_t>(part_hash(key) >> (64 - bits));
    CacheTab<K, PB> tab{table + table_off[p], table_off[p + 1] - table_off[p], false};
    uint32_t c = 0;
    tab.for_each(key, [&](uint32_t) { ++c; });
    if (c > 1) atomicOr(dup, 1u);
  }
}

// Slots of each partition's region (at least one more than its rows, so every
// probe walk ends at an empty slot) and probe tiles per partition.
__global__ void k_cache_sizes(const uint32_t *__restrict__ offR, const uint32_t *__restrict__ offS,
                              uint32_t F, float lf, uint32_t ctile, uint32_t *__restrict__ tsz,
                              uint32_t *__restrict__ tiles) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < F) {
    const uint32_t nr = offR[p + 1] - offR[p], ns = offS[p + 1] - offS[p];
    tsz[p] = nr ? static_cast<uint32_t>(ceil(static_cast<double>(nr) / static_cast<double>(lf))) + 1u : 0u;
    if (nr && tsz[p] <= nr) tsz[p] = nr + 1;
    tiles[p] = (nr && ns) ? (ns + ctile - 1) / ctile : 0u;
  }
  if (p == F) {
    tsz[p] = 0;
    tiles[p] = 0;
  }
}

template <typename K, typename PB>
__global__ void k_cache_build(const K *__restrict__ keys, const PB *__restrict__ pay, uint64_t n,
                              int bits, const uint32_t *__restrict__ table_off,
                              Slot<K, PB> *__restrict__ table) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    const K key = keys[r];
    const uint64_t h = fmix64(static_cast<uint64_t>(sext(key)));  // slot within the region
    const uint32_t p = static_cast<uint32_t>(part_hash(key) >> (64 - bits));
    const uint32_t base = table_off[p], ns = table_off[p + 1] - base;
    uint32_t i = fastrange32(h, ns);
    for (;;) {
      if (atomicCAS(&table[base + i].rowid, kEmpty, static_cast<uint32_t>(r)) == kEmpty) {
        table[base + i].key = key;
        table[base + i].pay = pay[r];
        break;
      }
      i = (i + 1 == ns) ? 0 : i + 1;
    }
  }
}

template <typename K, typename PB, typename PS>
__global__ void __launch_bounds__(kCNT)
    k_cache_probe(const Slot<K, PB> *__restrict__ table, const uint32_t *__restrict__ table_off,
                  const K *__restrict__ sk, const PS *__restrict__ sp, const uint32_t *__restrict__ sr,
                  const uint32_t *__restrict__ offS, const uint32_t *__restrict__ tile_off,
                  const uint32_t *__restrict__ tile_part, uint32_t F, uint32_t per_xcd, uint32_t ctile,
                  int shared_mall, const uint32_t *dup, EmitOut o) {
  __shared__ EmitLds<kCNT, kCSCAP> L;
  uint64_t fill = 0;
  uint64_t cs = 0;
  const bool unique = *dup == 0;
  const uint64_t T = tile_off[F];
  // L2 schedule: XCD x takes the x-th eighth of the tiles (its own partitions).
  // Shared schedule (regions too big for an L2): consecutive tiles go to
  // consecutive workgroups, so every XCD works on the same partition and its
  // region stays in the memory-side cache.
  const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const uint64_t xlo = shared_mall ? blockIdx.x : T * x / kXcds + j;
  const uint64_t xhi = shared_mall ? T : T * (x + 1) / kXcds;
  const uint64_t step = shared_mall ? gridDim.x : per_xcd;
  for (uint64_t t = xlo; t < xhi; t += step) {
    const uint32_t p = tile_part[t];
    const uint32_t s0 = offS[p] + static_cast<uint32_t>(t - tile_off[p]) * ctile;
    const uint32_t s1 = min(offS[p + 1], s0 + ctile);
    CacheTab<K, PB> tab{table + table_off[p], table_off[p + 1] - table_off[p], unique};
    probe_range<kCNT, kCIPT, kCSCAP>(tab, sk, sp, sr, s0, s1, L, fill, o, cs);
  }
  finish(L, o, fill, cs);
}

uint64_t cache_table_bound(uint64_t nR, float lf, uint32_t F) {
  return static_cast<uint64_t>(static_cast<double>(nR) / static_cast<double>(lf)) + 2ull * F + 64;
}

template <typename K, typename PB, typename PS>
int radix_cache_impl(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  int bits = a.plan.radix_bits;
  if (bits < 1) bits = 1;
  if (bits > kCacheMaxBits) bits = kCacheMaxBits;
  const uint32_t F = 1u << bits;
  float lf = a.plan.load_factor;
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  const PassPlan pp{{bits, 0}, 1};
  const uint64_t tbound = cache_table_bound(a.nR, lf, F);
  if (tbound >= (uint64_t(1) << 32))
    return fail(EIGER_ERR_TOO_LARGE, "RADIX_CACHE: table above 2^32 slots; raise the load factor");

  JoinCounters *c = ws.take<JoinCounters>(1);
  SideBufs<K, PS> S = side_layout<K, PS>(ws, a.nS, pp);
  uint32_t *seg1 = ws.take<uint32_t>(2), *cpre1 = ws.take<uint32_t>(2);
  uint32_t *offR = ws.take<uint32_t>(F + 1);
  const uint64_t nC = std::max(ub_chunks(a.nR, 1), ub_chunks(a.nS, 1)) << bits;
  uint32_t *C = ws.take<uint32_t>(nC);
  uint64_t *tmp = ws.take<uint64_t>(scan_tmp_elems(std::max<uint64_t>(nC, F + 1)));
  uint64_t *total = ws.take<uint64_t>(1);
  uint32_t *table_off = ws.take<uint32_t>(F + 1);
  uint32_t *tile_off = ws.take<uint32_t>(F + 1);
  // tiles hold at least 2048 probe rows, so a partition has at most ceil(rows / 2048)
  uint32_t *tile_part = ws.take<uint32_t>(uint64_t(F) + (a.nS + 2047) / 2048 + 1);
  uint32_t *dup = ws.take<uint32_t>(1);
  Slot<K, PB> *table = ws.take<Slot<K, PB>>(tbound);
  *ctr = c;
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if (a.nR == 0 || a.nS == 0) return EIGER_OK;
  const K *bk = static_cast<const K *>(a.bk);
  // build side: partition sizes only (histogram + scan), no scatter
  EIGER_LAUNCH("radix_seg", k_single_segment, dim3(1), dim3(64), 0, s, seg1, cpre1,
               static_cast<uint32_t>(a.nR));
  {
    const uint64_t ub = ub_chunks(a.nR, 1), nCR = ub << bits;
    if ((rc = fill_u32(C, nCR, 0, s))) return rc;
    EIGER_LAUNCH("radix_hist", k_part_hist<K>, dim3(unsigned(ub)), dim3(kPNT), 0, s, bk, seg1, cpre1, 1u,
                 64 - bits, bits, C);
    if ((rc = exclusive_scan_u32(C, C, nCR, tmp, total, s))) return rc;
    EIGER_LAUNCH("radix_offsets", k_part_offsets, dim3(unsigned((F + 1 + 255) / 256)), dim3(256), 0, s,
                 seg1, cpre1, 1u, bits, C, offR, static_cast<uint32_t>(a.nR));
  }
  // probe side: one partitioning pass
  Side<K, PS> fs;
  if ((rc = partition_side<K, PS>(static_cast<const K *>(a.pk), static_cast<const PS *>(a.pp), a.nS, S,
                                  pp, C, tmp, total, s, &fs)))
    return rc;
  // The workgroups of one XCD should cover about one partition at a time, so
  // that a single table region is live in that XCD's L2.
  const uint32_t per_xcd = static_cast<uint32_t>(std::max(1, device_cu_count() / kXcds)) * 4;
  const double region = static_cast<double>(a.nR) / F / lf * sizeof(Slot<K, PB>);
  const int shared_mall = region > kL2RegionMax ? 1 : 0;
  uint64_t ct = shared_mall ? kCTileMax : a.nS / F / per_xcd;
  ct = std::max<uint64_t>(2048, std::min<uint64_t>(kCTileMax, ct));
  const uint32_t ctile = static_cast<uint32_t>((ct + 2047) / 2048 * 2048);
  EIGER_LAUNCH("cache_sizes", k_cache_sizes, dim3((F + 1 + 255) / 256), dim3(256), 0, s, offR, S.off, F,
               lf, ctile, table_off, tile_off);
  if ((rc = exclusive_scan_u32(table_off, table_off, F + 1, tmp, total, s))) return rc;
  if ((rc = exclusive_scan_u32(tile_off, tile_off, F + 1, tmp, total, s))) return rc;
  EIGER_LAUNCH("cache_sizes", k_item_part, dim3((F + 255) / 256), dim3(256), 0, s, tile_off, F, tile_part);
  if ((rc = fill_u32(reinterpret_cast<uint32_t *>(table), tbound * sizeof(Slot<K, PB>) / 4, kEmpty, s)))
    return rc;
  EIGER_LAUNCH("cache_build", (k_cache_build<K, PB>), dim3(grid_for_rows(a.nR)), dim3(256), 0, s, bk,
               static_cast<const PB *>(a.bp), a.nR, bits, table_off, table);
  if ((rc = fill_u32(dup, 1, 0, s))) return rc;
  EIGER_LAUNCH("cache_unique", (k_cache_unique<K, PB>), dim3(grid_for_rows(a.nR)), dim3(256), 0, s, bk, a.nR,
               bits, table_off, table, dup);
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  EIGER_LAUNCH("cache_probe", (k_cache_probe<K, PB, PS>), dim3(per_xcd * kXcds), dim3(kCNT), 0, s, table,
               table_off, fs.k, fs.p, fs.r, S.off, tile_off, tile_part, F, per_xcd, ctile, shared_mall, dup, o);
  return EIGER_OK;
}

}  // namespace

int run_radix_cache(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const bool k64 = a.kdt == EIGER_INT64, b64 = a.bpdt == EIGER_INT64, p64 = a.ppdt == EIGER_INT64;
#define EIGER_DISPATCH(KT, BT, PT) return radix_cache_impl<KT, BT, PT>(a, ws, ctr)
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
