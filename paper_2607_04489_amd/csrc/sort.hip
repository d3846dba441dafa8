// sort.hip -- stable LSD radix sort of (key, row id) pairs, keys of 4 or 8 bytes.
//
// Section 3.6 (cases 1 and 2): a single numeric key, or several keys fused into
// one by smart key fusion, are sorted by radix sort. Each pass sorts by one digit
// of at most 8 bits, least significant digit first; the number of passes follows
// the key's significant width (the fused key's width), not its type.
//
// One pass = a per-tile digit histogram (k_sort_hist), one device-wide exclusive
// scan over the digit-major count table, and a scatter (k_sort_scatter). The
// scatter ranks each tile's items stably: every wave walks its own contiguous
// segment 64 items at a time, finds the lanes holding the same digit with one
// ballot per digit bit, and keeps per-wave running digit counts in LDS; items are
// then placed digit-major into an LDS copy of the tile and leave it in order, so
// each digit's run of the tile goes out as one contiguous block.
#include "common.hpp"
#include "sort.hpp"

namespace eiger {

namespace {

constexpr int kSNT = 256;
constexpr int kSWaves = kSNT / 64;
constexpr int kSDigitBits = 8;
constexpr int kSDigits = 1 << kSDigitBits;
static_assert(kSDigits == kSNT, "one thread per digit in the per-tile digit scan");

// Tiles of 8,192 items (4,096 for 8-byte keys): each digit's run of a tile
// averages 32 items, so its writes cover whole 128-byte lines more often
// (measured per 4-byte pass at 2^28 items: 2,048 items 3.8 ms, 4,096 2.7 ms,
// 6,144 1.9 ms, 8,192 1.7 ms).
template <typename K>
constexpr int items_per_thread() {
  return sizeof(K) == 8 ? 16 : 32;
}
// Workgroups per CU of the grids; workgroups loop over the remaining tiles. The
// histogram keeps one tile per workgroup; the scatter, whose workgroups hold
// up to 70 KB of LDS, runs best with a few resident workgroups per CU.
constexpr uint64_t kHistPerCu = 64;
constexpr uint64_t kScatPerCu = 8;

// Digit of a plain sort: bits [shift, shift + width) of the key.
template <typename K>
struct KeyDigit {
  static constexpr bool kStore = false;  // cheap: recomputed from the key
  int shift;
  uint32_t mask;
  __device__ __forceinline__ uint32_t operator()(K k) const { return static_cast<uint32_t>(k >> shift) & mask; }
};

// Digit of a key's partition id, the top `bits` bits of its partition hash
// (hash partitioning).
template <typename K>
struct PartDigit {
  static constexpr bool kStore = true;  // a hash per item: kept in LDS for the write-out
  int top;                              // 64 - partition bits
  int shift;
  uint32_t mask;
  __device__ __forceinline__ uint32_t operator()(K k) const {
    return static_cast<uint32_t>((part_hash(k) >> top) >> shift) & mask;
  }
};

// Workgroups loop over tiles (the grid is sized to the chip): one workgroup
// per tile was limited by how fast workgroups are dispatched, not by memory.
// kVec (16-byte aligned keys): each thread reads 16 bytes of consecutive keys
// per load (counting does not depend on which thread holds which key).
template <typename K, int kItems, typename D, bool kVec>
__global__ void __launch_bounds__(kSNT) k_sort_hist(const K *__restrict__ keys, uint64_t n, D dig, uint32_t ntiles,
                                                    uint32_t *__restrict__ cnt) {
  constexpr int T = kSNT * kItems;
  constexpr int V = 16 / static_cast<int>(sizeof(K));  // keys per 16-byte load
  constexpr int NV = T / V;                            // 16-byte loads per tile (T is a multiple of 256)
  __shared__ uint32_t h[kSDigits];
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(tile) * T;
    if constexpr (kVec) {
#pragma unroll
      for (int j = 0; j < (NV + kSNT - 1) / kSNT; ++j) {
        const int q = j * kSNT + static_cast<int>(threadIdx.x);
        if (q >= NV) break;
        const uint64_t i = base + static_cast<uint64_t>(q) * V;
        if (i + V <= n) {
          K v[V];
          *reinterpret_cast<uint4 *>(v) = *reinterpret_cast<const uint4 *>(keys + i);
#pragma unroll
          for (int u = 0; u < V; ++u) atomicAdd(&h[dig(v[u])], 1u);
        } else {
#pragma unroll
          for (int u = 0; u < V; ++u)
            if (i + u < n) atomicAdd(&h[dig(keys[i + u])], 1u);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const uint64_t i = base + static_cast<uint64_t>(j) * kSNT + threadIdx.x;
        if (i < n) atomicAdd(&h[dig(keys[i])], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x <= dig.mask) cnt[static_cast<uint64_t>(threadIdx.x) * ntiles + tile] = h[threadIdx.x];
    __syncthreads();
  }
}

// 32-bit value lanes moved along with the keys. Lane w of row i is
// src[w][i * stride[w]]; a NULL source lane means the row id i itself.
constexpr int kSortLanes = 4;
struct LanesIn {
  const uint32_t *src[kSortLanes];
  uint32_t stride[kSortLanes];
};
struct LanesOut {
  uint32_t *dst[kSortLanes];
};

// One LSD pass: rank each tile's items stably by digit, place them digit-major
// in LDS, write each digit's run of the tile to its global position.
template <typename K, int NW, int kItems, typename D>
__global__ void __launch_bounds__(kSNT) k_sort_scatter(const K *__restrict__ kin, LanesIn vin, uint64_t n, D dig,
                                                       int bits, uint32_t ntiles, const uint32_t *__restrict__ offs,
                                                       K *__restrict__ kout, LanesOut vout) {
  constexpr int T = kSNT * kItems;
  constexpr int NL = NW > 0 ? NW : 1;
  __shared__ K sk[T];
  __shared__ uint32_t sv[NL][NW > 0 ? T : 1];
  __shared__ uint8_t sd[D::kStore ? T : 1];
  __shared__ uint32_t wcnt[kSWaves][kSDigits];
  __shared__ uint32_t dstart[kSDigits];
  __shared__ uint32_t adj[kSDigits];
  __shared__ uint32_t scan_tmp[kSWaves + 1];
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
    for (int x = 0; x < kSWaves; ++x) wcnt[x][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(tile) * T;
    const uint64_t wbase = base + static_cast<uint64_t>(w) * (64 * kItems);
    K key[kItems];
    uint32_t val[NL][kItems], lo[kItems], dg[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      const bool ok = i < n;
      key[j] = ok ? kin[i] : K(0);
#pragma unroll
      for (int v = 0; v < NW; ++v)
        val[v][j] = ok ? (vin.src[v] ? vin.src[v][i * vin.stride[v]] : static_cast<uint32_t>(i)) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      const bool ok = i < n;
      const uint32_t d = dig(key[j]);
      dg[j] = d;
      uint64_t peers = __ballot(ok);
#pragma unroll
      for (int b = 0; b < kSDigitBits; ++b) {
        if (b < bits) {
          const bool set = (d >> b) & 1u;
          const uint64_t bb = __ballot(set);
          peers &= set ? bb : ~bb;
        }
      }
      const uint32_t before = lane_prefix(peers);
      // every lane reads the wave's running count before the group's first lane
      // (the only writer of this digit in this step) stores the new one; LDS
      // operations of one wave complete in order
      const uint32_t pre = ok ? wcnt[w][d] : 0u;
      if (ok && before == 0) wcnt[w][d] = pre + static_cast<uint32_t>(__popcll(peers));
      lo[j] = pre + before;
    }
    __syncthreads();
    // digit t: exclusive prefix over the waves (wave order = item order), tile total
    const int t = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int x = 0; x < kSWaves; ++x) {
      const uint32_t c = wcnt[x][t];
      wcnt[x][t] = tot;
      tot += c;
    }
    uint32_t all;
    const uint32_t ds = block_exclusive_scan<kSNT, uint32_t>(tot, scan_tmp, &all);
    dstart[t] = ds;
    // global start of this tile's run of digit t, minus its start inside the tile
    adj[t] = static_cast<uint32_t>(t) <= dig.mask ? offs[static_cast<uint64_t>(t) * ntiles + tile] - ds : 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      if (i < n) {
        const uint32_t d = D::kStore ? dg[j] : dig(key[j]);
        const uint32_t p = dstart[d] + wcnt[w][d] + lo[j];
        sk[p] = key[j];
#pragma unroll
        for (int v = 0; v < NW; ++v) sv[v][p] = val[v][j];
        if constexpr (D::kStore) sd[p] = static_cast<uint8_t>(d);
      }
    }
    __syncthreads();
    const uint32_t in_tile = static_cast<uint32_t>(min<uint64_t>(T, n - base));
    for (uint32_t p = threadIdx.x; p < in_tile; p += kSNT) {
      const K k = sk[p];
      uint32_t d;
      if constexpr (D::kStore)
        d = sd[p];
      else
        d = dig(k);
      const uint32_t o = adj[d] + p;
      kout[o] = k;
#pragma unroll
      for (int v = 0; v < NW; ++v) vout.dst[v][o] = sv[v][p];
    }
    __syncthreads();
  }
}

template <typename K>
__global__ void __launch_bounds__(256) k_sort_copy(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                   uint64_t n, K *__restrict__ kout, uint32_t *__restrict__ vout) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    kout[i] = kin[i];
    vout[i] = vin ? vin[i] : static_cast<uint32_t>(i);
  }
}

// Count-table and temporaries of the passes over n items in tiles of T.
template <typename K, int NW>
struct PassBufs {
  uint64_t ntiles;
  uint32_t *cnt;
  uint64_t *tmp, *total;
  K *k2;
  uint32_t *v2[NW > 0 ? NW : 1];
};

template <typename K, int NW>
PassBufs<K, NW> pass_bufs(Workspace &ws, uint64_t n, int T) {
  PassBufs<K, NW> b{};
  b.ntiles = (n + T - 1) / T;
  const uint64_t ncnt = b.ntiles * kSDigits;
  b.cnt = ws.take<uint32_t>(ncnt);
  b.tmp = ws.take<uint64_t>(scan_tmp_elems(ncnt));
  b.total = ws.take<uint64_t>(1);
  b.k2 = ws.take<K>(n);
  for (int v = 0; v < NW; ++v) b.v2[v] = ws.take<uint32_t>(n);
  return b;
}

// ceil(total_bits / digit_bits) stable passes of balanced digit widths, least
// significant digit first, alternating between (kout, vout) and the
// temporaries so that the last pass lands in (kout, vout). make(shift, mask)
// gives the pass's digit functor.
template <typename K, int NW, int kItems, typename MakeDigit>
int lsd_passes(const K *kin, LanesIn vin, uint64_t n, int total_bits, int digit_bits, K *kout, LanesOut vout,
               const PassBufs<K, NW> &b, MakeDigit make, hipStream_t s) {
  const int passes = (total_bits + digit_bits - 1) / digit_bits;
  const unsigned hist_grid =
      static_cast<unsigned>(std::min<uint64_t>(b.ntiles, uint64_t(device_cu_count()) * kHistPerCu));
  const unsigned scat_grid =
      static_cast<unsigned>(std::min<uint64_t>(b.ntiles, uint64_t(device_cu_count()) * kScatPerCu));
  int shift = 0;
  const K *src_k = kin;
  LanesIn src_v = vin;
  for (int p = 0; p < passes; ++p) {
    const int bits = (total_bits - shift + (passes - p) - 1) / (passes - p);
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    K *dk = to_out ? kout : b.k2;
    LanesOut dv{};
    for (int v = 0; v < NW; ++v) dv.dst[v] = to_out ? vout.dst[v] : b.v2[v];
    const auto dig = make(shift, (1u << bits) - 1u);
    if (reinterpret_cast<uintptr_t>(src_k) % 16 == 0)
      EIGER_LAUNCH("sort_hist", (k_sort_hist<K, kItems, decltype(dig), true>), dim3(hist_grid), dim3(kSNT), 0, s,
                   src_k, n, dig, static_cast<uint32_t>(b.ntiles), b.cnt);
    else
      EIGER_LAUNCH("sort_hist", (k_sort_hist<K, kItems, decltype(dig), false>), dim3(hist_grid), dim3(kSNT), 0, s,
                   src_k, n, dig, static_cast<uint32_t>(b.ntiles), b.cnt);
    int rc = exclusive_scan_u32(b.cnt, b.cnt, (static_cast<uint64_t>(dig.mask) + 1) * b.ntiles, b.tmp, b.total, s);
    if (rc) return rc;
    EIGER_LAUNCH("sort_scatter", (k_sort_scatter<K, NW, kItems, decltype(dig)>), dim3(scat_grid), dim3(kSNT), 0, s,
                 src_k, src_v, n, dig, bits, static_cast<uint32_t>(b.ntiles), b.cnt, dk, dv);
    src_k = dk;
    for (int v = 0; v < NW; ++v) {
      src_v.src[v] = dv.dst[v];
      src_v.stride[v] = 1;
    }
    shift += bits;
  }
  return EIGER_OK;
}

template <typename K>
int sort_impl(const K *kin, const uint32_t *vin, uint64_t n, int key_bits, K *kout, uint32_t *vout, Workspace &ws,
              hipStream_t s) {
  constexpr int kItems = items_per_thread<K>();
  const PassBufs<K, 1> b = pass_bufs<K, 1>(ws, n, kSNT * kItems);
  if (!ws.base || n == 0) return EIGER_OK;
  const int passes = (key_bits + kSDigitBits - 1) / kSDigitBits;
  if (passes == 0 || n == 1) {
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((n + 255) / 256, 4096));
    EIGER_LAUNCH("sort_copy", k_sort_copy<K>, dim3(grid), dim3(256), 0, s, kin, vin, n, kout, vout);
    return EIGER_OK;
  }
  LanesIn in{};
  in.src[0] = vin;
  in.stride[0] = 1;
  LanesOut out{};
  out.dst[0] = vout;
  return lsd_passes<K, 1, kItems>(kin, in, n, key_bits, kSDigitBits, kout, out, b,
                                  [](int shift, uint32_t mask) { return KeyDigit<K>{shift, mask}; }, s);
}

// Partition bounds: off[p] = first position whose partition id is >= p (the
// rows are sorted by partition id), off[F] = n.
template <typename K>
__global__ void __launch_bounds__(256) k_part_bounds(const K *__restrict__ keys, uint64_t n, int bits, uint32_t F,
                                                     uint32_t *__restrict__ off) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p <= F; p += stride) {
    uint64_t a = 0, b = n;
    while (a < b) {
      const uint64_t m = a + (b - a) / 2;
      if ((part_hash(keys[m]) >> (64 - bits)) < p)
        a = m + 1;
      else
        b = m;
    }
    off[p] = static_cast<uint32_t>(a);
  }
}

// Tile items for hash partitioning: the largest count (at most 32 per thread)
// whose LDS copy (key, lanes, digit byte) stays within 64 KB, two workgroups per CU.
template <typename K, int NW>
constexpr int part_items() {
  constexpr int per = 65536 / (kSNT * static_cast<int>(sizeof(K) + 4 * NW + 1));
  return per > 32 ? 32 : per;
}

// Widest digit of a partitioning pass: at least 32 items of a tile per digit on
// average, so each digit's run of the tile is written in whole lines more often
// (2^28 rows, 4-byte keys and two 4-byte lanes, 4,864-item tiles: 14 bits in
// two 7-bit passes 7.6 ms, 16 bits in two 8-bit passes 11.2 ms).
constexpr int part_digit_bits(int tile) {
  int b = 1;
  while (b < kSDigitBits && (tile >> (b + 1)) >= 32) ++b;
  return b;
}

template <typename K, int NW>
int partition_impl(const K *keys, uint64_t n, const PartLanes &cols, int bits, Workspace &ws, PartitionOut *out,
                   hipStream_t s, bool run) {
  constexpr int kItems = part_items<K, NW>();
  const uint32_t F = 1u << bits;
  K *ok = ws.take<K>(n ? n : 1);
  LanesOut ov{};
  for (int v = 0; v < NW; ++v) ov.dst[v] = ws.take<uint32_t>(n ? n : 1);
  uint32_t *off = ws.take<uint32_t>(uint64_t(F) + 1);
  const PassBufs<K, NW> b = pass_bufs<K, NW>(ws, n, kSNT * kItems);
  out->keys = ok;
  for (int v = 0; v < kSortLanes; ++v) out->words[v] = v < NW ? ov.dst[v] : nullptr;
  out->off = off;
  if (!ws.base || !run) return EIGER_OK;
  if (n > 0) {
    LanesIn in{};
    for (int v = 0; v < NW; ++v) {
      in.src[v] = cols.src[v];
      in.stride[v] = cols.stride[v];
    }
    const int top = 64 - bits;
    int rc = lsd_passes<K, NW, kItems>(
        keys, in, n, bits, part_digit_bits(kSNT * kItems), ok, ov, b,
        [top](int shift, uint32_t mask) { return PartDigit<K>{top, shift, mask}; }, s);
    if (rc) return rc;
  }
  EIGER_LAUNCH("part_bounds", k_part_bounds<K>, dim3(static_cast<unsigned>(std::min<uint64_t>((F + 256) / 256, 1024))),
               dim3(256), 0, s, ok, n, bits, F, off);
  return EIGER_OK;
}

template <typename K>
int partition_lanes(const K *keys, uint64_t n, const PartLanes &cols, int bits, Workspace &ws, PartitionOut *out,
                    hipStream_t s, bool run) {
  switch (cols.n) {
    case 0: return partition_impl<K, 0>(keys, n, cols, bits, ws, out, s, run);
    case 1: return partition_impl<K, 1>(keys, n, cols, bits, ws, out, s, run);
    case 2: return partition_impl<K, 2>(keys, n, cols, bits, ws, out, s, run);
    case 3: return partition_impl<K, 3>(keys, n, cols, bits, ws, out, s, run);
    default: return partition_impl<K, 4>(keys, n, cols, bits, ws, out, s, run);
  }
}

}  // namespace

int radix_partition_lanes(int key_bytes, const void *keys, uint64_t n, const PartLanes &cols, int bits, Workspace &ws,
                          PartitionOut *out, hipStream_t s, bool run) {
  if (bits < 1 || bits > 24 || cols.n < 0 || cols.n > kSortLanes)
    return fail(EIGER_ERR_INVALID_ARG, "radix partition: bits in [1, 24], at most 4 lanes");
  if (key_bytes == 8)
    return partition_lanes<int64_t>(static_cast<const int64_t *>(keys), n, cols, bits, ws, out, s, run);
  return partition_lanes<int32_t>(static_cast<const int32_t *>(keys), n, cols, bits, ws, out, s, run);
}

int radix_sort_pairs(int key_bytes, const void *kin, const uint32_t *vin, uint64_t n, int key_bits, void *kout,
                     uint32_t *vout, Workspace &ws, hipStream_t s) {
  if (key_bytes == 8)
    return sort_impl<uint64_t>(static_cast<const uint64_t *>(kin), vin, n, key_bits, static_cast<uint64_t *>(kout),
                               vout, ws, s);
  return sort_impl<uint32_t>(static_cast<const uint32_t *>(kin), vin, n, key_bits, static_cast<uint32_t *>(kout),
                             vout, ws, s);
}

}  // namespace eiger

using namespace eiger;

namespace {

int check_sort_args(int32_t key_bytes, int64_t n, int32_t key_bits) {
  if (key_bytes != 4 && key_bytes != 8) return fail(EIGER_ERR_INVALID_ARG, "eiger_sort_pairs: key_bytes must be 4 or 8");
  if (n < 0 || n > EIGER_MAX_ROWS) return fail(EIGER_ERR_TOO_LARGE, "eiger_sort_pairs: n outside [0, EIGER_MAX_ROWS]");
  if (key_bits < 0 || key_bits > 8 * key_bytes)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_sort_pairs: key_bits outside [0, 8 * key_bytes]");
  return EIGER_OK;
}

}  // namespace

extern "C" int eiger_sort_pairs_workspace_size(int32_t key_bytes, int64_t n, int32_t key_bits, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_sort_pairs_workspace_size: bytes is NULL");
  if (int rc = check_sort_args(key_bytes, n, key_bits)) return rc;
  Workspace ws(nullptr, 0);
  radix_sort_pairs(key_bytes, nullptr, nullptr, static_cast<uint64_t>(n), key_bits, nullptr, nullptr, ws, nullptr);
  *bytes = ws.used + 256;
  return EIGER_OK;
}

extern "C" int eiger_sort_pairs(int32_t key_bytes, const void *keys_in, const uint32_t *vals_in, int64_t n,
                                int32_t key_bits, void *keys_out, uint32_t *vals_out, void *workspace,
                                size_t workspace_bytes, void *stream) {
  if (int rc = check_sort_args(key_bytes, n, key_bits)) return rc;
  if (n > 0 && (!keys_in || !keys_out || !vals_out || !workspace))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_sort_pairs: NULL buffer");
  size_t need = 0;
  eiger_sort_pairs_workspace_size(key_bytes, n, key_bits, &need);
  if (workspace_bytes < need) return fail(EIGER_ERR_WORKSPACE, "eiger_sort_pairs: workspace too small");
  if (n > 0 && (keys_in == keys_out || (vals_in && vals_in == vals_out)))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_sort_pairs: outputs must not alias the inputs");
  Workspace ws(workspace, workspace_bytes);
  return radix_sort_pairs(key_bytes, keys_in, vals_in, static_cast<uint64_t>(n), key_bits, keys_out, vals_out, ws,
                          static_cast<hipStream_t>(stream));
}
