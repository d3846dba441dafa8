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
// 70 KB of LDS, runs best with a few resident workgroups per CU.
constexpr uint64_t kHistPerCu = 64;
constexpr uint64_t kScatPerCu = 8;

template <typename K>
constexpr int tile_items() {
  return kSNT * items_per_thread<K>();
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift, uint32_t mask) {
  return static_cast<uint32_t>(k >> shift) & mask;
}

// Workgroups loop over tiles (the grid is sized to the chip): one workgroup
// per tile was limited by how fast workgroups are dispatched, not by memory.
template <typename K>
__global__ void __launch_bounds__(kSNT) k_sort_hist(const K *__restrict__ keys, uint64_t n, int shift,
                                                    uint32_t mask, uint32_t ntiles, uint32_t *__restrict__ cnt) {
  constexpr int kItems = items_per_thread<K>();
  __shared__ uint32_t h[kSDigits];
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(tile) * tile_items<K>();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = base + static_cast<uint64_t>(j) * kSNT + threadIdx.x;
      if (i < n) atomicAdd(&h[digit_of(keys[i], shift, mask)], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= mask) cnt[static_cast<uint64_t>(threadIdx.x) * ntiles + tile] = h[threadIdx.x];
    __syncthreads();
  }
}

// vin == nullptr: the values are the row ids (first pass of a permutation sort).
template <typename K>
__global__ void __launch_bounds__(kSNT) k_sort_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                       uint64_t n, int shift, int bits, uint32_t ntiles,
                                                       const uint32_t *__restrict__ offs, K *__restrict__ kout,
                                                       uint32_t *__restrict__ vout) {
  constexpr int kItems = items_per_thread<K>();
  constexpr int T = tile_items<K>();
  __shared__ K sk[T];
  __shared__ uint32_t sv[T];
  __shared__ uint32_t wcnt[kSWaves][kSDigits];
  __shared__ uint32_t dstart[kSDigits];
  __shared__ uint32_t adj[kSDigits];
  __shared__ uint32_t scan_tmp[kSWaves + 1];
  const uint32_t mask = (1u << bits) - 1u;
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
    for (int x = 0; x < kSWaves; ++x) wcnt[x][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(tile) * T;
    const uint64_t wbase = base + static_cast<uint64_t>(w) * (64 * kItems);
    K key[kItems];
    uint32_t val[kItems], lo[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      const bool ok = i < n;
      key[j] = ok ? kin[i] : K(0);
      val[j] = ok ? (vin ? vin[i] : static_cast<uint32_t>(i)) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      const bool ok = i < n;
      const uint32_t d = digit_of(key[j], shift, mask);
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
    adj[t] = static_cast<uint32_t>(t) <= mask ? offs[static_cast<uint64_t>(t) * ntiles + tile] - ds : 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = wbase + static_cast<uint64_t>(j) * 64 + lane;
      if (i < n) {
        const uint32_t d = digit_of(key[j], shift, mask);
        const uint32_t p = dstart[d] + wcnt[w][d] + lo[j];
        sk[p] = key[j];
        sv[p] = val[j];
      }
    }
    __syncthreads();
    const uint32_t in_tile = static_cast<uint32_t>(min<uint64_t>(T, n - base));
    for (uint32_t p = threadIdx.x; p < in_tile; p += kSNT) {
      const K k = sk[p];
      const uint32_t o = adj[digit_of(k, shift, mask)] + p;
      kout[o] = k;
      vout[o] = sv[p];
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

template <typename K>
int sort_impl(const K *kin, const uint32_t *vin, uint64_t n, int key_bits, K *kout, uint32_t *vout, Workspace &ws,
              hipStream_t s) {
  constexpr int T = tile_items<K>();
  const uint64_t ntiles = (n + T - 1) / T;
  const uint64_t ncnt = ntiles * kSDigits;
  uint32_t *cnt = ws.take<uint32_t>(ncnt);
  uint64_t *tmp = ws.take<uint64_t>(scan_tmp_elems(ncnt));
  uint64_t *total = ws.take<uint64_t>(1);
  K *k2 = ws.take<K>(n);
  uint32_t *v2 = ws.take<uint32_t>(n);
  if (!ws.base || n == 0) return EIGER_OK;
  const int passes = (key_bits + kSDigitBits - 1) / kSDigitBits;
  if (passes == 0 || n == 1) {
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((n + 255) / 256, 4096));
    EIGER_LAUNCH("sort_copy", k_sort_copy<K>, dim3(grid), dim3(256), 0, s, kin, vin, n, kout, vout);
    return EIGER_OK;
  }
  // balanced digit widths, least significant digit first; the last pass lands in out
  const unsigned hist_grid = static_cast<unsigned>(std::min<uint64_t>(ntiles, uint64_t(device_cu_count()) * kHistPerCu));
  const unsigned scat_grid = static_cast<unsigned>(std::min<uint64_t>(ntiles, uint64_t(device_cu_count()) * kScatPerCu));
  int shift = 0;
  const K *src_k = kin;
  const uint32_t *src_v = vin;
  for (int p = 0; p < passes; ++p) {
    const int bits = (key_bits - shift + (passes - p) - 1) / (passes - p);
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    K *dk = to_out ? kout : k2;
    uint32_t *dv = to_out ? vout : v2;
    const uint32_t mask = (1u << bits) - 1u;
    EIGER_LAUNCH("sort_hist", k_sort_hist<K>, dim3(hist_grid), dim3(kSNT), 0, s, src_k, n,
                 shift, mask, static_cast<uint32_t>(ntiles), cnt);
    int rc = exclusive_scan_u32(cnt, cnt, (static_cast<uint64_t>(mask) + 1) * ntiles, tmp, total, s);
    if (rc) return rc;
    EIGER_LAUNCH("sort_scatter", k_sort_scatter<K>, dim3(scat_grid), dim3(kSNT), 0, s, src_k,
                 src_v, n, shift, bits, static_cast<uint32_t>(ntiles), cnt, dk, dv);
    src_k = dk;
    src_v = dv;
    shift += bits;
  }
  return EIGER_OK;
}

}  // namespace

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
