// util.hip -- fills and a device-wide exclusive scan (reduce, scan of block sums, rescan).
#include "common.hpp"

namespace eiger {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;  // elements per thread
constexpr int kScanTile = kScanThreads * kScanItems;

// Fills: each workgroup stores one contiguous chunk of the 16-byte-aligned
// body with 16-byte stores (a stand-alone 2 GiB fill ran at 5.8 TB/s this way,
// 5.5 with 4-byte grid-stride stores and 4.0 with 16-byte grid-stride stores);
// the unaligned head and the tail take single words.
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t head = min(n, static_cast<uint64_t>((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4);
  const uint64_t nv = (n - head) / 4, done = head + nv * 4;
  if (blockIdx.x == 0) {
    if (threadIdx.x < head) p[threadIdx.x] = v;
    if (threadIdx.x < n - done) p[done + threadIdx.x] = v;
  }
  uint4 *__restrict__ q = reinterpret_cast<uint4 *>(p + head);
  const uint4 vv = make_uint4(v, v, v, v);
  const uint64_t per = (nv + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = uint64_t(blockIdx.x) * per, hi = min(nv, lo + per);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) q[i] = vv;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t head = min(n, static_cast<uint64_t>((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 8);
  const uint64_t nv = (n - head) / 2, done = head + nv * 2;
  if (blockIdx.x == 0) {
    if (threadIdx.x < head) p[threadIdx.x] = v;
    if (threadIdx.x < n - done) p[done + threadIdx.x] = v;
  }
  ulonglong2 *__restrict__ q = reinterpret_cast<ulonglong2 *>(p + head);
  const ulonglong2 vv = make_ulonglong2(v, v);
  const uint64_t per = (nv + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = uint64_t(blockIdx.x) * per, hi = min(nv, lo + per);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) q[i] = vv;
}

// Phase 1: sum of each tile of kScanTile counts.
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *__restrict__ in,
                                                              uint64_t n,
                                                              uint64_t *__restrict__ tile_sums) {
  __shared__ uint64_t red[kScanThreads / 64];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    uint64_t i = base + uint64_t(k) * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum_u64<kScanThreads>(s, red);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = s;
}

// Phase 2: one workgroup turns tile sums into exclusive tile offsets (in place)
// and writes the grand total.
__global__ void __launch_bounds__(1024) k_scan_tiles(uint64_t *__restrict__ tile_sums,
                                                     uint64_t ntiles,
                                                     uint64_t *__restrict__ total) {
  __shared__ uint64_t part[1024];
  const uint64_t per = (ntiles + 1023) / 1024;
  const uint64_t lo = threadIdx.x * per;
  const uint64_t hi = lo + per < ntiles ? lo + per : ntiles;
  uint64_t s = 0;
  for (uint64_t i = lo; i < hi; ++i) s += tile_sums[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (int t = 0; t < 1024; ++t) {
      uint64_t v = part[t];
      part[t] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  uint64_t run = part[threadIdx.x];
  for (uint64_t i = lo; i < hi; ++i) {
    uint64_t v = tile_sums[i];
    tile_sums[i] = run;
    run += v;
  }
}

// Phase 3: exclusive scan inside each tile, offset by the tile's prefix.
// Each thread owns kScanItems consecutive elements.
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const uint32_t *in, uint32_t *out,
                                                            uint64_t n,
                                                            const uint64_t *__restrict__ tile_off) {
  __shared__ uint32_t scratch[kScanThreads / 64 + 1];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan<kScanThreads>(s, scratch, &total) +
                 static_cast<uint32_t>(tile_off[blockIdx.x]);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

}  // namespace

static unsigned fill_grid(uint64_t n) {  // n words; up to 1024 chunks of >= 4 KiB
  uint64_t g = (n + 1023) / 1024;
  if (g > 1024) g = 1024;
  return static_cast<unsigned>(g ? g : 1);
}

int fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return EIGER_OK;
  EIGER_LAUNCH("fill_u32", k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  return EIGER_OK;
}

int fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return EIGER_OK;
  EIGER_LAUNCH("fill_u64", k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  return EIGER_OK;
}

size_t scan_tmp_elems(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

int exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint64_t *tmp,
                       uint64_t *total_dev, hipStream_t s) {
  const uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles == 0) return fill_u64(total_dev, 1, 0, s);
  EIGER_LAUNCH("scan_reduce", k_scan_reduce, dim3(unsigned(ntiles)), dim3(kScanThreads), 0, s, in,
               n, tmp);
  EIGER_LAUNCH("scan_tiles", k_scan_tiles, dim3(1), dim3(1024), 0, s, tmp, ntiles, total_dev);
  EIGER_LAUNCH("scan_down", k_scan_down, dim3(unsigned(ntiles)), dim3(kScanThreads), 0, s, in, out,
               n, tmp);
  return EIGER_OK;
}

}  // namespace eiger
