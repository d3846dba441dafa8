// util.hip -- fills and a device-wide exclusive scan (reduce, scan of block sums, rescan).
#include "common.hpp"

namespace eiger {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;  // elements per thread
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
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

static unsigned fill_grid(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
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
