// calibrate.hip -- bandwidth ceilings for the measurement reports (diagnostics;
// not on the join path): a streaming copy with 16-byte loads and stores, and
// random 32-byte reads from a table, each timed with HIP events on the stream.
#include "common.hpp"

namespace eiger {
namespace {

__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Each thread reads `per` random 32-byte slots (8 in flight) of a table of
// `slots` slots (a power of two) and folds them into one word, written once
// per thread so the loads are kept.
__global__ void __launch_bounds__(256) k_random_reads(const uint4 *__restrict__ table, uint64_t slots, uint32_t per,
                                                     uint64_t nthreads, uint32_t *__restrict__ sink) {
  const uint64_t tid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= nthreads) return;
  const uint64_t mask = slots - 1;
  uint32_t acc = 0;
  for (uint32_t r = 0; r < per; r += 8) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint64_t s = fmix64(tid * 0x9E3779B97F4A7C15ull + r + u) & mask;
      v[u] = table[2 * s];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].w;
  }
  sink[tid] = acc;
}

}  // namespace
}  // namespace eiger

using namespace eiger;

extern "C" int eiger_calibrate(int32_t kind, void *a, void *b, int64_t n_bytes, int64_t reads, double *ms,
                               void *stream) {
  if (!ms || !a || n_bytes <= 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_calibrate: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t cus = static_cast<uint64_t>(device_cu_count());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EIGER_HIP(hipEventCreate(&e0));
  EIGER_HIP(hipEventCreate(&e1));
  int rc = EIGER_OK;
  if (kind == 0) {  // copy n_bytes (a multiple of 16) from a to b
    if (!b || n_bytes % 16) {
      rc = fail(EIGER_ERR_INVALID_ARG, "eiger_calibrate: copy needs a destination and a multiple of 16 bytes");
    } else {
      const uint64_t n = static_cast<uint64_t>(n_bytes) / 16;
      const dim3 grid(static_cast<unsigned>(cus * 16));
      (void)hipEventRecord(e0, s);
      hipLaunchKernelGGL(k_copy16, grid, dim3(256), 0, s, static_cast<const uint4 *>(a), static_cast<uint4 *>(b), n);
      (void)hipEventRecord(e1, s);
    }
  } else if (kind == 1) {  // `reads` random 32-byte reads from the table a of n_bytes; b receives one word per thread
    uint64_t slots = 1;
    while (slots * 2 * 32 <= static_cast<uint64_t>(n_bytes)) slots *= 2;
    const uint32_t per = 64;
    const uint64_t threads = (static_cast<uint64_t>(reads) + per - 1) / per;
    if (!b || reads <= 0 || threads > (uint64_t(1) << 31)) {
      rc = fail(EIGER_ERR_INVALID_ARG, "eiger_calibrate: random reads need a sink of one word per 64 reads");
    } else {
      const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
      (void)hipEventRecord(e0, s);
      hipLaunchKernelGGL(k_random_reads, grid, dim3(256), 0, s, static_cast<const uint4 *>(a), slots, per, threads,
                         static_cast<uint32_t *>(b));
      (void)hipEventRecord(e1, s);
    }
  } else {
    rc = fail(EIGER_ERR_INVALID_ARG, "eiger_calibrate: kind must be 0 (copy) or 1 (random reads)");
  }
  if (rc == EIGER_OK) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) rc = hip_fail(e, "eiger_calibrate");
    *ms = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
