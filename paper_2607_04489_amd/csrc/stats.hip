// stats.hip -- one pass over a key column: count, min, max and HLL registers.
//
// Section 4 of the paper: min/max (and mean) of intermediate data at close to
// memory bandwidth; Section 4.1: an HLL++ sketch for the distinct count.
// Each workgroup keeps a private copy of the 2^14 registers in LDS (one u32 per
// register, updated with LDS atomic max after a plain read filters out the
// common no-change case), then writes it out packed four to a word; a second
// small kernel takes the byte-wise max over the workgroups.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace eiger {

namespace {

constexpr int kStatsThreads = 512;
constexpr int kStatsUnroll = 4;  // 16-byte loads in flight per thread and iteration
constexpr int kWords = kHllM / 4;

template <typename K>
struct Vec16;
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef int64_t v2i64 __attribute__((ext_vector_type(2)));
template <>
struct Vec16<int32_t> {
  using T = v4i32;
  static constexpr int N = 4;
  __device__ static int64_t get(const T &v, int k) { return v[k]; }
};
template <>
struct Vec16<int64_t> {
  using T = v2i64;
  static constexpr int N = 2;
  __device__ static int64_t get(const T &v, int k) { return v[k]; }
};

struct StatsLane {
  int64_t mn = INT64_MAX;
  int64_t mx = INT64_MIN;
  __device__ __forceinline__ void visit(int64_t x, uint32_t *regs) {
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
    const uint64_t h = fmix64(static_cast<uint64_t>(x));
    const uint32_t idx = static_cast<uint32_t>(h >> (64 - kHllP));
    const uint64_t w = h << kHllP;
    const uint32_t rank = w ? static_cast<uint32_t>(__clzll(w)) + 1u : uint32_t(64 - kHllP + 1);
    if (rank > regs[idx]) atomicMax(&regs[idx], rank);
  }
};

template <typename K>
__global__ void __launch_bounds__(kStatsThreads)
    k_stats_partial(const K *__restrict__ keys, uint64_t n, uint32_t *__restrict__ part_regs,
                    int64_t *__restrict__ part_mm) {
  __shared__ uint32_t regs[kHllM];
  __shared__ int64_t red[2][kStatsThreads / 64];
  for (int i = threadIdx.x; i < kHllM; i += kStatsThreads) regs[i] = 0;
  __syncthreads();

  using V = Vec16<K>;
  StatsLane lane;
  const uint64_t gtid = uint64_t(blockIdx.x) * kStatsThreads + threadIdx.x;
  const uint64_t stride = uint64_t(gridDim.x) * kStatsThreads;
  // scalar head up to the first 16-byte boundary, then 16-byte vectors
  uint64_t head = ((16 - (reinterpret_cast<uintptr_t>(keys) & 15)) & 15) / sizeof(K);
  if (head > n) head = n;
  if (gtid < head) lane.visit(sext(keys[gtid]), regs);
  keys += head;
  n -= head;
  const uint64_t nvec = n / V::N;
  const typename V::T *vk = reinterpret_cast<const typename V::T *>(keys);
  uint64_t v = gtid;
  for (; v + (kStatsUnroll - 1) * stride < nvec; v += kStatsUnroll * stride) {
    typename V::T buf[kStatsUnroll];
#pragma unroll
    for (int u = 0; u < kStatsUnroll; ++u) buf[u] = __builtin_nontemporal_load(&vk[v + u * stride]);
#pragma unroll
    for (int u = 0; u < kStatsUnroll; ++u)
#pragma unroll
      for (int k = 0; k < V::N; ++k) lane.visit(V::get(buf[u], k), regs);
  }
  for (; v < nvec; v += stride) {
    typename V::T b = __builtin_nontemporal_load(&vk[v]);
#pragma unroll
    for (int k = 0; k < V::N; ++k) lane.visit(V::get(b, k), regs);
  }
  for (uint64_t i = nvec * V::N + gtid; i < n; i += stride) lane.visit(sext(keys[i]), regs);

  int64_t mn = wave_min_i64(lane.mn), mx = wave_max_i64(lane.mx);
  const int wave = threadIdx.x / 64;
  if (__lane_id() == 0) {
    red[0][wave] = mn;
    red[1][wave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kStatsThreads / 64; ++w) {
      mn = red[0][w] < mn ? red[0][w] : mn;
      mx = red[1][w] > mx ? red[1][w] : mx;
    }
    part_mm[2 * blockIdx.x] = mn;
    part_mm[2 * blockIdx.x + 1] = mx;
  }
  uint32_t *out = part_regs + uint64_t(blockIdx.x) * kWords;
  for (int i = threadIdx.x; i < kWords; i += kStatsThreads)
    out[i] = regs[4 * i] | (regs[4 * i + 1] << 8) | (regs[4 * i + 2] << 16) | (regs[4 * i + 3] << 24);
}

__device__ __forceinline__ uint32_t bytewise_max(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    uint32_t x = (a >> k) & 255u, y = (b >> k) & 255u;
    r |= (x > y ? x : y) << k;
  }
  return r;
}

// Registers are merged by byte-wise max. Above 2 * kSlices workgroups this
// takes two stages, so that many loads are in flight: stage 1 reduces slice y
// of the per-workgroup register arrays (groups g = y, y + kSlices, ...) for 256
// words per block; stage 2 merges the slices and, in block 0, the
// per-workgroup min/max. (One thread per word over all workgroups took ~0.12 ms
// for 512 workgroups; two stages take ~0.016 ms.)
constexpr int kSlices = 16;

__global__ void __launch_bounds__(256) k_stats_merge(const uint32_t *__restrict__ part_regs, int groups,
                                                     uint32_t *__restrict__ slice_regs) {
  const int word = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  uint32_t r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int g = y;
  for (; g + 7 * kSlices < groups; g += 8 * kSlices) {
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = bytewise_max(r[u], part_regs[uint64_t(g + u * kSlices) * kWords + word]);
  }
  for (; g < groups; g += kSlices) r[0] = bytewise_max(r[0], part_regs[uint64_t(g) * kWords + word]);
#pragma unroll
  for (int u = 1; u < 8; ++u) r[0] = bytewise_max(r[0], r[u]);
  slice_regs[uint64_t(y) * kWords + word] = r[0];
}

__global__ void __launch_bounds__(256) k_stats_final(const uint32_t *__restrict__ slice_regs, int slices,
                                                     uint32_t *__restrict__ regs_out,
                                                     const int64_t *__restrict__ part_mm, int groups,
                                                     int64_t *__restrict__ mm_out) {
  const int word = blockIdx.x * 256 + threadIdx.x;
  uint32_t r = 0;
  for (int y = 0; y < slices; ++y) r = bytewise_max(r, slice_regs[uint64_t(y) * kWords + word]);
  regs_out[word] = r;
  if (blockIdx.x == 0) {
    __shared__ int64_t red[2][4];
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int g = threadIdx.x; g < groups; g += 256) {
      int64_t a = part_mm[2 * g], b = part_mm[2 * g + 1];
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    mn = wave_min_i64(mn);
    mx = wave_max_i64(mx);
    if (__lane_id() == 0) {
      red[0][threadIdx.x / 64] = mn;
      red[1][threadIdx.x / 64] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w) {
        mn = red[0][w] < mn ? red[0][w] : mn;
        mx = red[1][w] > mx ? red[1][w] : mx;
      }
      mm_out[0] = mn;
      mm_out[1] = mx;
    }
  }
}

int stats_groups(int64_t n, int32_t dtype) {
  const int64_t per_group = int64_t(kStatsThreads) * (16 / dtype_size(dtype)) * kStatsUnroll * 4;
  int64_t g = (n + per_group - 1) / per_group;
  const int64_t cap = int64_t(device_cu_count()) * 2;  // 64 KiB LDS each: two per CU
  if (g > cap) g = cap;
  return static_cast<int>(g < 1 ? 1 : g);
}

struct StatsLayout {
  uint32_t *part_regs;
  uint32_t *slice_regs;
  int64_t *part_mm;
  uint32_t *regs;
  int64_t *mm;
};

StatsLayout stats_layout(Workspace &ws, int groups) {
  StatsLayout L;
  L.part_regs = ws.take<uint32_t>(size_t(groups) * kWords);
  L.slice_regs = ws.take<uint32_t>(size_t(kSlices) * kWords);
  L.part_mm = ws.take<int64_t>(size_t(groups) * 2);
  L.regs = ws.take<uint32_t>(kWords);
  L.mm = ws.take<int64_t>(2);
  return L;
}

// sigma(x) = x + sum_{k>=1} x^(2^k) 2^(k-1)
double ertl_sigma(double x) {
  if (x == 1.0) return INFINITY;
  double z = x, y = 1.0;
  for (;;) {
    x *= x;
    const double z_old = z;
    z += x * y;
    y += y;
    if (z == z_old) return z;
  }
}

// tau(x) = (1 - x - sum_{k>=1} (1 - x^(2^-k))^2 2^-k) / 3
double ertl_tau(double x) {
  if (x == 0.0 || x == 1.0) return 0.0;
  double z = 1.0 - x, y = 1.0;
  for (;;) {
    x = std::sqrt(x);
    const double z_old = z;
    y *= 0.5;
    z -= (1.0 - x) * (1.0 - x) * y;
    if (z == z_old) return z / 3.0;
  }
}

}  // namespace

// Distinct-count estimate from dense registers: O. Ertl's table-free improved
// estimator, alpha_inf m^2 / (m sigma(C0/m) + sum_k C_k 2^-k + m tau(1 - C_{q+1}/m) 2^-q).
double hll_estimate(const uint8_t *regs) {
  constexpr int q = 64 - kHllP;
  int64_t c[q + 2] = {0};
  for (int j = 0; j < kHllM; ++j) c[regs[j]]++;
  const double m = kHllM;
  if (c[0] == kHllM) return 0.0;
  double z = m * ertl_tau(1.0 - double(c[q + 1]) / m);
  for (int k = q; k >= 1; --k) z = 0.5 * (z + double(c[k]));
  z += m * ertl_sigma(double(c[0]) / m);
  return m * m / (2.0 * std::log(2.0)) / z;
}

}  // namespace eiger

using namespace eiger;

extern "C" size_t eiger_stats_workspace_size(int64_t n, int32_t dtype) {
  if (n < 0 || (dtype != EIGER_INT32 && dtype != EIGER_INT64)) return 0;
  Workspace ws(nullptr, 0);
  stats_layout(ws, stats_groups(n, dtype));
  return ws.used;
}

extern "C" int eiger_stats(eiger_column keys, eiger_stats_t *out, uint8_t *hll_regs_host, void *ws_ptr,
                           size_t ws_bytes, void *stream) {
  if (!out) return fail(EIGER_ERR_INVALID_ARG, "eiger_stats: out is NULL");
  if (keys.dtype != EIGER_INT32 && keys.dtype != EIGER_INT64)
    return fail(EIGER_ERR_DTYPE, "eiger_stats: key dtype must be EIGER_INT32 or EIGER_INT64");
  if (keys.n < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_stats: negative row count");
  if (keys.n > EIGER_MAX_ROWS)
    return fail(EIGER_ERR_TOO_LARGE, "eiger_stats: more than EIGER_MAX_ROWS = 2^32 - 2^16 rows");
  if (keys.n > 0 && !keys.data) return fail(EIGER_ERR_INVALID_ARG, "eiger_stats: keys.data is NULL");
  if (keys.n > 0 && (reinterpret_cast<uintptr_t>(keys.data) % dtype_size(keys.dtype)) != 0)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_stats: keys.data is not aligned to its dtype");
  *out = eiger_stats_t{};
  out->dtype = keys.dtype;
  out->hll_p = kHllP;
  if (keys.n == 0) {
    out->flags = EIGER_STATS_EMPTY;
    if (hll_regs_host) std::memset(hll_regs_host, 0, kHllM);
    return EIGER_OK;
  }
  const int groups = stats_groups(keys.n, keys.dtype);
  Workspace ws(ws_ptr, ws_bytes);
  StatsLayout L = stats_layout(ws, groups);
  if (!ws_ptr || ws.used > ws_bytes)
    return fail(EIGER_ERR_WORKSPACE, "eiger_stats: workspace too small (need " +
                                         std::to_string(ws.used) + " bytes)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (keys.dtype == EIGER_INT32) {
    EIGER_LAUNCH("stats_partial", k_stats_partial<int32_t>, dim3(groups), dim3(kStatsThreads), 0, s,
                 static_cast<const int32_t *>(keys.data), uint64_t(keys.n), L.part_regs, L.part_mm);
  } else {
    EIGER_LAUNCH("stats_partial", k_stats_partial<int64_t>, dim3(groups), dim3(kStatsThreads), 0, s,
                 static_cast<const int64_t *>(keys.data), uint64_t(keys.n), L.part_regs, L.part_mm);
  }
  if (groups <= 2 * kSlices) {  // few workgroups: one merge launch over them all
    EIGER_LAUNCH("stats_final", k_stats_final, dim3(kWords / 256), dim3(256), 0, s, L.part_regs, groups, L.regs,
                 L.part_mm, groups, L.mm);
  } else {
    EIGER_LAUNCH("stats_final", k_stats_merge, dim3(kWords / 256, kSlices), dim3(256), 0, s, L.part_regs,
                 groups, L.slice_regs);
    EIGER_LAUNCH("stats_final", k_stats_final, dim3(kWords / 256), dim3(256), 0, s, L.slice_regs, kSlices,
                 L.regs, L.part_mm, groups, L.mm);
  }
  std::vector<uint8_t> regs(kHllM);
  int64_t mm[2];
  EIGER_HIP(hipMemcpyAsync(regs.data(), L.regs, kHllM, hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipMemcpyAsync(mm, L.mm, sizeof(mm), hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipStreamSynchronize(s));
  out->n = keys.n;
  out->min = mm[0];
  out->max = mm[1];
  out->ndv = hll_estimate(regs.data());
  if (hll_regs_host) std::memcpy(hll_regs_host, regs.data(), kHllM);
  return EIGER_OK;
}
