// common.hpp -- shared device helpers and host plumbing of the gfx950 join library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "eiger.h"

namespace eiger {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // empty-slot marker in every table's row-id field
constexpr int kHllP = EIGER_HLL_P;
constexpr int kHllM = 1 << kHllP;

// ---------------------------------------------------------------- device math

// MurmurHash3 64-bit finalizer (Appleby): the key hash of the sketch registers,
// of hash-table slots and of radix partition ids of 8-byte keys.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

template <typename T>
__device__ __forceinline__ int64_t sext(T v) {
  return static_cast<int64_t>(v);
}

// Partition hash: radix partitions are the top bits of this value. 8-byte keys
// take fmix64; 4-byte keys the 32-bit MurmurHash3 finalizer (Appleby) in the
// upper half, a third of the instructions for the same top-bit mixing.
template <typename K>
__device__ __forceinline__ uint64_t part_hash(K key) {
  if constexpr (sizeof(K) == 4) {
    uint32_t h = static_cast<uint32_t>(key);
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return static_cast<uint64_t>(h) << 32;
  } else {
    return fmix64(static_cast<uint64_t>(sext(key)));
  }
}

// Lane-level exclusive prefix of a 64-lane mask: number of set bits below this lane.
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Inclusive wave64 scan with shuffles (T = uint32_t or uint64_t).
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    int64_t t = __shfl_xor(v, d, 64);
    v = t < v ? t : v;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    int64_t t = __shfl_xor(v, d, 64);
    v = t > v ? t : v;
  }
  return v;
}

// Exclusive scan over a workgroup of NT threads (T = uint32_t or uint64_t).
// `scratch` must hold NT/64 + 1 values of T in LDS. Returns this thread's
// exclusive prefix; *total gets the sum. Contains __syncthreads(): every
// thread of the workgroup must call it.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *scratch, T *total) {
  constexpr int NW = NT / 64;
  const int lane = __lane_id();
  const int wave = threadIdx.x / 64;
  T inc = wave_inclusive_scan<T>(v);
  if (lane == 63) scratch[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < NW; ++w) {
      T t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[NW] = run;
  }
  __syncthreads();
  T r = scratch[wave] + inc - v;
  *total = scratch[NW];
  __syncthreads();
  return r;
}

// Sum of a u64 over a workgroup (result valid in thread 0). `scratch` holds NT/64 u64.
template <int NT>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *scratch) {
  constexpr int NW = NT / 64;
  v = wave_sum_u64(v);
  if (__lane_id() == 0) scratch[threadIdx.x / 64] = v;
  __syncthreads();
  uint64_t s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) s += scratch[w];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- host plumbing

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Per-kernel event timing (enabled by eiger_profile_enable).
struct ProfScope {
  ProfScope(const char *name, hipStream_t s);
  ~ProfScope();
  const char *name_;
  hipStream_t stream_;
  hipEvent_t start_ = nullptr;
};

int device_cu_count();

#define EIGER_HIP(call)                                   \
  do {                                                    \
    hipError_t _e = (call);                               \
    if (_e != hipSuccess) return ::eiger::hip_fail(_e, #call); \
  } while (0)

#define EIGER_LAUNCH(name, kernel, grid, block, shmem, stream, ...)          \
  do {                                                                       \
    ::eiger::ProfScope _ps(name, stream);                                    \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);     \
    hipError_t _e = hipGetLastError();                                       \
    if (_e != hipSuccess) return ::eiger::hip_fail(_e, name);                \
  } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only sizes.
struct Workspace {
  char *base;
  size_t cap;
  size_t used = 0;
  Workspace(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
  template <typename T>
  T *take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

inline size_t dtype_size(int32_t dt) { return dt == EIGER_INT64 ? 8 : 4; }

// ---- internal launchers shared across translation units -----------------
int fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
int fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
// Exclusive scan of n u32 counts into out (may alias in), writing the total to
// *total_dev (device u64). tmp needs scan_tmp_elems(n) u64.
size_t scan_tmp_elems(uint64_t n);
int exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint64_t *tmp,
                       uint64_t *total_dev, hipStream_t s);

}  // namespace eiger
