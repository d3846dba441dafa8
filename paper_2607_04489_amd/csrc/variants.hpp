// variants.hpp -- interface between the ABI layer and the join variants.
#pragma once

#include "common.hpp"

namespace eiger {

struct JoinArgs {
  const void *bk, *bp, *pk, *pp;  // build keys/payload, probe keys/payload (device)
  uint64_t nR, nS;
  int32_t kdt, bpdt, ppdt;        // eiger_dtype of keys, build payload, probe payload
  eiger_plan_t plan;
  uint32_t *ob, *op;              // outputs (device) or null in count-only mode
  uint64_t cap;
  hipStream_t s;
};

// Device words every variant leaves behind for the host to read.
struct JoinCounters {
  uint64_t count;     // pairs found (may exceed cap)
  uint64_t checksum;  // sum of payload products mod 2^64
  uint64_t flags;     // kFlag* bits
  uint64_t pad;
};

constexpr uint64_t kFlagBuildOutOfRange = 1;  // DIRECT: a build key outside [build_min, build_max]

// Each variant lays out its buffers in `ws` (sizing only when ws.base is null)
// and, when not sizing, enqueues its kernels on a.s. `ctr` points into ws and
// must be zeroed by the variant before use.
int run_direct(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);
int run_global_hash(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);
int run_radix(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);
int run_radix_cache(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);
int run_sort_merge(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);

// Wide joins: payload columns as 32-bit word lanes (an 8-byte column is two
// lanes, low word then high word, each with stride 2).
constexpr int kMaxWords = 8;
struct WordCols {
  const uint32_t *src[kMaxWords];
  uint32_t stride[kMaxWords];
  int n;
};
// Where a wide join's materialization reads from: the partitioned row ids and
// word arrays of one side (GFTR), filled in by run_radix_wide.
struct WideSource {
  const uint32_t *rows;
  const uint32_t *words[kMaxWords];
};
// RADIX join of the keys in a (payloads ignored) carrying the word lanes of
// both sides through the partitioning (GFTR); the output pairs are positions
// in the final partitioned arrays, described by *outR / *outS.
int run_radix_wide(const JoinArgs &a, const WordCols &colsR, const WordCols &colsS, Workspace &ws, JoinCounters **ctr,
                   WideSource *outR, WideSource *outS);
// Dispatch of eiger_join's variants (abi.hip).
int run_join_variant(const JoinArgs &a, Workspace &ws, JoinCounters **ctr);

// Largest key range the DIRECT variant accepts (its offset table is 4 B per key value).
constexpr uint64_t kDirectMaxRange = uint64_t(1) << 30;

// Slots of a global hash table for n build rows at load factor lf (power of two).
uint64_t hash_slots(uint64_t n, float lf);

// RADIX join configuration (LDS budget of the per-partition tables).
struct RadixLimits {
  uint32_t max_slots;   // LDS table slots for this key/payload width
  uint32_t max_build;   // build rows one LDS table holds at load factor lf
};
RadixLimits radix_limits(int32_t kdt, int32_t bpdt, float lf);

// RADIX_CACHE: largest partition-bit count of its single partitioning pass.
constexpr int kCacheMaxBits = 10;
// Bytes of one slot of the device-memory hash tables (GLOBAL_HASH, RADIX_CACHE).
inline size_t slot_bytes(int32_t kdt, int32_t bpdt) {
  return (dtype_size(kdt) + dtype_size(bpdt) + 4 <= 16) ? 16 : 32;
}

// Learned selector (selector.hip).
void selector_features(const eiger_stats_t &b, const eiger_stats_t &p, float *out);
int class_plan(int32_t cls, const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out);
// Sets *in_domain = false (and leaves *out alone) when the features lie
// outside the installed model's training box.
int learned_plan(const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out, bool *in_domain);

}  // namespace eiger
