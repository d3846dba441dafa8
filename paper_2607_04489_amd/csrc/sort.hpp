// sort.hpp -- the radix sort shared by the sort entry points and smart key fusion.
#pragma once

#include "common.hpp"

namespace eiger {

// Stable LSD radix sort of n (key, value) pairs by the low key_bits bits of the
// key (key_bytes 4 or 8). vin == nullptr sorts the row ids 0..n-1 along. Outputs
// must not alias the inputs. With ws.base == nullptr it only sizes the workspace.
int radix_sort_pairs(int key_bytes, const void *kin, const uint32_t *vin, uint64_t n, int key_bits, void *kout,
                     uint32_t *vout, Workspace &ws, hipStream_t s);

// Hash partitioning with value lanes: rows are ordered by partition id, the top
// `bits` bits of the key's partition hash (part_hash), by stable passes of the same
// sort (digits of at most 8 bits, narrower for wide rows); up to 4 32-bit lanes move along (lane w of row i is
// src[w][i * stride[w]]). out receives the partitioned keys, the lanes (stride 1)
// and off[0..2^bits] (partition p is [off[p], off[p + 1])). Always lays out
// the workspace; enqueues only with a workspace base and `run`.
struct PartLanes {
  const uint32_t *src[4];
  uint32_t stride[4];
  int n;
};
struct PartitionOut {
  const void *keys;
  const uint32_t *words[4];
  const uint32_t *off;
};
int radix_partition_lanes(int key_bytes, const void *keys, uint64_t n, const PartLanes &cols, int bits, Workspace &ws,
                          PartitionOut *out, hipStream_t s, bool run);

}  // namespace eiger
