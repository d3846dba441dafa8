// sort.hpp -- the radix sort shared by the sort entry points and smart key fusion.
#pragma once

#include "common.hpp"

namespace eiger {

// Stable LSD radix sort of n (key, value) pairs by the low key_bits bits of the
// key (key_bytes 4 or 8). vin == nullptr sorts the row ids 0..n-1 along. Outputs
// must not alias the inputs. With ws.base == nullptr it only sizes the workspace.
int radix_sort_pairs(int key_bytes, const void *kin, const uint32_t *vin, uint64_t n, int key_bits, void *kout,
                     uint32_t *vout, Workspace &ws, hipStream_t s);

}  // namespace eiger
