// skf.hip -- smart key fusion (Section 4.3) and the order-preserving dictionary
// encoding it uses (Algorithm 1).
//
// Dictionary encoding, per key column (one relation, or two read as one column):
//   1. insert: every row inserts its key into an open-addressing table (CAS on an
//      empty slot; the winner is the value's leader) and records its slot id;
//   2. retrieve: the occupied slots are compacted into (value - min, slot) pairs,
//      and their number is the exact distinct count;
//   3. the pairs are radix-sorted by value (width of max - min);
//   4. scatter: the slot of the i-th smallest value receives code i;
//   5. gather: each row reads the code of its slot -- done inside the fusion
//      kernel, so codes are never stored on their own.
// The slot id plays the role of the leader's row id as group id: it indexes an
// array of table size instead of one of column size, which stays in L2.
//
// Fusion: one kernel reads every key column (frame-of-reference keys) or slot
// ids (dictionary keys) of a row, forms each code, complements it within its
// width for a descending key, and ORs it into place: 4- or 8-byte output.
#include <cmath>

#include "common.hpp"
#include "sort.hpp"

namespace eiger {

namespace {

// INT64_MIN marks empty slots; rows holding that key use the extra slot `slots`.
constexpr unsigned long long kDeEmpty = 0x8000000000000000ull;
constexpr int kDeNT = 256;
// Longest probe sequence an insert walks before it reports overflow: far beyond
// what a table at most half full needs, and it bounds the work when the
// distinct estimate was much too low (the caller then retries with more slots).
constexpr uint64_t kDeMaxProbe = 2048;

struct DeTable {
  unsigned long long *key;  // slots entries
  uint64_t mask;            // slots - 1
  uint32_t *ctr;            // [0] distinct count, [1] INT64_MIN present, [2] overflow
};

// One logical column over the rows of one or two relations.
template <typename K>
struct Rows {
  const K *a;
  const K *b;
  uint64_t na, n;
  __device__ __forceinline__ const K *at(uint64_t i) const { return i < na ? a + i : b + (i - na); }
};

// Rows a fusion thread handles together: all their loads are issued before any
// result is used, so each thread keeps several memory accesses in flight.
constexpr int kDeBatch = 8;

// Step 1 for one value: its slot in the global table (claimed if new). The
// value kDeEmpty (INT64_MIN) has the extra slot mask + 1; a full walk gives
// mask + 2 and raises the overflow flag.
__device__ __forceinline__ uint64_t de_slot(const DeTable &t, unsigned long long k) {
  if (k == kDeEmpty) {
    t.ctr[1] = 1u;
    return t.mask + 1;
  }
  uint64_t h = fmix64(k) & t.mask;
  const uint64_t limit = t.mask < kDeMaxProbe ? t.mask + 1 : kDeMaxProbe;
  for (uint64_t probe = 0; probe < limit; ++probe) {
    unsigned long long cur = t.key[h];
    if (cur == kDeEmpty) cur = atomicCAS(&t.key[h], kDeEmpty, k);
    if (cur == kDeEmpty || cur == k) return h;
    h = (h + 1) & t.mask;
  }
  t.ctr[2] = 1u;
  return t.mask + 2;
}

// One row per thread and step: a batched form (all rows' first table reads in
// flight before any is resolved) measured slower on a hot, L2-resident table.
template <typename K>
__global__ void __launch_bounds__(kDeNT) k_de_insert(Rows<K> rows, DeTable t, uint32_t *__restrict__ loc) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDeNT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kDeNT + threadIdx.x; i < rows.n; i += stride) {
    const unsigned long long k = static_cast<unsigned long long>(static_cast<int64_t>(*rows.at(i)));
    loc[i] = static_cast<uint32_t>(de_slot(t, k));
  }
}

// Step 1 for tables of few distinct values: each workgroup keeps the distinct
// values it has met, with their global slots, in an LDS table for all of its
// chunks of kDeNT * kDeLdsRows rows. A chunk first enters its rows' values into
// the LDS table, then the values new to the workgroup are claimed in the
// global table (one walk per value and workgroup, not per row), then every row
// takes its value's slot from LDS. A value that finds no LDS slot within
// kDeLdsProbe steps takes the global walk itself, as does INT64_MIN. The
// global table has at most kDeLdsMaxTable slots, so at most half as many
// distinct values: the LDS table stays at most half full.
constexpr uint32_t kDeLdsSlots = 4096;
constexpr int kDeLdsRows = 16;
constexpr uint32_t kDeLdsProbe = 64;
constexpr uint32_t kDeLdsNone = 0xFFFFFFFFu;
constexpr uint64_t kDeLdsMaxTable = 4096;  // global tables up to this many slots use it
constexpr int kDeLdsPerCu = 3;             // 48 KB of LDS per workgroup

// kVec: 4-byte keys from one 16-byte aligned array (and a 16-byte aligned loc):
// each thread loads and stores four consecutive rows at once.
template <typename K, bool kVec>
__global__ void __launch_bounds__(kDeNT) k_de_insert_lds(Rows<K> rows, DeTable t, uint32_t *__restrict__ loc) {
  __shared__ unsigned long long lk[kDeLdsSlots];
  __shared__ uint32_t lg[kDeLdsSlots];
  constexpr uint64_t C = static_cast<uint64_t>(kDeNT) * kDeLdsRows;
  const uint64_t nch = (rows.n + C - 1) / C;
  for (uint32_t j = threadIdx.x; j < kDeLdsSlots; j += kDeNT) {
    lk[j] = kDeEmpty;
    lg[j] = kDeLdsNone;
  }
  __syncthreads();
  for (uint64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    // row r of this thread: kVec groups of four consecutive rows, else rows
    // kDeNT apart
    auto row = [&](int r) -> uint64_t {
      if constexpr (kVec)
        return ch * C + (static_cast<uint64_t>(r / 4) * kDeNT + threadIdx.x) * 4 + (r % 4);
      else
        return ch * C + threadIdx.x + static_cast<uint64_t>(r) * kDeNT;
    };
    unsigned long long key[kDeLdsRows];
    uint32_t li[kDeLdsRows];
    if constexpr (kVec) {
#pragma unroll
      for (int q = 0; q < kDeLdsRows; q += 4) {
        const uint64_t i = row(q);
        if (i + 3 < rows.n) {
          const int4 v = *reinterpret_cast<const int4 *>(rows.a + i);
          key[q] = static_cast<unsigned long long>(static_cast<int64_t>(v.x));
          key[q + 1] = static_cast<unsigned long long>(static_cast<int64_t>(v.y));
          key[q + 2] = static_cast<unsigned long long>(static_cast<int64_t>(v.z));
          key[q + 3] = static_cast<unsigned long long>(static_cast<int64_t>(v.w));
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            key[q + u] = i + u < rows.n ? static_cast<unsigned long long>(static_cast<int64_t>(rows.a[i + u])) : kDeEmpty;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < kDeLdsRows; ++r) {
        const uint64_t i = row(r);
        key[r] = i < rows.n ? static_cast<unsigned long long>(static_cast<int64_t>(*rows.at(i))) : kDeEmpty;
      }
    }
#pragma unroll
    for (int r = 0; r < kDeLdsRows; ++r) {
      li[r] = kDeLdsNone;
      if (key[r] == kDeEmpty) continue;
      uint32_t h = static_cast<uint32_t>(fmix64(key[r])) & (kDeLdsSlots - 1);
      for (uint32_t probe = 0; probe < kDeLdsProbe; ++probe) {
        unsigned long long cur = lk[h];
        if (cur == kDeEmpty) cur = atomicCAS(&lk[h], kDeEmpty, key[r]);
        if (cur == kDeEmpty || cur == key[r]) {
          li[r] = h;
          break;
        }
        h = (h + 1) & (kDeLdsSlots - 1);
      }
    }
    __syncthreads();
    // values new to this workgroup: claim them in the global table
    for (uint32_t j = threadIdx.x; j < kDeLdsSlots; j += kDeNT) {
      if (lg[j] != kDeLdsNone) continue;
      const unsigned long long k = lk[j];
      if (k != kDeEmpty) lg[j] = static_cast<uint32_t>(de_slot(t, k));
    }
    __syncthreads();
    // (the next chunk only claims empty LDS slots and fills their lg entries,
    // which no row of this chunk reads, so no barrier follows)
    uint32_t out[kDeLdsRows];
#pragma unroll
    for (int r = 0; r < kDeLdsRows; ++r)
      out[r] = li[r] != kDeLdsNone ? lg[li[r]] : (row(r) < rows.n ? static_cast<uint32_t>(de_slot(t, key[r])) : 0u);
    if constexpr (kVec) {
#pragma unroll
      for (int q = 0; q < kDeLdsRows; q += 4) {
        const uint64_t i = row(q);
        if (i + 3 < rows.n) {
          *reinterpret_cast<uint4 *>(loc + i) = make_uint4(out[q], out[q + 1], out[q + 2], out[q + 3]);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (i + u < rows.n) loc[i + u] = out[q + u];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < kDeLdsRows; ++r) {
        const uint64_t i = row(r);
        if (i < rows.n) loc[i] = out[r];
      }
    }
  }
}

// Compacts occupied slots into (key - base, slot) pairs; one atomic per wave.
__global__ void __launch_bounds__(kDeNT) k_de_retrieve(DeTable t, uint64_t base, unsigned long long *__restrict__ ukey,
                                                       uint32_t *__restrict__ uslot) {
  const uint64_t slots = t.mask + 1;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDeNT;
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * kDeNT + threadIdx.x;
  // every lane of a wave runs the same number of iterations (ballots below)
  const uint64_t wave0 = first - __lane_id();
  for (uint64_t i0 = wave0; i0 < slots; i0 += stride) {
    const uint64_t i = i0 + __lane_id();
    const unsigned long long k = i < slots ? t.key[i] : kDeEmpty;
    const bool occ = k != kDeEmpty;
    const uint64_t m = __ballot(occ);
    uint32_t at = 0;
    if (__lane_id() == 0 && m) at = atomicAdd(&t.ctr[0], static_cast<uint32_t>(__popcll(m)));
    at = __shfl(at, 0, 64) + lane_prefix(m);
    if (occ) {
      ukey[at] = k - base;
      uslot[at] = static_cast<uint32_t>(i);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && t.ctr[1]) {
    const uint32_t at = atomicAdd(&t.ctr[0], 1u);
    ukey[at] = kDeEmpty - base;
    uslot[at] = static_cast<uint32_t>(slots);
  }
}

// Step 4: the slot of the i-th smallest distinct value gets code i.
__global__ void __launch_bounds__(kDeNT) k_de_scatter(const uint32_t *__restrict__ sorted_slot, uint64_t ndv,
                                                      uint32_t *__restrict__ code_of_slot) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kDeNT + threadIdx.x;
  if (i < ndv) code_of_slot[sorted_slot[i]] = static_cast<uint32_t>(i);
}

// Step 5 for the stand-alone encoding, and the dictionary itself.
__global__ void __launch_bounds__(kDeNT) k_de_gather(const uint32_t *__restrict__ loc, uint64_t n,
                                                     const uint32_t *__restrict__ code_of_slot,
                                                     uint32_t *__restrict__ codes) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDeNT;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kDeNT + threadIdx.x; i < n; i += stride)
    codes[i] = code_of_slot[loc[i]];
}

template <typename K>
__global__ void __launch_bounds__(kDeNT) k_de_dict(const unsigned long long *__restrict__ sorted_key, uint64_t ndv,
                                                   uint64_t base, K *__restrict__ dict) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kDeNT + threadIdx.x;
  if (i < ndv) dict[i] = static_cast<K>(static_cast<int64_t>(sorted_key[i] + base));
}

struct FuseKey {
  const void *a;
  const void *b;
  const uint32_t *loc;           // DICT: slot of each row
  const uint32_t *code_of_slot;  // DICT: code of each slot
  uint64_t base;                 // FOR: minimum (two's-complement bits)
  uint64_t flip;                 // all-ones over the width for a descending key, else 0
  int32_t wide;                  // 8-byte key column
  int32_t dict;
  uint32_t slots1;               // DICT: entries of code_of_slot (table slots + 1)
  int32_t bits;
  int32_t shift;
};

struct FuseArgs {
  FuseKey k[EIGER_SKF_MAX_KEYS];
  int32_t nk;
  uint64_t na, n;
  void *out_a;
  void *out_b;
};

template <typename F>
__global__ void __launch_bounds__(kDeNT) k_skf_fuse(FuseArgs A) {
  constexpr uint64_t span = uint64_t(kDeNT) * kDeBatch;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * span;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * span + threadIdx.x; base < A.n;
       base += stride) {
    F f[kDeBatch];
#pragma unroll
    for (int b = 0; b < kDeBatch; ++b) f[b] = 0;
    for (int c = 0; c < A.nk; ++c) {
      const FuseKey &k = A.k[c];
      if (k.bits == 0) continue;
      uint64_t code[kDeBatch];
      if (k.dict) {
        uint32_t sl[kDeBatch];
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) {
          const uint64_t i = base + uint64_t(b) * kDeNT;
          sl[b] = i < A.n ? k.loc[i] : 0u;
        }
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) {
          const uint64_t i = base + uint64_t(b) * kDeNT;
          code[b] = i < A.n ? k.code_of_slot[sl[b]] : 0u;
        }
      } else if (k.wide) {
        int64_t v[kDeBatch];
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) {
          const uint64_t i = base + uint64_t(b) * kDeNT;
          if (i < A.n) v[b] = i < A.na ? static_cast<const int64_t *>(k.a)[i] : static_cast<const int64_t *>(k.b)[i - A.na];
        }
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) code[b] = static_cast<uint64_t>(v[b]) - k.base;
      } else {
        int32_t v[kDeBatch];
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) {
          const uint64_t i = base + uint64_t(b) * kDeNT;
          if (i < A.n) v[b] = i < A.na ? static_cast<const int32_t *>(k.a)[i] : static_cast<const int32_t *>(k.b)[i - A.na];
        }
        // exact: every key is at least the minimum
#pragma unroll
        for (int b = 0; b < kDeBatch; ++b) code[b] = static_cast<uint64_t>(static_cast<int64_t>(v[b])) - k.base;
      }
#pragma unroll
      for (int b = 0; b < kDeBatch; ++b) f[b] |= static_cast<F>((code[b] ^ k.flip) << k.shift);
    }
#pragma unroll
    for (int b = 0; b < kDeBatch; ++b) {
      const uint64_t i = base + uint64_t(b) * kDeNT;
      if (i < A.na)
        static_cast<F *>(A.out_a)[i] = f[b];
      else if (i < A.n)
        static_cast<F *>(A.out_b)[i - A.na] = f[b];
    }
  }
}

unsigned grid_for(uint64_t n, int nt = kDeNT) {
  const uint64_t blocks = (n + nt - 1) / nt;
  return static_cast<unsigned>(std::max<uint64_t>(1, std::min<uint64_t>(blocks, 8192)));
}

int bit_width_u64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

uint64_t de_slots(double est) {
  uint64_t s = 1024;
  while (static_cast<double>(s) < 2.0 * (1.05 * est + 16.0)) s <<= 1;
  return s;
}

void plan_shifts(eiger_skf_plan_t *p) {
  int total = 0;
  for (int c = 0; c < p->n_keys; ++c) total += p->key[c].bits;
  p->total_bits = total;
  p->fused_bytes = total <= 32 ? 4 : (total <= 64 ? 8 : 0);
  int pos = total;
  for (int c = 0; c < p->n_keys; ++c) {
    pos -= p->key[c].bits;
    p->key[c].shift = pos;
  }
}

void plan_key(const eiger_stats_t &st, int descending, int for_max_bits, int64_t dict_max_ndv, eiger_skf_key_t *k) {
  *k = eiger_skf_key_t{};
  k->dtype = st.dtype;
  k->descending = descending ? 1 : 0;
  if (st.n == 0) {
    k->code = EIGER_SKF_FOR;
    return;
  }
  const uint64_t range = static_cast<uint64_t>(st.max) - static_cast<uint64_t>(st.min);
  const int w = bit_width_u64(range);
  k->base = st.min;
  k->range_bits = w;
  if (w <= for_max_bits) {
    k->code = EIGER_SKF_FOR;
    k->bits = w;
  } else if (st.ndv <= static_cast<double>(dict_max_ndv)) {
    const double est = std::max(1.0, st.ndv);
    k->code = EIGER_SKF_DICT;
    k->ndv = static_cast<int64_t>(std::llround(est));
    k->slots = static_cast<int64_t>(de_slots(est));
    k->bits = bit_width_u64(static_cast<uint64_t>(std::max<int64_t>(k->ndv, 1) - 1));
  } else {
    k->code = EIGER_SKF_FOR;
    k->bits = w;
  }
}

int check_plan(const eiger_skf_plan_t *p, const char *who) {
  if (!p || p->n_keys < 1 || p->n_keys > EIGER_SKF_MAX_KEYS)
    return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": plan with 1..8 keys expected");
  for (int c = 0; c < p->n_keys; ++c) {
    const eiger_skf_key_t &k = p->key[c];
    if (k.dtype != EIGER_INT32 && k.dtype != EIGER_INT64)
      return fail(EIGER_ERR_DTYPE, std::string(who) + ": key dtype must be int32 or int64");
    if (k.code == EIGER_SKF_DICT) {
      if (k.slots < 2 || (k.slots & (k.slots - 1)) || k.slots > (int64_t(1) << 31))
        return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": dictionary slots must be a power of two <= 2^31");
      if (k.range_bits < 0 || k.range_bits > 64) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": range_bits");
    } else if (k.code != EIGER_SKF_FOR || k.bits < 0 || k.bits > 64) {
      return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": bad key code or width");
    }
  }
  return EIGER_OK;
}

// Per dictionary key: the table, the slot of every row, the sorted distinct
// values with their slots, and the code of every slot.
struct DictBufs {
  DeTable t;
  uint32_t *loc;
  unsigned long long *ukey, *skey;
  uint32_t *uslot, *sslot, *code_of_slot;
};

struct SkfLayout {
  DictBufs d[EIGER_SKF_MAX_KEYS];
  uint32_t *ctr;  // 4 words per key
  void *fused;    // sort: fused keys before sorting
  void *sorted;   // sort: sorted keys when the caller passes none
};

// Fusion over 16-byte accesses: each thread takes groups of four consecutive
// rows, reads each key column (or dictionary slot ids) four rows at a time and
// writes four fused keys at once. Used when every column is one array with
// 16-byte aligned rows. With kLdsCodes the dictionaries' code tables (at most
// kFuseLdsCodes entries in all) are first copied into LDS, so the per-row code
// lookups are LDS reads.
constexpr uint32_t kFuseLdsCodes = 9216;  // 36 KB
constexpr int kFuseGroups = 2;            // groups of four rows per thread and step

template <typename F, bool kLdsCodes>
__global__ void __launch_bounds__(kDeNT) k_skf_fuse_vec(FuseArgs A, uint32_t lds_off0, uint32_t lds_total) {
  __shared__ uint32_t codes[kLdsCodes ? kFuseLdsCodes : 1];
  uint32_t lds_off[EIGER_SKF_MAX_KEYS];
  if constexpr (kLdsCodes) {
    uint32_t o = lds_off0;
    for (int c = 0; c < A.nk; ++c) {
      lds_off[c] = o;
      if (A.k[c].dict && A.k[c].bits) {
        const uint32_t m = A.k[c].slots1;
        for (uint32_t j = threadIdx.x; j < m; j += kDeNT) codes[o + j] = A.k[c].code_of_slot[j];
        o += m;
      }
    }
    (void)lds_total;
    __syncthreads();
  }
  constexpr uint64_t span = uint64_t(kDeNT) * 4 * kFuseGroups;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * span;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * span; base < A.n; base += stride) {
    uint64_t i0[kFuseGroups];
    bool full[kFuseGroups];
#pragma unroll
    for (int g = 0; g < kFuseGroups; ++g) {
      i0[g] = base + (static_cast<uint64_t>(g) * kDeNT + threadIdx.x) * 4;
      full[g] = i0[g] + 3 < A.n;
    }
    F f[kFuseGroups][4];
#pragma unroll
    for (int g = 0; g < kFuseGroups; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) f[g][u] = 0;
    for (int c = 0; c < A.nk; ++c) {
      const FuseKey &k = A.k[c];
      if (k.bits == 0) continue;
      uint64_t code[kFuseGroups][4];
#pragma unroll
      for (int g = 0; g < kFuseGroups; ++g) {
        const uint64_t i = i0[g];
        if (k.dict) {
          uint32_t sl[4] = {0u, 0u, 0u, 0u};
          if (full[g]) {
            const uint4 v = *reinterpret_cast<const uint4 *>(k.loc + i);
            sl[0] = v.x; sl[1] = v.y; sl[2] = v.z; sl[3] = v.w;
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) sl[u] = i + u < A.n ? k.loc[i + u] : 0u;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if constexpr (kLdsCodes)
              code[g][u] = codes[lds_off[c] + sl[u]];
            else
              code[g][u] = i + u < A.n ? k.code_of_slot[sl[u]] : 0u;
          }
        } else if (k.wide) {
          const int64_t *a = static_cast<const int64_t *>(k.a);
          int64_t v[4] = {0, 0, 0, 0};
          if (full[g]) {
            const longlong2 x = *reinterpret_cast<const longlong2 *>(a + i);
            const longlong2 y = *reinterpret_cast<const longlong2 *>(a + i + 2);
            v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = i + u < A.n ? a[i + u] : 0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) code[g][u] = static_cast<uint64_t>(v[u]) - k.base;
        } else {
          const int32_t *a = static_cast<const int32_t *>(k.a);
          int32_t v[4] = {0, 0, 0, 0};
          if (full[g]) {
            const int4 x = *reinterpret_cast<const int4 *>(a + i);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = i + u < A.n ? a[i + u] : 0;
          }
          // exact: every key is at least the minimum
#pragma unroll
          for (int u = 0; u < 4; ++u) code[g][u] = static_cast<uint64_t>(static_cast<int64_t>(v[u])) - k.base;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) f[g][u] |= static_cast<F>((code[g][u] ^ k.flip) << k.shift);
      }
    }
#pragma unroll
    for (int g = 0; g < kFuseGroups; ++g) {
      F *out = static_cast<F *>(A.out_a);
      const uint64_t i = i0[g];
      if (full[g]) {
        if constexpr (sizeof(F) == 4) {
          *reinterpret_cast<uint4 *>(out + i) = make_uint4(f[g][0], f[g][1], f[g][2], f[g][3]);
        } else {
          *reinterpret_cast<ulonglong2 *>(out + i) = make_ulonglong2(f[g][0], f[g][1]);
          *reinterpret_cast<ulonglong2 *>(out + i + 2) = make_ulonglong2(f[g][2], f[g][3]);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i + u < A.n) out[i + u] = f[g][u];
      }
    }
  }
}

// Sizes the sort workspace for the largest distinct-value sort and the row sort.
size_t sort_ws_bytes(int key_bytes, uint64_t n, int bits) {
  Workspace w(nullptr, 0);
  radix_sort_pairs(key_bytes, nullptr, nullptr, n, bits, nullptr, nullptr, w, nullptr);
  return w.used + 256;
}

size_t skf_layout(Workspace &ws, const eiger_skf_plan_t &p, uint64_t n, bool sort, SkfLayout *L) {
  *L = SkfLayout{};
  L->ctr = ws.take<uint32_t>(4 * EIGER_SKF_MAX_KEYS);
  uint64_t max_slots = 0;
  for (int c = 0; c < p.n_keys; ++c) {
    if (p.key[c].code != EIGER_SKF_DICT) continue;
    const uint64_t slots = static_cast<uint64_t>(p.key[c].slots);
    max_slots = std::max(max_slots, slots);
    DictBufs &d = L->d[c];
    d.t.key = ws.take<unsigned long long>(slots);
    d.t.mask = slots - 1;
    d.t.ctr = L->ctr ? L->ctr + 4 * c : nullptr;
    d.loc = ws.take<uint32_t>(n);
    d.ukey = ws.take<unsigned long long>(slots + 1);
    d.skey = ws.take<unsigned long long>(slots + 1);
    d.uslot = ws.take<uint32_t>(slots + 1);
    d.sslot = ws.take<uint32_t>(slots + 1);
    d.code_of_slot = ws.take<uint32_t>(slots + 1);
  }
  if (sort) {
    L->fused = ws.take<uint64_t>(n);
    L->sorted = ws.take<uint64_t>(n);
  }
  // one shared region for every radix sort of this call (they run one after another)
  const size_t need = std::max(max_slots ? sort_ws_bytes(8, max_slots + 1, 64) : 0,
                               sort ? sort_ws_bytes(8, n, 64) : 0);
  return need;
}

template <typename K>
int de_launch_insert(const DictBufs &d, const void *a, const void *b, uint64_t na, uint64_t n, hipStream_t s) {
  Rows<K> r{static_cast<const K *>(a), static_cast<const K *>(b), na, n};
  if (d.t.mask + 1 <= kDeLdsMaxTable) {
    const uint64_t chunks = (n + uint64_t(kDeNT) * kDeLdsRows - 1) / (uint64_t(kDeNT) * kDeLdsRows);
    const unsigned grid =
        static_cast<unsigned>(std::max<uint64_t>(1, std::min<uint64_t>(chunks, uint64_t(device_cu_count()) * kDeLdsPerCu)));
    bool vec = false;
    if constexpr (sizeof(K) == 4) {
      vec = na == n && reinterpret_cast<uintptr_t>(a) % 16 == 0 && reinterpret_cast<uintptr_t>(d.loc) % 16 == 0;
      if (vec) EIGER_LAUNCH("dict_insert", (k_de_insert_lds<K, true>), dim3(grid), dim3(kDeNT), 0, s, r, d.t, d.loc);
    }
    if (!vec) EIGER_LAUNCH("dict_insert", (k_de_insert_lds<K, false>), dim3(grid), dim3(kDeNT), 0, s, r, d.t, d.loc);
  } else {
    EIGER_LAUNCH("dict_insert", k_de_insert<K>, dim3(grid_for(n)), dim3(kDeNT), 0, s, r, d.t, d.loc);
  }
  return EIGER_OK;
}

// Steps 1-2 for every dictionary key, one read-back of the counts, then steps 3-4.
// Fills the exact counts and widths into *out.
int dict_steps(const eiger_skf_plan_t &p, const eiger_column *ka, const eiger_column *kb, uint64_t na, uint64_t n,
               SkfLayout &L, void *sort_ws, size_t sort_ws_size, eiger_skf_plan_t *out, hipStream_t s) {
  bool any = false;
  for (int c = 0; c < p.n_keys; ++c) {
    if (p.key[c].code != EIGER_SKF_DICT) continue;
    any = true;
    DictBufs &d = L.d[c];
    int rc = fill_u64(reinterpret_cast<uint64_t *>(d.t.key), d.t.mask + 1, kDeEmpty, s);
    if (rc) return rc;
    if ((rc = fill_u32(d.t.ctr, 4, 0u, s))) return rc;
    const void *a = ka[c].data, *b = kb ? kb[c].data : nullptr;
    rc = p.key[c].dtype == EIGER_INT64 ? de_launch_insert<int64_t>(d, a, b, na, n, s)
                                       : de_launch_insert<int32_t>(d, a, b, na, n, s);
    if (rc) return rc;
    EIGER_LAUNCH("dict_retrieve", k_de_retrieve, dim3(grid_for(d.t.mask + 1)), dim3(kDeNT), 0, s, d.t,
                 static_cast<uint64_t>(p.key[c].base), d.ukey, d.uslot);
  }
  *out = p;
  if (!any) return EIGER_OK;
  uint32_t host[4 * EIGER_SKF_MAX_KEYS];
  EIGER_HIP(hipMemcpyAsync(host, L.ctr, sizeof(host), hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < p.n_keys; ++c) {
    if (p.key[c].code != EIGER_SKF_DICT) continue;
    const uint64_t ndv = host[4 * c];
    if (host[4 * c + 2] || ndv > static_cast<uint64_t>(p.key[c].slots) / 2)
      return fail(EIGER_ERR_TOO_LARGE, "smart key fusion: more distinct values than half the dictionary slots");
    out->key[c].ndv = static_cast<int64_t>(ndv);
    out->key[c].bits = bit_width_u64(ndv ? ndv - 1 : 0);
  }
  plan_shifts(out);
  for (int c = 0; c < p.n_keys; ++c) {
    if (p.key[c].code != EIGER_SKF_DICT) continue;
    DictBufs &d = L.d[c];
    const uint64_t ndv = static_cast<uint64_t>(out->key[c].ndv);
    Workspace sw(sort_ws, sort_ws_size);
    int rc = radix_sort_pairs(8, d.ukey, d.uslot, ndv, p.key[c].range_bits, d.skey, d.sslot, sw, s);
    if (rc) return rc;
    if (ndv)
      EIGER_LAUNCH("dict_scatter", k_de_scatter, dim3(grid_for(ndv)), dim3(kDeNT), 0, s, d.sslot, ndv,
                   d.code_of_slot);
  }
  return EIGER_OK;
}

int launch_fuse(const eiger_skf_plan_t &p, const eiger_column *ka, const eiger_column *kb, uint64_t na, uint64_t n,
                const SkfLayout &L, void *out_a, void *out_b, hipStream_t s) {
  if (n == 0) return EIGER_OK;
  FuseArgs A{};
  A.nk = p.n_keys;
  A.na = na;
  A.n = n;
  A.out_a = out_a;
  A.out_b = out_b;
  for (int c = 0; c < p.n_keys; ++c) {
    const eiger_skf_key_t &k = p.key[c];
    FuseKey &f = A.k[c];
    f.a = ka[c].data;
    f.b = kb ? kb[c].data : nullptr;
    f.wide = k.dtype == EIGER_INT64;
    f.dict = k.code == EIGER_SKF_DICT;
    f.loc = L.d[c].loc;
    f.code_of_slot = L.d[c].code_of_slot;
    f.slots1 = f.dict ? static_cast<uint32_t>(k.slots + 1) : 0u;
    f.base = static_cast<uint64_t>(k.base);
    f.bits = k.bits;
    f.shift = k.shift;
    f.flip = k.descending && k.bits ? (k.bits == 64 ? ~0ull : ((1ull << k.bits) - 1)) : 0ull;
  }
  // 16-byte form: every column one 16-byte aligned array, output too
  bool vec = na == n && reinterpret_cast<uintptr_t>(out_a) % 16 == 0;
  uint64_t lds_codes = 0;
  for (int c = 0; c < p.n_keys; ++c) {
    vec = vec && reinterpret_cast<uintptr_t>(ka[c].data) % 16 == 0;
    if (p.key[c].code == EIGER_SKF_DICT && p.key[c].bits) lds_codes += A.k[c].slots1;
  }
  if (vec) {
    const uint64_t units = (n + 4 * kFuseGroups - 1) / (4 * kFuseGroups);
    const unsigned g = grid_for(units);
    const bool lds = lds_codes <= kFuseLdsCodes;
    const uint32_t lt = static_cast<uint32_t>(lds_codes);
    if (p.fused_bytes == 4) {
      if (lds)
        EIGER_LAUNCH("skf_fuse", (k_skf_fuse_vec<uint32_t, true>), dim3(g), dim3(kDeNT), 0, s, A, 0u, lt);
      else
        EIGER_LAUNCH("skf_fuse", (k_skf_fuse_vec<uint32_t, false>), dim3(g), dim3(kDeNT), 0, s, A, 0u, lt);
    } else {
      if (lds)
        EIGER_LAUNCH("skf_fuse", (k_skf_fuse_vec<uint64_t, true>), dim3(g), dim3(kDeNT), 0, s, A, 0u, lt);
      else
        EIGER_LAUNCH("skf_fuse", (k_skf_fuse_vec<uint64_t, false>), dim3(g), dim3(kDeNT), 0, s, A, 0u, lt);
    }
    return EIGER_OK;
  }
  const unsigned grid = grid_for((n + kDeBatch - 1) / kDeBatch);
  if (p.fused_bytes == 4) {
    EIGER_LAUNCH("skf_fuse", k_skf_fuse<uint32_t>, dim3(grid), dim3(kDeNT), 0, s, A);
  } else {
    EIGER_LAUNCH("skf_fuse", k_skf_fuse<uint64_t>, dim3(grid), dim3(kDeNT), 0, s, A);
  }
  return EIGER_OK;
}

int check_keys(const eiger_column *keys, int32_t n_keys, const eiger_skf_plan_t &p, int64_t *n, const char *who) {
  if (!keys) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": NULL key array");
  if (n_keys != p.n_keys) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": n_keys differs from the plan");
  *n = keys[0].n;
  for (int c = 0; c < n_keys; ++c) {
    if (keys[c].n != *n) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": key columns of unequal length");
    if (keys[c].dtype != p.key[c].dtype) return fail(EIGER_ERR_DTYPE, std::string(who) + ": key dtype differs from the plan");
    if (keys[c].n > 0 && !keys[c].data) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": NULL key column");
  }
  if (*n < 0 || *n > EIGER_MAX_ROWS) return fail(EIGER_ERR_TOO_LARGE, std::string(who) + ": rows outside [0, EIGER_MAX_ROWS]");
  return EIGER_OK;
}

size_t skf_total_bytes(const eiger_skf_plan_t &p, uint64_t n, bool sort) {
  Workspace ws(nullptr, 0);
  SkfLayout L;
  const size_t sort_need = skf_layout(ws, p, n, sort, &L);
  ws.take<char>(sort_need);
  return ws.used + 256;
}

// eiger_skf_fuse and eiger_sort_multikey share this body.
int skf_run(const eiger_column *ka, const eiger_column *kb, int32_t n_keys, const eiger_skf_plan_t *plan, void *out_a,
            void *out_b, bool sort, uint32_t *perm, void *sorted, eiger_skf_plan_t *out_plan, void *wsp,
            size_t ws_bytes, hipStream_t s, const char *who) {
  if (int rc = check_plan(plan, who)) return rc;
  if (!out_plan) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": out_plan is NULL");
  int64_t na = 0, nb = 0;
  if (int rc = check_keys(ka, n_keys, *plan, &na, who)) return rc;
  if (kb)
    if (int rc = check_keys(kb, n_keys, *plan, &nb, who)) return rc;
  const uint64_t n = static_cast<uint64_t>(na + nb);
  if (n > static_cast<uint64_t>(EIGER_MAX_ROWS)) return fail(EIGER_ERR_TOO_LARGE, std::string(who) + ": too many rows");
  if (n > 0 && !sort && (!out_a || (nb > 0 && !out_b)))
    return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": NULL output");
  if (n > 0 && sort && !perm) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": out_perm is NULL");
  if (ws_bytes < skf_total_bytes(*plan, n, sort))
    return fail(EIGER_ERR_WORKSPACE, std::string(who) + ": workspace too small");
  if (n > 0 && !wsp) return fail(EIGER_ERR_INVALID_ARG, std::string(who) + ": NULL workspace");
  Workspace ws(wsp, ws_bytes);
  SkfLayout L;
  const size_t sort_need = skf_layout(ws, *plan, n, sort, &L);
  void *sort_ws = ws.take<char>(sort_need);
  int rc = dict_steps(*plan, ka, kb, static_cast<uint64_t>(na), n, L, sort_ws, sort_need, out_plan, s);
  if (rc) return rc;
  if (out_plan->fused_bytes == 0)
    return fail(EIGER_ERR_UNSUPPORTED, std::string(who) + ": the key codes need more than 64 bits");
  if (!sort) return launch_fuse(*out_plan, ka, kb, static_cast<uint64_t>(na), n, L, out_a, out_b, s);
  if ((rc = launch_fuse(*out_plan, ka, nullptr, n, n, L, L.fused, nullptr, s))) return rc;
  Workspace sw(sort_ws, sort_need);
  return radix_sort_pairs(out_plan->fused_bytes, L.fused, nullptr, n, out_plan->total_bits,
                          sorted ? sorted : L.sorted, perm, sw, s);
}

}  // namespace

}  // namespace eiger

using namespace eiger;

extern "C" int eiger_skf_plan(const eiger_stats_t *stats, const int32_t *descending, int32_t n_keys,
                              int32_t for_max_bits, int64_t dict_max_ndv, eiger_skf_plan_t *out) {
  if (!stats || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_skf_plan: NULL argument");
  if (n_keys < 1 || n_keys > EIGER_SKF_MAX_KEYS) return fail(EIGER_ERR_INVALID_ARG, "eiger_skf_plan: 1..8 keys");
  eiger_skf_plan_t p{};
  p.n_keys = n_keys;
  for (int c = 0; c < n_keys; ++c) {
    if (stats[c].dtype != EIGER_INT32 && stats[c].dtype != EIGER_INT64)
      return fail(EIGER_ERR_DTYPE, "eiger_skf_plan: key dtype must be int32 or int64");
    plan_key(stats[c], descending ? descending[c] : 0, for_max_bits, dict_max_ndv, &p.key[c]);
  }
  plan_shifts(&p);
  *out = p;
  return EIGER_OK;
}

extern "C" int eiger_skf_plan_join(const eiger_stats_t *build_stats, const eiger_stats_t *probe_stats, int32_t n_keys,
                                   int32_t for_max_bits, int64_t dict_max_ndv, eiger_skf_plan_t *out) {
  if (!build_stats || !probe_stats || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_skf_plan_join: NULL argument");
  if (n_keys < 1 || n_keys > EIGER_SKF_MAX_KEYS) return fail(EIGER_ERR_INVALID_ARG, "eiger_skf_plan_join: 1..8 keys");
  eiger_skf_plan_t p{};
  p.n_keys = n_keys;
  for (int c = 0; c < n_keys; ++c) {
    const eiger_stats_t &b = build_stats[c], &q = probe_stats[c];
    if (b.dtype != q.dtype || (b.dtype != EIGER_INT32 && b.dtype != EIGER_INT64))
      return fail(EIGER_ERR_DTYPE, "eiger_skf_plan_join: both sides' key dtypes must match (int32 or int64)");
    eiger_stats_t u = b;
    u.n = b.n + q.n;
    if (b.n == 0) {
      u.min = q.min;
      u.max = q.max;
    } else if (q.n > 0) {
      u.min = std::min(b.min, q.min);
      u.max = std::max(b.max, q.max);
    }
    u.ndv = b.ndv + q.ndv;  // at least the distinct count of the union
    plan_key(u, 0, for_max_bits, dict_max_ndv, &p.key[c]);
  }
  plan_shifts(&p);
  *out = p;
  return EIGER_OK;
}

extern "C" int eiger_skf_workspace_size(const eiger_skf_plan_t *plan, int64_t n_a, int64_t n_b, int32_t sort,
                                        size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_skf_workspace_size: bytes is NULL");
  if (int rc = check_plan(plan, "eiger_skf_workspace_size")) return rc;
  if (n_a < 0 || n_b < 0 || n_a + n_b > EIGER_MAX_ROWS)
    return fail(EIGER_ERR_TOO_LARGE, "eiger_skf_workspace_size: rows outside [0, EIGER_MAX_ROWS]");
  *bytes = skf_total_bytes(*plan, static_cast<uint64_t>(n_a + n_b), sort != 0);
  return EIGER_OK;
}

extern "C" int eiger_skf_fuse(const eiger_column *keys_a, const eiger_column *keys_b, int32_t n_keys,
                              const eiger_skf_plan_t *plan, void *out_a, void *out_b, eiger_skf_plan_t *out_plan,
                              void *ws, size_t ws_bytes, void *stream) {
  return skf_run(keys_a, keys_b, n_keys, plan, out_a, out_b, false, nullptr, nullptr, out_plan, ws, ws_bytes,
                 static_cast<hipStream_t>(stream), "eiger_skf_fuse");
}

extern "C" int eiger_sort_multikey(const eiger_column *keys, int32_t n_keys, const eiger_skf_plan_t *plan,
                                   uint32_t *out_perm, void *out_sorted, eiger_skf_plan_t *out_plan, void *ws,
                                   size_t ws_bytes, void *stream) {
  return skf_run(keys, nullptr, n_keys, plan, nullptr, nullptr, true, out_perm, out_sorted, out_plan, ws, ws_bytes,
                 static_cast<hipStream_t>(stream), "eiger_sort_multikey");
}

extern "C" int eiger_dict_encode_workspace_size(eiger_column col, int64_t slots, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_dict_encode_workspace_size: bytes is NULL");
  if (col.n < 0 || col.n > EIGER_MAX_ROWS) return fail(EIGER_ERR_TOO_LARGE, "eiger_dict_encode: rows outside range");
  eiger_skf_plan_t p{};
  p.n_keys = 1;
  p.key[0].code = EIGER_SKF_DICT;
  p.key[0].dtype = col.dtype;
  p.key[0].slots = slots;
  p.key[0].range_bits = 64;
  if (int rc = check_plan(&p, "eiger_dict_encode")) return rc;
  *bytes = skf_total_bytes(p, static_cast<uint64_t>(col.n), false);
  return EIGER_OK;
}

extern "C" int eiger_dict_encode(eiger_column col, int64_t slots, uint32_t *out_codes, void *out_dict,
                                 int64_t dict_capacity, int64_t *out_ndv, void *wsp, size_t ws_bytes, void *stream) {
  size_t need = 0;
  if (int rc = eiger_dict_encode_workspace_size(col, slots, &need)) return rc;
  if (!out_ndv) return fail(EIGER_ERR_INVALID_ARG, "eiger_dict_encode: out_ndv is NULL");
  if (col.n > 0 && (!col.data || !out_codes || !wsp)) return fail(EIGER_ERR_INVALID_ARG, "eiger_dict_encode: NULL buffer");
  if (ws_bytes < need) return fail(EIGER_ERR_WORKSPACE, "eiger_dict_encode: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  eiger_skf_plan_t p{};
  p.n_keys = 1;
  p.key[0].code = EIGER_SKF_DICT;
  p.key[0].dtype = col.dtype;
  p.key[0].slots = slots;
  p.key[0].range_bits = 64;  // values are sorted as key - INT64_MIN over the full width
  p.key[0].base = INT64_MIN;
  *out_ndv = 0;
  if (col.n == 0) return EIGER_OK;
  Workspace ws(wsp, ws_bytes);
  SkfLayout L;
  const size_t sort_need = skf_layout(ws, p, static_cast<uint64_t>(col.n), false, &L);
  void *sort_ws = ws.take<char>(sort_need);
  eiger_skf_plan_t fin;
  int rc = dict_steps(p, &col, nullptr, static_cast<uint64_t>(col.n), static_cast<uint64_t>(col.n), L, sort_ws,
                      sort_need, &fin, s);
  if (rc) return rc;
  const uint64_t ndv = static_cast<uint64_t>(fin.key[0].ndv);
  *out_ndv = fin.key[0].ndv;
  if (out_dict && fin.key[0].ndv > dict_capacity)
    return fail(EIGER_ERR_CAPACITY, "eiger_dict_encode: more distinct values than dict_capacity");
  const DictBufs &d = L.d[0];
  EIGER_LAUNCH("dict_gather", k_de_gather, dim3(grid_for(static_cast<uint64_t>(col.n))), dim3(kDeNT), 0, s, d.loc,
               static_cast<uint64_t>(col.n), d.code_of_slot, out_codes);
  if (out_dict) {
    if (col.dtype == EIGER_INT64) {
      EIGER_LAUNCH("dict_values", k_de_dict<int64_t>, dim3(grid_for(ndv)), dim3(kDeNT), 0, s, d.skey, ndv,
                   static_cast<uint64_t>(INT64_MIN), static_cast<int64_t *>(out_dict));
    } else {
      EIGER_LAUNCH("dict_values", k_de_dict<int32_t>, dim3(grid_for(ndv)), dim3(kDeNT), 0, s, d.skey, ndv,
                   static_cast<uint64_t>(INT64_MIN), static_cast<int32_t *>(out_dict));
    }
  }
  EIGER_HIP(hipStreamSynchronize(s));
  return EIGER_OK;
}
