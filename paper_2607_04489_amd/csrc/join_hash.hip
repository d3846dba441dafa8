// join_hash.hip -- GLOBAL_HASH variant: one open-addressing table in HBM.
//
// This is the non-partitioned hash join of the paper (Section 3.2, Table 1),
// laid out for gfx950: the key, row id and payload of a build row share one
// 16-byte slot (32 bytes when key and payload are both 8 bytes), so a probe
// touches one cache line per slot group instead of gathering keys through
// tuple ids (the cost the paper blames for the hash join's losses, Section
// 5.2.1). Slots are claimed by CAS on the key word with a sentinel key outside
// the build range (duplicates show up during the build), or, when the build
// keys reach both ends of the key domain, by CAS on the row-id word followed
// by a duplicate check. Empty slots have row id 0xFFFFFFFF either way. The
// table is a multiset: duplicate build keys occupy several slots and a probe
// walks the whole cluster (linear probing) until an empty slot.
#include <limits>
#include <type_traits>

#include "join_common.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr int kNT = 256;
constexpr int kIPT = 5;
constexpr int kSCAP = 4096;

template <typename K, typename PB>
struct HashTab {
  static constexpr bool kHashed = true;
  static constexpr bool kRuns = false;
  using SlotT = Slot<K, PB>;
  using Index = uint64_t;  // a table may hold more than 2^32 slots
  const Slot<K, PB> *__restrict__ slots;
  uint64_t mask;
  const uint32_t *dup;  // device flag: nonzero when some build key occurs twice
  bool unique;          // set in the kernel from *dup

  __device__ __forceinline__ void init() { unique = dup && *dup == 0; }
  __device__ __forceinline__ uint64_t home(K key) const {
    return fmix64(static_cast<uint64_t>(sext(key))) & mask;
  }
  __device__ __forceinline__ uint64_t next(uint64_t i) const { return (i + 1) & mask; }
  __device__ __forceinline__ SlotT load(uint64_t i) const { return slots[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint64_t i = home(key);
    for (;;) {
      const Slot<K, PB> s = slots[i];
      if (s.rowid == kEmpty) break;
      if (s.key == key) f(s.rowid);
      i = next(i);
    }
  }
};

// Sets *dup when some build key occurs more than once: every build row walks
// its key's cluster and counts equal keys. Afterwards probes of a table with
// distinct keys stop at their first match.
template <typename K, typename PB>
__global__ void k_hash_unique(const K *__restrict__ keys, uint64_t n, HashTab<K, PB> tab,
                              uint32_t *dup) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    if (*static_cast<volatile uint32_t *>(dup)) return;
    const K key = keys[r];
    uint32_t c = 0;
    tab.for_each(key, [&](uint32_t) { ++c; });
    if (c > 1) atomicOr(dup, 1u);
  }
}

template <typename K, typename PB>
__global__ void k_hash_build(const K *__restrict__ keys, const PB *__restrict__ pay, uint64_t n,
                             Slot<K, PB> *__restrict__ slots, uint64_t mask) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    const K key = keys[r];
    uint64_t i = fmix64(static_cast<uint64_t>(sext(key))) & mask;
    // The table has more slots than rows, so an empty slot is always found.
    for (;;) {
      if (atomicCAS(&slots[i].rowid, kEmpty, static_cast<uint32_t>(r)) == kEmpty) {
        slots[i].key = key;
        slots[i].pay = pay[r];
        break;
      }
      i = (i + 1) & mask;
    }
  }
}

// Table clear for the key-claiming build: key = sentinel, row id = empty. Slots
// are 16 or 32 bytes (one or two 16-byte words); each workgroup stores one
// contiguous chunk of the table with 16-byte stores, as the library's fills do.
template <typename K, typename PB>
__global__ void __launch_bounds__(256) k_hash_clear(Slot<K, PB> *__restrict__ slots, uint64_t n, K sentinel) {
  constexpr int kWords = sizeof(Slot<K, PB>) / 16;
  static_assert(kWords == 1 || kWords == 2, "16- or 32-byte slots");
  Slot<K, PB> e{};
  e.key = sentinel;
  e.rowid = kEmpty;
  uint4 w[kWords];
  __builtin_memcpy(w, &e, sizeof(e));
  uint4 *__restrict__ q = reinterpret_cast<uint4 *>(slots);
  const uint64_t nw = n * kWords;
  const uint64_t per = (nw + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = uint64_t(blockIdx.x) * per, hi = min(nw, lo + per);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) q[i] = w[i % kWords];
}

// Build that claims a slot by CAS on its key word (empty = a sentinel value no
// build key takes), so a row that meets its own key on the way has found a
// duplicate: the distinctness flag comes out of the build, without a second
// walk per build row. A key equal to the sentinel (the plan's key range was
// wrong) is reported through the counters' flags.
template <typename K, typename PB>
__global__ void k_hash_build_keys(const K *__restrict__ keys, const PB *__restrict__ pay, uint64_t n,
                                  Slot<K, PB> *__restrict__ slots, uint64_t mask, K sentinel, uint32_t *dup,
                                  uint64_t *flags) {
  using W = typename std::conditional<sizeof(K) == 8, unsigned long long, unsigned int>::type;
  const W empty = static_cast<W>(sentinel);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  bool seen = false;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    const K key = keys[r];
    if (key == sentinel) {
      atomicOr(reinterpret_cast<unsigned long long *>(flags), kFlagBuildOutOfRange);
      continue;
    }
    uint64_t i = fmix64(static_cast<uint64_t>(sext(key))) & mask;
    // The table has more slots than rows, so an empty slot is always found.
    for (;;) {
      const W old = atomicCAS(reinterpret_cast<W *>(&slots[i].key), empty, static_cast<W>(key));
      if (old == empty) {
        slots[i].rowid = static_cast<uint32_t>(r);
        slots[i].pay = pay[r];
        break;
      }
      seen |= old == static_cast<W>(key);
      i = (i + 1) & mask;
    }
  }
  if (seen) atomicOr(dup, 1u);
}

// A key value outside the plan's build range, if the key type has one.
template <typename K>
bool hash_sentinel(const JoinArgs &a, K *out) {
  const int64_t lo = static_cast<int64_t>(std::numeric_limits<K>::min());
  const int64_t hi = static_cast<int64_t>(std::numeric_limits<K>::max());
  if (a.nR == 0 || a.plan.build_min > lo) {
    *out = std::numeric_limits<K>::min();
    return true;
  }
  if (a.plan.build_max < hi) {
    *out = std::numeric_limits<K>::max();
    return true;
  }
  return false;
}

// Each workgroup streams a contiguous range of probe rows (an equal share of
// whole sub-tiles).
template <class Tab, typename K, typename PS>
__global__ void __launch_bounds__(kNT) k_probe(Tab tab, const K *__restrict__ pk,
                                               const PS *__restrict__ pp, uint64_t n, EmitOut o) {
  __shared__ EmitLds<kNT, kSCAP> L;
  uint64_t fill = 0;
  uint64_t cs = 0;
  tab.init();
  constexpr uint64_t sub = uint64_t(kNT) * kIPT;
  const uint64_t nsub = (n + sub - 1) / sub;
  const uint64_t per = (nsub + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = blockIdx.x * per * sub;
  const uint64_t hi = lo + per * sub < n ? lo + per * sub : n;
  probe_range<kNT, kIPT, kSCAP>(tab, pk, pp, static_cast<const uint32_t *>(nullptr), lo, hi, L, fill,
                                o, cs);
  finish(L, o, fill, cs);
}

unsigned grid_for(uint64_t work, uint64_t per_block, int per_cu) {
  uint64_t g = (work + per_block - 1) / per_block;
  const uint64_t cap = uint64_t(device_cu_count()) * per_cu;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g ? g : 1);
}

template <typename K, typename PB, typename PS>
int hash_impl(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const uint64_t nslots = hash_slots(a.nR, a.plan.load_factor);
  JoinCounters *c = ws.take<JoinCounters>(1);
  uint32_t *dup = ws.take<uint32_t>(1);
  Slot<K, PB> *slots = ws.take<Slot<K, PB>>(nslots);
  *ctr = c;
  if (!ws.base) return EIGER_OK;
  hipStream_t s = a.s;
  int rc;
  if ((rc = fill_u64(reinterpret_cast<uint64_t *>(c), 4, 0, s))) return rc;
  if (a.nR == 0 || a.nS == 0) return EIGER_OK;
  if ((rc = fill_u32(dup, 1, 0, s))) return rc;
  HashTab<K, PB> tab{slots, nslots - 1, dup, false};
  K sentinel;
  if (hash_sentinel<K>(a, &sentinel)) {
    EIGER_LAUNCH("hash_clear", (k_hash_clear<K, PB>),
                 dim3(static_cast<unsigned>(std::min<uint64_t>((nslots + 1023) / 1024, uint64_t(device_cu_count()) * 16))),
                 dim3(256), 0, s, slots, nslots, sentinel);
    EIGER_LAUNCH("hash_build", (k_hash_build_keys<K, PB>), dim3(grid_for(a.nR, 256 * 2, 8)), dim3(256), 0, s,
                 static_cast<const K *>(a.bk), static_cast<const PB *>(a.bp), a.nR, slots, nslots - 1, sentinel,
                 dup, &c->flags);
  } else {
    // keys at both ends of the domain: claim by row id, then a duplicate check
    if ((rc = fill_u32(reinterpret_cast<uint32_t *>(slots), nslots * sizeof(Slot<K, PB>) / 4, kEmpty, s)))
      return rc;
    EIGER_LAUNCH("hash_build", (k_hash_build<K, PB>), dim3(grid_for(a.nR, 256 * 2, 8)), dim3(256), 0, s,
                 static_cast<const K *>(a.bk), static_cast<const PB *>(a.bp), a.nR, slots, nslots - 1);
    EIGER_LAUNCH("hash_unique", (k_hash_unique<K, PB>), dim3(grid_for(a.nR, 256 * 2, 8)), dim3(256), 0, s,
                 static_cast<const K *>(a.bk), a.nR, tab, dup);
  }
  EmitOut o{a.ob, a.op, a.cap, &c->count, &c->checksum};
  EIGER_LAUNCH("hash_probe", (k_probe<HashTab<K, PB>, K, PS>),
               dim3(grid_for(a.nS, uint64_t(kNT) * kIPT, 4)), dim3(kNT), 0, s, tab,
               static_cast<const K *>(a.pk), static_cast<const PS *>(a.pp), a.nS, o);
  return EIGER_OK;
}

}  // namespace

uint64_t hash_slots(uint64_t n, float lf) {
  if (!(lf > 0.f) || lf > 0.9f) lf = 0.5f;
  uint64_t want = static_cast<uint64_t>(static_cast<double>(n) / lf) + 1;
  uint64_t s = 64;
  while (s < want) s <<= 1;
  return s;
}

int run_global_hash(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  const bool k64 = a.kdt == EIGER_INT64, b64 = a.bpdt == EIGER_INT64, p64 = a.ppdt == EIGER_INT64;
#define EIGER_DISPATCH(KT, BT, PT) return hash_impl<KT, BT, PT>(a, ws, ctr)
  if (!k64 && !b64 && !p64) EIGER_DISPATCH(int32_t, int32_t, int32_t);
  if (!k64 && !b64 && p64) EIGER_DISPATCH(int32_t, int32_t, int64_t);
  if (!k64 && b64 && !p64) EIGER_DISPATCH(int32_t, int64_t, int32_t);
  if (!k64 && b64 && p64) EIGER_DISPATCH(int32_t, int64_t, int64_t);
  if (k64 && !b64 && !p64) EIGER_DISPATCH(int64_t, int32_t, int32_t);
  if (k64 && !b64 && p64) EIGER_DISPATCH(int64_t, int32_t, int64_t);
  if (k64 && b64 && !p64) EIGER_DISPATCH(int64_t, int64_t, int32_t);
  EIGER_DISPATCH(int64_t, int64_t, int64_t);
#undef EIGER_DISPATCH
}

}  // namespace eiger
