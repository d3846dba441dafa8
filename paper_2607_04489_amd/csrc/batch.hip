// batch.hip -- many independent joins in one hipGraph launch.
//
// All joins of a batch go through the same stages, each one persistent kernel
// over a flat list of work items (join, row range) built on the host:
//   reset     per-join state (min/max, counters, flags) and the table arena
//   minmax    min/max of every join's build keys (the statistics the per-join
//             choice needs; Section 4 of the paper: runtime statistics)
//   plan      per join: a table indexed by key - min when the key range fits the
//             join's slot budget (dense keys), else an open-addressing table
//   build     insert build rows; a direct slot claimed twice flags a duplicate
//   unique    hash joins: every build row counts its key; more than one -> flag
//   probe     probe tiles against their join's table, materialize pairs into
//             the join's output range (first-match walks: build keys distinct)
//   radix     joins of size buckets tuned to the partitioned join run the RADIX
//             variant's own kernels (histograms, scans, scatters, LDS-table
//             join) inside the same graph, one join after another, each into
//             its own output range; a collect kernel copies their counters
// Stages never wait on each other inside a kernel, so no workgroup spins.
#include <algorithm>
#include <vector>

#include "join_common.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

constexpr uint32_t kBuildTile = 16384;
constexpr int kBNT = 256;
constexpr int kBIPT = 4;
constexpr int kBSCAP = 4096;
constexpr uint32_t kVarDirect = 0, kVarHash = 1, kVarRadix = 2;

struct BatchJoinDev {
  const void *bk, *bp, *pk, *pp;
  uint64_t nR, nS;
  uint64_t out_off;  // first output position of this join
  uint64_t tab_off;  // first slot of this join's table region
  uint64_t slots;    // slots of the region (power of two)
};

struct BatchState {
  int64_t mn, mx;
  uint64_t count, checksum;
  uint32_t variant, flags;
};

struct Item {
  uint32_t join, pad;
  uint64_t lo, hi;
};

__global__ void k_batch_reset(BatchState *__restrict__ st, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  st[j].mn = INT64_MAX;
  st[j].mx = INT64_MIN;
  st[j].count = 0;
  st[j].checksum = 0;
  st[j].variant = kVarHash;
  st[j].flags = 0;
}

template <typename K>
__global__ void __launch_bounds__(256) k_batch_minmax(const Item *__restrict__ items, uint32_t n_items,
                                                      const BatchJoinDev *__restrict__ J, BatchState *__restrict__ st) {
  __shared__ int64_t red[2][4];
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    const K *keys = static_cast<const K *>(J[w.join].bk);
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (uint64_t i = w.lo + threadIdx.x; i < w.hi; i += 256) {
      const int64_t k = sext(keys[i]);
      mn = k < mn ? k : mn;
      mx = k > mx ? k : mx;
    }
    mn = wave_min_i64(mn);
    mx = wave_max_i64(mx);
    if (__lane_id() == 0) {
      red[0][threadIdx.x / 64] = mn;
      red[1][threadIdx.x / 64] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < 4; ++q) {
        mn = red[0][q] < mn ? red[0][q] : mn;
        mx = red[1][q] > mx ? red[1][q] : mx;
      }
      atomicMin(reinterpret_cast<long long *>(&st[w.join].mn), static_cast<long long>(mn));
      atomicMax(reinterpret_cast<long long *>(&st[w.join].mx), static_cast<long long>(mx));
    }
    __syncthreads();
  }
}

__global__ void k_batch_plan(const BatchJoinDev *__restrict__ J, BatchState *__restrict__ st, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t range = static_cast<uint64_t>(st[j].mx) - static_cast<uint64_t>(st[j].mn) + 1;
  st[j].variant = (J[j].nR > 0 && range != 0 && range <= J[j].slots) ? kVarDirect : kVarHash;
}

template <typename K, typename P>
__global__ void __launch_bounds__(256) k_batch_build(const Item *__restrict__ items, uint32_t n_items,
                                                     const BatchJoinDev *__restrict__ J, BatchState *__restrict__ st,
                                                     Slot<K, P> *__restrict__ arena) {
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    const BatchJoinDev d = J[w.join];
    const K *keys = static_cast<const K *>(d.bk);
    const P *pay = static_cast<const P *>(d.bp);
    Slot<K, P> *tab = arena + d.tab_off;
    const bool direct = st[w.join].variant == kVarDirect;
    const uint64_t mn = static_cast<uint64_t>(st[w.join].mn), mask = d.slots - 1;
    for (uint64_t r = w.lo + threadIdx.x; r < w.hi; r += 256) {
      const K key = keys[r];
      if (direct) {
        const uint64_t s = static_cast<uint64_t>(sext(key)) - mn;  // < range <= slots
        if (atomicCAS(&tab[s].rowid, kEmpty, static_cast<uint32_t>(r)) == kEmpty) {
          tab[s].key = key;
          tab[s].pay = pay[r];
        } else {
          atomicOr(&st[w.join].flags, EIGER_BATCH_DUPLICATE_BUILD);
        }
      } else {
        uint64_t s = fmix64(static_cast<uint64_t>(sext(key))) & mask;
        for (;;) {  // slots >= 2 rows: an empty slot exists
          if (atomicCAS(&tab[s].rowid, kEmpty, static_cast<uint32_t>(r)) == kEmpty) {
            tab[s].key = key;
            tab[s].pay = pay[r];
            break;
          }
          s = (s + 1) & mask;
        }
      }
    }
  }
}

template <typename K, typename P>
__global__ void __launch_bounds__(256) k_batch_unique(const Item *__restrict__ items, uint32_t n_items,
                                                      const BatchJoinDev *__restrict__ J, BatchState *__restrict__ st,
                                                      const Slot<K, P> *__restrict__ arena) {
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    if (st[w.join].variant != kVarHash) continue;
    const BatchJoinDev d = J[w.join];
    const K *keys = static_cast<const K *>(d.bk);
    const Slot<K, P> *tab = arena + d.tab_off;
    const uint64_t mask = d.slots - 1;
    for (uint64_t r = w.lo + threadIdx.x; r < w.hi; r += 256) {
      const K key = keys[r];
      uint64_t s = fmix64(static_cast<uint64_t>(sext(key))) & mask;
      uint32_t c = 0;
      for (;;) {
        const Slot<K, P> v = tab[s];
        if (v.rowid == kEmpty) break;
        c += v.key == key;
        s = (s + 1) & mask;
      }
      if (c > 1) atomicOr(&st[w.join].flags, EIGER_BATCH_DUPLICATE_BUILD);
    }
  }
}

template <typename K, typename P>
struct BatchDirectTab {
  static constexpr bool kHashed = false;
  static constexpr bool kRuns = false;
  const Slot<K, P> *slots;
  uint64_t mn, range;
  __device__ __forceinline__ uint32_t lookup(K key, uint32_t &first, uint64_t &psum) const {
    const uint64_t d = static_cast<uint64_t>(sext(key)) - mn;
    if (d >= range) return 0;
    const Slot<K, P> s = slots[d];
    if (s.rowid == kEmpty || s.key != key) return 0;
    first = s.rowid;
    psum += static_cast<uint64_t>(sext(s.pay));
    return 1;
  }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint32_t first;
    uint64_t ps = 0;
    if (lookup(key, first, ps)) f(first);
  }
};

template <typename K, typename P>
struct BatchHashTab {
  static constexpr bool kHashed = true;
  static constexpr bool kRuns = false;
  using SlotT = Slot<K, P>;
  using Index = uint64_t;
  const Slot<K, P> *slots;
  uint64_t mask;
  bool unique;
  __device__ __forceinline__ uint64_t home(K key) const {
    return fmix64(static_cast<uint64_t>(sext(key))) & mask;
  }
  __device__ __forceinline__ uint64_t next(uint64_t i) const { return (i + 1) & mask; }
  __device__ __forceinline__ SlotT load(uint64_t i) const { return slots[i]; }
  template <class F>
  __device__ __forceinline__ void for_each(K key, F f) const {
    uint64_t i = home(key);
    for (;;) {
      const SlotT s = slots[i];
      if (s.rowid == kEmpty) break;
      if (s.key == key) f(s.rowid);
      i = next(i);
    }
  }
};

template <typename K, typename P>
__global__ void __launch_bounds__(kBNT) k_batch_probe(const Item *__restrict__ items, uint32_t n_items,
                                                      const BatchJoinDev *__restrict__ J, BatchState *__restrict__ st,
                                                      const Slot<K, P> *__restrict__ arena, uint32_t *ob,
                                                      uint32_t *op) {
  __shared__ EmitLds<kBNT, kBSCAP> L;
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    const BatchJoinDev d = J[w.join];
    BatchState *s = st + w.join;
    EmitOut o{ob + d.out_off, op + d.out_off, d.nS, &s->count, &s->checksum};
    uint64_t fill = 0, cs = 0;
    const K *pk = static_cast<const K *>(d.pk);
    const P *pp = static_cast<const P *>(d.pp);
    if (s->variant == kVarDirect) {
      const uint64_t mn = static_cast<uint64_t>(s->mn);
      BatchDirectTab<K, P> tab{arena + d.tab_off, mn, static_cast<uint64_t>(s->mx) - mn + 1};
      probe_range<kBNT, kBIPT, kBSCAP>(tab, pk, pp, static_cast<const uint32_t *>(nullptr), w.lo, w.hi, L, fill,
                                       o, cs);
    } else {
      BatchHashTab<K, P> tab{arena + d.tab_off, d.slots - 1, true};
      probe_range<kBNT, kBIPT, kBSCAP>(tab, pk, pp, static_cast<const uint32_t *>(nullptr), w.lo, w.hi, L, fill,
                                       o, cs);
    }
    finish(L, o, fill, cs);
    __syncthreads();
  }
}

// Counters of a RADIX join run inside the graph -> its batch state.
__global__ void k_batch_collect(const JoinCounters *__restrict__ c, BatchState *__restrict__ st, uint64_t cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->count = c->count;
    st->checksum = c->checksum;
    st->variant = kVarRadix;
    st->flags = c->count > cap ? EIGER_BATCH_CAPACITY : 0u;
  }
}

int bucket_of_rows(int64_t n) {
  int b = 0;
  while (b < EIGER_BATCH_BUCKETS - 1 && (int64_t(2) << b) <= n) ++b;
  return b;
}

eiger_batch_tune tune_for(const eiger_batch_tune *tune, int64_t n) {
  eiger_batch_tune t{0.5f, 16384, 0};
  if (tune) {
    const eiger_batch_tune &u = tune[bucket_of_rows(n)];
    if (u.load_factor > 0.f && u.load_factor <= 0.9f) t.load_factor = u.load_factor;
    if (u.probe_tile >= 256 && u.probe_tile <= (1 << 20)) t.probe_tile = u.probe_tile;
    if (u.radix_bits >= 1 && u.radix_bits <= 16) t.radix_bits = u.radix_bits;
  }
  return t;
}

// A join of the batch that runs the RADIX variant inside the graph.
struct RadixJob {
  int32_t join;
  JoinArgs args;   // outputs and stream are filled in at capture
  size_t ws_off, ws_bytes;
};

// Host-side description of a batch (descriptors, work items, sizes).
struct BatchPlan {
  std::vector<BatchJoinDev> joins;
  std::vector<Item> build, probe;
  std::vector<RadixJob> radix;
  uint64_t arena_slots = 0, out_total = 0;
  size_t radix_ws = 0;
};

int plan_batch(const eiger_batch_join *joins, int32_t n, int32_t kdt, int32_t pdt, const eiger_batch_tune *tune,
               BatchPlan *bp) {
  if (!joins || n <= 0) return fail(EIGER_ERR_INVALID_ARG, "batch: no joins");
  if ((kdt != EIGER_INT32 && kdt != EIGER_INT64) || (pdt != EIGER_INT32 && pdt != EIGER_INT64))
    return fail(EIGER_ERR_DTYPE, "batch: dtypes must be EIGER_INT32 or EIGER_INT64");
  bp->joins.resize(n);
  for (int32_t j = 0; j < n; ++j) {
    const eiger_batch_join &q = joins[j];
    if (q.n_build < 0 || q.n_probe < 0) return fail(EIGER_ERR_INVALID_ARG, "batch: negative row count");
    if (q.n_build > EIGER_MAX_ROWS || q.n_probe > EIGER_MAX_ROWS)
      return fail(EIGER_ERR_TOO_LARGE, "batch: a join side has more than EIGER_MAX_ROWS = 2^32 - 2^16 rows");
    if ((q.n_build > 0 && (!q.build_keys || !q.build_payload)) || (q.n_probe > 0 && (!q.probe_keys || !q.probe_payload)))
      return fail(EIGER_ERR_INVALID_ARG, "batch: NULL column of a non-empty side");
    const size_t ks = dtype_size(kdt), ps = dtype_size(pdt);
    if (reinterpret_cast<uintptr_t>(q.build_keys) % ks || reinterpret_cast<uintptr_t>(q.probe_keys) % ks ||
        reinterpret_cast<uintptr_t>(q.build_payload) % ps || reinterpret_cast<uintptr_t>(q.probe_payload) % ps)
      return fail(EIGER_ERR_INVALID_ARG, "batch: column not aligned to its dtype");
    const eiger_batch_tune t = tune_for(tune, q.n_build);
    if (t.radix_bits > 0 && q.n_build > 0 && q.n_probe > 0) {
      BatchJoinDev &d = bp->joins[j];
      d = BatchJoinDev{q.build_keys, q.build_payload, q.probe_keys, q.probe_payload, uint64_t(q.n_build),
                       uint64_t(q.n_probe), bp->out_total, bp->arena_slots, 0};
      RadixJob job{};
      job.join = j;
      JoinArgs &a = job.args;
      a.bk = q.build_keys;
      a.bp = q.build_payload;
      a.pk = q.probe_keys;
      a.pp = q.probe_payload;
      a.nR = uint64_t(q.n_build);
      a.nS = uint64_t(q.n_probe);
      a.kdt = kdt;
      a.bpdt = pdt;
      a.ppdt = pdt;
      a.plan = eiger_plan_t{};
      a.plan.variant = EIGER_RADIX;
      a.plan.key_dtype = kdt;
      a.plan.radix_bits = t.radix_bits;
      a.plan.radix_passes = t.radix_bits > 8 ? 2 : 1;
      a.plan.load_factor = t.load_factor;
      a.cap = uint64_t(q.n_probe);
      Workspace dry(nullptr, 0);
      JoinCounters *unused = nullptr;
      if (int rc = run_join_variant(a, dry, &unused)) return rc;
      // the partitioned joins run one after another on the graph's stream, so
      // they share one workspace region sized for the largest
      job.ws_off = 0;
      job.ws_bytes = dry.used + 256;
      bp->radix_ws = std::max(bp->radix_ws, (job.ws_bytes + 255) & ~size_t(255));
      bp->radix.push_back(job);
      bp->out_total += uint64_t(q.n_probe);
      continue;
    }
    uint64_t slots = 64;
    const double want = static_cast<double>(q.n_build) / t.load_factor + 1.0;
    while (static_cast<double>(slots) < want) slots <<= 1;
    if (slots < 2 * static_cast<uint64_t>(q.n_build)) slots <<= 1;  // >= 2 rows per... keep an empty slot
    BatchJoinDev &d = bp->joins[j];
    d = BatchJoinDev{q.build_keys, q.build_payload, q.probe_keys, q.probe_payload, uint64_t(q.n_build),
                     uint64_t(q.n_probe), bp->out_total, bp->arena_slots, slots};
    bp->out_total += uint64_t(q.n_probe);
    bp->arena_slots += slots;
    for (uint64_t lo = 0; lo < uint64_t(q.n_build); lo += kBuildTile)
      bp->build.push_back(Item{uint32_t(j), 0, lo, std::min<uint64_t>(q.n_build, lo + kBuildTile)});
    if (q.n_build > 0)
      for (uint64_t lo = 0; lo < uint64_t(q.n_probe); lo += uint64_t(t.probe_tile))
        bp->probe.push_back(Item{uint32_t(j), 0, lo, std::min<uint64_t>(q.n_probe, lo + t.probe_tile)});
  }
  if (bp->build.size() >= (1ull << 32) || bp->probe.size() >= (1ull << 32))
    return fail(EIGER_ERR_TOO_LARGE, "batch: too many work items");
  return EIGER_OK;
}

struct BatchLayout {
  BatchJoinDev *joins;
  BatchState *state;
  Item *build, *probe;
  void *arena;
  char *radix_ws;
};

BatchLayout batch_layout(Workspace &ws, const BatchPlan &bp, size_t slot_bytes_) {
  BatchLayout L;
  L.joins = ws.take<BatchJoinDev>(bp.joins.size());
  L.state = ws.take<BatchState>(bp.joins.size());
  L.build = ws.take<Item>(std::max<size_t>(bp.build.size(), 1));
  L.probe = ws.take<Item>(std::max<size_t>(bp.probe.size(), 1));
  L.arena = ws.take<char>(bp.arena_slots * slot_bytes_);
  L.radix_ws = ws.take<char>(bp.radix_ws);
  return L;
}

struct BatchHandle {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n = 0;
  BatchState *state = nullptr;
};

template <typename K, typename P>
int enqueue_batch(const BatchPlan &bp, const BatchLayout &L, uint32_t *ob, uint32_t *op, hipStream_t s) {
  const int n = static_cast<int>(bp.joins.size());
  const unsigned nb = static_cast<unsigned>(bp.build.size()), np = static_cast<unsigned>(bp.probe.size());
  const unsigned cus = static_cast<unsigned>(device_cu_count());
  int rc;
  EIGER_LAUNCH("batch_reset", k_batch_reset, dim3((n + 255) / 256), dim3(256), 0, s, L.state, n);
  if ((rc = fill_u32(static_cast<uint32_t *>(L.arena), bp.arena_slots * sizeof(Slot<K, P>) / 4, kEmpty, s))) return rc;
  if (nb) {
    EIGER_LAUNCH("batch_minmax", k_batch_minmax<K>, dim3(std::min(nb, cus * 8)), dim3(256), 0, s, L.build, nb,
                 L.joins, L.state);
  }
  EIGER_LAUNCH("batch_plan", k_batch_plan, dim3((n + 255) / 256), dim3(256), 0, s, L.joins, L.state, n);
  if (nb) {
    Slot<K, P> *arena = static_cast<Slot<K, P> *>(L.arena);
    EIGER_LAUNCH("batch_build", (k_batch_build<K, P>), dim3(std::min(nb, cus * 8)), dim3(256), 0, s, L.build, nb,
                 L.joins, L.state, arena);
    EIGER_LAUNCH("batch_unique", (k_batch_unique<K, P>), dim3(std::min(nb, cus * 8)), dim3(256), 0, s, L.build, nb,
                 L.joins, L.state, arena);
  }
  if (np) {
    EIGER_LAUNCH("batch_probe", (k_batch_probe<K, P>), dim3(std::min(np, cus * 4)), dim3(kBNT), 0, s, L.probe, np,
                 L.joins, L.state, static_cast<const Slot<K, P> *>(L.arena), ob, op);
  }
  for (const RadixJob &job : bp.radix) {
    JoinArgs a = job.args;
    const uint64_t off = bp.joins[job.join].out_off;
    a.ob = ob + off;
    a.op = op + off;
    a.s = s;
    Workspace w(L.radix_ws + job.ws_off, job.ws_bytes);
    JoinCounters *c = nullptr;
    if ((rc = run_join_variant(a, w, &c))) return rc;
    EIGER_LAUNCH("batch_collect", k_batch_collect, dim3(1), dim3(64), 0, s, c, L.state + job.join, a.cap);
  }
  return EIGER_OK;
}

size_t batch_slot_bytes(int32_t kdt, int32_t pdt) { return slot_bytes(kdt, pdt); }

}  // namespace

}  // namespace eiger

using namespace eiger;

extern "C" int eiger_join_batch_workspace_size(const eiger_batch_join *joins, int32_t n_joins, int32_t key_dtype,
                                               int32_t payload_dtype, const eiger_batch_tune *tune, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "batch: bytes is NULL");
  BatchPlan bp;
  int rc = plan_batch(joins, n_joins, key_dtype, payload_dtype, tune, &bp);
  if (rc) return rc;
  Workspace ws(nullptr, 0);
  batch_layout(ws, bp, batch_slot_bytes(key_dtype, payload_dtype));
  *bytes = ws.used;
  return EIGER_OK;
}

extern "C" int eiger_join_batch_create(const eiger_batch_join *joins, int32_t n_joins, int32_t key_dtype,
                                       int32_t payload_dtype, const eiger_batch_tune *tune, uint32_t *out_build_rowid,
                                       uint32_t *out_probe_rowid, void *ws_ptr, size_t ws_bytes, void *stream,
                                       void **handle) {
  if (!handle) return fail(EIGER_ERR_INVALID_ARG, "batch: handle is NULL");
  *handle = nullptr;
  BatchPlan bp;
  int rc = plan_batch(joins, n_joins, key_dtype, payload_dtype, tune, &bp);
  if (rc) return rc;
  if (bp.out_total > 0 && (!out_build_rowid || !out_probe_rowid))
    return fail(EIGER_ERR_INVALID_ARG, "batch: NULL output arrays");
  Workspace ws(ws_ptr, ws_bytes);
  BatchLayout L = batch_layout(ws, bp, batch_slot_bytes(key_dtype, payload_dtype));
  if (!ws_ptr || ws.used > ws_bytes)
    return fail(EIGER_ERR_WORKSPACE, "batch: workspace too small (need " + std::to_string(ws.used) + " bytes)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // descriptors and work items, copied once (outside the graph)
  EIGER_HIP(hipMemcpyAsync(L.joins, bp.joins.data(), bp.joins.size() * sizeof(BatchJoinDev), hipMemcpyHostToDevice, s));
  if (!bp.build.empty())
    EIGER_HIP(hipMemcpyAsync(L.build, bp.build.data(), bp.build.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  if (!bp.probe.empty())
    EIGER_HIP(hipMemcpyAsync(L.probe, bp.probe.data(), bp.probe.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  EIGER_HIP(hipStreamSynchronize(s));
  auto *h = new BatchHandle();
  h->n = n_joins;
  h->state = L.state;
  // The caller's stream may be the legacy default stream, which cannot be
  // captured: record the graph on a private stream (default priority).
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipStreamCreateWithFlags");
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    delete h;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  const bool k64 = key_dtype == EIGER_INT64, p64 = payload_dtype == EIGER_INT64;
  if (!k64 && !p64) rc = enqueue_batch<int32_t, int32_t>(bp, L, out_build_rowid, out_probe_rowid, cs);
  else if (!k64 && p64) rc = enqueue_batch<int32_t, int64_t>(bp, L, out_build_rowid, out_probe_rowid, cs);
  else if (k64 && !p64) rc = enqueue_batch<int64_t, int32_t>(bp, L, out_build_rowid, out_probe_rowid, cs);
  else rc = enqueue_batch<int64_t, int64_t>(bp, L, out_build_rowid, out_probe_rowid, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    delete h;
    return rc ? rc : hip_fail(e, "hipStreamEndCapture");
  }
  h->graph = g;
  e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete h;
    return hip_fail(e, "hipGraphInstantiate");
  }
  *handle = h;
  return EIGER_OK;
}

extern "C" int eiger_join_batch_launch(void *handle, void *stream) {
  if (!handle) return fail(EIGER_ERR_INVALID_ARG, "batch: handle is NULL");
  auto *h = static_cast<BatchHandle *>(handle);
  EIGER_HIP(hipGraphLaunch(h->exec, static_cast<hipStream_t>(stream)));
  return EIGER_OK;
}

extern "C" int eiger_join_batch_results(void *handle, int64_t *counts, int64_t *checksums, int32_t *variants,
                                        uint32_t *flags, void *stream) {
  if (!handle) return fail(EIGER_ERR_INVALID_ARG, "batch: handle is NULL");
  auto *h = static_cast<BatchHandle *>(handle);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<BatchState> st(h->n);
  EIGER_HIP(hipMemcpyAsync(st.data(), h->state, sizeof(BatchState) * h->n, hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < h->n; ++j) {
    if (counts) counts[j] = static_cast<int64_t>(st[j].count);
    if (checksums) checksums[j] = static_cast<int64_t>(st[j].checksum);
    if (variants)
      variants[j] = st[j].variant == kVarDirect ? EIGER_DIRECT
                    : st[j].variant == kVarRadix ? EIGER_RADIX
                                                 : EIGER_GLOBAL_HASH;
    if (flags) flags[j] = st[j].flags;
  }
  return EIGER_OK;
}

extern "C" int eiger_join_batch_destroy(void *handle) {
  if (!handle) return EIGER_OK;
  auto *h = static_cast<BatchHandle *>(handle);
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  delete h;
  return EIGER_OK;
}
