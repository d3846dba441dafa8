// abi.hip -- the extern "C" surface: argument checks, planning, workspace sizing,
// variant dispatch, error strings and per-kernel event timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "variants.hpp"

namespace eiger {

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return EIGER_ERR_HIP;
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

// ------------------------------------------------------------------ profiling

namespace {

struct Pending {
  const char *name;
  hipEvent_t start, stop;
};

struct ProfTable {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  std::vector<eiger_kernel_time_t> rows;

  void resolve_locked() {
    for (auto &p : pending) {
      float ms = 0.f;
      if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
        auto it = std::find_if(rows.begin(), rows.end(),
                               [&](const eiger_kernel_time_t &r) { return std::strcmp(r.name, p.name) == 0; });
        if (it == rows.end()) {
          eiger_kernel_time_t r{};
          std::strncpy(r.name, p.name, sizeof(r.name) - 1);
          rows.push_back(r);
          it = rows.end() - 1;
        }
        it->launches += 1;
        it->total_ms += ms;
      }
      (void)hipEventDestroy(p.start);
      (void)hipEventDestroy(p.stop);
    }
    pending.clear();
  }
};

ProfTable &prof() {
  static ProfTable t;
  return t;
}

}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), stream_(s) {
  ProfTable &t = prof();
  if (!t.on) return;
  // no timing events inside a stream capture (they would become graph nodes)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&start_) != hipSuccess) {
    start_ = nullptr;
    return;
  }
  (void)hipEventRecord(start_, s);
}

ProfScope::~ProfScope() {
  if (!start_) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess) {
    (void)hipEventDestroy(start_);
    return;
  }
  (void)hipEventRecord(stop, stream_);
  ProfTable &t = prof();
  std::lock_guard<std::mutex> g(t.mu);
  t.pending.push_back(Pending{name_, start_, stop});
}

// ------------------------------------------------------------------ checks

namespace {

int check_column(const eiger_column &c, const char *what, bool key) {
  if (c.dtype != EIGER_INT32 && c.dtype != EIGER_INT64)
    return fail(EIGER_ERR_DTYPE, std::string(what) + ": dtype must be EIGER_INT32 or EIGER_INT64");
  if (c.n < 0) return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": negative row count");
  if (c.n > EIGER_MAX_ROWS)
    return fail(EIGER_ERR_TOO_LARGE, std::string(what) + ": more than EIGER_MAX_ROWS = 2^32 - 2^16 rows");
  if (c.n > 0 && !c.data) return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": data is NULL");
  if (c.n > 0 && reinterpret_cast<uintptr_t>(c.data) % dtype_size(c.dtype) != 0)
    return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": data is not aligned to its dtype");
  (void)key;
  return EIGER_OK;
}

int check_join_inputs(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                      const eiger_column &pp, const eiger_plan_t *plan) {
  int rc;
  if ((rc = check_column(bk, "build_keys", true))) return rc;
  if ((rc = check_column(bp, "build_payload", false))) return rc;
  if ((rc = check_column(pk, "probe_keys", true))) return rc;
  if ((rc = check_column(pp, "probe_payload", false))) return rc;
  if (bk.dtype != pk.dtype) return fail(EIGER_ERR_DTYPE, "build and probe key dtypes differ");
  if (bk.n != bp.n) return fail(EIGER_ERR_INVALID_ARG, "build_payload has a different row count than build_keys");
  if (pk.n != pp.n) return fail(EIGER_ERR_INVALID_ARG, "probe_payload has a different row count than probe_keys");
  if (!plan) return fail(EIGER_ERR_INVALID_ARG, "plan is NULL");
  if (plan->variant < EIGER_DIRECT || plan->variant > EIGER_SORT_MERGE)
    return fail(EIGER_ERR_INVALID_ARG, "plan.variant is not an eiger_variant");
  if (plan->key_dtype != bk.dtype) return fail(EIGER_ERR_DTYPE, "plan.key_dtype differs from the key columns");
  if (plan->variant == EIGER_DIRECT && bk.n > 0) {
    if (plan->build_max < plan->build_min)
      return fail(EIGER_ERR_INVALID_ARG, "DIRECT plan: build_max < build_min");
    const uint64_t range = static_cast<uint64_t>(plan->build_max) - static_cast<uint64_t>(plan->build_min) + 1;
    if (range == 0 || range > kDirectMaxRange)
      return fail(EIGER_ERR_UNSUPPORTED, "DIRECT plan: key range above 2^30 values");
  }
  if (plan->variant == EIGER_SORT_MERGE && bk.n > 0 && plan->build_max < plan->build_min)
    return fail(EIGER_ERR_INVALID_ARG, "SORT_MERGE plan: build_max < build_min");
  if (plan->variant != EIGER_DIRECT && plan->variant != EIGER_SORT_MERGE &&
      !(plan->load_factor > 0.f && plan->load_factor <= 0.9f))
    return fail(EIGER_ERR_INVALID_ARG, "plan.load_factor must be in (0, 0.9]");
  if (plan->variant == EIGER_RADIX) {
    if (plan->radix_bits < 1 || plan->radix_bits > 18)
      return fail(EIGER_ERR_INVALID_ARG, "plan.radix_bits must be in [1, 18]");
    if (plan->radix_passes < 1 || plan->radix_passes > 2)
      return fail(EIGER_ERR_INVALID_ARG, "plan.radix_passes must be 1 or 2");
  }
  if (plan->variant == EIGER_RADIX_CACHE && (plan->radix_bits < 1 || plan->radix_bits > kCacheMaxBits))
    return fail(EIGER_ERR_INVALID_ARG, "RADIX_CACHE plan.radix_bits must be in [1, 10]");
  return EIGER_OK;
}

JoinArgs make_args(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                   const eiger_column &pp, const eiger_plan_t *plan, uint32_t *ob, uint32_t *op,
                   int64_t cap, void *stream) {
  JoinArgs a{};
  a.bk = bk.data;
  a.bp = bp.data;
  a.pk = pk.data;
  a.pp = pp.data;
  a.nR = static_cast<uint64_t>(bk.n);
  a.nS = static_cast<uint64_t>(pk.n);
  a.kdt = bk.dtype;
  a.bpdt = bp.dtype;
  a.ppdt = pp.dtype;
  a.plan = *plan;
  a.ob = ob;
  a.op = op;
  a.cap = static_cast<uint64_t>(cap);
  a.s = static_cast<hipStream_t>(stream);
  return a;
}

int run_variant(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) {
  switch (a.plan.variant) {
    case EIGER_DIRECT: return run_direct(a, ws, ctr);
    case EIGER_GLOBAL_HASH: return run_global_hash(a, ws, ctr);
    case EIGER_RADIX: return run_radix(a, ws, ctr);
    case EIGER_SORT_MERGE: return run_sort_merge(a, ws, ctr);
    default: return run_radix_cache(a, ws, ctr);
  }
}

}  // namespace

int run_join_variant(const JoinArgs &a, Workspace &ws, JoinCounters **ctr) { return run_variant(a, ws, ctr); }

int check_join_inputs_public(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                             const eiger_column &pp, const eiger_plan_t *plan) {
  return check_join_inputs(bk, bp, pk, pp, plan);
}

namespace {

// ------------------------------------------------------------------ planning

constexpr double kHashTableBudget = 4.0 * 1024 * 1024 * 1024;  // bytes a GLOBAL_HASH table may take

uint64_t key_range(const eiger_stats_t &s) {
  if (s.n == 0) return 0;
  const uint64_t r = static_cast<uint64_t>(s.max) - static_cast<uint64_t>(s.min) + 1;
  return r == 0 ? UINT64_MAX : r;  // the whole 64-bit domain saturates
}

constexpr double kCacheRegionBudget = 1.5 * 1024 * 1024;  // bytes of one RADIX_CACHE table region

// Partition bits that bring one RADIX_CACHE table region under the L2 budget
// (8-byte build payloads assumed: the statistics do not carry payload widths).
int cache_bits_for(uint64_t n_build, int32_t kdt, float lf) {
  const double bytes = static_cast<double>(n_build) / lf * static_cast<double>(slot_bytes(kdt, EIGER_INT64));
  int bits = 1;
  while (bits < kCacheMaxBits && bytes / std::ldexp(1.0, bits) > kCacheRegionBudget) ++bits;
  return bits;
}

int radix_bits_for(uint64_t n_build, int32_t kdt, int32_t bpdt, float lf) {
  const RadixLimits lim = radix_limits(kdt, bpdt, lf);
  const double target = 0.6 * lim.max_build;  // headroom for uneven partitions
  int bits = 1;
  while (bits < 18 && static_cast<double>(n_build) / std::ldexp(1.0, bits) > target) ++bits;
  return bits;
}

void fill_common(const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out) {
  out->key_dtype = b.dtype;
  out->build_min = b.min;
  out->build_max = b.max;
  const double nd = std::max(std::max(b.ndv, p.ndv), 1.0);
  out->predicted_out = (b.n == 0 || p.n == 0)
                           ? 0
                           : static_cast<int64_t>(std::min(9.0e18, double(b.n) * double(p.n) / nd));
}

void rule_plan(const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out) {
  const uint64_t range = key_range(b);
  // Duplicated build keys share a home slot, so open-addressing clusters grow
  // with the copies of a key; those builds go to CSR runs (dense ranges) or to
  // LDS tables after partitioning.
  const bool duplicated = b.ndv < 0.9 * static_cast<double>(b.n);
  // DIRECT only for duplicated keys: with distinct keys a hash slot holds key,
  // row id and payload in one line, while a CSR probe reads three (offsets, row
  // id, payload); measured 1.1-2.3x slower than GLOBAL_HASH on dense distinct
  // builds of 2^16..2^26 rows
  if (b.n > 0 && duplicated && range <= kDirectMaxRange && range <= 4 * static_cast<uint64_t>(b.n)) {
    out->variant = EIGER_DIRECT;
    out->load_factor = 0.f;
    return;
  }
  const float lf = 0.5f;
  // payload width is not part of the statistics: size the slot for 8-byte payloads
  const double slot = b.dtype == EIGER_INT64 ? 32.0 : 16.0;
  const double table = static_cast<double>(hash_slots(static_cast<uint64_t>(b.n), lf)) * slot;
  // 16-byte slots (4-byte keys): the partitioned join overtakes the in-place
  // probe above a 1 GiB table (2^24 distinct build rows, a 1 GiB table: 8.3 vs
  // 8.2 ms; 2^26 rows, 4 GiB: 16.9 vs 12.3 ms, probe side 2^28 rows); 32-byte
  // slots keep the in-place probe up to the whole budget
  const double budget = b.dtype == EIGER_INT64 ? kHashTableBudget : kHashTableBudget / 4;
  if (table <= budget && (!duplicated || table <= 64.0 * 1024 * 1024)) {
    out->variant = EIGER_GLOBAL_HASH;
    out->load_factor = lf;
    return;
  }
  // Large probes: one pass over the probe side with L2-sized table regions
  // when a region fits at <= 2^10 partitions; otherwise LDS tables.
  const double region = table / std::ldexp(1.0, kCacheMaxBits);
  if (!duplicated && region <= kCacheRegionBudget) {
    out->variant = EIGER_RADIX_CACHE;
    out->load_factor = lf;
    out->radix_bits = cache_bits_for(static_cast<uint64_t>(b.n), b.dtype, lf);
    out->radix_passes = 1;
    return;
  }
  // LDS tables at a low load factor: short walks matter more than fan-out.
  out->variant = EIGER_RADIX;
  out->load_factor = 0.25f;
  // at most two passes of 8 bits (256 buckets each); larger partitions build
  // their LDS table in several chunks
  out->radix_bits = std::min(16, radix_bits_for(static_cast<uint64_t>(b.n), b.dtype, EIGER_INT64, out->load_factor));
  out->radix_passes = out->radix_bits > 8 ? 2 : 1;
  (void)p;
}

}  // namespace

}  // namespace eiger

using namespace eiger;

extern "C" const char *eiger_last_error(void) { return g_last_error.c_str(); }

extern "C" int eiger_version(void) { return 100; }

extern "C" int eiger_profile_enable(int on) {
  ProfTable &t = prof();
  std::lock_guard<std::mutex> g(t.mu);
  t.resolve_locked();
  t.rows.clear();
  t.on = on != 0;
  return EIGER_OK;
}

extern "C" int eiger_profile_read(eiger_kernel_time_t *out, int max_entries, int *n_out) {
  if (!n_out || max_entries < 0 || (max_entries > 0 && !out))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_profile_read: bad arguments");
  ProfTable &t = prof();
  std::lock_guard<std::mutex> g(t.mu);
  t.resolve_locked();
  const int n = static_cast<int>(t.rows.size());
  for (int i = 0; i < n && i < max_entries; ++i) out[i] = t.rows[i];
  *n_out = n;
  return EIGER_OK;
}

extern "C" int eiger_join_plan(const eiger_stats_t *build, const eiger_stats_t *probe, int32_t selector,
                               const eiger_plan_t *forced, eiger_plan_t *out) {
  if (!build || !probe || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_plan: NULL argument");
  if (build->dtype != probe->dtype) return fail(EIGER_ERR_DTYPE, "eiger_join_plan: key dtypes differ");
  if (build->dtype != EIGER_INT32 && build->dtype != EIGER_INT64)
    return fail(EIGER_ERR_DTYPE, "eiger_join_plan: unsupported key dtype");
  if (build->n < 0 || probe->n < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_plan: negative row count");
  eiger_plan_t p{};
  fill_common(*build, *probe, &p);
  switch (selector) {
    case EIGER_SEL_RULE:
      rule_plan(*build, *probe, &p);
      break;
    case EIGER_SEL_FIXED_HASH:
      p.variant = EIGER_GLOBAL_HASH;
      p.load_factor = 0.5f;
      break;
    case EIGER_SEL_FORCED:
      if (!forced) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_plan: EIGER_SEL_FORCED needs `forced`");
      if (forced->variant < EIGER_DIRECT || forced->variant > EIGER_SORT_MERGE)
        return fail(EIGER_ERR_INVALID_ARG, "eiger_join_plan: forced.variant is not an eiger_variant");
      p.variant = forced->variant;
      p.load_factor = forced->load_factor;
      p.radix_bits = forced->radix_bits;
      p.radix_passes = forced->radix_passes;
      if (p.variant != EIGER_DIRECT && !(p.load_factor > 0.f && p.load_factor <= 0.9f)) p.load_factor = 0.5f;
      if (p.variant == EIGER_RADIX) {
        if (p.radix_bits < 1 || p.radix_bits > 18)
          p.radix_bits = radix_bits_for(static_cast<uint64_t>(build->n), build->dtype, EIGER_INT64, p.load_factor);
        if (p.radix_passes < 1 || p.radix_passes > 2) p.radix_passes = p.radix_bits > 8 ? 2 : 1;
      }
      if (p.variant == EIGER_RADIX_CACHE) {
        if (p.radix_bits < 1 || p.radix_bits > kCacheMaxBits)
          p.radix_bits = cache_bits_for(static_cast<uint64_t>(build->n), build->dtype, p.load_factor);
        p.radix_passes = 1;
      }
      if (p.variant == EIGER_DIRECT && build->n > 0 && key_range(*build) > kDirectMaxRange)
        return fail(EIGER_ERR_UNSUPPORTED, "eiger_join_plan: DIRECT over a key range above 2^30 values");
      break;
    case EIGER_SEL_LEARNED: {
      bool in_domain = true;
      const int rc = learned_plan(*build, *probe, &p, &in_domain);
      if (rc) return rc;
      if (!in_domain) {
        rule_plan(*build, *probe, &p);
        p.flags |= EIGER_PLAN_RULE_FALLBACK;
      }
      break;
    }
    default:
      return fail(EIGER_ERR_INVALID_ARG, "eiger_join_plan: selector is not an eiger_selector");
  }
  *out = p;
  return EIGER_OK;
}

namespace eiger {

// Workspace bytes of a join (host only; the columns' data pointers are not read).
int join_workspace_bytes(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                         const eiger_column &pp, const eiger_plan_t *plan, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_workspace_size: bytes is NULL");
  // sizing never reads data: give the checks a dummy aligned address
  static const int64_t dummy[1] = {0};
  eiger_column cols[4] = {bk, bp, pk, pp};
  for (auto &c : cols)
    if (c.n > 0) c.data = dummy;
  int rc = check_join_inputs(cols[0], cols[1], cols[2], cols[3], plan);
  if (rc) return rc;
  JoinArgs a = make_args(cols[0], cols[1], cols[2], cols[3], plan, nullptr, nullptr, 0, nullptr);
  Workspace ws(nullptr, 0);
  JoinCounters *ctr = nullptr;
  if ((rc = run_variant(a, ws, &ctr))) return rc;
  *bytes = ws.used;
  return EIGER_OK;
}

}  // namespace eiger

extern "C" int eiger_join_workspace_size(const eiger_plan_t *plan, eiger_column build_keys,
                                         eiger_column build_payload, eiger_column probe_keys,
                                         eiger_column probe_payload, size_t *bytes) {
  return join_workspace_bytes(build_keys, build_payload, probe_keys, probe_payload, plan, bytes);
}

namespace eiger {

// eiger_join with the argument checks done: sizes the plan's workspace, runs
// the variant in (ws_ptr, ws_bytes), reads the counters back.
int join_checked(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk, const eiger_column &pp,
                 const eiger_plan_t *plan, uint32_t *ob, uint32_t *op, int64_t cap, int64_t *out_count,
                 int64_t *out_checksum, void *ws_ptr, size_t ws_bytes, void *stream) {
  JoinArgs a = make_args(bk, bp, pk, pp, plan, ob, op, cap, stream);
  int rc;
  {
    Workspace dry(nullptr, 0);
    JoinCounters *unused = nullptr;
    if ((rc = run_variant(a, dry, &unused))) return rc;
    if (!ws_ptr || dry.used > ws_bytes)
      return fail(EIGER_ERR_WORKSPACE,
                  "eiger_join: workspace too small (need " + std::to_string(dry.used) + " bytes)");
  }
  Workspace ws(ws_ptr, ws_bytes);
  JoinCounters *ctr = nullptr;
  if ((rc = run_variant(a, ws, &ctr))) return rc;
  JoinCounters host{};
  EIGER_HIP(hipMemcpyAsync(&host, ctr, sizeof(host), hipMemcpyDeviceToHost, a.s));
  EIGER_HIP(hipStreamSynchronize(a.s));
  if (host.flags & kFlagBuildOutOfRange)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join: a build key lies outside the plan's [build_min, build_max]");
  *out_count = static_cast<int64_t>(host.count);
  *out_checksum = static_cast<int64_t>(host.checksum);
  if (ob && host.count > static_cast<uint64_t>(cap))
    return fail(EIGER_ERR_CAPACITY, "eiger_join: " + std::to_string(host.count) +
                                        " result pairs exceed out_capacity " + std::to_string(cap));
  return EIGER_OK;
}

// Checks shared by the join entry points (everything but the workspace).
int check_join_call(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk, const eiger_column &pp,
                    const eiger_plan_t *plan, uint32_t *ob, uint32_t *op, int64_t cap, int64_t *out_count,
                    int64_t *out_checksum) {
  int rc = check_join_inputs(bk, bp, pk, pp, plan);
  if (rc) return rc;
  if (!out_count || !out_checksum) return fail(EIGER_ERR_INVALID_ARG, "eiger_join: out_count/out_checksum is NULL");
  if (cap < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_join: negative out_capacity");
  if ((ob == nullptr) != (op == nullptr))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join: give both output arrays or neither");
  if (cap > 0 && !ob) return fail(EIGER_ERR_INVALID_ARG, "eiger_join: out_capacity > 0 with NULL output arrays");
  return EIGER_OK;
}

}  // namespace eiger

extern "C" int eiger_join(eiger_column build_keys, eiger_column build_payload, eiger_column probe_keys,
                          eiger_column probe_payload, const eiger_plan_t *plan, uint32_t *out_build_rowid,
                          uint32_t *out_probe_rowid, int64_t out_capacity, int64_t *out_count,
                          int64_t *out_checksum, void *ws_ptr, size_t ws_bytes, void *stream) {
  int rc = check_join_call(build_keys, build_payload, probe_keys, probe_payload, plan, out_build_rowid,
                           out_probe_rowid, out_capacity, out_count, out_checksum);
  if (rc) return rc;
  return join_checked(build_keys, build_payload, probe_keys, probe_payload, plan, out_build_rowid, out_probe_rowid,
                      out_capacity, out_count, out_checksum, ws_ptr, ws_bytes, stream);
}
