// join_wide.hip -- wide joins: the equi-join with the payload columns of both
// relations materialized for every result pair (the paper's "wide join",
// Section 5.2.1), by either of its two materialization strategies (Section 3.2):
//  GFUR  gather from the untransformed relations: join the keys with any
//        variant into (build row, probe row) pairs, then gather every payload
//        column of both sides from the caller's columns by row id;
//  GFTR  gather from the transformed relations (RADIX only): the payload
//        columns travel with the keys through the partitioning passes, the join
//        emits positions in the partitioned arrays, and each output block
//        gathers its payloads from one partition's contiguous range.
// Both give the same result; which is faster depends on the match ratio and
// the sizes (Section 5.2.3), so EIGER_MAT_AUTO chooses from the plan.
#include <cmath>
#include <string>

#include "variants.hpp"

namespace eiger {

int check_join_inputs_public(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                             const eiger_column &pp, const eiger_plan_t *plan);

namespace {

constexpr int kMaxCols = 4;            // payload columns per side
constexpr float kGftrMinMatch = 0.25f;  // AUTO: GFTR from this estimated match ratio up

// One side's materialization: sources (column c as its low / high 32-bit word
// arrays with a stride in words; hi null for 4-byte columns), optional map from
// emitted position to row id, and the output columns.
struct GatherSide {
  const uint32_t *rows;
  const uint32_t *lo[kMaxCols];
  const uint32_t *hi[kMaxCols];
  uint32_t stride[kMaxCols];
  void *dst[kMaxCols];
  int n;
};

__device__ __forceinline__ void gather_row(const GatherSide &g, uint32_t src, uint64_t t) {
  for (int c = 0; c < g.n; ++c) {
    const uint64_t at = uint64_t(src) * g.stride[c];
    const uint32_t lo = g.lo[c][at];
    if (g.hi[c]) {
      const uint64_t v = (uint64_t(g.hi[c][at]) << 32) | lo;
      static_cast<uint64_t *>(g.dst[c])[t] = v;
    } else {
      static_cast<uint32_t *>(g.dst[c])[t] = lo;
    }
  }
}

// Materialize result rows [0, min(count, cap)): payload words of both sides at
// the emitted (build, probe) indices, then (GFTR) the indices replaced by row ids.
__global__ void __launch_bounds__(256)
    k_wide_gather(uint32_t *__restrict__ ob, uint32_t *__restrict__ op, const JoinCounters *__restrict__ ctr,
                  uint64_t cap, GatherSide R, GatherSide S) {
  const uint64_t n = ctr->count < cap ? ctr->count : cap;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const uint32_t b = ob[t], p = op[t];
    gather_row(R, b, t);
    gather_row(S, p, t);
    if (R.rows) ob[t] = R.rows[b];
    if (S.rows) op[t] = S.rows[p];
  }
}

int check_cols(const eiger_column *cols, int32_t n, int64_t rows, const char *what) {
  if (n < 0 || n > kMaxCols)
    return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": between 0 and 4 payload columns");
  if (n > 0 && !cols) return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": NULL column array");
  for (int32_t c = 0; c < n; ++c) {
    if (cols[c].dtype != EIGER_INT32 && cols[c].dtype != EIGER_INT64)
      return fail(EIGER_ERR_DTYPE, std::string(what) + ": payload dtype must be EIGER_INT32 or EIGER_INT64");
    if (cols[c].n != rows) return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": a payload column's row count differs from its keys'");
    if (rows > 0 && !cols[c].data) return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": NULL payload column");
    if (rows > 0 && reinterpret_cast<uintptr_t>(cols[c].data) % dtype_size(cols[c].dtype))
      return fail(EIGER_ERR_INVALID_ARG, std::string(what) + ": payload column not aligned to its dtype");
  }
  return EIGER_OK;
}

// The columns as word lanes (GFTR carries them through the partitioning).
WordCols word_cols(const eiger_column *cols, int32_t n) {
  WordCols w{};
  for (int32_t c = 0; c < n; ++c) {
    const uint32_t *base = static_cast<const uint32_t *>(cols[c].data);
    if (cols[c].dtype == EIGER_INT64) {
      w.src[w.n] = base;
      w.stride[w.n++] = 2;
      w.src[w.n] = base ? base + 1 : nullptr;
      w.stride[w.n++] = 2;
    } else {
      w.src[w.n] = base;
      w.stride[w.n++] = 1;
    }
  }
  return w;
}

int resolve_mat(const eiger_plan_t *plan, int32_t mat, int32_t nb_cols, int32_t np_cols, int64_t n_probe,
                int32_t *out) {
  if (mat != EIGER_MAT_GFUR && mat != EIGER_MAT_GFTR && mat != EIGER_MAT_AUTO)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: materialize must be an eiger_materialize");
  if (mat == EIGER_MAT_GFTR && plan->variant != EIGER_RADIX)
    return fail(EIGER_ERR_UNSUPPORTED, "eiger_join_wide: GFTR needs a RADIX plan (it gathers from the "
                                       "partitioned relations)");
  if (mat == EIGER_MAT_AUTO) {
    const double match = n_probe > 0 ? static_cast<double>(plan->predicted_out) / static_cast<double>(n_probe) : 0.0;
    mat = (plan->variant == EIGER_RADIX && match >= kGftrMinMatch) ? EIGER_MAT_GFTR : EIGER_MAT_GFUR;
  }
  // without payload columns there is nothing to carry: both strategies coincide
  if (nb_cols == 0 && np_cols == 0) mat = EIGER_MAT_GFUR;
  *out = mat;
  return EIGER_OK;
}

JoinArgs key_join_args(const eiger_column &bk, const eiger_column &pk, const eiger_plan_t *plan, uint32_t *ob,
                       uint32_t *op, int64_t cap, void *stream) {
  JoinArgs a{};
  a.bk = bk.data;
  a.bp = bk.data;  // the keys stand in for the narrow join's payloads
  a.pk = pk.data;
  a.pp = pk.data;
  a.nR = static_cast<uint64_t>(bk.n);
  a.nS = static_cast<uint64_t>(pk.n);
  a.kdt = a.bpdt = a.ppdt = bk.dtype;
  a.plan = *plan;
  a.ob = ob;
  a.op = op;
  a.cap = static_cast<uint64_t>(cap);
  a.s = static_cast<hipStream_t>(stream);
  return a;
}

// Lays out (ws.base null: only sizes) and, with a base, runs the key join of
// the chosen strategy. *src* are filled for GFTR.
int run_wide(const JoinArgs &a, int32_t mat, const WordCols &wr, const WordCols &wp, Workspace &ws,
             JoinCounters **ctr, WideSource *srcR, WideSource *srcS) {
  if (mat == EIGER_MAT_GFTR) return run_radix_wide(a, wr, wp, ws, ctr, srcR, srcS);
  return run_join_variant(a, ws, ctr);
}

GatherSide gather_side(const eiger_column *cols, int32_t n, void *const *dst, const WideSource *src) {
  GatherSide g{};
  g.n = n;
  g.rows = src ? src->rows : nullptr;
  int w = 0;
  for (int32_t c = 0; c < n; ++c) {
    const bool wide = cols[c].dtype == EIGER_INT64;
    if (src) {  // transformed: one word array per lane, stride 1
      g.lo[c] = src->words[w];
      g.hi[c] = wide ? src->words[w + 1] : nullptr;
      g.stride[c] = 1;
    } else {
      const uint32_t *base = static_cast<const uint32_t *>(cols[c].data);
      g.lo[c] = base;
      g.hi[c] = wide ? base + 1 : nullptr;
      g.stride[c] = wide ? 2 : 1;
    }
    w += wide ? 2 : 1;
    g.dst[c] = dst ? dst[c] : nullptr;
  }
  return g;
}

int check_wide(const eiger_column &bk, const eiger_column *bcols, int32_t nbc, const eiger_column &pk,
               const eiger_column *pcols, int32_t npc, const eiger_plan_t *plan) {
  int rc = check_join_inputs_public(bk, bk, pk, pk, plan);
  if (rc) return rc;
  if ((rc = check_cols(bcols, nbc, bk.n, "build"))) return rc;
  return check_cols(pcols, npc, pk.n, "probe");
}

}  // namespace
}  // namespace eiger

using namespace eiger;

extern "C" int eiger_join_wide_workspace_size(const eiger_plan_t *plan, int32_t materialize, eiger_column build_keys,
                                              const eiger_column *build_cols, int32_t n_build_cols,
                                              eiger_column probe_keys, const eiger_column *probe_cols,
                                              int32_t n_probe_cols, size_t *bytes) {
  if (!bytes) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide_workspace_size: bytes is NULL");
  // sizing never reads data: dummy aligned addresses for the checks
  static const int64_t dummy[1] = {0};
  eiger_column bk = build_keys, pk = probe_keys;
  eiger_column bc[kMaxCols], pc[kMaxCols];
  if (bk.n > 0) bk.data = dummy;
  if (pk.n > 0) pk.data = dummy;
  if (n_build_cols < 0 || n_build_cols > kMaxCols || n_probe_cols < 0 || n_probe_cols > kMaxCols)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: between 0 and 4 payload columns a side");
  for (int32_t c = 0; c < n_build_cols; ++c) {
    if (!build_cols) return fail(EIGER_ERR_INVALID_ARG, "build: NULL column array");
    bc[c] = build_cols[c];
    if (bc[c].n > 0) bc[c].data = dummy;
  }
  for (int32_t c = 0; c < n_probe_cols; ++c) {
    if (!probe_cols) return fail(EIGER_ERR_INVALID_ARG, "probe: NULL column array");
    pc[c] = probe_cols[c];
    if (pc[c].n > 0) pc[c].data = dummy;
  }
  int rc = check_wide(bk, bc, n_build_cols, pk, pc, n_probe_cols, plan);
  if (rc) return rc;
  int32_t mat;
  if ((rc = resolve_mat(plan, materialize, n_build_cols, n_probe_cols, pk.n, &mat))) return rc;
  JoinArgs a = key_join_args(bk, pk, plan, nullptr, nullptr, 0, nullptr);
  Workspace ws(nullptr, 0);
  JoinCounters *ctr = nullptr;
  WideSource sr{}, sp{};
  if ((rc = run_wide(a, mat, word_cols(bc, n_build_cols), word_cols(pc, n_probe_cols), ws, &ctr, &sr, &sp)))
    return rc;
  *bytes = ws.used;
  return EIGER_OK;
}

extern "C" int eiger_join_wide(eiger_column build_keys, const eiger_column *build_cols, int32_t n_build_cols,
                               eiger_column probe_keys, const eiger_column *probe_cols, int32_t n_probe_cols,
                               const eiger_plan_t *plan, int32_t materialize, uint32_t *out_build_rowid,
                               uint32_t *out_probe_rowid, void *const *out_build_cols, void *const *out_probe_cols,
                               int64_t out_capacity, int64_t *out_count, int32_t *out_materialized, void *ws_ptr,
                               size_t ws_bytes, void *stream) {
  int rc = check_wide(build_keys, build_cols, n_build_cols, probe_keys, probe_cols, n_probe_cols, plan);
  if (rc) return rc;
  if (!out_count) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: out_count is NULL");
  if (out_capacity < 0) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: negative out_capacity");
  if (out_capacity > 0) {
    if (!out_build_rowid || !out_probe_rowid)
      return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: out_capacity > 0 needs both row-id output arrays");
    if ((n_build_cols > 0 && !out_build_cols) || (n_probe_cols > 0 && !out_probe_cols))
      return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: NULL output column array");
    for (int32_t c = 0; c < n_build_cols; ++c)
      if (!out_build_cols[c]) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: NULL build output column");
    for (int32_t c = 0; c < n_probe_cols; ++c)
      if (!out_probe_cols[c]) return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: NULL probe output column");
  } else if (out_build_rowid || out_probe_rowid) {
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: out_capacity == 0 takes NULL outputs (count only)");
  }
  int32_t mat;
  if ((rc = resolve_mat(plan, materialize, n_build_cols, n_probe_cols, probe_keys.n, &mat))) return rc;
  if (out_materialized) *out_materialized = mat;
  const WordCols wr = word_cols(build_cols, n_build_cols), wp = word_cols(probe_cols, n_probe_cols);
  JoinArgs a = key_join_args(build_keys, probe_keys, plan, out_capacity > 0 ? out_build_rowid : nullptr,
                             out_capacity > 0 ? out_probe_rowid : nullptr, out_capacity, stream);
  {
    Workspace dry(nullptr, 0);
    JoinCounters *unused = nullptr;
    WideSource sr{}, sp{};
    if ((rc = run_wide(a, mat, wr, wp, dry, &unused, &sr, &sp))) return rc;
    if (!ws_ptr || dry.used > ws_bytes)
      return fail(EIGER_ERR_WORKSPACE,
                  "eiger_join_wide: workspace too small (need " + std::to_string(dry.used) + " bytes)");
  }
  Workspace ws(ws_ptr, ws_bytes);
  JoinCounters *ctr = nullptr;
  WideSource sr{}, sp{};
  if ((rc = run_wide(a, mat, wr, wp, ws, &ctr, &sr, &sp))) return rc;
  hipStream_t s = a.s;
  if (out_capacity > 0 && build_keys.n > 0 && probe_keys.n > 0) {
    const bool tr = mat == EIGER_MAT_GFTR;
    const GatherSide gr = gather_side(build_cols, n_build_cols, out_build_cols, tr ? &sr : nullptr);
    const GatherSide gp = gather_side(probe_cols, n_probe_cols, out_probe_cols, tr ? &sp : nullptr);
    const uint64_t want = static_cast<uint64_t>(out_capacity);
    uint64_t g = (want + 255) / 256;
    const uint64_t gmax = uint64_t(device_cu_count()) * 16;
    if (g > gmax) g = gmax;
    EIGER_LAUNCH("wide_gather", k_wide_gather, dim3(unsigned(g ? g : 1)), dim3(256), 0, s, out_build_rowid,
                 out_probe_rowid, ctr, want, gr, gp);
  }
  JoinCounters host{};
  EIGER_HIP(hipMemcpyAsync(&host, ctr, sizeof(host), hipMemcpyDeviceToHost, s));
  EIGER_HIP(hipStreamSynchronize(s));
  if (host.flags & kFlagBuildOutOfRange)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_join_wide: a build key lies outside the plan's [build_min, build_max]");
  *out_count = static_cast<int64_t>(host.count);
  if (out_capacity > 0 && host.count > static_cast<uint64_t>(out_capacity))
    return fail(EIGER_ERR_CAPACITY, "eiger_join_wide: " + std::to_string(host.count) +
                                        " result rows exceed out_capacity " + std::to_string(out_capacity));
  return EIGER_OK;
}
