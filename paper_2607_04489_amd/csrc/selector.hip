// selector.hip -- features, plan classes and the host-side MLP forward pass of
// the learned variant selector (EIGER_SEL_LEARNED).
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "mlp.hpp"
#include "variants.hpp"

namespace eiger {

namespace {

// The plan classes the selector chooses among.
struct ClassSpec {
  int32_t variant, bits, passes;
  float lf;
};
constexpr ClassSpec kClasses[kOut] = {
    {EIGER_DIRECT, 0, 0, 0.f},          {EIGER_GLOBAL_HASH, 0, 0, 0.25f}, {EIGER_GLOBAL_HASH, 0, 0, 0.5f},
    {EIGER_GLOBAL_HASH, 0, 0, 0.75f},   {EIGER_RADIX, 6, 1, 0.5f},        {EIGER_RADIX, 10, 2, 0.5f},
    {EIGER_RADIX, 12, 2, 0.25f},        {EIGER_RADIX, 14, 2, 0.25f},      {EIGER_RADIX, 16, 2, 0.25f},
    {EIGER_RADIX, 16, 2, 0.5f},         {EIGER_RADIX, 18, 2, 0.25f},      {EIGER_RADIX_CACHE, 2, 1, 0.5f},
    {EIGER_RADIX_CACHE, 4, 1, 0.3f},    {EIGER_RADIX_CACHE, 6, 1, 0.3f},  {EIGER_RADIX_CACHE, 8, 1, 0.3f},
    {EIGER_RADIX_CACHE, 10, 1, 0.3f},
};

// Predictions (log2 ms) of two GLOBAL_HASH load factors closer than log2(1.01)
// are taken as a tie: the selector then prefers the larger load factor, which
// halves the table's memory and its clear at no predicted cost.
constexpr float kTieLog2 = 0.0143552929770700f;

double range_of(const eiger_stats_t &s) {
  if (s.n <= 0) return 0.0;
  return static_cast<double>(static_cast<uint64_t>(s.max) - static_cast<uint64_t>(s.min)) + 1.0;
}

struct Model {
  std::mutex mu;
  bool loaded = false;
  bool has_domain = false;
  std::vector<float> params, mean, stdv, lo, hi;
};

Model &model() {
  static Model m;
  return m;
}

// Same arithmetic and order as the device forward (ordered fused sums).
void host_forward(const float *P, const float *x, float *y) {
  const MlpOffsets o;
  float h1[kHid], h2[kHid];
  for (int j = 0; j < kHid; ++j) {
    float acc = 0.f;
    for (int i = 0; i < kIn; ++i) acc = std::fmaf(x[i], P[o.W1 + i * kHid + j], acc);
    acc += P[o.b1 + j];
    h1[j] = acc < 0.f ? 0.f : acc;
  }
  for (int j = 0; j < kHid; ++j) {
    float acc = 0.f;
    for (int i = 0; i < kHid; ++i) acc = std::fmaf(h1[i], P[o.W2 + i * kHid + j], acc);
    acc += P[o.b2 + j];
    h2[j] = acc < 0.f ? 0.f : acc;
  }
  for (int j = 0; j < kOut; ++j) {
    float acc = 0.f;
    for (int i = 0; i < kHid; ++i) acc = std::fmaf(h2[i], P[o.W3 + i * kOut + j], acc);
    y[j] = acc + P[o.b3 + j];
  }
}

}  // namespace

void selector_features(const eiger_stats_t &b, const eiger_stats_t &p, float *out) {
  const double nR = std::max<double>(b.n, 0), nS = std::max<double>(p.n, 0);
  const double dR = std::max(b.ndv, 0.0), dS = std::max(p.ndv, 0.0);
  const double rR = range_of(b), rS = range_of(p);
  double overlap = 0.0;
  if (b.n > 0 && p.n > 0) {
    const double lo = static_cast<double>(std::max(b.min, p.min));
    const double hi = static_cast<double>(std::min(b.max, p.max));
    overlap = hi >= lo ? std::min(1.0, (hi - lo + 1.0) / std::max(rS, 1.0)) : 0.0;
  }
  const double f[kIn] = {
      std::log2(1.0 + nR),
      std::log2(1.0 + nS),
      std::log2(1.0 + dR),
      std::log2(1.0 + dS),
      std::log2(1.0 + rR),
      std::log2(1.0 + rS),
      b.dtype == EIGER_INT64 ? 1.0 : 0.0,
      std::min(1.0, dR / std::max(nR, 1.0)),
      std::min(1.0, dS / std::max(nS, 1.0)),
      std::max(0.0, std::log2(std::max(nR, 1.0) / std::max(dR, 1.0))),
      std::max(-64.0, std::min(0.0, std::log2(std::max(dR, 1.0) / std::max(rR, 1.0)))),
      overlap,
      std::log2(std::max(nS, 1.0) / std::max(nR, 1.0)),
      std::log2(1.0 + nR * nS / std::max(std::max(dR, dS), 1.0) * overlap),
      std::log2(1.0 + nS / std::max(dR, 1.0)),
      std::log2(1.0 + dS / std::max(dR, 1.0)),
  };
  for (int i = 0; i < kIn; ++i) out[i] = static_cast<float>(f[i]);
}

int class_plan(int32_t cls, const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out) {
  if (cls < 0 || cls >= kOut) return fail(EIGER_ERR_INVALID_ARG, "selector class out of range");
  const ClassSpec &c = kClasses[cls];
  if (c.variant == EIGER_DIRECT && b.n > 0 && range_of(b) > static_cast<double>(kDirectMaxRange))
    return fail(EIGER_ERR_UNSUPPORTED, "DIRECT class over a key range above 2^30 values");
  eiger_plan_t pl{};
  pl.variant = c.variant;
  pl.radix_bits = c.bits;
  pl.radix_passes = c.passes;
  pl.load_factor = c.lf;
  pl.key_dtype = b.dtype;
  pl.build_min = b.min;
  pl.build_max = b.max;
  const double nd = std::max(std::max(b.ndv, p.ndv), 1.0);
  pl.predicted_out = (b.n == 0 || p.n == 0) ? 0
                                           : static_cast<int64_t>(std::min(9.0e18, double(b.n) * double(p.n) / nd));
  *out = pl;
  return EIGER_OK;
}

int learned_plan(const eiger_stats_t &b, const eiger_stats_t &p, eiger_plan_t *out, bool *in_domain) {
  Model &m = model();
  std::vector<float> P, mean, stdv, lo, hi;
  bool has_domain;
  {
    std::lock_guard<std::mutex> g(m.mu);
    if (!m.loaded) return fail(EIGER_ERR_MODEL, "eiger_join_plan: no learned selector model is loaded");
    P = m.params;
    mean = m.mean;
    stdv = m.stdv;
    lo = m.lo;
    hi = m.hi;
    has_domain = m.has_domain;
  }
  float x[kIn], y[kOut];
  selector_features(b, p, x);
  *in_domain = true;
  if (has_domain)
    for (int i = 0; i < kIn; ++i)
      if (!(x[i] >= lo[i] && x[i] <= hi[i])) *in_domain = false;
  if (!*in_domain) return EIGER_OK;
  for (int i = 0; i < kIn; ++i) x[i] = (x[i] - mean[i]) / stdv[i];
  host_forward(P.data(), x, y);
  int best = -1;
  bool feasible[kOut];
  for (int c = 0; c < kOut; ++c) {
    eiger_plan_t tmp;
    feasible[c] = class_plan(c, b, p, &tmp) == EIGER_OK;
    if (!feasible[c]) continue;
    if (best < 0 || y[c] < y[best]) best = c;
  }
  if (best < 0) return fail(EIGER_ERR_MODEL, "learned selector: no feasible class");
  // Near-tie between GLOBAL_HASH load factors: take the largest load factor
  // (the smallest table) predicted within kTieLog2 of the best.
  if (kClasses[best].variant == EIGER_GLOBAL_HASH) {
    const int first = best;
    for (int c = 0; c < kOut; ++c)
      if (feasible[c] && kClasses[c].variant == EIGER_GLOBAL_HASH && kClasses[c].lf > kClasses[best].lf &&
          y[c] - y[first] <= kTieLog2)
        best = c;
  }
  set_error("");
  return class_plan(best, b, p, out);
}

}  // namespace eiger

using namespace eiger;

extern "C" int eiger_selector_features(const eiger_stats_t *build, const eiger_stats_t *probe, float *out) {
  if (!build || !probe || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_selector_features: NULL argument");
  selector_features(*build, *probe, out);
  return EIGER_OK;
}

extern "C" int eiger_selector_class_plan(int32_t cls, const eiger_stats_t *build, const eiger_stats_t *probe,
                                         eiger_plan_t *out) {
  if (!build || !probe || !out) return fail(EIGER_ERR_INVALID_ARG, "eiger_selector_class_plan: NULL argument");
  if (build->dtype != probe->dtype) return fail(EIGER_ERR_DTYPE, "eiger_selector_class_plan: key dtypes differ");
  return class_plan(cls, *build, *probe, out);
}

extern "C" int eiger_selector_load(const float *params, const float *feat_mean, const float *feat_std,
                                   const float *feat_lo, const float *feat_hi) {
  if (!params || !feat_mean || !feat_std) return fail(EIGER_ERR_INVALID_ARG, "eiger_selector_load: NULL argument");
  if (!feat_lo != !feat_hi)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_selector_load: give both feature bounds or neither");
  if (feat_lo)
    for (int i = 0; i < kIn; ++i)
      if (!(feat_lo[i] <= feat_hi[i]))
        return fail(EIGER_ERR_MODEL, "eiger_selector_load: feature bounds need lo <= hi (and no NaN)");
  for (int i = 0; i < kIn; ++i)
    if (!(feat_std[i] > 0.f) || !std::isfinite(feat_mean[i]))
      return fail(EIGER_ERR_MODEL, "eiger_selector_load: feature std must be > 0 and mean finite");
  for (int64_t i = 0; i < kParams; ++i)
    if (!std::isfinite(params[i])) return fail(EIGER_ERR_MODEL, "eiger_selector_load: non-finite parameter");
  Model &m = model();
  std::lock_guard<std::mutex> g(m.mu);
  m.params.assign(params, params + kParams);
  m.mean.assign(feat_mean, feat_mean + kIn);
  m.stdv.assign(feat_std, feat_std + kIn);
  m.has_domain = feat_lo != nullptr;
  if (feat_lo) {
    m.lo.assign(feat_lo, feat_lo + kIn);
    m.hi.assign(feat_hi, feat_hi + kIn);
  } else {
    m.lo.clear();
    m.hi.clear();
  }
  m.loaded = true;
  return EIGER_OK;
}

extern "C" int eiger_selector_loaded(void) {
  Model &m = model();
  std::lock_guard<std::mutex> g(m.mu);
  return m.loaded ? 1 : 0;
}
