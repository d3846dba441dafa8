// noalloc.hip -- eiger_join_noalloc: eiger_join whose scratch memory is a
// fixed device array of the library instead of a caller workspace, for callers
// that cannot allocate device memory.
//
// The array lives in the code object (file-scope __device__), so every GPU the
// library runs on holds its own copy until the process ends. In host code the
// array's name is only a stand-in: its device address is looked up once per
// device with hipGetSymbolAddress and that pointer is what the variants get as
// their workspace. Every call on one GPU shares that GPU's array, so calls that
// overlap on one GPU race; the variants clear whatever must start at zero
// (counters, tables) with their own fill kernels, as they do in a caller's
// workspace.
#include <mutex>

#include "variants.hpp"

namespace eiger {

int join_checked(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk, const eiger_column &pp,
                 const eiger_plan_t *plan, uint32_t *ob, uint32_t *op, int64_t cap, int64_t *out_count,
                 int64_t *out_checksum, void *ws_ptr, size_t ws_bytes, void *stream);
int check_join_call(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk, const eiger_column &pp,
                    const eiger_plan_t *plan, uint32_t *ob, uint32_t *op, int64_t cap, int64_t *out_count,
                    int64_t *out_checksum);
int join_workspace_bytes(const eiger_column &bk, const eiger_column &bp, const eiger_column &pk,
                         const eiger_column &pp, const eiger_plan_t *plan, size_t *bytes);

namespace {

static __device__ __align__(256) unsigned char scratch[EIGER_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (looked up once, with `dev` current).
int scratch_on(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EIGER_ERR_UNSUPPORTED, "eiger_join_noalloc: device index above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    EIGER_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(EIGER_ERR_HIP, "eiger_join_noalloc: hipGetSymbolAddress gave a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EIGER_OK;
}

}  // namespace
}  // namespace eiger

using namespace eiger;

extern "C" int eiger_join_noalloc(eiger_column build_keys, eiger_column build_payload, eiger_column probe_keys,
                                  eiger_column probe_payload, const eiger_plan_t *plan,
                                  uint32_t *out_build_rowid, uint32_t *out_probe_rowid, int64_t out_capacity,
                                  int64_t *out_count, int64_t *out_checksum, void *stream) {
  int rc = check_join_call(build_keys, build_payload, probe_keys, probe_payload, plan, out_build_rowid,
                           out_probe_rowid, out_capacity, out_count, out_checksum);
  if (rc) return rc;
  // the size check runs on the host only, before any HIP call
  size_t need = 0;
  if ((rc = join_workspace_bytes(build_keys, build_payload, probe_keys, probe_payload, plan, &need))) return rc;
  if (need > static_cast<size_t>(EIGER_NOALLOC_SCRATCH_BYTES))
    return fail(EIGER_ERR_TOO_LARGE, "eiger_join_noalloc: this plan needs " + std::to_string(need) +
                                         " bytes of scratch, above the fixed " +
                                         std::to_string(static_cast<size_t>(EIGER_NOALLOC_SCRATCH_BYTES)) +
                                         " (use eiger_join with a workspace)");
  int dev = 0;
  EIGER_HIP(hipGetDevice(&dev));
  if (stream) {
    int sdev = -1;
    EIGER_HIP(hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev));
    if (sdev != dev)
      return fail(EIGER_ERR_INVALID_ARG, "eiger_join_noalloc: the stream belongs to device " + std::to_string(sdev) +
                                             ", the current device is " + std::to_string(dev));
  }
  void *ws = nullptr;
  if ((rc = scratch_on(dev, &ws))) return rc;
  return join_checked(build_keys, build_payload, probe_keys, probe_payload, plan, out_build_rowid, out_probe_rowid,
                      out_capacity, out_count, out_checksum, ws, static_cast<size_t>(EIGER_NOALLOC_SCRATCH_BYTES),
                      stream);
}
