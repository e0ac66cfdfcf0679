// static_map.hip -- clm_map_static: the whole path (bin, sweep, reduce) of
// one map over a single or cross set with no device allocation and no
// caller workspace.  The cell list lives in `scratch`, a file-scope device
// array of kStaticScratchBytes that every GPU the library runs on holds until
// the process ends; its device address is looked up once per device with
// hipGetSymbolAddress (in host code the array's name is only a stand-in, so
// it is never passed to a kernel or a copy).
//
// Every call on one device uses that device's array and leaves the last
// call's contents in it; the build rewrites everything a map reads (counts
// are cleared by a fill kernel first), so no state carries over between
// calls.  Two calls that overlap on one device (different streams, or host
// threads) race on the array.
#include <mutex>

#include "clmap_state.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (nullptr: not yet)

// The device address of this device's `scratch`; `dev` must be current.
clm_status scratch_of(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CLM_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CLM_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    if (((uintptr_t)p & 255) != 0) return fail(CLM_E_DEVICE, "static scratch is not 256-byte aligned");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CLM_OK;
}

}  // namespace

extern "C" {

clm_status clm_map_static_max_bytes(size_t* bytes) {
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  *bytes = kStaticScratchBytes;
  return CLM_OK;
}

clm_status clm_map_static(clm_context* ctx, const clm_box* box, const double* x_dev, int64_t n_x,
                          const double* y_dev, int64_t n_y, clm_precision precision,
                          clm_map_kind kind, const clm_map_params* params, const clm_map_out* out) {
  if (!ctx || !box || !params || !out) return fail(CLM_E_INVALID_ARG, "NULL argument");
  size_t need = 0;
  clm_status s = clm_celllist_workspace_bytes(box, n_x, n_y, precision, &need);
  if (s != CLM_OK) return s;
  if (need > kStaticScratchBytes)
    return fail(CLM_E_CAPACITY,
                "clm_map_static: this cell list needs %zu bytes of scratch, the static scratch "
                "holds %zu (use clm_celllist_create with a workspace)",
                need, kStaticScratchBytes);
  CLM_HIP(hipSetDevice(ctx->device));
  void* ws = nullptr;
  s = scratch_of(ctx->device, &ws);
  if (s != CLM_OK) return s;
  clm_celllist cl;  // on the stack: nothing is allocated
  s = celllist_init(&cl, ctx, box, n_x, n_y, precision, ws, kStaticScratchBytes);
  if (s != CLM_OK) return s;
  cl.untimed = 1;
  s = celllist_build_gated(&cl, x_dev, y_dev, nullptr);
  if (s != CLM_OK) return s;
  return map_one(&cl, kind, params, out, true);
}

}  // extern "C"
