// calib_api.cpp -- the C-ABI of the device-rate microbenchmarks of
// libclmap.so (declared in include/clmap_calib.h; kernels in
// calib_kernels.hip).
#include <cstdint>

#include "../../include/clmap_calib.h"
#include "clmap_state.h"

namespace {

constexpr int kCalibIters = 8192;  // FMA steps per chain

size_t fma_scratch(int kind) {
  return (size_t)kCalibBlocks * kCalibThreads * (kind == CLM_CALIB_FMA_F64 ? sizeof(double) : sizeof(float));
}

}  // namespace

extern "C" {

clm_status clm_calibrate_scratch_bytes(int kind, size_t* bytes) {
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  if (kind == CLM_CALIB_FMA_F32 || kind == CLM_CALIB_FMA_F64) {
    *bytes = fma_scratch(kind);
    return CLM_OK;
  }
  if (kind == CLM_CALIB_COPY) {
    *bytes = 0;
    return CLM_OK;
  }
  return fail(CLM_E_INVALID_ARG, "unknown calibration kind %d", kind);
}

clm_status clm_calibrate(clm_context* ctx, int kind, const void* src, void* dst, size_t bytes, int reps,
                         double* ms, double* work) {
  if (!ctx) return fail(CLM_E_INVALID_ARG, "context is NULL");
  if (!ms || !work) return fail(CLM_E_INVALID_ARG, "an output is NULL");
  if (reps < 1) return fail(CLM_E_INVALID_ARG, "reps must be >= 1");
  if (!dst) return fail(CLM_E_INVALID_ARG, "dst_dev is NULL");
  const bool fma = kind == CLM_CALIB_FMA_F32 || kind == CLM_CALIB_FMA_F64;
  if (!fma && kind != CLM_CALIB_COPY) return fail(CLM_E_INVALID_ARG, "unknown calibration kind %d", kind);
  double w = 0.0;
  if (fma) {
    if (bytes < fma_scratch(kind))
      return fail(CLM_E_WORKSPACE, "dst_dev has %zu bytes, %zu needed", bytes, fma_scratch(kind));
    w = 2.0 * kCalibChains * (double)kCalibIters * kCalibBlocks * kCalibThreads;
  } else {
    if (!src) return fail(CLM_E_INVALID_ARG, "src_dev is NULL");
    if (bytes % 16 != 0 || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
      return fail(CLM_E_INVALID_ARG, "copy size and addresses must be multiples of 16");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (bytes > 0 && a < b + bytes && b < a + bytes)
      return fail(CLM_E_INVALID_ARG, "source and destination overlap");
    w = 2.0 * (double)bytes;
  }
  CLM_HIP(hipSetDevice(ctx->device));
  auto launch = [&]() -> hipError_t {
    if (fma) return launch_calib_fma(kind == CLM_CALIB_FMA_F64, dst, kCalibIters, ctx->stream);
    return launch_calib_copy(src, dst, (int64_t)(bytes / 16), ctx->stream);
  };
  CLM_HIP(launch());
  hipEvent_t e0, e1;
  CLM_HIP(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CLM_E_DEVICE, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  e = hipEventRecord(e0, ctx->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(CLM_E_DEVICE, "calibration failed: %s", hipGetErrorString(e));
  *ms = (double)t / reps;
  *work = w;
  return CLM_OK;
}

}  // extern "C"
