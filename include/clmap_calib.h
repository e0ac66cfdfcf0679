/*
 * clmap_calib.h -- device-rate microbenchmarks of libclmap.so.
 *
 * Not an operation of the method ("CellListMap.jl", Martinez, arXiv
 * 2202.06427): these calls measure what this device attains for the two
 * resources that bound the library's kernels, so that their achieved rates
 * can be compared with a measured ceiling as well as with the published one.
 * The cell sweep of the pair mapping (sections 2.3 and 2.8) is bound by
 * vector arithmetic, the cell-list build (section 2.6) by memory traffic.
 *
 *   CLM_CALIB_FMA_F32  FP32 fused multiply-adds on the vector ALU, built like
 *                      the rest of the library without packed FP32
 *                      instructions (one FMA per lane per instruction);
 *   CLM_CALIB_FMA_F64  FP64 fused multiply-adds;
 *   CLM_CALIB_COPY     a device-to-device copy in 16-byte vectors.
 *
 * Conventions are those of clmap.h (status codes, device pointers on the
 * context's device, caller-owned device memory).
 */
#ifndef CLMAP_CALIB_H
#define CLMAP_CALIB_H

#include "clmap.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum clm_calib_kind {
  CLM_CALIB_FMA_F32 = 0,
  CLM_CALIB_FMA_F64 = 1,
  CLM_CALIB_COPY = 2
} clm_calib_kind;

/* Device bytes that `dst_dev` must hold for an FMA kind (one value per
 * launched thread; the values themselves are meaningless).  For
 * CLM_CALIB_COPY *bytes receives 0 (the copy size is the caller's).
 * Errors: CLM_E_INVALID_ARG (unknown kind, bytes NULL). */
clm_status clm_calibrate_scratch_bytes(int kind, size_t* bytes);

/* Runs the microbenchmark `kind` once untimed, then `reps` times between two
 * events on the context's stream, and synchronizes that stream.
 *   FMA kinds: a fixed grid of independent FMA chains; `src_dev` is unused
 *     (may be NULL), `dst_dev` receives one value per thread and `bytes` is
 *     its size (>= clm_calibrate_scratch_bytes).
 *   CLM_CALIB_COPY: copies `bytes` (a multiple of 16) from `src_dev` to
 *     `dst_dev`, both 16-byte aligned and not overlapping.
 * Outputs (host): *ms the mean time of one launch in milliseconds, *work the
 * work of one launch: flops (2 per FMA) or bytes moved (read + written).
 * Errors: CLM_E_INVALID_ARG (unknown kind, reps < 1, NULL outputs, a copy
 * size or alignment that is not a multiple of 16), CLM_E_WORKSPACE (dst_dev
 * too small for an FMA kind), CLM_E_DEVICE. */
clm_status clm_calibrate(clm_context* ctx, int kind, const void* src_dev, void* dst_dev, size_t bytes,
                         int reps, double* ms, double* work);

#ifdef __cplusplus
}
#endif

#endif /* CLMAP_CALIB_H */
