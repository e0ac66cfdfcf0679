// device_util.h -- small wave-level helpers shared by the kernels of
// libclmap (gfx950, 64-lane wavefronts).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clm {

// A load through the constant address space with a wave-uniform address is
// emitted as a scalar (SMEM) load into SGPRs.  (The host compilation pass
// never runs device code; it only needs a body.)
template <typename T>
__device__ __forceinline__ T ldu(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)(p);
#else
  return *p;
#endif
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Rank of this lane among the set lanes of mask (lanes below it).
__device__ __forceinline__ int lane_rank(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// 1/v for FP64 pair terms: the hardware reciprocal refined by one Newton
// step (error about 1 ulp; one reciprocal serves both s^2/d^2 and the force
// factor instead of two IEEE divisions).  Membership never depends on it.
__device__ __forceinline__ double rcp64(double v) {
  double r = __builtin_amdgcn_rcp(v);
  const double e = __builtin_fma(-v, r, 1.0);
  return __builtin_fma(r, e, r);
}

}  // namespace clm
