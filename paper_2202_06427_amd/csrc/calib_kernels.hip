// calib_kernels.hip -- microbenchmarks for the denominators of the rooflines:
// the attainable vector FMA rate (FP32 without packed instructions, FP64) and
// the attainable HBM copy bandwidth of this device.  Not part of the method.
//
//   calib_fma_kernel<T>   kCalibThreads threads per block, kCalibChains
//                         independent FMA chains per thread, `iters` steps;
//                         each thread writes its sum (keeps the chains live)
//   calib_copy_kernel     grid-stride copy of 16-byte vectors, four in flight
#include "clmap_internal.h"

namespace clm {

template <typename T>
__global__ void __launch_bounds__(kCalibThreads) calib_fma_kernel(T* __restrict__ out, T b, T c, int iters) {
  const int t = blockIdx.x * kCalibThreads + threadIdx.x;
  T a[kCalibChains];
#pragma unroll
  for (int k = 0; k < kCalibChains; ++k) a[k] = (T)(t + k) * (T)1e-9;
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kCalibChains; ++k) a[k] = fma(a[k], b, c);
  }
  T s = (T)0;
#pragma unroll
  for (int k = 0; k < kCalibChains; ++k) s += a[k];
  out[t] = s;
}

__global__ void __launch_bounds__(256) calib_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {  // four loads in flight per thread
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_calib_fma(int fp64, void* out, int iters, hipStream_t s) {
  if (fp64)
    calib_fma_kernel<double><<<kCalibBlocks, kCalibThreads, 0, s>>>((double*)out, 0.9999999, 1e-7, iters);
  else
    calib_fma_kernel<float><<<kCalibBlocks, kCalibThreads, 0, s>>>((float*)out, 0.9999f, 1e-4f, iters);
  return hipGetLastError();
}

hipError_t launch_calib_copy(const void* src, void* dst, int64_t n16, hipStream_t s) {
  if (n16 == 0) return hipSuccess;
  const int64_t want = (n16 + 255) / 256;
  const unsigned blocks = (unsigned)(want < kCalibCopyBlocks ? want : kCalibCopyBlocks);
  calib_copy_kernel<<<blocks, 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

}  // namespace clm
