// kclosest_kernels.hip -- selection of the k closest pairs on gfx950 (paper
// section 3.2, Code 8).  The candidates come from a neighbour-list map at a
// threshold found with exact distance histograms; these kernels give each
// candidate its canonical squared distance and order them.
//
//   kc_inverse     one thread per sorted slot: caller index -> sorted slot
//   kc_keys        one thread per candidate: canonical d2 (minimum over the
//                  images K in {-1,0,1}^dim of the FP64 wrapped positions),
//                  record (d2 bits, i, j); padding records sort last
//   kc_sort_lds    one block: bitonic sort of up to kKcLdsRecords records in LDS
//   kc_sort_step   one compare-exchange stage of a bitonic sort in HBM
//   kc_output      the first k records to (i, j, d2), padding (-1, -1, +inf)
// All are latency-bound and small next to the sweeps that find the candidates.
#include "clmap_internal.h"

namespace clm {

namespace {

// Records order by (d2, i, j); d2 >= 0 so its bit pattern orders like its value.
__device__ __forceinline__ bool kc_less(const KcRecord& a, const KcRecord& b) {
  if (a.key != b.key) return a.key < b.key;
  if (a.i != b.i) return a.i < b.i;
  return a.j < b.j;
}

__device__ __forceinline__ void kc_order(KcRecord& a, KcRecord& b, bool up) {
  if (kc_less(b, a) == up) {
    const KcRecord t = a;
    a = b;
    b = t;
  }
}

}  // namespace

__global__ void __launch_bounds__(256) kc_inverse_kernel(const uint32_t* __restrict__ idx, int n,
                                                         uint32_t* __restrict__ inv) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s < n) inv[idx[s]] = (uint32_t)s;
}

__global__ void __launch_bounds__(256) kc_keys_kernel(KcKeys A) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= A.npow2) return;
  const unsigned long long cnt = *A.count;
  const int C = cnt < (unsigned long long)A.cap ? (int)cnt : A.cap;
  if (t >= C) {
    A.rec[t] = KcRecord{~0ull, ~0u, ~0u};
    return;
  }
  const uint32_t i = (uint32_t)A.pairs[2 * t], j = (uint32_t)A.pairs[2 * t + 1];
  const double4 ri = A.r64_x[A.inv_x[i]];
  const double4 rj = A.cross ? A.r64_y[A.inv_y[j]] : A.r64_x[A.inv_x[j]];
  double best = __longlong_as_double(0x7ff0000000000000ll);  // +inf
  const int kzlo = A.dim == 3 ? -1 : 0, kzhi = A.dim == 3 ? 1 : 0;
  for (int kz = kzlo; kz <= kzhi; ++kz)
    for (int ky = -1; ky <= 1; ++ky)
      for (int kx = -1; kx <= 1; ++kx) {
        const double* tk = &A.tK[kcode(kx, ky, kz) * 4];
        const double D0 = (rj.x - ri.x) + tk[0];
        const double D1 = (rj.y - ri.y) + tk[1];
        double d2 = D0 * D0 + D1 * D1;
        if (A.dim == 3) {
          const double D2 = (rj.z - ri.z) + tk[2];
          d2 = d2 + D2 * D2;
        }
        best = d2 < best ? d2 : best;
      }
  A.rec[t] = KcRecord{(unsigned long long)__double_as_longlong(best), i, j};
}

// One block of kKcLdsThreads threads sorts n (a power of two, <= kKcLdsRecords)
// records in LDS.
__global__ void __launch_bounds__(kKcLdsThreads) kc_sort_lds_kernel(KcRecord* __restrict__ rec, int n) {
  __shared__ KcRecord s[kKcLdsRecords];
  for (int t = threadIdx.x; t < n; t += kKcLdsThreads) s[t] = rec[t];
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = threadIdx.x; p < n / 2; p += kKcLdsThreads) {
        const int t = 2 * p - (p & (j - 1));  // bit j of t is clear
        kc_order(s[t], s[t + j], (t & k) == 0);
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < n; t += kKcLdsThreads) rec[t] = s[t];
}

__global__ void __launch_bounds__(256) kc_sort_step_kernel(KcRecord* __restrict__ rec, int n, int k,
                                                           int j) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n / 2) return;
  const int t = 2 * p - (p & (j - 1));
  KcRecord a = rec[t], b = rec[t + j];
  kc_order(a, b, (t & k) == 0);
  rec[t] = a;
  rec[t + j] = b;
}

__global__ void __launch_bounds__(256) kc_output_kernel(const KcRecord* __restrict__ rec, int k, int found,
                                                        int32_t* __restrict__ io, int32_t* __restrict__ jo,
                                                        double* __restrict__ d2o) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= k) return;
  if (t < found) {
    io[t] = (int32_t)rec[t].i;
    jo[t] = (int32_t)rec[t].j;
    d2o[t] = __longlong_as_double((long long)rec[t].key);
  } else {
    io[t] = -1;
    jo[t] = -1;
    d2o[t] = __longlong_as_double(0x7ff0000000000000ll);
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_kc_inverse(const uint32_t* idx, int n, uint32_t* inv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  kc_inverse_kernel<<<(n + 255) / 256, 256, 0, s>>>(idx, n, inv);
  return hipGetLastError();
}

hipError_t launch_kc_keys(const KcKeys& A, hipStream_t s) {
  kc_keys_kernel<<<(A.npow2 + 255) / 256, 256, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_kc_sort(KcRecord* rec, int n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  if (n <= kKcLdsRecords) {
    kc_sort_lds_kernel<<<1, kKcLdsThreads, 0, s>>>(rec, n);
    return hipGetLastError();
  }
  const unsigned nb = (unsigned)((n / 2 + 255) / 256);
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      kc_sort_step_kernel<<<nb, 256, 0, s>>>(rec, n, k, j);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t launch_kc_output(const KcRecord* rec, int k, int found, int32_t* io, int32_t* jo, double* d2o,
                            hipStream_t s) {
  kc_output_kernel<<<(k + 255) / 256, 256, 0, s>>>(rec, k, found, io, jo, d2o);
  return hipGetLastError();
}

}  // namespace clm
