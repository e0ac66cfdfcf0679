// md_kernels.hip -- velocity Verlet and a Verlet pair list on gfx950 (the
// molecular-dynamics use of the paper's section 4.2: Lennard-Jones forces,
// velocity Verlet, velocity rescaling, pair lists kept over several steps).
//
//   md_kick_drift   one thread per particle: v = lambda v + h f, x += dt v
//   md_kick         one thread per particle: v += h f, block sums of |v|^2
//   vl_drift        one thread per particle: largest |x - x_ref|^2 (atomic max
//                   on the bits of a non-negative double)
//   vl_decide       one thread: rebuild flag of this step, counters
//   vl_build        one wave per cell-list tile: every partner within the
//                   list cutoff, FP64, into a sliced column-major list
//   vl_refresh      one thread per sorted slot: frame position H (Hinv x - w)
//   vl_lj           one thread per sorted slot (row): FP64 LJ over the row,
//                   optional fused second half-kick, block partials
//   md_finalize     one block: fixed-order sum of the block partials
//
// All are HBM- or latency-bound except vl_lj, whose bound is the FP64 VALU
// work per listed partner and the gathers of partner positions.
#include "clmap_internal.h"

namespace clm {

namespace {

template <typename T>
__device__ __forceinline__ T ldu(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)(p);
#else
  return *p;
#endif
}

// 1/v to FP64 accuracy: hardware reciprocal estimate and one Newton step.
__device__ __forceinline__ double rcp64(double v) {
  double r = __builtin_amdgcn_rcp(v);
  const double e = __builtin_fma(-v, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Block of kMdBlock threads: sums of kMdPart doubles and one count into
// part[b * kMdPart + k] and pcount[b] (fixed order: waves, then wave 0..3).
__device__ __forceinline__ void block_partials(const double* acc, unsigned long long cnt,
                                               double* __restrict__ part,
                                               unsigned long long* __restrict__ pcount, int b) {
  __shared__ double red[kMdBlock / kWave][kMdPart];
  __shared__ unsigned long long redc[kMdBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[w][k] = s;
  }
  const unsigned long long c = wave_sum_u64(cnt);
  if (lane == 0) redc[w] = c;
  __syncthreads();
  if (threadIdx.x < kMdPart) {
    double s = 0.0;
    for (int q = 0; q < kMdBlock / kWave; ++q) s += red[q][threadIdx.x];
    part[(size_t)b * kMdPart + threadIdx.x] = s;
  }
  if (threadIdx.x == 0 && pcount) {
    unsigned long long s = 0;
    for (int q = 0; q < kMdBlock / kWave; ++q) s += redc[q];
    pcount[b] = s;
  }
}

// Blocks are dispatched to the 8 XCDs round-robin; give each XCD a
// contiguous range of rows (spatial neighbours share that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  if (nblk < 8) return b;
  const int per = nblk / 8, rem = nblk % 8;
  const int xcd = b % 8, k = b / 8;
  return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k;
}

}  // namespace

// ---------------------------------------------------------------- integrator
__global__ void __launch_bounds__(kMdBlock) md_kick_drift_kernel(double* __restrict__ x,
                                                                 double* __restrict__ v,
                                                                 const double* __restrict__ f,
                                                                 int64_t ncomp, double h, double dt,
                                                                 double target_ke,
                                                                 const double* __restrict__ ke) {
  const int64_t k = (int64_t)blockIdx.x * kMdBlock + threadIdx.x;
  if (k >= ncomp) return;
  double vk = v[k];
  if (target_ke > 0.0) vk = sqrt(target_ke / *ke) * vk;
  vk = vk + h * f[k];
  v[k] = vk;
  x[k] = x[k] + dt * vk;
}

__global__ void __launch_bounds__(kMdBlock) md_kick_kernel(double* __restrict__ v,
                                                           const double* __restrict__ f, int n,
                                                           int dim, double h,
                                                           double* __restrict__ part) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  double acc[kMdPart];
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) acc[k] = 0.0;
  if (i < n) {
    double q = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double va = v[(size_t)i * dim + a] + h * f[(size_t)i * dim + a];
      v[(size_t)i * dim + a] = va;
      q = a == 0 ? va * va : q + va * va;
    }
    acc[MP_KE] = q;
  }
  block_partials(acc, 0ull, part, nullptr, blockIdx.x);
}

// One block: fixed-order sums of nb partials.  energy = 2 eps sum(u) (every
// pair was seen from both ends), virial = 12 eps sum(f D D), count = pairs / 2,
// ke = mass / 2 sum |v|^2.
__global__ void __launch_bounds__(256) md_finalize_kernel(MdFinal F) {
  __shared__ double red[256];
  __shared__ unsigned long long redc[256];
  double keep[kMdPart];
  for (int k = 0; k < kMdPart; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < F.nb; b += 256) s += F.part[(size_t)b * kMdPart + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    keep[k] = red[0];
    __syncthreads();
  }
  unsigned long long c = 0;
  if (F.pcount)
    for (int b = threadIdx.x; b < F.nb; b += 256) c += F.pcount[b];
  redc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) redc[threadIdx.x] += redc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (F.energy) *F.energy = 2.0 * F.eps * keep[MP_E];
  if (F.virial) {
    const int d = F.dim;
    const int slot[3][3] = {{MP_W + 0, MP_W + 1, MP_W + 2},
                            {MP_W + 1, MP_W + 3, MP_W + 4},
                            {MP_W + 2, MP_W + 4, MP_W + 5}};
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) F.virial[a * d + b] = 12.0 * F.eps * keep[slot[a][b]];
  }
  if (F.count) *F.count = redc[0] / 2;
  if (F.ke_keep) {
    const double ke = 0.5 * F.mass * keep[MP_KE];
    *F.ke_keep = ke;
    if (F.ke) *F.ke = ke;
  }
}

// ---------------------------------------------------------------- Verlet list: maintenance
__global__ void __launch_bounds__(kMdBlock) vl_drift_kernel(const double* __restrict__ x,
                                                            const double* __restrict__ xref, int n,
                                                            int dim,
                                                            unsigned long long* __restrict__ maxd2) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  double m = 0.0;
  if (i < n) {
    double q = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double d = x[(size_t)i * dim + a] - xref[(size_t)i * dim + a];
      q = a == 0 ? d * d : q + d * d;
    }
    // a NaN displacement forces a rebuild
    m = q == q ? q : 1.0e300;
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0 && m > 0.0)
    atomicMax(maxd2, (unsigned long long)__double_as_longlong(m));
}

__global__ void vl_decide_kernel(VlFlags* __restrict__ fl, double lim2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double m = __longlong_as_double((long long)fl->maxd2);
  const bool g = fl->force != 0u || m > lim2;
  fl->gate = g ? 1u : 0u;
  fl->force = 0u;
  fl->maxd2 = 0ull;
  fl->updates += 1ull;
  if (g) {
    fl->rebuilds += 1ull;
    fl->entries = 0ull;
    fl->max_row = 0u;
  }
}

// Frame position of every sorted slot: r'' = H (Hinv x - w), the canonical
// wrap's operations without the floor; x_ref = x on a rebuild step.
__global__ void __launch_bounds__(kMdBlock) vl_refresh_kernel(VlRefresh A) {
  const int s = blockIdx.x * kMdBlock + threadIdx.x;
  if (s >= A.n) return;
  const uint32_t i = A.idx[s];
  const int4 w4 = A.wrap[s];
  const int w[3] = {w4.x, w4.y, w4.z};
  double r[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < A.dim; ++a) r[a] = A.x[(size_t)i * A.dim + a];
  double f[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < A.dim; ++a) {
    double acc = A.Hinv[a * 3 + 0] * r[0];
    acc = acc + A.Hinv[a * 3 + 1] * r[1];
    if (A.dim == 3) acc = acc + A.Hinv[a * 3 + 2] * r[2];
    f[a] = acc - (double)w[a];
  }
  double q[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < A.dim; ++a) {
    double acc = A.H[a * 3 + 0] * f[0];
    acc = acc + A.H[a * 3 + 1] * f[1];
    if (A.dim == 3) acc = acc + A.H[a * 3 + 2] * f[2];
    q[a] = acc;
  }
  A.pf[s] = make_double4(q[0], q[1], q[2], 0.0);
  if (*A.gate != 0u)
    for (int a = 0; a < A.dim; ++a) A.xref[(size_t)i * A.dim + a] = r[a];
}

// One wave per cell-list tile (<= 64 consecutive sorted particles of one
// cell row): every neighbouring cell of the full shell, every partner within
// the list cutoff (FP64 on the build's canonical positions), appended to the
// lane's row as (sorted partner << 5) | image code.  Row s lives in slice
// s / 64, column s % 64: entry k at list[(s / 64) cap 64 + k 64 + s % 64].
template <int DIM>
__global__ void __launch_bounds__(kWave) vl_build_kernel(VlBuild A) {
  if (*A.gate == 0u) return;
  const int ntiles = min((int)ldu(A.ntiles), A.max_tiles);
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  const Tile T = ldu(&A.tiles[t]);
  const int lane = threadIdx.x;
  const bool active = lane < (int)T.count;
  const uint32_t i = T.start + (uint32_t)(active ? lane : (int)T.count - 1);
  double ri[3];
  {
    const double4 r = A.r64[i];
    ri[0] = active ? r.x : 1e100;
    ri[1] = active ? r.y : 1e100;
    ri[2] = active ? r.z : 1e100;
  }
  uint32_t* row = A.list + (size_t)(i >> 6) * (size_t)A.cap * kWave + (i & 63u);
  uint32_t c = 0;
  const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
  const int cy = (int)(T.row % (uint32_t)ny);
  const int cz = DIM == 3 ? (int)(T.row / (uint32_t)ny) : 0;
  const int l = A.l, lx = A.lx;
  const int dzlo = DIM == 3 ? -l : 0, dzhi = DIM == 3 ? l : 0;
  for (int dz = dzlo; dz <= dzhi; ++dz) {
    for (int dy = -l; dy <= l; ++dy) {
      int uy = cy + dy, uz = cz + dz, py = 0, pz = 0;
      if (uy < 0) { uy += ny; py = -1; } else if (uy >= ny) { uy -= ny; py = 1; }
      if (DIM == 3) {
        if (uz < 0) { uz += nz; pz = -1; } else if (uz >= nz) { uz -= nz; pz = 1; }
      }
      const int rowbase = (uy + ny * uz) * nx;
      for (int ux = (int)T.cx0 - lx; ux <= (int)T.cx1 + lx; ++ux) {
        int uxw = ux, px = 0;
        if (uxw < 0) { uxw += nx; px = -1; } else if (uxw >= nx) { uxw -= nx; px = 1; }
        const int cell = rowbase + uxw;
        const uint32_t jb = ldu(&A.off[cell]), je = ldu(&A.off[cell + 1]);
        if (jb == je) continue;
        const int kc = kcode(px, py, pz);
        const double t0 = A.tK[kc * 4 + 0], t1 = A.tK[kc * 4 + 1], t2 = A.tK[kc * 4 + 2];
        for (uint32_t j = jb; j < je; ++j) {
          const double4 rj = ldu(&A.r64[j]);
          const double D0 = (rj.x - ri[0]) + t0;
          const double D1 = (rj.y - ri[1]) + t1;
          double d2 = D0 * D0 + D1 * D1;
          if (DIM == 3) {
            const double D2 = (rj.z - ri[2]) + t2;
            d2 = d2 + D2 * D2;
          }
          if (d2 <= A.rl2 && j != i) {
            if (c < (uint32_t)A.cap) row[(size_t)c * kWave] = (j << 5) | (uint32_t)kc;
            ++c;
          }
        }
      }
    }
  }
  unsigned long long stored = 0;
  if (active) {
    A.cnt[i] = c < (uint32_t)A.cap ? c : (uint32_t)A.cap;
    stored = c < (uint32_t)A.cap ? c : (uint32_t)A.cap;
    if (c > (uint32_t)A.cap) A.fl->overflow = 1u;
  }
  uint32_t cm = active ? c : 0u;
  for (int d = kWave / 2; d > 0; d >>= 1) cm = max(cm, (uint32_t)__shfl_xor((int)cm, d, kWave));
  stored = wave_sum_u64(stored);
  if (lane == 0) {
    atomicMax(&A.fl->max_row, cm);
    atomicAdd(&A.fl->entries, stored);
  }
}

// ---------------------------------------------------------------- Verlet list: forces
// One thread per row (sorted slot s): canonical FP64 displacement in the
// frame, membership d2 <= rc2, Lennard-Jones u and f, sums over the row.
template <int DIM, bool KICK, bool VIR>
__global__ void __launch_bounds__(kMdBlock) vl_lj_kernel(VlForce A) {
  __shared__ double tk[27 * 4];
  for (int k = threadIdx.x; k < 27 * 4; k += kMdBlock) tk[k] = A.tK[k];
  __syncthreads();
  const int nblk = (A.n + kMdBlock - 1) / kMdBlock;
  const int b = xcd_block(blockIdx.x, nblk);
  const int s = b * kMdBlock + threadIdx.x;
  double acc[kMdPart];
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) acc[k] = 0.0;
  unsigned long long npair = 0;
  if (s < A.n) {
    const double4 rs = A.pf[s];
    const uint32_t cnt = A.cnt[s];
    const uint32_t* __restrict__ row = A.list + (size_t)(s >> 6) * (size_t)A.cap * kWave + (s & 63);
    double G[3] = {0.0, 0.0, 0.0};
    double E = 0.0;
    double W[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double rc2 = A.rc2, s2 = A.s2;
    uint32_t k = 0;
    for (; k < cnt; ++k) {
      const uint32_t e = row[(size_t)k * kWave];
      const uint32_t j = e >> 5;
      const int kc = (int)(e & 31u);
      const double4 rj = A.pf[j];
      double D[3];
      D[0] = (rj.x - rs.x) + tk[kc * 4 + 0];
      D[1] = (rj.y - rs.y) + tk[kc * 4 + 1];
      double d2 = D[0] * D[0] + D[1] * D[1];
      if (DIM == 3) {
        D[2] = (rj.z - rs.z) + tk[kc * 4 + 2];
        d2 = d2 + D[2] * D[2];
      } else {
        D[2] = 0.0;
      }
      if (d2 <= rc2) {
        const double r = rcp64(d2);
        const double x = s2 * r;
        const double x3 = x * x * x;
        E += x3 * x3 - x3;
        const double f = (2.0 * x3 * x3 - x3) * r;
#pragma unroll
        for (int a = 0; a < DIM; ++a) G[a] += f * D[a];
        if constexpr (VIR) {
          W[0] += f * D[0] * D[0];
          W[1] += f * D[0] * D[1];
          W[3] += f * D[1] * D[1];
          if (DIM == 3) {
            W[2] += f * D[0] * D[2];
            W[4] += f * D[1] * D[2];
            W[5] += f * D[2] * D[2];
          }
        }
        ++npair;
      }
    }
    const uint32_t i = A.idx[s];
    const double m24 = -24.0 * A.eps;
    double q = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double Fa = m24 * G[a];
      A.forces[(size_t)i * DIM + a] = Fa;
      if constexpr (KICK) {
        const double va = A.v[(size_t)i * DIM + a] + A.h * Fa;
        A.v[(size_t)i * DIM + a] = va;
        q = a == 0 ? va * va : q + va * va;
      }
    }
    acc[MP_E] = E;
#pragma unroll
    for (int w = 0; w < 6; ++w) acc[MP_W + w] = W[w];
    acc[MP_KE] = q;
  }
  block_partials(acc, npair, A.part, A.pcount, b);
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_md_kick_drift(double* x, double* v, const double* f, int64_t ncomp, double h,
                                double dt, double target_ke, const double* ke, hipStream_t s) {
  if (ncomp == 0) return hipSuccess;
  md_kick_drift_kernel<<<blocks_for(ncomp, kMdBlock), kMdBlock, 0, s>>>(x, v, f, ncomp, h, dt,
                                                                        target_ke, ke);
  return hipGetLastError();
}

hipError_t launch_md_kick(double* v, const double* f, int n, int dim, double h, double* part,
                          hipStream_t s) {
  md_kick_kernel<<<blocks_for(n, kMdBlock), kMdBlock, 0, s>>>(v, f, n, dim, h, part);
  return hipGetLastError();
}

hipError_t launch_md_finalize(const MdFinal& F, hipStream_t s) {
  md_finalize_kernel<<<1, 256, 0, s>>>(F);
  return hipGetLastError();
}

hipError_t launch_vl_drift(const double* x, const double* xref, int n, int dim,
                           unsigned long long* maxd2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  vl_drift_kernel<<<blocks_for(n, kMdBlock), kMdBlock, 0, s>>>(x, xref, n, dim, maxd2);
  return hipGetLastError();
}

hipError_t launch_vl_decide(VlFlags* fl, double lim2, hipStream_t s) {
  vl_decide_kernel<<<1, 64, 0, s>>>(fl, lim2);
  return hipGetLastError();
}

hipError_t launch_vl_refresh(const VlRefresh& A, hipStream_t s) {
  if (A.n == 0) return hipSuccess;
  vl_refresh_kernel<<<blocks_for(A.n, kMdBlock), kMdBlock, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_vl_build(int dim, const VlBuild& A, hipStream_t s) {
  if (A.max_tiles <= 0) return hipSuccess;
  if (dim == 3)
    vl_build_kernel<3><<<A.max_tiles, kWave, 0, s>>>(A);
  else
    vl_build_kernel<2><<<A.max_tiles, kWave, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_vl_lj(int dim, bool kick, bool vir, const VlForce& A, hipStream_t s) {
  const unsigned nb = blocks_for(A.n, kMdBlock);
#define CLM_VL_LJ(D, K, V) vl_lj_kernel<D, K, V><<<nb, kMdBlock, 0, s>>>(A)
  if (dim == 3) {
    if (kick) { if (vir) CLM_VL_LJ(3, true, true); else CLM_VL_LJ(3, true, false); }
    else { if (vir) CLM_VL_LJ(3, false, true); else CLM_VL_LJ(3, false, false); }
  } else {
    if (kick) { if (vir) CLM_VL_LJ(2, true, true); else CLM_VL_LJ(2, true, false); }
    else { if (vir) CLM_VL_LJ(2, false, true); else CLM_VL_LJ(2, false, false); }
  }
#undef CLM_VL_LJ
  return hipGetLastError();
}

}  // namespace clm
