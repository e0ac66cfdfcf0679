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
#include "device_util.h"

namespace clm {

namespace {

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
    const double s = wave_sum_d(acc[k]);
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
      double va = v[(size_t)i * dim + a];
      if (f) {  // f == NULL: kinetic energy of v only
        va = va + h * f[(size_t)i * dim + a];
        v[(size_t)i * dim + a] = va;
      }
      q = a == 0 ? va * va : q + va * va;
    }
    acc[MP_KE] = q;
  }
  block_partials(acc, 0ull, part, nullptr, blockIdx.x);
}

// v = sqrt(target_ke / KE) v, KE the integrator's kept kinetic energy.
__global__ void __launch_bounds__(kMdBlock) md_rescale_kernel(double* __restrict__ v, int64_t ncomp,
                                                              double target_ke,
                                                              const double* __restrict__ ke) {
  const int64_t k = (int64_t)blockIdx.x * kMdBlock + threadIdx.x;
  if (k >= ncomp) return;
  v[k] = sqrt(target_ke / *ke) * v[k];
}

// One block: fixed-order sums of nb partials (each thread sums rows t,
// t + 256, ... of all components, then waves and the block combine in a fixed
// order).  energy = 2 eps sum(u) (every pair was seen from both ends), virial
// = 12 eps sum(f D D), count = pairs / 2, ke = mass / 2 sum |v|^2.
__global__ void __launch_bounds__(256) md_finalize_kernel(MdFinal F) {
  __shared__ double red[4][kMdPart];
  __shared__ unsigned long long redc[4];
  double acc[kMdPart];
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) acc[k] = 0.0;
  unsigned long long c = 0;
  for (int b = threadIdx.x; b < F.nb; b += 256) {
#pragma unroll
    for (int k = 0; k < kMdPart; ++k) acc[k] += F.part[(size_t)b * kMdPart + k];
    if (F.pcount) c += F.pcount[b];
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) {
    const double v = wave_sum_d(acc[k]);
    if (lane == 0) red[w][k] = v;
  }
  c = wave_sum_u64(c);
  if (lane == 0) redc[w] = c;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double keep[kMdPart];
  for (int k = 0; k < kMdPart; ++k) keep[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  const unsigned long long cnt = redc[0] + redc[1] + redc[2] + redc[3];
  if (F.energy) *F.energy = 2.0 * F.eps * keep[MP_E];
  if (F.virial) {
    const int d = F.dim;
    const int slot[3][3] = {{MP_W + 0, MP_W + 1, MP_W + 2},
                            {MP_W + 1, MP_W + 3, MP_W + 4},
                            {MP_W + 2, MP_W + 4, MP_W + 5}};
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) F.virial[a * d + b] = 12.0 * F.eps * keep[slot[a][b]];
  }
  if (F.count) *F.count = cnt / 2;
  if (F.ke_keep) {
    const double ke = 0.5 * F.mass * keep[MP_KE];
    *F.ke_keep = ke;
    if (F.ke) *F.ke = ke;
  }
}

// ---------------------------------------------------------------- Verlet list: maintenance
// Largest squared displacement since the last rebuild: per-block maxima
// (grid-stride over the particles, at most kDriftBlocks blocks), no atomics.
__global__ void __launch_bounds__(kMdBlock) vl_drift_kernel(const double* __restrict__ x,
                                                            const double* __restrict__ xref, int n,
                                                            int dim, double* __restrict__ bmax) {
  double m = 0.0;
  for (int i = blockIdx.x * kMdBlock + threadIdx.x; i < n; i += gridDim.x * kMdBlock) {
    double q = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double d = x[(size_t)i * dim + a] - xref[(size_t)i * dim + a];
      q = a == 0 ? d * d : q + d * d;
    }
    // a NaN displacement forces a rebuild
    m = fmax(m, q == q ? q : 1.0e300);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, kWave));
  __shared__ double wm[kMdBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = wm[0];
    for (int k = 1; k < kMdBlock / kWave; ++k) b = fmax(b, wm[k]);
    bmax[blockIdx.x] = b;
  }
}

// One block: the largest of the block maxima against (skin / 2)^2 decides
// this step's rebuild; counters.
__global__ void __launch_bounds__(256) vl_decide_kernel(const double* __restrict__ bmax, int nb,
                                                        double lim2, VlFlags* __restrict__ fl) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) m = fmax(m, bmax[b]);
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, kWave));
  __shared__ double wm[4];
  if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double mx = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
  const bool g = fl->force != 0u || mx > lim2;
  fl->gate = g ? 1u : 0u;
  fl->force = 0u;
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

// After a rebuild: row lengths (capped at the capacity), overflow flag, the
// longest row and the number of stored entries.
__global__ void __launch_bounds__(kMdBlock) vl_rowstats_kernel(uint32_t* __restrict__ cnt, int n,
                                                               int cap, VlFlags* __restrict__ fl,
                                                               const uint32_t* __restrict__ gate) {
  if (*gate == 0u) return;
  const int s = blockIdx.x * kMdBlock + threadIdx.x;
  uint32_t c = 0;
  if (s < n) {
    c = cnt[s];
    if (c > (uint32_t)cap) {
      fl->overflow = 1u;
      cnt[s] = (uint32_t)cap;
    }
  }
  uint32_t cm = c;
  unsigned long long st = c < (uint32_t)cap ? c : (uint32_t)cap;
  for (int d = kWave / 2; d > 0; d >>= 1) cm = max(cm, (uint32_t)__shfl_xor((int)cm, d, kWave));
  st = wave_sum_u64(st);
  __shared__ uint32_t wm[kMdBlock / kWave];
  __shared__ unsigned long long ws[kMdBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) {
    wm[threadIdx.x / kWave] = cm;
    ws[threadIdx.x / kWave] = st;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    unsigned long long t = 0;
    for (int k = 0; k < kMdBlock / kWave; ++k) {
      m = max(m, wm[k]);
      t += ws[k];
    }
    atomicMax(&fl->max_row, m);
    atomicAdd(&fl->entries, t);
  }
}

// One wave per (cell-list tile, neighbouring cell row): a tile is <= 64
// consecutive sorted particles of one cell row; blockIdx.y picks one of the
// (2 l + 1)^2 (3D) or 2 l + 1 (2D) rows of the full shell.  Every partner
// within the list cutoff (FP64 on the build's canonical positions) is
// appended to the lane's row as (sorted partner << 5) | image code: the lane
// counts its partners in the row, reserves space with one atomic add on its
// row length, and writes them in a second pass (so the order of a row's
// entries depends on the order in which its waves ran).  Layout (P lanes per
// row in the force kernel, cap a multiple of P): entry k of row s at
//   (s / 64) cap 64 + (k / P) 64 P + (s % 64) P + k % P,
// so that the P lanes of each of 64 / P consecutive rows read 64 consecutive
// words.
// Stores the WC entries of a chunk (WC = P: one row's P consecutive words).
template <int WC>
__device__ __forceinline__ void vl_store_chunk(uint32_t* p, const uint32_t* buf) {
#pragma unroll
  for (int q = 0; q < WC / 4; ++q)
    reinterpret_cast<uint4*>(p)[q] = make_uint4(buf[4 * q], buf[4 * q + 1], buf[4 * q + 2], buf[4 * q + 3]);
}

// WC > 0 (= P, 4..16): entries are gathered in buf, one chunk of P
// consecutive words of the row, and stored a chunk at a time (16-byte
// stores instead of 4-byte ones); the caller stores the last partial chunk.
template <int DIM, bool WRITE, int WC>
__device__ __forceinline__ uint32_t vl_scan_row(const VlBuild& A, const Tile& T, uint32_t i,
                                                const double* ri, int dz, int dy, uint32_t* row,
                                                uint32_t c, uint32_t* buf) {
  const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
  const int cy = (int)(T.row % (uint32_t)ny);
  const int cz = DIM == 3 ? (int)(T.row / (uint32_t)ny) : 0;
  const uint32_t lgP = (uint32_t)A.lgP, pm = (uint32_t)A.P - 1u;
  int uy = cy + dy, uz = cz + dz, py = 0, pz = 0;
  if (uy < 0) { uy += ny; py = -1; } else if (uy >= ny) { uy -= ny; py = 1; }
  if (DIM == 3) {
    if (uz < 0) { uz += nz; pz = -1; } else if (uz >= nz) { uz -= nz; pz = 1; }
  }
  const int rowbase = (uy + ny * uz) * nx;
  uint32_t found = 0;
  for (int ux = (int)T.cx0 - A.lx; ux <= (int)T.cx1 + A.lx; ++ux) {
    int uxw = ux, px = 0;
    if (uxw < 0) { uxw += nx; px = -1; } else if (uxw >= nx) { uxw -= nx; px = 1; }
    const int cell = rowbase + uxw;
    const uint32_t jb = ldu(&A.off[cell]), je = ldu(&A.off[cell + 1]);
    if (jb == je) continue;
    const int kc = kcode(px, py, pz);
    const double t0 = A.tK[kc * 4 + 0], t1 = A.tK[kc * 4 + 1], t2 = A.tK[kc * 4 + 2];
    auto test = [&](const double4& rj, uint32_t j) {
      const double D0 = (rj.x - ri[0]) + t0;
      const double D1 = (rj.y - ri[1]) + t1;
      double d2 = D0 * D0 + D1 * D1;
      if (DIM == 3) {
        const double D2 = (rj.z - ri[2]) + t2;
        d2 = d2 + D2 * D2;
      }
      if (d2 <= A.rl2 && j != i) {
        if (WRITE) {
          const uint32_t k = c + found;
          const uint32_t e = (j << 5) | (uint32_t)kc;
          if constexpr (WC > 0) {
#pragma unroll
            for (int q = 0; q < WC; ++q) buf[q] = (k & (uint32_t)(WC - 1)) == (uint32_t)q ? e : buf[q];
            if ((k & (uint32_t)(WC - 1)) == (uint32_t)(WC - 1) && k < (uint32_t)A.cap)
              vl_store_chunk<WC>(row + (size_t)(k >> lgP) * (kWave << lgP), buf);
          } else if (k < (uint32_t)A.cap) {
            row[(size_t)(k >> lgP) * (kWave << lgP) + (k & pm)] = e;
          }
        }
        ++found;
      }
    };
    // four partner records requested before any is tested
    uint32_t j = jb;
    for (; j + 4 <= je; j += 4) {
      const double4 a0 = ldu(&A.r64[j]), a1 = ldu(&A.r64[j + 1]);
      const double4 a2 = ldu(&A.r64[j + 2]), a3 = ldu(&A.r64[j + 3]);
      test(a0, j);
      test(a1, j + 1);
      test(a2, j + 2);
      test(a3, j + 3);
    }
    for (; j < je; ++j) test(ldu(&A.r64[j]), j);
  }
  return found;
}

// The grid is bounded (kBuildBlocks): when no rebuild is due the launch
// costs next to nothing; otherwise each block walks work items with a grid
// stride.  With A.split a work item is (tile, neighbour row): many waves per
// tile for lists of few particles, rows filled through atomic reservations
// (two passes).  Without it a work item is a whole tile: one pass, each
// lane owns its row and stores its length.
template <int DIM, int WC>
__global__ void __launch_bounds__(kBuildWaves * kWave) vl_build_kernel(VlBuild A) {
  if (*A.gate == 0u) return;
  const int ntiles = min((int)ldu(A.ntiles), A.max_tiles);
  const int side = 2 * A.l + 1;
  const int nrow = DIM == 3 ? side * side : side;
  const int per = A.split ? nrow : 1;
  const int64_t items = (int64_t)ntiles * per;
  const int lane = threadIdx.x & (kWave - 1);
  // the wave index, made visibly wave-uniform so partner records stay scalar loads
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int64_t w0 = (int64_t)blockIdx.x * kBuildWaves + wid;
  for (int64_t w = w0; w < items; w += (int64_t)gridDim.x * kBuildWaves) {
    const int t = (int)(w / per), r = (int)(w % per);
    const Tile T = ldu(&A.tiles[t]);
    const bool active = lane < (int)T.count;
    const uint32_t i = T.start + (uint32_t)(active ? lane : (int)T.count - 1);
    double ri[3];
    {
      const double4 p = A.r64[i];
      ri[0] = active ? p.x : 1e100;
      ri[1] = active ? p.y : 1e100;
      ri[2] = active ? p.z : 1e100;
    }
    uint32_t* row = A.list + (size_t)(i >> 6) * (size_t)A.cap * kWave + (size_t)(i & 63u) * A.P;
    if (A.split) {
      const int dy = r % side - A.l;
      const int dz = DIM == 3 ? r / side - A.l : 0;
      const uint32_t found = vl_scan_row<DIM, false, 0>(A, T, i, ri, dz, dy, row, 0, nullptr);
      if (active && found != 0) {
        const uint32_t c = atomicAdd(&A.cnt[i], found);
        if (c < (uint32_t)A.cap) vl_scan_row<DIM, true, 0>(A, T, i, ri, dz, dy, row, c, nullptr);
      }
    } else {
      uint32_t c = 0;
      uint32_t buf[WC > 0 ? WC : 1];
#pragma unroll
      for (int q = 0; q < (WC > 0 ? WC : 1); ++q) buf[q] = 0u;
      for (int rr = 0; rr < nrow; ++rr) {
        const int dy = rr % side - A.l;
        const int dz = DIM == 3 ? rr / side - A.l : 0;
        c += vl_scan_row<DIM, true, WC>(A, T, i, ri, dz, dy, row, c, buf);
      }
      if constexpr (WC > 0) {  // the last, partial chunk (its unused words are never read)
        const uint32_t k0 = c & ~(uint32_t)(WC - 1);
        if ((c & (uint32_t)(WC - 1)) != 0u && k0 < (uint32_t)A.cap)
          vl_store_chunk<WC>(row + (size_t)(k0 >> (uint32_t)A.lgP) * (kWave << A.lgP), buf);
      }
      if (active) A.cnt[i] = c;
    }
  }
}

// ---------------------------------------------------------------- Verlet list: forces
// P lanes per row (sorted slot s), each taking every P-th entry, four entries
// per iteration with their loads issued first: canonical FP64 displacement
// in the frame, membership d2 <= rc2, Lennard-Jones u and f.  The P partial
// sums of a row meet through shuffles; its first lane writes the force (and
// applies the second half-kick).
template <int DIM, bool VIR>
__device__ __forceinline__ void vl_pair(const double4& rs, const double4& rj, const double* tk,
                                        int kc, double rc2, double s2, double* G, double& E,
                                        double* W, unsigned long long& npair) {
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

template <int DIM, bool KICK, bool VIR, int P>
__global__ void __launch_bounds__(kMdBlock) vl_lj_kernel(VlForce A) {
  __shared__ double tk[27 * 4];
  for (int k = threadIdx.x; k < 27 * 4; k += kMdBlock) tk[k] = A.tK[k];
  __syncthreads();
  constexpr int kRows = kMdBlock / P;  // rows per block
  const int nblk = (A.n + kRows - 1) / kRows;
  const int b = xcd_block(blockIdx.x, nblk);
  const int s = b * kRows + (int)threadIdx.x / P;
  const int q = (int)threadIdx.x % P;
  double G[3] = {0.0, 0.0, 0.0};
  double E = 0.0;
  double W[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  unsigned long long npair = 0;
  double4 rs = make_double4(0.0, 0.0, 0.0, 0.0);
  if (s < A.n) {
    rs = A.pf[s];
    const int cnt = (int)A.cnt[s];
    const uint32_t* __restrict__ row =
        A.list + (size_t)(s >> 6) * (size_t)A.cap * kWave + (size_t)(s & 63) * P + q;
    constexpr size_t kStep = (size_t)kWave * P;
    const int T = cnt > q ? (cnt - q + P - 1) / P : 0;
    const double rc2 = A.rc2, s2 = A.s2;
    // groups of four entries; the partner positions of the next group are
    // requested before the current group is evaluated
    const int ng = T / 4;
    uint32_t e0[4], e1[4];
    double4 r0[4];
    if (ng > 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) e0[u] = row[(size_t)u * kStep];
#pragma unroll
      for (int u = 0; u < 4; ++u) r0[u] = A.pf[e0[u] >> 5];
    }
    for (int g = 0; g < ng; ++g) {
      double4 r1[4];
      const bool more = g + 1 < ng;
      if (more) {
#pragma unroll
        for (int u = 0; u < 4; ++u) e1[u] = row[(size_t)(4 * (g + 1) + u) * kStep];
#pragma unroll
        for (int u = 0; u < 4; ++u) r1[u] = A.pf[e1[u] >> 5];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        vl_pair<DIM, VIR>(rs, r0[u], tk, (int)(e0[u] & 31u), rc2, s2, G, E, W, npair);
      if (more) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          e0[u] = e1[u];
          r0[u] = r1[u];
        }
      }
    }
    for (int t = 4 * ng; t < T; ++t) {
      const uint32_t e = row[(size_t)t * kStep];
      vl_pair<DIM, VIR>(rs, A.pf[e >> 5], tk, (int)(e & 31u), rc2, s2, G, E, W, npair);
    }
  }
#pragma unroll
  for (int o = P / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) G[a] += __shfl_xor(G[a], o, kWave);
    E += __shfl_xor(E, o, kWave);
    if constexpr (VIR) {
#pragma unroll
      for (int w = 0; w < 6; ++w) W[w] += __shfl_xor(W[w], o, kWave);
    }
    npair += __shfl_xor(npair, o, kWave);
  }
  double acc[kMdPart];
#pragma unroll
  for (int k = 0; k < kMdPart; ++k) acc[k] = 0.0;
  unsigned long long np = 0;
  if (s < A.n && q == 0) {
    const uint32_t i = A.idx[s];
    const double m24 = -24.0 * A.eps;
    double qq = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double Fa = m24 * G[a];
      A.forces[(size_t)i * DIM + a] = Fa;
      if constexpr (KICK) {
        const double va = A.v[(size_t)i * DIM + a] + A.h * Fa;
        A.v[(size_t)i * DIM + a] = va;
        qq = a == 0 ? va * va : qq + va * va;
      }
    }
    acc[MP_E] = E;
#pragma unroll
    for (int w = 0; w < 6; ++w) acc[MP_W + w] = W[w];
    acc[MP_KE] = qq;
    np = npair;
  }
  block_partials(acc, np, A.part, A.pcount, b);
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

hipError_t launch_md_rescale(double* v, int64_t ncomp, double target_ke, const double* ke,
                             hipStream_t s) {
  if (ncomp == 0) return hipSuccess;
  md_rescale_kernel<<<blocks_for(ncomp, kMdBlock), kMdBlock, 0, s>>>(v, ncomp, target_ke, ke);
  return hipGetLastError();
}

hipError_t launch_md_finalize(const MdFinal& F, hipStream_t s) {
  md_finalize_kernel<<<1, 256, 0, s>>>(F);
  return hipGetLastError();
}

int vl_drift_blocks(int64_t n) {
  const int64_t b = (n + kMdBlock - 1) / kMdBlock;
  return (int)(b < 1 ? 1 : (b > kDriftBlocks ? kDriftBlocks : b));
}

hipError_t launch_vl_drift(const double* x, const double* xref, int n, int dim, double lim2,
                           double* bmax, VlFlags* fl, hipStream_t s) {
  const int nb = vl_drift_blocks(n);
  vl_drift_kernel<<<nb, kMdBlock, 0, s>>>(x, xref, n, dim, bmax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  vl_decide_kernel<<<1, 256, 0, s>>>(bmax, nb, lim2, fl);
  return hipGetLastError();
}

hipError_t launch_vl_rowstats(uint32_t* cnt, int n, int cap, VlFlags* fl, const uint32_t* gate,
                              hipStream_t s) {
  vl_rowstats_kernel<<<blocks_for(n, kMdBlock), kMdBlock, 0, s>>>(cnt, n, cap, fl, gate);
  return hipGetLastError();
}

hipError_t launch_vl_refresh(const VlRefresh& A, hipStream_t s) {
  if (A.n == 0) return hipSuccess;
  vl_refresh_kernel<<<blocks_for(A.n, kMdBlock), kMdBlock, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_vl_build(int dim, const VlBuild& A, hipStream_t s) {
  if (A.max_tiles <= 0) return hipSuccess;
  const int64_t side = 2 * (int64_t)A.l + 1;
  const int64_t items = (int64_t)A.max_tiles * (A.split ? (dim == 3 ? side * side : side) : 1);
  const int64_t want = (items + kBuildWaves - 1) / kBuildWaves;
  const unsigned nb = (unsigned)(want < kBuildBlocks ? want : kBuildBlocks);
  // one pass per tile: entries stored a row chunk (P words) at a time
  const int wc = !A.split && (A.P == 4 || A.P == 8 || A.P == 16) ? A.P : 0;
#define CLM_VL_BUILD(D)                                                     \
  switch (wc) {                                                             \
    case 4: vl_build_kernel<D, 4><<<nb, kBuildWaves * kWave, 0, s>>>(A); break;   \
    case 8: vl_build_kernel<D, 8><<<nb, kBuildWaves * kWave, 0, s>>>(A); break;   \
    case 16: vl_build_kernel<D, 16><<<nb, kBuildWaves * kWave, 0, s>>>(A); break; \
    default: vl_build_kernel<D, 0><<<nb, kBuildWaves * kWave, 0, s>>>(A); break;  \
  }
  if (dim == 3) {
    CLM_VL_BUILD(3)
  } else {
    CLM_VL_BUILD(2)
  }
#undef CLM_VL_BUILD
  return hipGetLastError();
}

int vl_rows_per_lane_group(int64_t n) {
  // enough waves to keep many partner gathers in flight: P n / 64 >= 32768
  // (measured on Neon at 10^6 atoms: P = 4 takes 2.6 ms per step, P = 1
  // 3.9 ms, P = 8 2.7 ms, P = 16 2.9 ms)
  int P = 1;
  while (P < 16 && (int64_t)P * n < (int64_t)32768 * kWave) P *= 2;
  return P;
}

hipError_t launch_vl_lj(int dim, bool kick, bool vir, int P, const VlForce& A, hipStream_t s) {
  const unsigned nb = blocks_for((int64_t)A.n * P, kMdBlock);
#define CLM_VL_LJ(D, K, V, PP) vl_lj_kernel<D, K, V, PP><<<nb, kMdBlock, 0, s>>>(A)
#define CLM_VL_P(D, K, V)                        \
  switch (P) {                                   \
    case 1: CLM_VL_LJ(D, K, V, 1); break;        \
    case 2: CLM_VL_LJ(D, K, V, 2); break;        \
    case 4: CLM_VL_LJ(D, K, V, 4); break;        \
    case 8: CLM_VL_LJ(D, K, V, 8); break;        \
    default: CLM_VL_LJ(D, K, V, 16); break;      \
  }
  if (dim == 3) {
    if (kick) { if (vir) CLM_VL_P(3, true, true) else CLM_VL_P(3, true, false) }
    else { if (vir) CLM_VL_P(3, false, true) else CLM_VL_P(3, false, false) }
  } else {
    if (kick) { if (vir) CLM_VL_P(2, true, true) else CLM_VL_P(2, true, false) }
    else { if (vir) CLM_VL_P(2, false, true) else CLM_VL_P(2, false, false) }
  }
#undef CLM_VL_P
#undef CLM_VL_LJ
  return hipGetLastError();
}

}  // namespace clm
