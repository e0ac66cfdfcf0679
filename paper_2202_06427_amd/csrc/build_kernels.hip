// build_kernels.hip -- cell-list construction on gfx950 (paper section 2.6:
// particles assigned to cells by their coordinates, with a contiguous copy of
// every cell's coordinates; section 2.8: cell side = cutoff / lcell).
//
// The build is a two-level counting sort whose counters all live in LDS:
//   count    per block of particles: canonical FP64 wrap into the primary
//            cell, the cell index written out, and an LDS histogram over
//            buckets of consecutive cells (a few thousand particles each)
//   scan     exclusive prefix of the (bucket, block) table, bucket-major:
//            every block's first slot in every bucket
//   bucket   per block: (index, cell) records to the bucket-ordered array,
//            slots from LDS counters seeded with the block's offsets
//   place    one block per bucket: LDS histogram over its cells, their
//            offsets (written to the cell-offset array), then every record
//            takes its slot from an LDS counter, its position is gathered,
//            wrapped again and written as the FP32 cell-local offset, the
//            FP64 wrapped position, the original index and the wrap integers
//   tiles    one wave per cell row: greedy work units of <= 64 particles
// Device-wide atomics on random addresses run at a fixed rate of a few tens
// of G/s on this chip whatever the XCD layout, so none are used; the one
// random access per particle is the gather of its 24-byte position, and
// every output of a bucket lands in one contiguous range.  Every kernel is
// HBM- or latency-bound; nothing here is a dense contraction.
#include <algorithm>

#include "clmap_internal.h"

namespace clm {

// Canonical wrap of one position (definitions in clmap.h).  Non-finite or
// absurdly large inputs are clamped so that every index stays in bounds.
__device__ __forceinline__ void wrap_one(const BuildGeom& g, const double* __restrict__ r,
                                         double* f, int* w, double* rw) {
  const int dim = g.dim;
  double s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      double acc = g.Hinv[a * 3 + 0] * r[0];
      acc = acc + g.Hinv[a * 3 + 1] * r[1];
      if (dim == 3) acc = acc + g.Hinv[a * 3 + 2] * r[2];
      s[a] = acc;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      double fl = floor(s[a]);
      double fa = s[a] - fl;
      if (fa >= 1.0) {
        fa = 0.0;
        fl = fl + 1.0;
      }
      if (!(fa >= 0.0 && fa < 1.0)) fa = 0.0;              // NaN input
      if (!(fl > -1073741824.0 && fl < 1073741824.0)) fl = 0.0;  // out of int range
      f[a] = fa;
      w[a] = (int)fl;
    } else {
      f[a] = 0.0;
      w[a] = 0;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      double acc = g.H[a * 3 + 0] * f[0];
      acc = acc + g.H[a * 3 + 1] * f[1];
      if (dim == 3) acc = acc + g.H[a * 3 + 2] * f[2];
      rw[a] = acc;
    } else {
      rw[a] = 0.0;
    }
  }
}

// Every build kernel takes a gate: a device flag that, when it reads 0, makes
// the kernel return at once (a rebuild decided on the device, with no host
// round trip).  NULL means always run.
__device__ __forceinline__ bool gate_closed(const uint32_t* gate) {
  return gate != nullptr && *gate == 0u;
}

__device__ __forceinline__ void cell_of(const BuildGeom& g, const double* f, int* c) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < g.dim) {
      int k = (int)(f[a] * (double)g.n[a]);
      c[a] = k >= g.n[a] ? g.n[a] - 1 : (k < 0 ? 0 : k);
    } else {
      c[a] = 0;
    }
  }
}

// Pass 1: cell of every particle, bucket histogram of the block in LDS.
__global__ void __launch_bounds__(kBinThreads) bin_count_kernel(const double* __restrict__ x, int n,
                                                                BuildGeom g, BinPlan P,
                                                                uint32_t* __restrict__ key,
                                                                uint32_t* __restrict__ hist,
                                                                const uint32_t* __restrict__ gate) {
  __shared__ uint32_t sh[kMaxBuckets];
  if (gate_closed(gate)) return;
  for (int b = threadIdx.x; b < P.nbk; b += kBinThreads) sh[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBinThreads * P.per;
#pragma unroll 4
  for (int k = 0; k < P.per; ++k) {
    const int64_t i = base + (int64_t)k * kBinThreads + threadIdx.x;
    if (i < n) {
      double r[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < g.dim; ++a) r[a] = x[(size_t)i * g.dim + a];
      double f[3], rw[3];
      int w[3], c[3];
      wrap_one(g, r, f, w, rw);
      cell_of(g, f, c);
      const uint32_t lin = (uint32_t)(c[0] + g.n[0] * (c[1] + g.n[1] * c[2]));
      key[i] = lin;
      atomicAdd(&sh[lin / (uint32_t)P.cpb], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < P.nbk; b += kBinThreads) hist[(size_t)b * P.nblk + blockIdx.x] = sh[b];
}

// Pass 2: records (position as given, index, cell) into bucket order; the
// records of one block and bucket are consecutive.
__global__ void __launch_bounds__(kBinThreads) bin_bucket_kernel(const double* __restrict__ x, int n,
                                                                 int dim, BinPlan P,
                                                                 const uint32_t* __restrict__ key,
                                                                 const uint32_t* __restrict__ hist,
                                                                 BinRec* __restrict__ rec,
                                                                 const uint32_t* __restrict__ gate) {
  __shared__ uint32_t cur[kMaxBuckets];
  if (gate_closed(gate)) return;
  for (int b = threadIdx.x; b < P.nbk; b += kBinThreads) cur[b] = hist[(size_t)b * P.nblk + blockIdx.x];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBinThreads * P.per;
#pragma unroll 4
  for (int k = 0; k < P.per; ++k) {
    const int64_t i = base + (int64_t)k * kBinThreads + threadIdx.x;
    if (i < n) {
      const uint32_t lin = key[i];
      BinRec R;
      R.x = x[(size_t)i * dim];
      R.y = x[(size_t)i * dim + 1];
      R.z = dim == 3 ? x[(size_t)i * dim + 2] : 0.0;
      R.i = (uint32_t)i;
      R.cell = lin;
      rec[atomicAdd(&cur[lin / (uint32_t)P.cpb], 1u)] = R;
    }
  }
}

// Exclusive scan over a block of kBinThreads threads; *total receives the
// block sum.  Every thread of the block must call it (it has barriers).
__device__ __forceinline__ uint32_t block_excl_scan_bin(uint32_t v, uint32_t* total) {
  constexpr int kWaves = kBinThreads / kWave;
  __shared__ uint32_t wsum[kWaves];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += t;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    pre += k < wid ? wsum[k] : 0u;
    tot += wsum[k];
  }
  *total = tot;
  __syncthreads();  // wsum is reused by the next call
  return pre + incl - v;
}

// Pass 3: one block per bucket.  Cell histogram and offsets in LDS (the
// offsets also go to the cell-offset array), then every record takes its
// slot from an LDS counter and is wrapped into its four outputs.  A bucket
// of at most kPlaceCap particles is assembled in LDS and written out with
// consecutive stores; a larger one (clustered input) is written in place.
__global__ void __launch_bounds__(kBinThreads) bin_place_kernel(
    int n, BuildGeom g, BinPlan P, int ncells, const uint32_t* __restrict__ hist,
    const BinRec* __restrict__ rec, uint32_t* __restrict__ off, float4* __restrict__ pos,
    double4* __restrict__ r64, uint32_t* __restrict__ idx, int4* __restrict__ wrap,
    const uint32_t* __restrict__ gate) {
  __shared__ uint32_t cnt[kMaxBucketCells];
  __shared__ uint32_t cur[kMaxBucketCells];
  __shared__ float4 s_pos[kPlaceCap];
  __shared__ double4 s_r64[kPlaceCap];
  __shared__ int4 s_wrap[kPlaceCap];
  __shared__ uint32_t s_idx[kPlaceCap];
  if (gate_closed(gate)) return;
  const int b = blockIdx.x;
  const uint32_t lo = hist[(size_t)b * P.nblk];
  const uint32_t hi = b + 1 < P.nbk ? hist[(size_t)(b + 1) * P.nblk] : (uint32_t)n;
  const int c0 = b * P.cpb;
  const int nc = min(P.cpb, ncells - c0);
  const bool staged = hi - lo <= (uint32_t)kPlaceCap;
  for (int c = threadIdx.x; c < nc; c += kBinThreads) cnt[c] = 0;
  __syncthreads();
  for (uint32_t s = lo + threadIdx.x; s < hi; s += kBinThreads)
    atomicAdd(&cnt[rec[s].cell - (uint32_t)c0], 1u);
  __syncthreads();
  uint32_t carry = lo;
  for (int base = 0; base < nc; base += kBinThreads) {
    const int c = base + threadIdx.x;
    const uint32_t v = c < nc ? cnt[c] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan_bin(v, &tot);
    if (c < nc) {
      cur[c] = carry + ex;
      off[c0 + c] = carry + ex;
    }
    carry += tot;
  }
  if (b == P.nbk - 1 && threadIdx.x == 0) off[ncells] = (uint32_t)n;
  __syncthreads();
  for (uint32_t s = lo + threadIdx.x; s < hi; s += kBinThreads) {
    const BinRec R = rec[s];
    const uint32_t dst = atomicAdd(&cur[R.cell - (uint32_t)c0], 1u);
    const double r[3] = {R.x, R.y, R.z};
    double f[3], rw[3];
    int w[3], c[3];
    wrap_one(g, r, f, w, rw);
    cell_of(g, f, c);
    // cell origin H (c / n) in FP64, then the FP32 offset from it
    double u[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) u[q] = (double)c[q] / (double)g.n[q];
    float o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double O = g.H[a * 3 + 0] * u[0] + g.H[a * 3 + 1] * u[1] + g.H[a * 3 + 2] * u[2];
      o[a] = a < g.dim ? (float)(rw[a] - O) : 0.0f;
    }
    const float4 po = make_float4(o[0], o[1], o[2], 0.0f);
    const double4 ro = make_double4(rw[0], rw[1], rw[2], 0.0);
    if (staged) {
      const uint32_t d = dst - lo;
      s_pos[d] = po;
      s_r64[d] = ro;
      s_wrap[d] = make_int4(w[0], w[1], w[2], (int)(R.cell - (uint32_t)c0));  // .w: the cell in the bucket
      s_idx[d] = R.i;
    } else {
      const int4 wo = make_int4(w[0], w[1], w[2], 0);
      pos[dst] = po;
      r64[dst] = ro;
      wrap[dst] = wo;
      idx[dst] = R.i;
    }
  }
  if (!staged) return;  // uniform over the block
  __syncthreads();
  // Within a cell of at most kSortCell particles the order is by wrapped
  // Cartesian x, then by original index: a rebuild from the same positions
  // gives the same order, and a split of a row's run of particles (the
  // sweep's tile halves) splits it along x.  (Larger cells keep the order
  // in which the placements above were made.)
  for (uint32_t d = threadIdx.x; d < hi - lo; d += kBinThreads) {
    const int4 wv = s_wrap[d];
    const uint32_t e = cur[wv.w] - lo, k = cnt[wv.w], st = e - k;
    uint32_t p = d;
    if (k <= (uint32_t)kSortCell) {
      const double xd = s_r64[d].x;
      const uint32_t id = s_idx[d];
      p = st;
      for (uint32_t q = st; q < e; ++q) {
        const double xq = s_r64[q].x;
        p += (xq < xd || (xq == xd && s_idx[q] < id)) ? 1u : 0u;
      }
    }
    pos[lo + p] = s_pos[d];
    r64[lo + p] = s_r64[d];
    wrap[lo + p] = make_int4(wv.x, wv.y, wv.z, 0);
    idx[lo + p] = s_idx[d];
  }
}

// ---------------------------------------------------------------- scan
// Exclusive prefix of n uint32 counts into out[0..n] (out[n] = total).
// Two passes: per-chunk sums, then per-chunk apply (each block adds up the
// sums of the chunks before it); a single chunk takes one pass.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

// Exclusive scan across the block; *total receives the block sum.  Every
// thread of the block must call it (it contains barriers).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  constexpr int kWaves = kScanThreads / kWave;
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t wpre[kWaves];
  __shared__ uint32_t tot;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t t = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += t;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int k = 0; k < kWaves; ++k) {
      wpre[k] = s;
      s += wsum[k];
    }
    tot = s;
  }
  __syncthreads();
  uint32_t res = wpre[wid] + incl - v;
  *total = tot;
  __syncthreads();  // the shared slots are reused by the next call
  return res;
}

__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(const uint32_t* __restrict__ in,
                                                                 int n, uint32_t* __restrict__ sums,
                                                                 const uint32_t* __restrict__ gate) {
  if (gate_closed(gate)) return;
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < (size_t)n) s += in[base + k];
  __shared__ uint32_t red[kScanThreads / kWave];
  for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kScanThreads / kWave; ++k) t += red[k];
    sums[blockIdx.x] = t;
  }
}

// Per chunk: its exclusive prefix, offset by the sum of the chunk sums
// before it (each block adds those up itself: at most a few thousand).
template <bool ONE>
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(const uint32_t* __restrict__ in,
                                                                  int n,
                                                                  const uint32_t* __restrict__ sums,
                                                                  uint32_t* __restrict__ out,
                                                                  const uint32_t* __restrict__ gate) {
  if (gate_closed(gate)) return;
  uint32_t pre = 0;
  if constexpr (!ONE) {
    uint32_t part = 0;
    for (int k = (int)threadIdx.x; k < (int)blockIdx.x; k += kScanThreads) part += sums[k];
    block_excl_scan(part, &pre);
  }
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < (size_t)n ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot) + pre;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < (size_t)n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = pre + tot;
}

// ---------------------------------------------------------------- tiles
// One wave per cell row (cy, cz): tiles of 64 consecutive sorted particles
// of the row (the last one of the rest), cut where a tile would span more
// than smax cells; a tile may begin or end inside a cell (the particles of a
// cell are ordered by x, so it splits the cell along x).  The lanes load
// the row's cell offsets (64 cells per load); the walk then runs on
// wave-uniform values read from the lanes, so a row costs one load round
// trip per 64 cells instead of one per cell.
constexpr int kTileRowsPerBlock = 256 / kWave;

template <bool EMIT>
__device__ uint32_t walk_row_seq(const uint32_t* __restrict__ off, const TileGeom& g, int row,
                                 Tile* __restrict__ tiles, uint32_t t0, int lane) {
  const int nx = g.n[0];
  const uint32_t* o = off + (size_t)row * nx;
  uint32_t nt = 0;
  bool open = false;  // a tile of cells c0..last (tcount particles from a0) is open
  int c0 = 0, last = 0;
  uint32_t a0 = 0, tcount = 0;
  auto emit = [&]() {
    if (EMIT && lane == 0 && t0 + nt < g.max_tiles)
      tiles[t0 + nt] = Tile{a0, (uint32_t)row, (uint16_t)tcount, (uint16_t)c0, (uint16_t)last, (uint16_t)g.job};
    ++nt;
    open = false;
  };
  for (int cs = 0; cs < nx; cs += kWave) {
    uint32_t av = 0u, bv = 0u;
    if (cs + lane < nx) {
      av = o[cs + lane];
      bv = o[cs + lane + 1];
    }
    const int nch = nx - cs < kWave ? nx - cs : kWave;
    for (int L = 0; L < nch; ++L) {
      const int cx = cs + L;
      const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)av, L);
      const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)bv, L) - a;
      if (cnt == 0u) continue;
      if (open && cx - c0 >= g.smax) emit();  // the open tile would span too many cells
      uint32_t s = a;  // next particle of the cell to place
      while (s < a + cnt) {
        if (!open) {
          open = true;
          c0 = cx;
          a0 = s;
          tcount = 0;
        }
        const uint32_t take = min(a + cnt - s, (uint32_t)kTileMax - tcount);
        tcount += take;
        last = cx;
        s += take;
        if (tcount == (uint32_t)kTileMax) emit();
      }
    }
  }
  if (open) emit();
  return nt;
}

// Cell (x index) of sorted particle a of a row whose cell offsets are
// o[0..nx]: the last cell c with o[c] <= a.
__device__ __forceinline__ int cell_of_particle(const uint32_t* __restrict__ o, int nx, uint32_t a) {
  int lo = 0, hi = nx - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (o[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The tiles of a row.  When no run of 64 consecutive particles of the row
// spans more than smax cells, they are the row's 64-particle chunks: one
// lane per tile finds its first and last cells by binary search (the walk
// above gives the same tiles, one cell at a time); otherwise the walk.
template <bool EMIT>
__device__ uint32_t walk_row(const uint32_t* __restrict__ off, const TileGeom& g, int row,
                             Tile* __restrict__ tiles, uint32_t t0, int lane) {
  const int nx = g.n[0];
  const uint32_t* o = off + (size_t)row * nx;
  const uint32_t rs = o[0], re = o[nx];
  const uint32_t nt = (re - rs + (uint32_t)kTileMax - 1) / (uint32_t)kTileMax;
  bool wide = false;  // a chunk spans more than smax cells
  for (uint32_t tb = 0; tb < nt; tb += kWave) {
    const uint32_t t = tb + (uint32_t)lane;
    if (t < nt) {
      const uint32_t a0 = rs + t * (uint32_t)kTileMax;
      const uint32_t a1 = min(a0 + (uint32_t)kTileMax, re) - 1u;
      wide |= cell_of_particle(o, nx, a1) - cell_of_particle(o, nx, a0) >= g.smax;
    }
  }
  if (__builtin_amdgcn_ballot_w64(wide) != 0ull) return walk_row_seq<EMIT>(off, g, row, tiles, t0, lane);
  if (EMIT) {
    for (uint32_t tb = 0; tb < nt; tb += kWave) {
      const uint32_t t = tb + (uint32_t)lane;
      if (t < nt && t0 + t < g.max_tiles) {
        const uint32_t a0 = rs + t * (uint32_t)kTileMax;
        const uint32_t a1 = min(a0 + (uint32_t)kTileMax, re) - 1u;
        tiles[t0 + t] = Tile{a0, (uint32_t)row, (uint16_t)(a1 - a0 + 1u), (uint16_t)cell_of_particle(o, nx, a0),
                             (uint16_t)cell_of_particle(o, nx, a1), (uint16_t)g.job};
      }
    }
  }
  return nt;
}

__global__ void __launch_bounds__(256) tiles_count_kernel(const uint32_t* __restrict__ off, TileGeom g,
                                                          uint32_t* __restrict__ row_tiles,
                                                          const uint32_t* __restrict__ gate) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int row = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kTileRowsPerBlock + threadIdx.x / kWave));
  if (row >= g.nrows || gate_closed(gate)) return;
  const uint32_t nt = walk_row<false>(off, g, row, nullptr, 0, lane);
  if (lane == 0) row_tiles[row] = nt;
}
__global__ void __launch_bounds__(256) tiles_emit_kernel(const uint32_t* __restrict__ off, TileGeom g,
                                                         const uint32_t* __restrict__ row_off,
                                                         Tile* __restrict__ tiles,
                                                         const uint32_t* __restrict__ gate) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int row = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kTileRowsPerBlock + threadIdx.x / kWave));
  if (row >= g.nrows || gate_closed(gate)) return;
  walk_row<true>(off, g, row, tiles, row_off[row], lane);
}

// ---------------------------------------------------------------- small helpers
__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v, const uint32_t* __restrict__ gate) {
  if (gate_closed(gate)) return;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, size_t n, unsigned long long v, const uint32_t* __restrict__ gate) {
  if (gate_closed(gate)) return;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_f64_kernel(double* p, size_t n, double v, const uint32_t* __restrict__ gate) {
  if (gate_closed(gate)) return;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Sorted FP32 copy of the velocities and the largest |component| (as float
// bits; all values are >= 0 so the unsigned order is the float order).
__global__ void __launch_bounds__(256) gather_vel_kernel(const double* __restrict__ v, int dim,
                                                         const uint32_t* __restrict__ idx, int n,
                                                         float4* __restrict__ v32,
                                                         unsigned int* __restrict__ vmax_bits) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.0f;
  if (s < n) {
    uint32_t i = idx[s];
    float c[3] = {0.0f, 0.0f, 0.0f};
    for (int a = 0; a < dim; ++a) {
      double va = v[(size_t)i * dim + a];
      c[a] = (float)va;
      double av = fabs(va);
      // round the magnitude up so that the bound covers the FP64 value
      float af = (float)av;
      if ((double)af < av) af = __int_as_float(__float_as_int(af) + 1);
      if (!(af <= 3.0e38f)) af = 3.0e38f;
      m = fmaxf(m, af);
    }
    v32[s] = make_float4(c[0], c[1], c[2], 0.0f);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0 && m > 0.0f) atomicMax(vmax_bits, __float_as_uint(m));
}

// Weights of a weighted map into the unused 4th components of the sorted
// records (FP32 for the FP32 sweep, FP64 for the FP64 sweep and re-tests).
__global__ void __launch_bounds__(256) gather_weights_kernel(const double* __restrict__ w,
                                                             const uint32_t* __restrict__ idx, int n,
                                                             float4* __restrict__ pos,
                                                             double4* __restrict__ r64) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const double v = w[idx[s]];
  pos[s].w = (float)v;
  r64[s].w = v;
}

// ---------------------------------------------------------------- extrema
// Per-block minima and maxima of each coordinate (grid stride, at most
// kExtremaBlocks blocks), then one block combines them: the bounding box of
// a non-periodic computation (paper section 4.1).
__global__ void __launch_bounds__(256) extrema_kernel(const double* __restrict__ x, int64_t n, int dim,
                                                      double* __restrict__ part) {
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  double lo[3] = {inf, inf, inf}, hi[3] = {-inf, -inf, -inf};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    for (int a = 0; a < dim; ++a) {
      const double v = x[i * dim + a];
      lo[a] = fmin(lo[a], v);
      hi[a] = fmax(hi[a], v);
    }
  __shared__ double red[4][6];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int a = 0; a < 3; ++a) {
    double l = lo[a], h = hi[a];
    for (int d = kWave / 2; d > 0; d >>= 1) {
      l = fmin(l, __shfl_xor(l, d, kWave));
      h = fmax(h, __shfl_xor(h, d, kWave));
    }
    if (lane == 0) {
      red[w][a] = l;
      red[w][3 + a] = h;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = red[0][threadIdx.x];
    for (int q = 1; q < 4; ++q) v = threadIdx.x < 3 ? fmin(v, red[q][threadIdx.x]) : fmax(v, red[q][threadIdx.x]);
    part[blockIdx.x * 6 + threadIdx.x] = v;
  }
}

// One block: thread t takes the partials t, t + 256, ... (independent loads),
// then a tree in LDS (minimum and maximum are exact in any order).
__global__ void __launch_bounds__(256) extrema_final_kernel(const double* __restrict__ part, int nb,
                                                            double* __restrict__ out) {
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  const int t = threadIdx.x;
  double v[6] = {inf, inf, inf, -inf, -inf, -inf};
  for (int b = t; b < nb; b += 256)
    for (int a = 0; a < 6; ++a) v[a] = a < 3 ? fmin(v[a], part[b * 6 + a]) : fmax(v[a], part[b * 6 + a]);
  __shared__ double red[6][256];
  for (int a = 0; a < 6; ++a) red[a][t] = v[a];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int a = 0; a < 6; ++a)
        red[a][t] = a < 3 ? fmin(red[a][t], red[a][t + st]) : fmax(red[a][t], red[a][t + st]);
    __syncthreads();
  }
  if (t < 6) out[t] = red[t][0];
}

// ---------------------------------------------------------------- launchers
static inline unsigned grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s, const uint32_t* gate) {
  if (n == 0) return hipSuccess;
  fill_u32_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n, v, gate);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s, const uint32_t* gate) {
  if (n == 0) return hipSuccess;
  fill_u64_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n, v, gate);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s, const uint32_t* gate) {
  if (n == 0) return hipSuccess;
  fill_f64_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n, v, gate);
  return hipGetLastError();
}

size_t scan_scratch_elems(int n) { return (size_t)(n + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_scan(const uint32_t* in, int n, uint32_t* sums, uint32_t* out, hipStream_t s,
                       const uint32_t* gate) {
  int nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb <= 1) {  // one chunk: one block
    scan_apply_kernel<true><<<1, kScanThreads, 0, s>>>(in, n, sums, out, gate);
    return hipGetLastError();
  }
  scan_sums_kernel<<<nb, kScanThreads, 0, s>>>(in, n, sums, gate);
  scan_apply_kernel<false><<<nb, kScanThreads, 0, s>>>(in, n, sums, out, gate);
  return hipGetLastError();
}

BinPlan bin_plan(int64_t ncells, int64_t n) {
  BinPlan P;
  // about kPlaceTarget particles per bucket, so that nearly every bucket
  // fits the LDS assembly of the place pass; at most kMaxBuckets buckets and
  // kMaxBucketCells cells per bucket (LDS tables)
  int64_t cpb = n > 0 ? (kPlaceTarget * ncells) / n : ncells;
  cpb = std::min<int64_t>(cpb, kMaxBucketCells);
  cpb = std::max<int64_t>(cpb, (ncells + kMaxBuckets - 1) / kMaxBuckets);
  cpb = std::min<int64_t>(std::max<int64_t>(cpb, 1), std::max<int64_t>(ncells, 1));
  P.cpb = (int)cpb;
  P.nbk = (int)((std::max<int64_t>(ncells, 1) + cpb - 1) / cpb);
  // particles per thread of the count and bucket passes: about one block per CU
  const int64_t per = (n + (int64_t)kBinThreads * 256 - 1) / ((int64_t)kBinThreads * 256);
  P.per = (int)std::min<int64_t>(std::max<int64_t>(per, 1), 256);
  P.nblk = (int)std::max<int64_t>(1, (n + (int64_t)kBinThreads * P.per - 1) / ((int64_t)kBinThreads * P.per));
  return P;
}

hipError_t launch_bin(const double* x, int n, const BuildGeom& g, int ncells, const BinPlan& P,
                      uint32_t* key, uint32_t* hist, uint32_t* scan_scratch, BinRec* rec, uint32_t* off,
                      float4* pos, double4* r64, uint32_t* idx, int4* wrap, hipStream_t s,
                      const uint32_t* gate) {
  bin_count_kernel<<<P.nblk, kBinThreads, 0, s>>>(x, n, g, P, key, hist, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(hist, P.nbk * P.nblk, scan_scratch, hist, s, gate);
  if (e != hipSuccess) return e;
  bin_bucket_kernel<<<P.nblk, kBinThreads, 0, s>>>(x, n, g.dim, P, key, hist, rec, gate);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  bin_place_kernel<<<P.nbk, kBinThreads, 0, s>>>(n, g, P, ncells, hist, rec, off, pos, r64, idx, wrap,
                                                  gate);
  return hipGetLastError();
}

hipError_t launch_tiles(const uint32_t* off, const TileGeom& g, uint32_t* row_tiles,
                        uint32_t* row_off, uint32_t* scan_scratch, Tile* tiles, hipStream_t s,
                        const uint32_t* gate) {
  const int nb = (g.nrows + kTileRowsPerBlock - 1) / kTileRowsPerBlock;
  tiles_count_kernel<<<nb, 256, 0, s>>>(off, g, row_tiles, gate);
  hipError_t e = launch_scan(row_tiles, g.nrows, scan_scratch, row_off, s, gate);
  if (e != hipSuccess) return e;
  tiles_emit_kernel<<<nb, 256, 0, s>>>(off, g, row_off, tiles, gate);
  return hipGetLastError();
}

int extrema_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > kExtremaBlocks ? kExtremaBlocks : b));
}

hipError_t launch_extrema(const double* x, int64_t n, int dim, double* part, double* out, hipStream_t s) {
  const int nb = extrema_blocks(n);
  extrema_kernel<<<nb, 256, 0, s>>>(x, n, dim, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  extrema_final_kernel<<<1, 256, 0, s>>>(part, nb, out);
  return hipGetLastError();
}

hipError_t launch_gather_weights(const double* w, const uint32_t* idx, int n, float4* pos, double4* r64,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  gather_weights_kernel<<<(n + 255) / 256, 256, 0, s>>>(w, idx, n, pos, r64);
  return hipGetLastError();
}

hipError_t launch_gather_vel(const double* v, int dim, const uint32_t* idx, int n, float4* v32,
                             unsigned int* vmax_bits, hipStream_t s) {
  if (n == 0) return hipSuccess;
  gather_vel_kernel<<<(n + 255) / 256, 256, 0, s>>>(v, dim, idx, n, v32, vmax_bits);
  return hipGetLastError();
}

}  // namespace clm
