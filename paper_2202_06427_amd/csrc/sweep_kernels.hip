// sweep_kernels.hip -- the cell-pair sweep and its fused map-reduce back ends
// on gfx950 (paper section 2.8: loop over each cell and its neighbour cells,
// half of them for symmetric pairs; sections 2.3/2.7: a function applied to
// every pair within the cutoff and reduced; section 2.8: per-task output
// copies summed at the end).
//
// Work decomposition: one wavefront (one launched block) per tile of <= 64
// consecutive sorted particles (one per lane) of one cell row.  For every neighbour cell the
// wave visits, the cell's particles are streamed in order; the j-th record is
// the same for all 64 lanes, so it is read with scalar loads into SGPRs and
// consumed as an SGPR operand by the vector ALU (no LDS broadcast, whose VGPR
// write-back would cost as much as the arithmetic).
//
// Half shell (single set, symmetric maps): neighbour cells with offset
// (dz, dy) > 0 lexicographically, plus the home row where j > i in sorted
// order (the sorted order follows the cells along x).  Full shell (LJ
// forces as a gather, cross sets): every neighbour cell.  A neighbour row's
// cell offsets are loaded once, one cell per lane; with few tiles the rows
// of a tile are spread over several waves (sweep_split), each with its own
// partial slot.  Neighbour lists take their output offsets from a counting
// sweep over the same work items (or slots from a shared counter).
//
// Precision forms:
//  FP64 (canonical): D = (r'_j - r'_i) + H K, d2 = (Dx^2 + Dy^2) + Dz^2 with
//   separately rounded operations -- exactly the pair set of clmap.h.
//  FP32 + guard: q_i = fl32(r'_i - O_u) (i relative to the visited cell's
//   origin, computed in FP64) and o_j (FP32 offset of j from its cell
//   origin): D = o_j - q_i, d2 by FMA.  A rigorous bound on |d2_32 - d2|
//   (the band, computed on the host) classifies each candidate as certainly
//   in, certainly out, or uncertain; uncertain candidates (and histogram
//   values within the band of a bin edge, and LJ pairs closer than the near
//   threshold) are queued per wave in LDS and recomputed in canonical FP64,
//   64 at a time.
#include "clmap_internal.h"
#include "device_util.h"

namespace clm {

// ---------------------------------------------------------------- histogram bins
// Canonical bin of v against E64[0..nb] (first k with v <= E_{k+1}; v = 0 ->
// bin 0; beyond E_nb -> nb), FP64.  The edges are (k h)^2 (the last possibly
// rc^2), so the smallest m with v <= E_m is guessed from sqrt(v) / h and
// settled against the table itself: the result depends only on the table.
__device__ __forceinline__ int bin64(const double* __restrict__ E, int nb, double inv_h, double v) {
  if (!(v <= E[nb])) return nb;
  const double g = ceil(sqrt(v) * inv_h);
  int m = g > 0.0 ? (g < (double)nb ? (int)g : nb) : 0;
  while (m > 0 && v <= E[m - 1]) --m;
  while (!(v <= E[m])) ++m;  // stops at nb at the latest: v <= E_nb
  return m == 0 ? 0 : m - 1;
}

// FP32 bin with certainty flag.  The edges are formed in FP32, E_m =
// (m h)^2 for m < nb and E_nb = elast (the canonical last edge rounded to
// FP32): each is within 5 units of 2^-24 (relative) of the canonical FP64
// edge.  The bin is certain when v is farther than band from both of its
// edges; band covers the FP32 error of v plus 8 * 2^-24 * elast.
__device__ __forceinline__ float edge32(const float* Et, int m, int nb, float h, float elast) {
  if constexpr (kHistEdgeTable) return Et[m];
  const float e = (float)m * h;
  return m >= nb ? elast : e * e;
}
__device__ __forceinline__ int bin32(const float* Et, int nb, float h, float inv_h, float elast, float v,
                                     float band, bool* certain) {
  const float sq = __builtin_sqrtf(v);
  int k = (int)ceilf(sq * inv_h) - 1;
  k = k < 0 ? 0 : (k > nb ? nb : k);
  if (k < nb && k > 0 && v <= edge32(Et, k, nb, h, elast)) --k;
  else if (k < nb && v > edge32(Et, k + 1, nb, h, elast)) ++k;
  if (k >= nb) {
    *certain = (v - elast) > band;
    return nb;
  }
  const float lo = edge32(Et, k, nb, h, elast), hi = edge32(Et, k + 1, nb, h, elast);
  *certain = (k == 0 ? true : (v - lo) > band) && (hi - v) > band && v > lo && v <= hi;
  return k;
}

// ---------------------------------------------------------------- per-wave LDS
struct WaveLds {
  uint32_t* hist;     // copies x (nbins+1)
  double* hsum;       // copies x nbins
  float* E32;         // nbins+1 (when the FP32 edges come from a table)
  uint32_t* nl_ij;    // kNLStage*2
  double* nl_d;       // kNLStage
  int* nl_fill;       // 1
};

// ---------------------------------------------------------------- the sweep
// All members of Sweep are per-lane registers or wave-uniform values loaded
// with scalar loads; every method is inlined so nothing lives in memory.
template <int DIM, bool FP32, int KIND>
struct Sweep {
  static constexpr bool kLJF = KIND == K_LJ_F || KIND == K_LJ_FV;
  static constexpr bool kVir = KIND == K_LJ_FV;
  static constexpr bool kLJ = KIND == K_LJ_E || kLJF;
  static constexpr bool kDV = KIND == K_HIST_DV;
  static constexpr bool kHist = KIND == K_HIST_DIST || KIND == K_HIST_REL || kDV;
  static constexpr bool kRel = KIND == K_HIST_REL;
  static constexpr bool kVel = kRel || kDV;
  // rows may be spread over waves unless each particle's output is written
  // by the wave that holds it
  static constexpr bool kRowSplit = !(KIND == K_LJ_F || KIND == K_LJ_FV);
  static constexpr bool kW = KIND == K_SUM_W;
  static constexpr bool kNL = KIND == K_NL;
  static constexpr bool kSum = KIND == K_SUM_D || KIND == K_SUM_INV_D || kW || kLJ;

  // ---- uniform job constants
  const JobDesc* J;
  int cross, full, l, lx, nx, ny, nz;
  double Hn0[3];     // H[a][0] / n[0]: origin step between cells of a row
  double rc2;
  float lo32, hi32;
  float s2f, near2f;
  double s2, inv_s2;
  int nbins;
  float inv_h;
  float h32, elast;  // FP32 bin width and last edge
  int hC;            // histogram copies
  uint32_t* hist_l;  // this lane's copy: counters (nbins+1)
  double* hsum_l;    // and sums (nbins)
  double inv_h64;
  float bandh;       // histogram edge band (FP32)
  int want_sums, with_dist;
  const float4* P;       // j positions (FP32)
  const double4* R;      // j positions (FP64)
  const uint32_t* IDXJ;  // j original indices
  const float4* VJ;      // j velocities FP32
  const double* VJ64;    // j velocities FP64 (original order)
  const uint32_t* OFF;
  const double* E64;
  WaveLds L;
  // FP64 re-evaluation queue (FP32 form): ring of kQueueCap entries
  // (j, lane | kcode << 8 | count_it << 16) in LDS; head/tail are uniform
  uint2* Q;
  double* GA;          // per-lane FP64 force accumulators fed by the queue
  uint32_t qhead, qtail;
  uint32_t tstart;
  // ---- per lane
  int lane;
  bool active;
  uint32_t i, i_orig;
  double ri[3];
  float vi[3];
  double vi64[3];
  double wi64, wj64;   // weights of the lane's particle and of the candidate (FP64 form)
  double accE;
  double G[3];
  double S[3];       // FP64 form, per visited cell: sum of f_s D (folded into G and B)
  double W[6];
  double B[9];
  unsigned long long cnt_wave, cnt_lane;
  uint32_t qband, qnear;   // FP64 re-evaluations done by this lane (summed per tile)
  bool qe;                 // neighbour list: this lane's queued entry is a member (qa, qb, qd)
  uint32_t qa, qb;
  double qd;
  unsigned long long nl_base;  // neighbour list: next output slot of this work item
  // ---- visit
  float q[3];
  double t[3];
  int p[3];

  __device__ __forceinline__ void load_job(const JobDesc* job) {
    J = job;
    cross = ldu(&J->cross);
    full = ldu(&J->full_shell) || cross;
    l = ldu(&J->lcell);
    lx = ldu(&J->lcell_x);
    nx = ldu(&J->n[0]);
    ny = ldu(&J->n[1]);
    nz = ldu(&J->n[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) Hn0[a] = ldu(&J->Hn[a * 3]);
    rc2 = ldu(&J->rc2);
    lo32 = ldu(&J->lo32);
    hi32 = ldu(&J->hi32);
    bandh = hi32 - lo32;
    if constexpr (kLJ) {
      s2 = ldu(&J->s2);
      inv_s2 = 1.0 / s2;
      s2f = ldu(&J->s2f);
      near2f = ldu(&J->near2f);
    }
    if constexpr (kHist) {
      nbins = ldu(&J->nbins);
      inv_h = ldu(&J->inv_h);
      inv_h64 = (double)nbins / ldu(&J->hist_hi);
      E64 = ldu(&J->E64);
      h32 = (float)(ldu(&J->hist_hi) / (double)nbins);
      elast = ldu(&ldu(&J->E32)[nbins]);
      hC = hist_copies(KIND, nbins);
    }
    if constexpr (kVel) {
      VJ = cross ? ldu(&J->vel32_y) : ldu(&J->vel32_x);
      VJ64 = cross ? ldu(&J->vel64_y) : ldu(&J->vel64_x);
    }
    if constexpr (kRel) {
      want_sums = ldu(&J->want_sums);
      bandh = (float)ldu(ldu(&J->bandq));
    }
    if constexpr (kHist) bandh += 4.77e-7f * elast;  // 8 * 2^-24 * elast: the FP32 edges
    if constexpr (kNL) with_dist = ldu(&J->with_dist);
    P = cross ? ldu(&J->pos_y) : ldu(&J->pos_x);
    R = cross ? ldu(&J->r64_y) : ldu(&J->r64_x);
    IDXJ = cross ? ldu(&J->idx_y) : ldu(&J->idx_x);
    OFF = cross ? ldu(&J->off_y) : ldu(&J->off_x);
  }

  // ---------------- neighbour-list staging
  __device__ __forceinline__ void nl_emit(uint32_t a, uint32_t b, double d, unsigned long long g) {
    if ((long long)g < ldu(&J->capacity)) {
      int32_t* pairs = ldu(&J->pairs);
      pairs[2 * g] = (int32_t)a;
      pairs[2 * g + 1] = (int32_t)b;
      if (with_dist) ldu(&J->dist)[g] = d;
    }
  }

  __device__ __forceinline__ void nl_flush() {
    int n = uniform(*(volatile int*)L.nl_fill);
    n = n > kNLStage ? kNLStage : n;
    if (n > 0) {
      unsigned long long base = 0;
      if (ldu(&J->nl_offsets)) {  // this work item's slots follow its offset
        base = nl_base;
        nl_base += (unsigned long long)n;
      } else {
        if (lane == 0) base = atomicAdd(ldu(&J->nl_counter), (unsigned long long)n);
        base = __shfl(base, 0, kWave);
      }
      for (int s = lane; s < n; s += kWave) nl_emit(L.nl_ij[2 * s], L.nl_ij[2 * s + 1], L.nl_d[s], base + s);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) *L.nl_fill = 0;
    __builtin_amdgcn_wave_barrier();
  }

  __device__ __forceinline__ void nl_pair(uint32_t j, uint32_t* a, uint32_t* b) {
    uint32_t jo = ldu(&IDXJ[j]);
    uint32_t x0 = i_orig, x1 = jo;
    if (!cross && x0 > x1) { uint32_t tmp = x0; x0 = x1; x1 = tmp; }
    *a = x0;
    *b = x1;
  }

  // certain members of one iteration (same j for every lane)
  __device__ __forceinline__ void nl_stage_wave(unsigned long long m, uint32_t j, double d) {
    if (m == 0) return;
    uint32_t a = 0u, b = 0u;
    if (__builtin_amdgcn_inverse_ballot_w64(m)) nl_pair(j, &a, &b);
    nl_stage_lanes(m, a, b, d);
  }

  // the lanes of m stage their pair (a, b, d); called by the whole wave
  __device__ __forceinline__ void nl_stage_lanes(unsigned long long m, uint32_t a, uint32_t b, double d) {
    if (m == 0) return;
    const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
    int cnt = __popcll(m);
    int base = uniform(*(volatile int*)L.nl_fill);
    if (base + cnt > kNLStage) {
      nl_flush();
      base = 0;
    }
    if (in) {
      int slot = base + lane_rank(m);
      L.nl_ij[2 * slot] = a;
      L.nl_ij[2 * slot + 1] = b;
      L.nl_d[slot] = d;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) *L.nl_fill = base + cnt;
    __builtin_amdgcn_wave_barrier();
  }

  // a single lane (divergent FP64 path): straight to global memory
  __device__ __forceinline__ void nl_one(uint32_t j, double d) {
    uint32_t a, b;
    nl_pair(j, &a, &b);
    unsigned long long g = atomicAdd(ldu(&J->nl_counter), 1ull);
    nl_emit(a, b, d, g);
  }

  // |v_j - v_i| in FP64 for partner jo (caller index) and the velocity vo of
  // the particle on the other end (the oracle's operation order)
  __device__ __forceinline__ double speed64(uint32_t jo, const double* vo) const {
    double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) dv[a] = VJ64[(size_t)jo * DIM + a] - vo[a];
    double qq = dv[0] * dv[0] + dv[1] * dv[1];
    if (DIM == 3) qq = qq + dv[2] * dv[2];
    return sqrt(qq);
  }

  // ---------------- FP64 epilogue for one member pair (canonical d2, D)
  __device__ __forceinline__ void pair64(double d2, const double* D, uint32_t j, bool count_it) {
    if (count_it) cnt_lane += 1;
    if constexpr (KIND == K_SUM_D) accE += sqrt(d2);
    if constexpr (KIND == K_SUM_INV_D) accE += 1.0 / sqrt(d2);
    if constexpr (kW) accE += (wi64 * wj64) / sqrt(d2);
    if constexpr (kLJ) {
      const double r = rcp64(d2);
      double x = s2 * r;
      double x3 = x * x * x;
      double u = x3 * x3 - x3;
      if constexpr (KIND == K_LJ_E) {
        accE += u;
      } else {
        double f = (2.0 * x3 * x3 - x3) * r;  // f_s / (24 eps)
        accE += 0.5 * u;
#pragma unroll
        for (int a = 0; a < DIM; ++a) S[a] += f * D[a];
        if constexpr (kVir) {
          W[0] += 0.5 * f * D[0] * D[0];
          W[1] += 0.5 * f * D[0] * D[1];
          W[3] += 0.5 * f * D[1] * D[1];
          if (DIM == 3) {
            W[2] += 0.5 * f * D[0] * D[2];
            W[4] += 0.5 * f * D[1] * D[2];
            W[5] += 0.5 * f * D[2] * D[2];
          }
        }
      }
    }
    if constexpr (KIND == K_HIST_DIST) {
      int k = bin64(E64, nbins, inv_h64, d2);
      hist_add(k);
    }
    if constexpr (kDV) {
      const int k = bin64(E64, nbins, inv_h64, d2);
      hist_add(k);
      if (k < nbins) hsum_add(k, speed64(ldu(&IDXJ[j]), vi64));
    }
    if constexpr (kRel) {
      uint32_t jo = ldu(&IDXJ[j]);
      double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < DIM; ++a) dv[a] = ldu(&VJ64[(size_t)jo * DIM + a]) - vi64[a];
      double qq = dv[0] * dv[0] + dv[1] * dv[1];
      if (DIM == 3) qq = qq + dv[2] * dv[2];
      int k = bin64(E64, nbins, inv_h64, qq);
      hist_add(k);
      if (want_sums && k < nbins) hsum_add(k, sqrt(qq));
    }
    if constexpr (kNL) nl_one(j, sqrt(d2));
  }

  // ---------------- private histogram (this lane's copy)
  __device__ __forceinline__ void hist_add(int k) { atomicAdd(&hist_l[k], 1u); }
  __device__ __forceinline__ void hsum_add(int k, double v) { atomicAdd(&hsum_l[k], v); }

  // ---------------- FP64 re-evaluation queue (FP32 form)
  // Append this iteration's special lanes (uniform control flow).
  // m: lanes to queue, band: lanes whose membership FP64 decides (counted
  // there); both are wave masks.
  __device__ __forceinline__ void enqueue(unsigned long long m, uint32_t j, int kc,
                                          unsigned long long band) {
    if (m == 0) return;
    const uint32_t t0 = (uint32_t)uniform((int)qtail);
    if (__builtin_amdgcn_inverse_ballot_w64(m)) {
      const uint32_t slot = (t0 + (uint32_t)lane_rank(m)) & (uint32_t)(kQueueCap - 1);
      const bool b = __builtin_amdgcn_inverse_ballot_w64(band);
      Q[slot] = make_uint2(j, (uint32_t)lane | ((uint32_t)kc << 8) | (b ? (1u << 16) : 0u));
    }
    qtail = (uint32_t)uniform((int)(t0 + (uint32_t)__popcll(m)));
  }

  // Canonical FP64 evaluation of one queued candidate by this lane; results
  // of the owning lane's particle go through LDS atomics.
  __device__ __forceinline__ void process(const uint2 e) {
    const uint32_t j = e.x;
    const int own = (int)(e.y & 63u);
    const int kc = (int)((e.y >> 8) & 31u);
    const bool count_it = ((e.y >> 16) & 1u) != 0u;
    const uint32_t iL = tstart + (uint32_t)own;
    const double4 rI = ldu(&J->r64_x)[iL];
    const double4 rJ = R[j];
    const double* tk = &J->tK[kc * 4];
    double D[3];
    D[0] = (rJ.x - rI.x) + tk[0];
    D[1] = (rJ.y - rI.y) + tk[1];
    double d2 = D[0] * D[0] + D[1] * D[1];
    if (DIM == 3) {
      D[2] = (rJ.z - rI.z) + tk[2];
      d2 = d2 + D[2] * D[2];
    } else {
      D[2] = 0.0;
    }
    if (!(d2 <= rc2)) return;
    if (count_it) cnt_lane += 1;
    if constexpr (KIND == K_SUM_D) accE += sqrt(d2);
    if constexpr (KIND == K_SUM_INV_D) accE += 1.0 / sqrt(d2);
    if constexpr (kW) accE += (rI.w * rJ.w) / sqrt(d2);
    if constexpr (kLJ) {
      const double r = rcp64(d2);
      const double x = s2 * r;
      const double x3 = x * x * x;
      const double u = x3 * x3 - x3;
      if constexpr (KIND == K_LJ_E) {
        accE += u;
      } else {
        const double f = (2.0 * x3 * x3 - x3) * r;
        accE += 0.5 * u;
#pragma unroll
        for (int a = 0; a < DIM; ++a) atomicAdd(&GA[own * 3 + a], f * D[a]);
        const int pk[3] = {kc % 3 - 1, (kc / 3) % 3 - 1, kc / 9 - 1};
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int b = 0; b < DIM; ++b) B[a * 3 + b] += 0.5 * f * D[a] * (double)pk[b];
        if constexpr (kVir) {
          W[0] += 0.5 * f * D[0] * D[0];
          W[1] += 0.5 * f * D[0] * D[1];
          W[3] += 0.5 * f * D[1] * D[1];
          if (DIM == 3) {
            W[2] += 0.5 * f * D[0] * D[2];
            W[4] += 0.5 * f * D[1] * D[2];
            W[5] += 0.5 * f * D[2] * D[2];
          }
        }
      }
    }
    if constexpr (KIND == K_HIST_DIST) hist_add(bin64(E64, nbins, inv_h64, d2));
    if constexpr (kDV) {
      const int k = bin64(E64, nbins, inv_h64, d2);
      hist_add(k);
      if (k < nbins) {
        const uint32_t io = ldu(&J->idx_x)[iL];
        const double* v64 = ldu(&J->vel64_x);
        double vo[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) vo[a] = v64[(size_t)io * DIM + a];
        hsum_add(k, speed64(IDXJ[j], vo));
      }
    }
    if constexpr (kRel) {
      const uint32_t io = ldu(&J->idx_x)[iL];
      const double* v64 = ldu(&J->vel64_x);
      const uint32_t jo = IDXJ[j];
      double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < DIM; ++a) dv[a] = VJ64[(size_t)jo * DIM + a] - v64[(size_t)io * DIM + a];
      double qq = dv[0] * dv[0] + dv[1] * dv[1];
      if (DIM == 3) qq = qq + dv[2] * dv[2];
      const int k = bin64(E64, nbins, inv_h64, qq);
      hist_add(k);
      if (want_sums && k < nbins) hsum_add(k, sqrt(qq));
    }
    if constexpr (kNL) {  // staged by the whole wave after this batch (drain)
      uint32_t a = ldu(&J->idx_x)[iL], b = IDXJ[j];
      if (!cross && a > b) { uint32_t tmp = a; a = b; b = tmp; }
      qe = true;
      qa = a;
      qb = b;
      qd = sqrt(d2);
    }
  }

  // Process queued entries 64 at a time (all: also a final partial batch).
  __device__ __forceinline__ void drain(bool all) {
    uint32_t h = (uint32_t)uniform((int)qhead);
    const uint32_t tl = (uint32_t)uniform((int)qtail);
    while (tl - h >= (uint32_t)kWave || (all && tl != h)) {
      const uint32_t nb = min(tl - h, (uint32_t)kWave);
      if constexpr (kNL) qe = false;
      if ((uint32_t)lane < nb) {
        const uint2 e = Q[(h + (uint32_t)lane) & (uint32_t)(kQueueCap - 1)];
        const uint32_t b = (e.y >> 16) & 1u;  // band entries carry count_it
        qband += b;
        qnear += 1u - b;
        process(e);
      }
      if constexpr (kNL) nl_stage_lanes(__builtin_amdgcn_ballot_w64(qe), qa, qb, qd);
      h = (uint32_t)uniform((int)(h + nb));
    }
    qhead = h;
  }

  // ---------------- one candidate
  // Lanes of this tile that may pair with candidate j (a wave mask, built on
  // the scalar unit from the tile's first sorted index): mode 0 all, mode 1
  // j > i (home row of the half shell), mode 2 j != i (own cells, full shell).
  // Lane L holds sorted index tstart + L; inactive lanes sit far away.
  __device__ __forceinline__ unsigned long long filter_mask(int mode, uint32_t j) const {
    if (mode == 0) return ~0ull;
    const int k = (int)(j - tstart);
    if (mode == 1) return k <= 0 ? 0ull : (k >= kWave ? ~0ull : ((1ull << k) - 1ull));
    return (k >= 0 && k < kWave) ? ~(1ull << k) : ~0ull;
  }

  // One candidate (same j in every lane), okm: filter_mask.
  __device__ __forceinline__ void cand32(uint32_t j, const float4& pj, unsigned long long okm,
                                         float& visE, float* g32, float* w32, int kc) {
    const float dx = pj.x - q[0];
    const float dy = pj.y - q[1];
    const float dz = DIM == 3 ? pj.z - q[2] : 0.0f;
    const float d2 = DIM == 3 ? __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx))
                              : __builtin_fmaf(dy, dy, dx * dx);
    // classification as wave masks (one compare each, logic on the scalar unit)
    const unsigned long long mlo = __builtin_amdgcn_ballot_w64(d2 <= lo32);
    const unsigned long long mhi = __builtin_amdgcn_ballot_w64(d2 <= hi32);
    const unsigned long long in_m = mlo & okm;
    const unsigned long long band_m = mhi & ~mlo & okm;
    unsigned long long spec_m = band_m;
    const bool in = __builtin_amdgcn_inverse_ballot_w64(in_m);
    bool spec = false;  // per-lane extra reasons (histogram edges)
    cnt_wave += (unsigned long long)__popcll(in_m);
    if constexpr (KIND == K_SUM_D || KIND == K_SUM_INV_D || kW) {
      const float r = __builtin_amdgcn_rsqf(d2);
      const float term = KIND == K_SUM_D ? d2 * r : (kW ? pj.w * r : r);
      visE += in ? term : 0.0f;
    } else if constexpr (kLJ) {
      // near2f < lo32: near pairs are members, evaluated in FP64
      const unsigned long long near_m = __builtin_amdgcn_ballot_w64(d2 < near2f) & okm;
      const bool fast = __builtin_amdgcn_inverse_ballot_w64(in_m & ~near_m);
      spec_m |= near_m;
      // x = s^2/d^2 masked once: u and f vanish together on other lanes.
      // f s^2 = (2 x^6 - x^3) x = (2u + x^3) x; the 1/s^2 is applied when
      // the visit's sums are folded into FP64.
      const float x = fast ? s2f * __builtin_amdgcn_rcpf(d2) : 0.0f;
      const float x3 = x * x * x;
      const float u = __builtin_fmaf(x3, x3, -x3);
      visE += u;
      if constexpr (kLJF) {
        const float f = __builtin_fmaf(2.0f, u, x3) * x;
        g32[0] = __builtin_fmaf(f, dx, g32[0]);
        g32[1] = __builtin_fmaf(f, dy, g32[1]);
        if (DIM == 3) g32[2] = __builtin_fmaf(f, dz, g32[2]);
        if constexpr (kVir) {
          w32[0] = __builtin_fmaf(f * dx, dx, w32[0]);
          w32[1] = __builtin_fmaf(f * dx, dy, w32[1]);
          w32[3] = __builtin_fmaf(f * dy, dy, w32[3]);
          if (DIM == 3) {
            w32[2] = __builtin_fmaf(f * dx, dz, w32[2]);
            w32[4] = __builtin_fmaf(f * dy, dz, w32[4]);
            w32[5] = __builtin_fmaf(f * dz, dz, w32[5]);
          }
        }
      }
    } else if constexpr (kHist) {
      float v = d2;
      if constexpr (kRel) {
        const float4 vj = ldu(&VJ[j]);
        const float ex = vj.x - vi[0], ey = vj.y - vi[1];
        const float ez = DIM == 3 ? vj.z - vi[2] : 0.0f;
        v = DIM == 3 ? __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex))
                     : __builtin_fmaf(ey, ey, ex * ex);
      }
      if (in) {
        bool certain;
        const int k = bin32(L.E32, nbins, h32, inv_h, elast, v, bandh, &certain);
        if (certain) {
          hist_add(k);
          if (kRel && want_sums && k < nbins) hsum_add(k, (double)__builtin_sqrtf(v));
          if (kDV && k < nbins) {
            const float4 vj = ldu(&VJ[j]);
            const float ex = vj.x - vi[0], ey = vj.y - vi[1];
            const float ez = DIM == 3 ? vj.z - vi[2] : 0.0f;
            const float qq = DIM == 3 ? __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex))
                                      : __builtin_fmaf(ey, ey, ex * ex);
            hsum_add(k, (double)__builtin_sqrtf(qq));
          }
        } else {
          spec = true;
        }
      }
    } else if constexpr (kNL) {
      nl_stage_wave(in_m, j, (double)__builtin_sqrtf(d2));
    }
    if constexpr (kHist) spec_m |= __builtin_amdgcn_ballot_w64(spec);
    enqueue(spec_m, j, kc, band_m);
  }

  __device__ __forceinline__ void cand64(uint32_t j, const double4& rj, unsigned long long okm) {
    if constexpr (kW) wj64 = rj.w;
    double D[3];
    D[0] = (rj.x - ri[0]) + t[0];
    D[1] = (rj.y - ri[1]) + t[1];
    double d2 = D[0] * D[0] + D[1] * D[1];
    if (DIM == 3) {
      D[2] = (rj.z - ri[2]) + t[2];
      d2 = d2 + D[2] * D[2];
    } else {
      D[2] = 0.0;
    }
    const unsigned long long in_m = __builtin_amdgcn_ballot_w64(d2 <= rc2) & okm;
    const bool in = __builtin_amdgcn_inverse_ballot_w64(in_m);
    cnt_wave += (unsigned long long)__popcll(in_m);
    if constexpr (kNL) {
      nl_stage_wave(in_m, j, sqrt(d2));
    } else if constexpr (KIND != K_COUNT) {
      if (in) pair64(d2, D, j, false);
    }
  }

  // ---------------- one visited cell: j in [jb, je)
  // G += S, B += S p^T / 2 at the end of a visited cell
  __device__ __forceinline__ void fold_visit() {
    if constexpr (kLJF) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) G[a] += S[a];
      if (p[0] != 0 || p[1] != 0 || p[2] != 0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int b = 0; b < DIM; ++b) B[a * 3 + b] += 0.5 * S[a] * (double)p[b];
      }
    }
  }

  // FP32 form: the visit's FP32 sums go straight into the FP64 lane
  // accumulators (G, and B when the visited cell is a periodic image).
  // The unfiltered loop (nearly every visit) and the filtered one are
  // separate so the common one computes no masks.
  template <bool FILT>
  __device__ __forceinline__ void loop32(uint32_t jb, uint32_t je, int mode, float& visE, float* g32,
                                         float* w32, int kc) {
    uint32_t j = jb;
    for (; j + 4 <= je; j += 4) {
      const float4 p0 = ldu(&P[j]), p1 = ldu(&P[j + 1]), p2 = ldu(&P[j + 2]), p3 = ldu(&P[j + 3]);
      cand32(j, p0, FILT ? filter_mask(mode, j) : ~0ull, visE, g32, w32, kc);
      cand32(j + 1, p1, FILT ? filter_mask(mode, j + 1) : ~0ull, visE, g32, w32, kc);
      cand32(j + 2, p2, FILT ? filter_mask(mode, j + 2) : ~0ull, visE, g32, w32, kc);
      cand32(j + 3, p3, FILT ? filter_mask(mode, j + 3) : ~0ull, visE, g32, w32, kc);
      drain(false);
    }
    // at most 3 more candidates: the ring (kQueueCap >= 4 * 64 + 63 + 3 * 64)
    // holds them without a drain in between
    for (; j < je; ++j) cand32(j, ldu(&P[j]), FILT ? filter_mask(mode, j) : ~0ull, visE, g32, w32, kc);
    drain(false);
  }

  __device__ __forceinline__ void visit(uint32_t jb, uint32_t je, int mode) {
    if constexpr (FP32) {
      float visE = 0.0f;
      float g32[3] = {0.0f, 0.0f, 0.0f};
      float w32[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      const int kc = kcode(p[0], p[1], p[2]);
      if (mode == 0)
        loop32<false>(jb, je, 0, visE, g32, w32, kc);
      else
        loop32<true>(jb, je, mode, visE, g32, w32, kc);
      if constexpr (kSum) accE += kLJF ? 0.5 * (double)visE : (kW ? wi64 * (double)visE : (double)visE);
      if constexpr (kLJF) {
        double ga[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          ga[a] = (double)g32[a] * inv_s2;
          G[a] += ga[a];
        }
        if (p[0] != 0 || p[1] != 0 || p[2] != 0) {
#pragma unroll
          for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) B[a * 3 + b] += 0.5 * ga[a] * (double)p[b];
        }
        if constexpr (kVir) {
#pragma unroll
          for (int k = 0; k < 6; ++k) W[k] += 0.5 * inv_s2 * (double)w32[k];
        }
      }
    } else {
      if constexpr (kLJF) {
        S[0] = 0.0; S[1] = 0.0; S[2] = 0.0;
      }
      if (mode == 0) {
        for (uint32_t j = jb; j < je; ++j) cand64(j, ldu(&R[j]), ~0ull);
      } else {
        for (uint32_t j = jb; j < je; ++j) cand64(j, ldu(&R[j]), filter_mask(mode, j));
      }
      fold_visit();
    }
  }

  // ---------------- one tile
  // Rows r (in visiting order) with r % ngrp == grp; partial slot
  // tile * ngrp + grp.
  __device__ __forceinline__ void run(const Tile& T, int tile_id, int grp, int ngrp) {
    const int cy = (int)(T.row % (uint32_t)ny);
    const int cz = DIM == 3 ? (int)(T.row / (uint32_t)ny) : 0;
    const int count = T.count;
    const int cx0 = T.cx0, cx1 = T.cx1;
    active = lane < count;
    i = T.start + (uint32_t)(active ? lane : count - 1);
    i_orig = ldu(&J->idx_x)[i];
    {
      // inactive lanes are placed 1e100 away: no candidate can reach them
      const double4 r = ldu(&J->r64_x)[i];
      ri[0] = active ? r.x : 1e100;
      ri[1] = active ? r.y : 1e100;
      ri[2] = active ? r.z : 1e100;
      if constexpr (kW) wi64 = active ? r.w : 0.0;
    }
    if constexpr (kVel) {
      const float4 v = ldu(&J->vel32_x)[i];
      vi[0] = v.x; vi[1] = v.y; vi[2] = v.z;
      const double* v64 = ldu(&J->vel64_x);
#pragma unroll
      for (int a = 0; a < DIM; ++a) vi64[a] = v64[(size_t)i_orig * DIM + a];
    }
    accE = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) G[a] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) W[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) B[k] = 0.0;
    cnt_wave = 0;
    cnt_lane = 0;
    qband = 0;
    qnear = 0;
    tstart = T.start;
    const int local = (tile_id - ldu(&J->tile_begin)) * ngrp + grp;  // this job's partial slot
    if constexpr (kNL) {
      const unsigned long long* no = ldu(&J->nl_offsets);
      nl_base = no ? ldu(&no[local]) : 0ull;
    }
    qhead = 0;
    qtail = 0;
    if constexpr (FP32 && kLJF) {
#pragma unroll
      for (int a = 0; a < 3; ++a) GA[lane * 3 + a] = 0.0;
      __builtin_amdgcn_wave_barrier();
    }

    const int dzlo = DIM == 3 ? -l : 0, dzhi = DIM == 3 ? l : 0;
    int r = -1, next = grp;  // rows grp, grp + ngrp, ... (split maps)
    for (int dz = dzlo; dz <= dzhi; ++dz) {
      for (int dy = -l; dy <= l; ++dy) {
        if (!full && (dz < 0 || (dz == 0 && dy < 0))) continue;
        if constexpr (kRowSplit) {
          if (++r != next) continue;
          next += ngrp;
        }
        const bool home = !full && dz == 0 && dy == 0;
        const int uy = cy + dy, uz = cz + dz;
        int uyw = uy, uzw = uz, py = 0, pz = 0;
        if (uyw < 0) { uyw += ny; py = -1; } else if (uyw >= ny) { uyw -= ny; py = 1; }
        if (DIM == 3) {
          if (uzw < 0) { uzw += nz; pz = -1; } else if (uzw >= nz) { uzw -= nz; pz = 1; }
        }
        const int rowbase = (uyw + ny * uzw) * nx;
        const int xlo = home ? cx0 : cx0 - lx;
        const int xhi = cx1 + lx;
        // origin of the row's cell 0 (unwrapped row index), FP64
        double Orow[3] = {0.0, 0.0, 0.0};
        if constexpr (FP32) {
          const double u1 = (double)uy, u2 = DIM == 3 ? (double)uz : 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) Orow[a] = ldu(&J->Hn[a * 3 + 1]) * u1 + ldu(&J->Hn[a * 3 + 2]) * u2;
        }
        // The row's cells in chunks of up to 64: lane L loads the offsets of
        // cell cs + L (one vector load per chunk instead of a dependent
        // scalar load per cell), empty cells drop out of a ballot mask.
        for (int cs = xlo; cs <= xhi; cs += kWave) {
          uint32_t jbv = 0u, jev = 0u;
          {
            const int ux = cs + lane;
            if (ux <= xhi) {
              const int uxw = ux < 0 ? ux + nx : (ux >= nx ? ux - nx : ux);
              jbv = OFF[rowbase + uxw];
              jev = OFF[rowbase + uxw + 1];
            }
          }
          unsigned long long cells = __builtin_amdgcn_ballot_w64(jev != jbv);
          while (cells) {
            const int L = (int)__builtin_ctzll(cells);
            cells &= cells - 1ull;
            const int ux = cs + L;
            const int px = ux < 0 ? -1 : (ux >= nx ? 1 : 0);
            const uint32_t jb = (uint32_t)__builtin_amdgcn_readlane((int)jbv, L);
            const uint32_t je = (uint32_t)__builtin_amdgcn_readlane((int)jev, L);
            p[0] = px; p[1] = py; p[2] = pz;
            const int kc = kcode(px, py, pz);
            t[0] = ldu(&J->tK[kc * 4 + 0]);
            t[1] = ldu(&J->tK[kc * 4 + 1]);
            t[2] = ldu(&J->tK[kc * 4 + 2]);
            if constexpr (FP32) {
              // origin of the visited cell (unwrapped index u), FP64
              const double u0 = (double)ux;
#pragma unroll
              for (int a = 0; a < DIM; ++a) {
                const double O = Orow[a] + Hn0[a] * u0;
                q[a] = active ? (float)(ri[a] - O) : 1e18f;
              }
              if (DIM == 2) q[2] = 0.0f;
            }
            const bool own = !cross && dz == 0 && dy == 0 && px == 0 && ux >= cx0 && ux <= cx1;
            visit(jb, je, (home && px == 0) ? 1 : ((full && own) ? 2 : 0));
          }
        }
      }
    }

    // ---- tile epilogue
    if constexpr (FP32) drain(true);
    if constexpr (FP32 && kLJF) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int a = 0; a < DIM; ++a) G[a] += GA[lane * 3 + a];
    }
    if constexpr (kLJF) {
      const double* up = ldu(&J->upstream);
      const double mult = up ? ldu(up) : ldu(&J->scale);
      const double sc = mult * 24.0 * ldu(&J->eps);
      double* forces = ldu(&J->forces);
      if (active) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) forces[(size_t)i_orig * DIM + a] = sc * G[a];
      }
      const int4 w = ldu(&J->wrap_x)[i];
      const int wv[3] = {w.x, w.y, w.z};
      if (active) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int b = 0; b < DIM; ++b) B[a * 3 + b] += G[a] * (double)wv[b];
      }
    }
    if constexpr (kNL) nl_flush();
    const unsigned long long cnt = cnt_wave + wave_sum_u64(cnt_lane);
    double* Pp = ldu(&J->partials) + (size_t)local * kPartialD;
    // every lane may hold queued FP64 contributions of other lanes' particles:
    // reduce over all lanes (inactive lanes contribute nothing of their own)
    const double e = wave_sum_d(accE);
    if constexpr (FP32) {
      const unsigned long long gb = wave_sum_u64(qband), gn = wave_sum_u64(qnear);
      if (lane == 0 && (gb | gn)) {
        unsigned long long* g = ldu(&J->guard);
        atomicAdd(&g[0], gb);
        atomicAdd(&g[1], gn);
      }
    }
    if (lane == 0) {
      ldu(&J->pcount)[local] = cnt;
      Pp[P_SUM] = e;
    }
    if constexpr (kLJF) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double b = wave_sum_d(B[k]);
        if (lane == 0) Pp[P_BOX + k] = b;
      }
      if constexpr (kVir) {
        constexpr int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        double ws[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) ws[k] = wave_sum_d(W[k]);
        if (lane == 0) {
#pragma unroll
          for (int m = 0; m < 9; ++m) Pp[P_VIR + m] = ws[map[m]];
        }
      }
    }
  }
};

template <int DIM, bool FP32, int KIND>
__global__ void __launch_bounds__(kBlock) sweep_kernel(const JobDesc* __restrict__ jobs,
                                                       const Tile* __restrict__ tiles,
                                                       const uint32_t* __restrict__ ntiles_dev,
                                                       int split_rows) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool kHist = KIND == K_HIST_DIST || KIND == K_HIST_REL || KIND == K_HIST_DV;
  constexpr bool kNL = KIND == K_NL;
  const int lane = (int)__lane_id();
  const int wid = uniform((int)(threadIdx.x / kWave));
  // the tile count is produced on the device; never trust it past the array
  constexpr int kWpb = kSweepWaves;
  const int cap = (int)(gridDim.x * kWpb);
  const int ntiles = min((int)ldu(ntiles_dev), cap);
  // G waves per tile when the tiles are few (G * ntiles <= cap); maps with
  // per-particle outputs keep one wave per tile (compiled out)
  constexpr bool kSplit = Sweep<DIM, FP32, KIND>::kRowSplit;
  const int G = kSplit ? sweep_split(ntiles, cap, split_rows) : 1;
  const int nitems = ntiles * G;
  // The grid is sized by an upper bound on the tile count; only the first
  // nblk blocks have work.  Blocks are dispatched to the 8 XCDs round-robin,
  // so block b (b < nblk) runs on XCD b % 8: give each XCD a contiguous
  // range of tiles (neighbouring cells share their rows in that XCD's L2).
  const int nblk = (nitems + kWpb - 1) / kWpb;
  int b = blockIdx.x;
  if (b >= nblk) return;
  if (nblk >= 8) {
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = b % 8, k = b / 8;
    b = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k;
  }
  const int item = uniform(b * kWpb + wid);
  if (item >= nitems) return;
  const int tile_id = kSplit ? item / G : item, grp = kSplit ? item - tile_id * G : 0;
  const Tile T = ldu(&tiles[tile_id]);

  Sweep<DIM, FP32, KIND> S;
  S.lane = lane;
  S.load_job(&jobs[T.job]);
  {
    const int nb = kHist ? S.nbins : 0;
    unsigned char* base = smem + sweep_lds_per_wave(KIND, nb, FP32) * wid;
    if constexpr (FP32) {
      S.Q = (uint2*)base;
      S.GA = (double*)(base + (size_t)kQueueCap * 8);
    }
    base += sweep_lds_queue_bytes(KIND, FP32);
    if constexpr (kHist) {
      const int C = S.hC;
      S.L.hist = (uint32_t*)base;
      S.L.hsum = (double*)(((uintptr_t)(base + (size_t)C * (nb + 1) * 4) + 7) & ~(uintptr_t)7);
      for (int k = lane; k < C * (nb + 1); k += kWave) S.L.hist[k] = 0u;
      if constexpr (hist_has_sums(KIND))
        for (int k = lane; k < C * nb; k += kWave) S.L.hsum[k] = 0.0;
      // copy q of the counters at q * (nb + 1), of the sums at q * nb
      const int q = lane & (C - 1);
      S.hist_l = S.L.hist + q * (nb + 1);
      S.hsum_l = S.L.hsum + q * nb;
      if constexpr (kHistEdgeTable) {
        S.L.E32 = (float*)(S.L.hsum + (hist_has_sums(KIND) ? (size_t)C * nb : 0));
        const float* E32g = ldu(&S.J->E32);
        for (int k = lane; k <= nb; k += kWave) S.L.E32[k] = E32g[k];
      }
    } else if constexpr (kNL) {
      S.L.nl_ij = (uint32_t*)base;
      S.L.nl_d = (double*)(base + (size_t)kNLStage * 8);
      S.L.nl_fill = (int*)(base + (size_t)kNLStage * 16);
      if (lane == 0) *S.L.nl_fill = 0;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }
  S.run(T, tile_id, grp, G);
  if constexpr (kHist) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int nb = S.nbins;
    unsigned long long* hist = ldu(&S.J->hist);
    double* hsums = ldu(&S.J->hist_sums);
    const int C = S.hC;
    for (int k = lane; k <= nb; k += kWave) {  // copies summed in a fixed order
      uint32_t c = 0u;
      for (int q = 0; q < C; ++q) c += S.L.hist[q * (nb + 1) + k];
      if (c) atomicAdd(&hist[k], (unsigned long long)c);
      if (((KIND == K_HIST_REL && S.want_sums) || KIND == K_HIST_DV) && k < nb) {
        double sm = 0.0;
        for (int q = 0; q < C; ++q) sm += S.L.hsum[q * nb + k];
        if (sm != 0.0) atomicAdd(&hsums[k], sm);
      }
    }
  }
}

// ---------------------------------------------------------------- small box
// Brute force over all pairs with the exact minimum-image search (used when
// not even cells as wide as the cutoff fit three times along every axis),
// FP64 only.  The nearest image of one pair: every K whose image can lie
// within the reach.
__device__ __forceinline__ double min_image64(const BruteArgs& A, const double* ri, const double* rj,
                                              double* D, int* Kb) {
  const int dim = A.dim;
  double dr[3] = {rj[0] - ri[0], rj[1] - ri[1], dim == 3 ? rj[2] - ri[2] : 0.0};
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    double fs = A.Hinv[d * 3 + 0] * dr[0] + A.Hinv[d * 3 + 1] * dr[1] + A.Hinv[d * 3 + 2] * dr[2];
    // images farther than half the sum of the lattice-vector lengths can never
    // be the nearest one, so the search radius is min(rc, reach_max)
    double R = A.reach / A.w[d] * (1.0 + 1e-6) + 1e-9;
    lo[d] = (int)ceil(-fs - R);
    hi[d] = (int)floor(-fs + R);
  }
  double best = __builtin_inf();
  for (int k0 = lo[0]; k0 <= hi[0]; ++k0)
    for (int k1 = lo[1]; k1 <= hi[1]; ++k1)
      for (int k2 = (dim == 3 ? lo[2] : 0); k2 <= (dim == 3 ? hi[2] : 0); ++k2) {
        double K[3] = {(double)k0, (double)k1, (double)k2};
        double E[3];
        for (int a = 0; a < dim; ++a) {
          double tt = A.H[a * 3 + 0] * K[0];
          tt = tt + A.H[a * 3 + 1] * K[1];
          if (dim == 3) tt = tt + A.H[a * 3 + 2] * K[2];
          E[a] = (rj[a] - ri[a]) + tt;
        }
        double d2 = E[0] * E[0] + E[1] * E[1];
        if (dim == 3) d2 = d2 + E[2] * E[2];
        if (d2 < best) {
          best = d2;
          for (int a = 0; a < 3; ++a) {
            D[a] = a < dim ? E[a] : 0.0;
            Kb[a] = a == 0 ? k0 : (a == 1 ? k1 : k2);
          }
        }
      }
  return best;
}

// The work is split over (64 particles i) x (a chunk of j): one wave per
// block, its partial sums in partial row blockIdx.x + gridDim.x * blockIdx.y;
// LJ forces go to per-chunk rows of FB (summed in chunk order afterwards).
__global__ void __launch_bounds__(64) brute_kernel(const JobDesc* __restrict__ jobs, BruteArgs A,
                                                   int jchunk, double* __restrict__ FB) {
  const JobDesc& J = jobs[0];
  const int dim = A.dim;
  const int lane = (int)threadIdx.x;
  const int ii = blockIdx.x * kWave + lane;
  const bool act = ii < A.n_x;
  const int ny = A.cross ? A.n_y : A.n_x;
  const int jlo = blockIdx.y * jchunk, jhi = min(ny, jlo + jchunk);
  double accE = 0.0, G[3] = {0, 0, 0}, W[9] = {0}, B[9] = {0};
  unsigned long long cnt = 0;
  if (act) {
    const int i = ii;
    const uint32_t io = J.idx_x[i];
    const double4 r = J.r64_x[i];
    const double ri[3] = {r.x, r.y, r.z};
    double vi[3] = {0, 0, 0};
    if (A.kind == K_HIST_REL || A.kind == K_HIST_DV)
      for (int a = 0; a < dim; ++a) vi[a] = J.vel64_x[(size_t)io * dim + a];
    const double4* __restrict__ R = A.cross ? J.r64_y : J.r64_x;
    const uint32_t* __restrict__ IX = A.cross ? J.idx_y : J.idx_x;
    const bool gather = A.kind == K_LJ_F;
    const int j0 = (A.cross || gather) ? jlo : max(jlo, i + 1);
    for (int j = j0; j < jhi; ++j) {
      if (!A.cross && j == i) continue;
      const double4 rr = R[j];
      const double rj[3] = {rr.x, rr.y, rr.z};
      double D[3];
      int K[3];
      double d2 = min_image64(A, ri, rj, D, K);
      if (!(d2 <= A.rc2)) continue;
      const bool own = A.cross || !gather || i < j;  // unordered contributions once
      if (own) cnt += 1;
      switch (A.kind) {
        case K_SUM_D: accE += sqrt(d2); break;
        case K_SUM_INV_D: accE += 1.0 / sqrt(d2); break;
        case K_SUM_W: accE += (r.w * rr.w) / sqrt(d2); break;
        case K_HIST_DV: {
          const int k = bin64(J.E64, J.nbins, (double)J.nbins / J.hist_hi, d2);
          atomicAdd(&J.hist[k], 1ull);
          if (k < J.nbins) {
            const uint32_t jo = IX[j];
            const double* vv = A.cross ? J.vel64_y : J.vel64_x;
            double dv[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) dv[a] = vv[(size_t)jo * dim + a] - vi[a];
            double qq = dv[0] * dv[0] + dv[1] * dv[1];
            if (dim == 3) qq = qq + dv[2] * dv[2];
            atomicAdd(&J.hist_sums[k], sqrt(qq));
          }
          break;
        }
        case K_LJ_E: case K_LJ_F: {
          const double r = rcp64(d2);
          double x = J.s2 * r, x3 = x * x * x;
          double u = x3 * x3 - x3;
          if (A.kind == K_LJ_E) { accE += u; break; }
          double f = (2.0 * x3 * x3 - x3) * r;
          accE += 0.5 * u;
          for (int a = 0; a < dim; ++a) G[a] += f * D[a];
          for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
              W[a * 3 + b] += 0.5 * f * D[a] * D[b];
              B[a * 3 + b] += 0.5 * f * D[a] * (double)K[b];
            }
          break;
        }
        case K_HIST_DIST: {
          int k = bin64(J.E64, J.nbins, (double)J.nbins / J.hist_hi, d2);
          atomicAdd(&J.hist[k], 1ull);
          break;
        }
        case K_HIST_REL: {
          uint32_t jo = IX[j];
          const double* vv = A.cross ? J.vel64_y : J.vel64_x;
          double dv[3] = {0, 0, 0};
          for (int a = 0; a < dim; ++a) dv[a] = vv[(size_t)jo * dim + a] - vi[a];
          double qq = dv[0] * dv[0] + dv[1] * dv[1];
          if (dim == 3) qq = qq + dv[2] * dv[2];
          int k = bin64(J.E64, J.nbins, (double)J.nbins / J.hist_hi, qq);
          atomicAdd(&J.hist[k], 1ull);
          if (J.want_sums && k < J.nbins) atomicAdd(&J.hist_sums[k], sqrt(qq));
          break;
        }
        case K_NL: {
          uint32_t jo = IX[j];
          uint32_t a = io, b = jo;
          if (!A.cross && a > b) { uint32_t tt = a; a = b; b = tt; }
          unsigned long long g = atomicAdd(J.nl_counter, 1ull);
          if ((long long)g < J.capacity) {
            J.pairs[2 * g] = (int32_t)a;
            J.pairs[2 * g + 1] = (int32_t)b;
            if (J.with_dist) J.dist[g] = sqrt(d2);
          }
          break;
        }
        default: break;
      }
    }
    if (A.kind == K_LJ_F) {
      // this chunk's share of the force on i, and of the wrap term G w^T
      // (linear in G, so it can be summed per chunk)
      double* fb = FB + ((size_t)blockIdx.y * A.n_x + i) * 3;
      for (int a = 0; a < 3; ++a) fb[a] = a < dim ? G[a] : 0.0;
      const int4 w = J.wrap_x[i];
      const int wv[3] = {w.x, w.y, w.z};
      for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) B[a * 3 + b] += G[a] * (double)wv[b];
    }
  }
  const int row = blockIdx.x + gridDim.x * blockIdx.y;
  double* Pp = J.partials + (size_t)row * kPartialD;
  const unsigned long long c = wave_sum_u64(cnt);
  const double e = wave_sum_d(accE);
  if (lane == 0) {
    J.pcount[row] = c;
    Pp[P_SUM] = e;
  }
  if (A.kind == K_LJ_F) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double v = wave_sum_d(W[k]);
      const double b = wave_sum_d(B[k]);
      if (lane == 0) {
        Pp[P_VIR + k] = v;
        Pp[P_BOX + k] = b;
      }
    }
  }
}

// Forces of the brute-force path: the per-chunk rows summed in chunk order.
__global__ void __launch_bounds__(256) brute_forces_kernel(const JobDesc* __restrict__ jobs, int n,
                                                           int dim, int nchunks,
                                                           const double* __restrict__ FB) {
  const JobDesc& J = jobs[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double G[3] = {0, 0, 0};
  for (int c = 0; c < nchunks; ++c)
    for (int a = 0; a < 3; ++a) G[a] += FB[((size_t)c * n + i) * 3 + a];
  const double mult = J.upstream ? *J.upstream : J.scale;
  const double s = mult * 24.0 * J.eps;
  const uint32_t io = J.idx_x[i];
  for (int a = 0; a < dim; ++a) J.forces[(size_t)io * dim + a] = s * G[a];
}

// ---------------------------------------------------------------- finalize
// Two-level fixed-order reduction of the per-tile partials of one job into
// the outputs: block b sums a contiguous range of tiles (strided by thread,
// then a tree in shared memory); one block then sums the block results in
// order.
__device__ __forceinline__ int final_slots(int kind) {
  return (kind == K_LJ_F || kind == K_LJ_FV) ? kPartialD : 1;
}

__global__ void __launch_bounds__(256) finalize1_kernel(const JobDesc* __restrict__ jobs, FinalArgs F,
                                                        double* __restrict__ scratch,
                                                        unsigned long long* __restrict__ scount) {
  const JobDesc& J = jobs[0];
  __shared__ double red[4][kPartialD];
  __shared__ unsigned long long redc[4];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  int nparts = F.nparts_dev ? min((int)*F.nparts_dev, F.nparts) : F.nparts;
  if (F.nparts_dev) nparts *= sweep_split(nparts, F.nparts, F.split_rows);
  const int chunk = (nparts + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(nparts, lo + chunk);
  const int nslots = final_slots(F.kind);
  // every slot at once: thread sums, then a shuffle tree per wave, then the
  // four waves in order
  unsigned long long c = 0;
  double v[kPartialD];
#pragma unroll
  for (int q = 0; q < kPartialD; ++q) v[q] = 0.0;
  for (int k = lo + tid; k < hi; k += 256) {
    c += J.pcount[k];
#pragma unroll
    for (int q = 0; q < kPartialD; ++q)
      if (q < nslots) v[q] += J.partials[(size_t)k * kPartialD + q];
  }
  c = wave_sum_u64(c);
  if (lane == 0) redc[w] = c;
#pragma unroll
  for (int q = 0; q < kPartialD; ++q) {
    if (q < nslots) {
      const double t = wave_sum_d(v[q]);
      if (lane == 0) red[w][q] = t;
    }
  }
  __syncthreads();
  if (tid == 0) scount[blockIdx.x] = ((redc[0] + redc[1]) + redc[2]) + redc[3];
  if (tid < nslots) scratch[(size_t)blockIdx.x * kPartialD + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// One block of kFinalBlocks threads: the block results in a fixed order
// (shuffle trees, then the waves in order); thread q writes output slot q.
__global__ void __launch_bounds__(kFinalBlocks) finalize2_kernel(FinalArgs F,
                                                                 const double* __restrict__ scratch,
                                                                 const unsigned long long* __restrict__ scount) {
  constexpr int kW = kFinalBlocks / kWave;
  __shared__ double red[kW][kPartialD];
  __shared__ unsigned long long redc[kW];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int nslots = final_slots(F.kind);
  const unsigned long long c = wave_sum_u64(scount[tid]);
  if (lane == 0) redc[w] = c;
#pragma unroll
  for (int q = 0; q < kPartialD; ++q) {
    if (q < nslots) {
      const double t = wave_sum_d(scratch[(size_t)tid * kPartialD + q]);
      if (lane == 0) red[w][q] = t;
    }
  }
  __syncthreads();
  if (tid == 0 && F.count) {
    unsigned long long n = 0;
    for (int k = 0; k < kW; ++k) n += redc[k];
    *F.count = F.halve_count ? n / 2 : n;
  }
  if (tid < nslots) {
    const int slot = tid;
    double tot = 0.0;
    for (int k = 0; k < kW; ++k) tot += red[k][slot];
    if (slot == P_SUM && F.energy) {
      const bool lj = F.kind == K_LJ_E || F.kind == K_LJ_F || F.kind == K_LJ_FV;
      *F.energy = (lj ? 4.0 * F.eps : 1.0) * tot;
    } else if (slot >= P_VIR && slot < P_VIR + 9 && F.virial && F.want_virial) {
      const int k = slot - P_VIR, a = k / 3, b = k % 3;
      if (a < F.dim && b < F.dim) F.virial[a * F.dim + b] = 24.0 * F.eps * tot;
    } else if (slot >= P_BOX && slot < P_BOX + 9 && F.grad_box) {
      const int k = slot - P_BOX, a = k / 3, b = k % 3;
      const double g = F.upstream ? *F.upstream : F.box_mult;
      if (a < F.dim && b < F.dim) F.grad_box[a * F.dim + b] = -24.0 * F.eps * g * tot;
    }
  }
}

// Relative-speed band from the largest velocity component (see clmap_api).
__global__ void relspeed_band_kernel(const unsigned int* __restrict__ vmax_bits, double hi, int dim,
                                     double* __restrict__ bandq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double u = 5.9604644775390625e-08;  // 2^-24
    double vmax = (double)__uint_as_float(*vmax_bits);
    // per-component error of the FP32 velocity difference near an edge
    // (|dv| <= 1.01 hi): u (|v_i| + |v_j| + |dv|), plus FP64 slack
    double Ea = u * (2.0 * vmax + 1.01 * hi) * (1.0 + 1e-6) + 1e-300;
    double E = sqrt((double)dim) * Ea;
    // error of q = |dv|^2 (FMA chain: 3 roundings), doubled for safety, plus
    // the FP32 rounding of the edge table
    double b = 2.0 * (2.02 * hi * E + E * E + 4.1 * u * hi * hi) + 2.0 * u * hi * hi;
    *bandq = b;
  }
}

// Candidate pairs of the cell method on this grid (the roofline's unit):
// for every cell c, its particles times those of each cell of its stencil
// (the half shell: the lx cells after c in its row and the whole reach of
// the rows with (dz, dy) > (0, 0), plus the pairs within c; cross sets: the
// x particles of c times the y particles of the full stencil).  One thread
// per cell; block sums added to out[0] (integers: any order is exact).
__global__ void __launch_bounds__(256) candidates_kernel(const JobDesc* __restrict__ jobs, int full,
                                                         unsigned long long* out) {
  const JobDesc& J = jobs[0];
  const int nx = J.n[0], ny = J.n[1], nz = J.dim == 3 ? J.n[2] : 1;
  const int ncell = nx * ny * nz;
  const int cid = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c = 0;
  if (cid < ncell) {
    const int l = J.lcell, lx = J.lcell_x, dim = J.dim;
    const bool fs = full || J.cross;
    const uint32_t* offx = J.off_x;
    const uint32_t* offy = J.cross ? J.off_y : J.off_x;
    const int cx = cid % nx, cy = (cid / nx) % ny, cz = cid / (nx * ny);
    const unsigned long long ni = offx[cid + 1] - offx[cid];
    if (ni != 0ull) {
      unsigned long long nj = 0;  // candidates of one particle of c in other cells
      for (int dz = dim == 3 ? -l : 0; dz <= (dim == 3 ? l : 0); ++dz)
        for (int dy = -l; dy <= l; ++dy) {
          if (!fs && (dz < 0 || (dz == 0 && dy < 0))) continue;
          const bool home = dz == 0 && dy == 0;
          const int uy = (cy + dy + ny) % ny, uz = dim == 3 ? (cz + dz + nz) % nz : 0;
          const int rowbase = (uy + ny * uz) * nx;
          const int xlo = (home && !fs) ? cx + 1 : cx - lx;
          for (int ux = xlo; ux <= cx + lx; ++ux) {
            if (home && ux == cx) continue;  // the cell itself: below
            const int cc = rowbase + ((ux % nx) + nx) % nx;
            nj += offy[cc + 1] - offy[cc];
          }
        }
      c = ni * nj;
      if (J.cross) c += ni * (unsigned long long)(offy[cid + 1] - offy[cid]);
      else c += fs ? ni * (ni - 1ull) : ni * (ni - 1ull) / 2ull;
    }
  }
  __shared__ unsigned long long red[256 / kWave];
  for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < 256 / kWave; ++k) t += red[k];
    if (t) atomicAdd(out, t);
  }
}

// ---------------------------------------------------------------- job tables
__global__ void set_job_kernel(JobDesc jd, JobDesc* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = jd;
}

// Canonical histogram edges: h = hi/nb, e_k = k*h, E_k = e_k*e_k (FP64, each
// operation rounded on its own); E_nb = rc2 for a distance histogram up to
// the cutoff.  E32 = nearest FP32 value.
__global__ void hist_edges_kernel(double* E64, float* E32, int nb, double hi, int force_last,
                                  double rc2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nb) return;
  double h = hi / (double)nb;
  double e = (double)k * h;
  double E = e * e;
  if (force_last && k == nb) E = rc2;
  E64[k] = E;
  E32[k] = (float)E;
}

// ---------------------------------------------------------------- batched jobs
// Block b appends job b's tiles to the launched list: its offset is the sum
// of the preceding jobs' (device) tile counts; the job id and offset are
// recorded for the sweep and the finalize.
__global__ void __launch_bounds__(256) gather_tiles_kernel(JobDesc* __restrict__ jobs, int njobs,
                                                           Tile* __restrict__ tiles,
                                                           uint32_t* __restrict__ total) {
  const int b = blockIdx.x;
  __shared__ int begin_s;
  if (threadIdx.x == 0) {
    int beg = 0;
    for (int k = 0; k < b; ++k) beg += min((int)*jobs[k].own_ntiles, jobs[k].own_max_tiles);
    begin_s = beg;
    const int cnt = min((int)*jobs[b].own_ntiles, jobs[b].own_max_tiles);
    jobs[b].tile_begin = beg;
    jobs[b].tile_end = beg + cnt;
    if (b == njobs - 1) *total = (uint32_t)(beg + cnt);
  }
  __syncthreads();
  const int beg = begin_s;
  const int cnt = min((int)*jobs[b].own_ntiles, jobs[b].own_max_tiles);
  const Tile* src = jobs[b].own_tiles;
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    Tile t = src[k];
    t.job = (uint16_t)b;
    tiles[beg + k] = t;
  }
}

// One block per job: fixed-order reduction of the job's tile partials.
__global__ void __launch_bounds__(256) finalize_batch_kernel(const JobDesc* __restrict__ jobs,
                                                             const FinalArgs* __restrict__ FA) {
  const JobDesc& J = jobs[blockIdx.x];
  const FinalArgs F = FA[blockIdx.x];
  __shared__ double red[256];
  __shared__ unsigned long long redc[256];
  const int tid = threadIdx.x;
  const int nparts = J.tile_end - J.tile_begin;
  unsigned long long c = 0;
  for (int k = tid; k < nparts; k += 256) c += J.pcount[k];
  redc[tid] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) redc[tid] += redc[tid + st];
    __syncthreads();
  }
  if (tid == 0 && F.count) *F.count = F.halve_count ? redc[0] / 2 : redc[0];
  const int nslots = final_slots(F.kind);
  for (int slot = 0; slot < nslots; ++slot) {
    double v = 0.0;
    for (int k = tid; k < nparts; k += 256) v += J.partials[(size_t)k * kPartialD + slot];
    red[tid] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) {
      const double tot = red[0];
      if (slot == P_SUM && F.energy) {
        const bool lj = F.kind == K_LJ_E || F.kind == K_LJ_F || F.kind == K_LJ_FV;
        *F.energy = (lj ? 4.0 * F.eps : 1.0) * tot;
      } else if (slot >= P_VIR && slot < P_VIR + 9 && F.virial && F.want_virial) {
        const int k = slot - P_VIR, a = k / 3, b = k % 3;
        if (a < F.dim && b < F.dim) F.virial[a * F.dim + b] = 24.0 * F.eps * tot;
      } else if (slot >= P_BOX && slot < P_BOX + 9 && F.grad_box) {
        const int k = slot - P_BOX, a = k / 3, b = k % 3;
        const double g = F.upstream ? *F.upstream : F.box_mult;
        if (a < F.dim && b < F.dim) F.grad_box[a * F.dim + b] = -24.0 * F.eps * g * tot;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- neighbour-list offsets
// One block: exclusive prefix sums of the n = tiles * G per-item pair counts
// of a counting sweep; thread t scans a contiguous chunk.
__global__ void __launch_bounds__(1024) nl_offsets_kernel(const unsigned long long* __restrict__ pcount,
                                                          const uint32_t* __restrict__ ntiles_dev, int cap,
                                                          int split_rows, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[1024];
  const int nt = min((int)*ntiles_dev, cap);
  const int n = nt * sweep_split(nt, cap, split_rows);
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  unsigned long long s = 0;
  for (int k = lo; k < hi; ++k) s += pcount[k];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the chunk sums
    const unsigned long long v = t >= d ? part[t - d] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long run = part[t] - s;
  for (int k = lo; k < hi; ++k) {
    out[k] = run;
    run += pcount[k];
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_nl_offsets(const unsigned long long* pcount, const uint32_t* ntiles_dev, int max_tiles,
                             int split_rows, unsigned long long* offsets, hipStream_t s) {
  if (max_tiles <= 0) return hipSuccess;
  nl_offsets_kernel<<<1, 1024, 0, s>>>(pcount, ntiles_dev, max_tiles, split_rows, offsets);
  return hipGetLastError();
}

hipError_t launch_gather_tiles(JobDesc* jobs, int njobs, Tile* tiles, uint32_t* total,
                               hipStream_t s) {
  gather_tiles_kernel<<<njobs, 256, 0, s>>>(jobs, njobs, tiles, total);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const JobDesc* jobs, const FinalArgs* F, int njobs, hipStream_t s) {
  finalize_batch_kernel<<<njobs, 256, 0, s>>>(jobs, F);
  return hipGetLastError();
}

template <int DIM, bool FP32>
static hipError_t sweep_dispatch(int kind, dim3 grid, size_t lds, const JobDesc* jobs,
                                 const Tile* tiles, const uint32_t* nt, int split, hipStream_t s) {
  switch (kind) {
    case K_COUNT: sweep_kernel<DIM, FP32, K_COUNT><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_SUM_D: sweep_kernel<DIM, FP32, K_SUM_D><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_SUM_INV_D: sweep_kernel<DIM, FP32, K_SUM_INV_D><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_LJ_E: sweep_kernel<DIM, FP32, K_LJ_E><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_LJ_F: sweep_kernel<DIM, FP32, K_LJ_F><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_LJ_FV: sweep_kernel<DIM, FP32, K_LJ_FV><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_HIST_DIST: sweep_kernel<DIM, FP32, K_HIST_DIST><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_HIST_REL: sweep_kernel<DIM, FP32, K_HIST_REL><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_SUM_W: sweep_kernel<DIM, FP32, K_SUM_W><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_HIST_DV: sweep_kernel<DIM, FP32, K_HIST_DV><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    case K_NL: sweep_kernel<DIM, FP32, K_NL><<<grid, kSweepWaves * kWave, lds, s>>>(jobs, tiles, nt, split); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep(int dim, bool fp32, int kind, const JobDesc* jobs, const Tile* tiles,
                        const uint32_t* ntiles_dev, int max_tiles, int nbins, hipStream_t s,
                        int split_rows) {
  if (max_tiles <= 0) return hipSuccess;
  const int split = split_rows;
  const int waves = kSweepWaves;
  dim3 grid((max_tiles + waves - 1) / waves);
  size_t lds = sweep_lds_per_wave(kind, nbins, fp32) * waves;
  if (dim == 3)
    return fp32 ? sweep_dispatch<3, true>(kind, grid, lds, jobs, tiles, ntiles_dev, split, s)
                : sweep_dispatch<3, false>(kind, grid, lds, jobs, tiles, ntiles_dev, split, s);
  return fp32 ? sweep_dispatch<2, true>(kind, grid, lds, jobs, tiles, ntiles_dev, split, s)
              : sweep_dispatch<2, false>(kind, grid, lds, jobs, tiles, ntiles_dev, split, s);
}

hipError_t launch_brute(const JobDesc* jobs, const BruteArgs& A, double* FB, int* nparts_out,
                        hipStream_t s) {
  const int ny = A.cross ? A.n_y : A.n_x;
  const int nib = std::max(1, (A.n_x + kWave - 1) / kWave);
  const int njb = brute_chunks(ny);
  const int jchunk = std::max(1, (ny + njb - 1) / njb);
  *nparts_out = nib * njb;
  brute_kernel<<<dim3(nib, njb), kWave, 0, s>>>(jobs, A, jchunk, FB);
  if (A.kind == K_LJ_F && A.n_x > 0)
    brute_forces_kernel<<<(A.n_x + 255) / 256, 256, 0, s>>>(jobs, A.n_x, A.dim, njb, FB);
  return hipGetLastError();
}

hipError_t launch_finalize(const JobDesc* jobs, const FinalArgs& F, double* scratch,
                           unsigned long long* scount, hipStream_t s) {
  finalize1_kernel<<<kFinalBlocks, 256, 0, s>>>(jobs, F, scratch, scount);
  finalize2_kernel<<<1, kFinalBlocks, 0, s>>>(F, scratch, scount);
  return hipGetLastError();
}

hipError_t launch_candidates(const JobDesc* jobs, int ncells, int full, unsigned long long* out,
                             hipStream_t s) {
  hipError_t e = launch_fill_u64(out, 1, 0ull, s);
  if (e != hipSuccess) return e;
  if (ncells > 0) candidates_kernel<<<(ncells + 255) / 256, 256, 0, s>>>(jobs, full, out);
  return hipGetLastError();
}

hipError_t launch_set_job(const JobDesc& jd, JobDesc* dst, hipStream_t s) {
  set_job_kernel<<<1, 64, 0, s>>>(jd, dst);
  return hipGetLastError();
}

hipError_t launch_hist_edges(double* E64, float* E32, int nbins, double hi, int force_last,
                             double rc2, hipStream_t s) {
  hist_edges_kernel<<<(nbins + 1 + 255) / 256, 256, 0, s>>>(E64, E32, nbins, hi, force_last, rc2);
  return hipGetLastError();
}

hipError_t launch_relspeed_band(const unsigned int* vmax_bits, double hi, int dim, double* bandq,
                                hipStream_t s) {
  relspeed_band_kernel<<<1, 64, 0, s>>>(vmax_bits, hi, dim, bandq);
  return hipGetLastError();
}

}  // namespace clm
