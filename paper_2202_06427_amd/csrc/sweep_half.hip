// sweep_half.hip -- Lennard-Jones energy + forces (+ box gradient, virial)
// over the half shell in the FP32 + FP64-guard form: every unordered pair is
// evaluated once (paper section 2.8: a cell and half of its neighbour cells),
// both particles' force sums are kept, and no atomics decide the summation
// order (repeated maps give bitwise-identical results).
//
// Work item: (home cell row h, half-shell row offset rho).  A row is the run
// of cells (0..nx-1, cy, cz); rho = 0 is the home row itself (pairs j > i in
// sorted order, cells forward along x), rho > 0 the neighbour rows with
// (dz, dy) > (0, 0).  One wavefront runs one item: for each tile of row h
// (<= 64 consecutive sorted particles, one per lane) it scans the tile's
// reach in row r = h + offset(rho) (one to three pieces of consecutive
// cells, with their periodic images).  The tile's two halves (lanes 0..31:
// its first 32 particles; lanes 32..63: the others) keep separate candidate
// lists: a candidate enters a half's list when its distance to that half's
// bounding box is within the cutoff (the paper's section 2.8 pruning of
// candidates by their position, applied to 32 particles at a time).
//
// A block pairs up to 32 candidates of each list with its half in 32 steps
// (JW = 32; when neither list has more than 16 left, 16 steps with the 16
// candidates in both rows of the half).  In step (phase g, k) lane l pairs
// its i with the candidate that a DPP row rotation by k brings from its
// 16-lane row; between the two phases the candidates move by 16 lanes inside
// their half.  The rotation is folded into the subtractions (v_sub_f32 with
// a DPP source) and the candidate-side force term goes back through the
// inverse rotation folded into an add: a step is 26 VALU instructions (one
// of them a quarter-rate reciprocal) for 64 pairs.  Coordinates are in units
// of sigma, so x = sigma^2 / d^2 is one reciprocal.
//
// Force sums: per lane, the i-side FP32 sum of a block is folded into FP64;
// the candidate-side FP32 sum of a block (the copies added) is added (FP64
// arithmetic, one FP32 rounding) into a FP32 plane slot owned by this item
// and half alone:
//     plane 3 rho     : i-side sums of item (row(i), rho)
//     plane 3 rho + 1 : j-side sums of half A of item (row(j) - offset(rho), rho)
//     plane 3 rho + 2 : the same for half B
// All are indexed by sorted index, so every slot has exactly one writer; a
// gather kernel sums the 3 NR planes of each particle in FP64 in a fixed
// order.
//
// FP32 coordinates: relative to the centre O of the bounding box of the
// lane's half of the tile, x_i = fl32((r'_i - O) / sigma) and
// x_j = fl32((r'_j + t - O) / sigma), computed in FP64.  |x_i,a| <= C_a,
// half that box's extent (at most the tile's: span cells along x, one cell
// across), and |x_j,a| <= C_a + |D_a|, so
// |D32_a - D_a| <= u (2 C_a + 2 |D_a|) + FP64 roundings (in sigma units):
// the steep pairs (|D| near sigma) keep small errors when the tile is
// compact.  The membership band comes from that bound per tile span (host
// table).  Pairs within the band of rc^2, and pairs closer than the near
// threshold, are queued per wave and evaluated in canonical FP64.
#include "clmap_internal.h"
#include "device_util.h"

namespace clm {

namespace {

constexpr int kHQCap = 320;   // FP64 re-evaluation queue (>= 63 + 4 * 64 entries)
constexpr int kHLCap = 128;   // each half's packed candidate ring (power of two, >= 63 + 64)
constexpr uint32_t kCenter = 13u;  // image code of K = (0, 0, 0)

template <int K>
__device__ __forceinline__ float row_ror(float v) {  // lane p reads lane (p - K) mod 16 of its row
  if constexpr (K == 0) {
    return v;
  } else {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + K, 0xF, 0xF, true));
  }
}
template <int K>
__device__ __forceinline__ int row_ror_i(int v) {
  if constexpr (K == 0) {
    return v;
  } else {
    return __builtin_amdgcn_mov_dpp(v, 0x120 + K, 0xF, 0xF, true);
  }
}
// inverse of row_ror<K>
template <int K>
__device__ __forceinline__ float row_back(float v) {
  if constexpr (K == 0) {
    return v;
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + (16 - K),
                                                                0xF, 0xF, true));
  }
}

__device__ __forceinline__ float shfl_f(float v, int src_byte) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src_byte, __builtin_bit_cast(int, v)));
}

// The same lane moves for FP64 values (two 32-bit halves each).
template <int K>
__device__ __forceinline__ double row_ror(double v) {
  if constexpr (K == 0) {
    return v;
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x120 + K, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x120 + K, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
}
template <int K>
__device__ __forceinline__ double row_back(double v) {
  if constexpr (K == 0) {
    return v;
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x120 + (16 - K), 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x120 + (16 - K), 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
}
__device__ __forceinline__ double shfl_f(double v, int src_byte) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src_byte, (int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src_byte, (int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rcp_t(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_t(double v) { return rcp64(v); }

// (dy, dz) of half-shell row offset rho: 0 -> home row; then (0, 1..l);
// then dz = 1..l with dy = -l..l.  2D: dz = 0, dy = 0..l.
__device__ __forceinline__ void row_offset(int l, int rho, int* dy, int* dz) {
  if (rho == 0) {
    *dy = 0;
    *dz = 0;
    return;
  }
  if (rho <= l) {
    *dy = rho;
    *dz = 0;
    return;
  }
  const int q = rho - l - 1;  // 3D only
  *dz = 1 + q / (2 * l + 1);
  *dy = q % (2 * l + 1) - l;
}

template <int DIM, bool VIR, typename T>
struct Half {
  const JobDesc* J;
  int lane;
  // uniform
  double rc2, s2, inv_sig;
  T near2f;                // (near_factor)^2: sigma units
  T lo, hi;                // membership thresholds on d^2 / sigma^2
  // the tile's two halves (lanes 0..31 and 32..63): origins of the sweep's
  // coordinates, the centres of their bounding boxes (uniform)
  double OA[3], OB[3];
  // per lane (i side, fixed for a tile)
  T xi[3];                 // relative to the origin of the lane's half, sigma units
  double Fi[3];
  // per lane accumulators of the item
  double E64;
  double B[9];
  double W[6];
  uint32_t qband, qnear;
  unsigned long long cnt;  // wave-uniform
  unsigned long long ntested, nkept;  // wave-uniform: (tile particle, candidate) pairs before / after pruning
  // per block
  T xj[3];
  T acc[3];
  int key;                 // home row: candidate's sorted index (pairs only j > i), else INT_MAX
  T e32;
  T fi32[3];
  T w32[6];
  // LDS
  uint32_t* Q;             // queue of FP64 re-evaluations: i lane | candidate << 6 | band << 31
  double* GA;              // [64][3] FP64 i-side sums of queued pairs
  double* GJ;              // [64][3] FP64 sums of f D (i -> j) of queued pairs, by candidate
  uint2* LST;              // packed candidates (sorted index, image code): list A, then list B
  uint2* BC;               // [64] the current block's candidates by slot
  double* RI;              // [64][3] FP64 positions of the tile's particles, by lane
  double* RJ;              // [64][3] FP64 positions of the block's candidates, by slot
  uint32_t qtail;          // queued entries: Q[0 .. qtail)
  uint32_t lhA, ltA, lhB, ltB;  // ring positions of lists A and B
  uint32_t tstart;

  // ---------------------------------------------------------------- FP64 queue
  // Canonical FP64 evaluation of one queued pair (i lane il, candidate slot
  // jm of the current block).
  __device__ __forceinline__ void process(uint32_t e, bool* in_out) {
    const int il = (int)(e & 63u), jm = (int)((e >> 6) & 63u);
    const uint2 c = BC[jm];
    const double* rI = &RI[il * 3];
    const double* rJ = &RJ[jm * 3];
    const double* tk = &J->tK[c.y * 4];
    double D[3];
    D[0] = (rJ[0] - rI[0]) + tk[0];
    D[1] = (rJ[1] - rI[1]) + tk[1];
    double d2 = D[0] * D[0] + D[1] * D[1];
    if (DIM == 3) {
      D[2] = (rJ[2] - rI[2]) + tk[2];
      d2 = d2 + D[2] * D[2];
    } else {
      D[2] = 0.0;
    }
    *in_out = d2 <= rc2;
    if (!(d2 <= rc2)) return;
    const double r = rcp64(d2);
    const double x = s2 * r;
    const double x3 = x * x * x;
    const double u = x3 * x3 - x3;
    const double f = (2.0 * x3 * x3 - x3) * r;
    E64 += u;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      atomicAdd(&GA[il * 3 + a], f * D[a]);
      atomicAdd(&GJ[jm * 3 + a], f * D[a]);
    }
    // (the image term f D p^T of the box gradient is added with the block's
    // candidate-side sums, which include GJ)
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
  }

  __device__ __forceinline__ void drain(bool all) {
    uint32_t h = 0;
    const uint32_t tl = (uint32_t)uniform((int)qtail);
    while (tl - h >= (uint32_t)kWave || (all && tl != h)) {
      const uint32_t nb = min(tl - h, (uint32_t)kWave);
      bool band_in = false;
      if ((uint32_t)lane < nb) {
        const uint32_t e = Q[h + (uint32_t)lane];
        bool in = false;
        process(e, &in);
        const bool band = (e >> 31) != 0u;  // above lo in FP32: FP64 decides and counts
        qband += band ? 1u : 0u;
        qnear += band ? 0u : 1u;
        band_in = band && in;
      }
      cnt += (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(band_in));
      h = (uint32_t)uniform((int)(h + nb));
    }
    // what is left (fewer than 64 entries) moves to the front
    const uint32_t left = tl - h;
    if (h != 0u && left != 0u) {
      uint32_t e = 0u;
      if ((uint32_t)lane < left) e = Q[h + (uint32_t)lane];
      __builtin_amdgcn_wave_barrier();
      if ((uint32_t)lane < left) Q[lane] = e;
      __builtin_amdgcn_wave_barrier();
    }
    qtail = left;
  }

  // ---------------------------------------------------------------- one step
  // jtag: (candidate held by this lane) << 6.
  template <int K, bool SELF, int JW>
  __device__ __forceinline__ void step(int jtag) {
    const T dx = row_ror<K>(xj[0]) - xi[0];
    const T dy = row_ror<K>(xj[1]) - xi[1];
    const T dz = DIM == 3 ? row_ror<K>(xj[2]) - xi[2] : T(0);
    const T d2 = DIM == 3 ? fma_t(dz, dz, fma_t(dy, dy, dx * dx)) : fma_t(dy, dy, dx * dx);
    unsigned long long okm = ~0ull;
    if constexpr (SELF) okm = __builtin_amdgcn_ballot_w64(row_ror_i<K>(key) > (int)(tstart + (uint32_t)lane));
    const unsigned long long mlo = __builtin_amdgcn_ballot_w64(d2 <= lo) & okm;
    const unsigned long long mhi = __builtin_amdgcn_ballot_w64(d2 <= hi) & okm;
    const unsigned long long mnr = __builtin_amdgcn_ballot_w64(d2 < near2f) & okm;
    cnt += (unsigned long long)__popcll(mlo);
    const bool fast = __builtin_amdgcn_inverse_ballot_w64(mlo & ~mnr);
    const T x = fast ? rcp_t(d2) : T(0);  // sigma^2 / d^2
    const T x3 = x * x * x;
    const T u = fma_t(x3, x3, -x3);
    e32 += u;
    const T f = fma_t(T(2), u, x3) * x;
    const T tx = f * dx, ty = f * dy, tz = f * dz;
    fi32[0] += tx;
    fi32[1] += ty;
    acc[0] += row_back<K>(tx);
    acc[1] += row_back<K>(ty);
    if (DIM == 3) {
      fi32[2] += tz;
      acc[2] += row_back<K>(tz);
    }
    if constexpr (VIR) {
      w32[0] = fma_t(tx, dx, w32[0]);
      w32[1] = fma_t(tx, dy, w32[1]);
      w32[3] = fma_t(ty, dy, w32[3]);
      if (DIM == 3) {
        w32[2] = fma_t(tx, dz, w32[2]);
        w32[4] = fma_t(ty, dz, w32[4]);
        w32[5] = fma_t(tz, dz, w32[5]);
      }
    }
    // keep the accumulator updates in this step (an empty asm that reads and
    // redefines them): left free, the scheduler defers them past later steps
    // and spills the pending terms
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(fi32[0]), "+v"(fi32[1]),
                 "+v"(fi32[2]), "+v"(e32));
    if constexpr (VIR)
      asm volatile("" : "+v"(w32[0]), "+v"(w32[1]), "+v"(w32[2]), "+v"(w32[3]), "+v"(w32[4]),
                   "+v"(w32[5]));
    const unsigned long long band = mhi & ~mlo;
    const unsigned long long spec = band | mnr;
    if (spec) {
      // entry: i lane | candidate << 6 | band << 31 (jtag rotates with the
      // candidates; the DPP read happens with every lane active: a source
      // lane outside exec would read as 0)
      uint32_t ent = (uint32_t)row_ror_i<K>(jtag) | (uint32_t)lane;
      if (band) ent = __builtin_amdgcn_inverse_ballot_w64(band) ? (ent | 0x80000000u) : ent;  // rare
      const uint32_t t0 = qtail;
      // byte offset of the lane's slot in the ring
      if (__builtin_amdgcn_inverse_ballot_w64(spec)) Q[(uint32_t)lane_rank(spec) + t0] = ent;
      qtail = t0 + (uint32_t)__popcll(spec);
    }
  }

  // 16 steps; the queue is drained (64 entries at a time) after every 4
  // steps, so it never holds more than 63 + 4 * 64 entries
  template <bool SELF, int JW>
  __device__ __forceinline__ void phase(int jtag) {
    step<0, SELF, JW>(jtag); step<1, SELF, JW>(jtag); step<2, SELF, JW>(jtag); step<3, SELF, JW>(jtag);
    if (qtail >= (uint32_t)kWave) drain(false);
    step<4, SELF, JW>(jtag); step<5, SELF, JW>(jtag); step<6, SELF, JW>(jtag); step<7, SELF, JW>(jtag);
    if (qtail >= (uint32_t)kWave) drain(false);
    step<8, SELF, JW>(jtag); step<9, SELF, JW>(jtag); step<10, SELF, JW>(jtag); step<11, SELF, JW>(jtag);
    if (qtail >= (uint32_t)kWave) drain(false);
    step<12, SELF, JW>(jtag); step<13, SELF, JW>(jtag); step<14, SELF, JW>(jtag); step<15, SELF, JW>(jtag);
    if (qtail >= (uint32_t)kWave) drain(false);
  }

  // One block: nA (0..JW) candidates of list A from ring position bA for the
  // lanes 0..31 (the tile's first 32 particles) and nB of list B from bB for
  // the lanes 32..63 (the others).  JW = 32: a candidate per lane, rotating
  // by 16 lanes inside its half between the two phases; JW = 16: the 16
  // candidates of a half sit in both of its rows (two copies).  A candidate's
  // slot is its lane (JW = 32) or its lane in the half's first row (JW = 16).
  // pjA / pjB: this item's j-side planes of the two halves.
  template <bool SELF, int JW>
  __device__ __forceinline__ void block(uint32_t nA, uint32_t bA, uint32_t nB, uint32_t bB, T* pjA, T* pjB,
                                        size_t npad) {
    const bool hb = lane >= 32;  // lane in half B
    const int m = lane & (JW - 1);
    const bool jv = (uint32_t)m < (hb ? nB : nA);
    const bool canon = JW == 32 || (lane & 16) == 0;  // the lane that owns the candidate's sums
    const int slot = JW == 32 ? lane : ((lane & 15) | (lane & 32));
    const uint32_t pos = ((hb ? bB : bA) + (uint32_t)m) & (uint32_t)(kHLCap - 1);
    const uint2 c = jv ? LST[(hb ? kHLCap : 0) + pos] : make_uint2(0u, kCenter);
    T* pj = hb ? pjB : pjA;
    const double* tK = J->tK;
    {
      const double4 r = jv ? J->r64_x[c.x] : make_double4(0.0, 0.0, 0.0, 0.0);
      const double* t = &tK[c.y * 4];
      xj[0] = jv ? (T)(((r.x + t[0]) - (hb ? OB[0] : OA[0])) * inv_sig) : T(-1e18);
      xj[1] = jv ? (T)(((r.y + t[1]) - (hb ? OB[1] : OA[1])) * inv_sig) : T(-1e18);
      xj[2] = DIM == 3 ? (jv ? (T)(((r.z + t[2]) - (hb ? OB[2] : OA[2])) * inv_sig) : T(-1e18)) : T(0);
      if (canon) {  // the candidate's FP64 position for queued pairs
        RJ[slot * 3 + 0] = r.x;
        RJ[slot * 3 + 1] = r.y;
        RJ[slot * 3 + 2] = r.z;
      }
    }
    if constexpr (SELF) key = (jv && c.y == kCenter) ? (int)c.x : 0x7fffffff;
    T jold[3] = {T(0), T(0), T(0)};
    if (jv && canon) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) jold[a] = pj[(size_t)a * npad + c.x];
    }
    if (canon) BC[slot] = c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc[a] = T(0);
      fi32[a] = T(0);
      GJ[lane * 3 + a] = 0.0;
    }
    e32 = T(0);
    if constexpr (VIR) {
#pragma unroll
      for (int k = 0; k < 6; ++k) w32[k] = T(0);
    }
    __builtin_amdgcn_wave_barrier();
    int jtag = slot << 6;
    if constexpr (JW == 32) {
      const int src = ((lane & 32) | ((lane + 16) & 31)) << 2;  // 16 lanes on inside the half
      phase<SELF, JW>(jtag);
#pragma unroll
      for (int a = 0; a < DIM; ++a) xj[a] = shfl_f(xj[a], src);
      if constexpr (SELF) key = __builtin_amdgcn_ds_bpermute(src, key);
#pragma unroll
      for (int a = 0; a < DIM; ++a) acc[a] = shfl_f(acc[a], src);
      jtag = __builtin_amdgcn_ds_bpermute(src, jtag);
      phase<SELF, JW>(jtag);
#pragma unroll
      for (int a = 0; a < DIM; ++a) acc[a] = shfl_f(acc[a], src);  // back in place
    } else {
      phase<SELF, JW>(jtag);
      // the two copies of each candidate's sums
#pragma unroll
      for (int a = 0; a < DIM; ++a) acc[a] += shfl_f(acc[a], (lane ^ 16) << 2);
    }
    drain(true);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // fold the block into FP64 (sigma units: forces times 1/sigma, virial as is)
    E64 += (double)e32;
#pragma unroll
    for (int a = 0; a < DIM; ++a) Fi[a] += (double)fi32[a] * inv_sig;
    if constexpr (VIR) {
#pragma unroll
      for (int k = 0; k < 6; ++k) W[k] += (double)w32[k];
    }
    if (jv && canon) {
      double S[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        S[a] = (double)acc[a] * inv_sig + GJ[slot * 3 + a];
        pj[(size_t)a * npad + c.x] = (T)((double)jold[a] - S[a]);
      }
      if (c.y != kCenter) {  // a periodic image: the box-gradient term S p^T
        const int p[3] = {(int)(c.y % 3u) - 1, (int)((c.y / 3u) % 3u) - 1, (int)(c.y / 9u) - 1};
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int b = 0; b < DIM; ++b) B[a * 3 + b] += S[a] * (double)p[b];
      }
    }
  }

  // Blocks while both lists hold 32 candidates or one holds 64: afterwards
  // each holds fewer than 64, so the next scan (at most 64 more per list)
  // stays within the ring.
  template <bool SELF>
  __device__ __forceinline__ void run_full(T* pjA, T* pjB, size_t npad) {
    for (;;) {
      const uint32_t a = ltA - lhA, b = ltB - lhB;
      if (!((a >= 32u && b >= 32u) || a >= 64u || b >= 64u)) break;
      const uint32_t nA = min(a, 32u), nB = min(b, 32u);
      block<SELF, 32>(nA, lhA, nB, lhB, pjA, pjB, npad);
      lhA += nA;
      lhB += nB;
    }
  }

  // The rest of both lists at the end of a tile: blocks of 32, the last one
  // of 16 when neither list has more than 16 left.
  template <bool SELF>
  __device__ __forceinline__ void run_tail(T* pjA, T* pjB, size_t npad) {
    for (;;) {
      const uint32_t a = ltA - lhA, b = ltB - lhB;
      if (a == 0u && b == 0u) break;
      if (a > 16u || b > 16u) {
        const uint32_t nA = min(a, 32u), nB = min(b, 32u);
        block<SELF, 32>(nA, lhA, nB, lhB, pjA, pjB, npad);
        lhA += nA;
        lhB += nB;
      } else {
        block<SELF, 16>(a, lhA, b, lhB, pjA, pjB, npad);
        lhA += a;
        lhB += b;
      }
    }
  }
};

template <int DIM, bool VIR, typename T, bool SELF>
__device__ __forceinline__ void run_tiles(Half<DIM, VIR, T>& S, const HalfArgs& A, int h, int py, int pz,
                                          int rbase, T* part_i, T* pjA, T* pjB) {
  const JobDesc* J = S.J;
  const int lane = S.lane;
  const int nx = ldu(&J->n[0]), lx = ldu(&J->lcell_x);
  const uint32_t* off = ldu(&J->off_x);
  const size_t npad = A.npad;
  const uint32_t* row_off = A.row_off;
  const int t0 = (int)ldu(&row_off[h]), t1 = min((int)ldu(&row_off[h + 1]), A.max_tiles);
  const Tile* tiles = A.tiles;
  // pruning threshold: above the cutoff by far more than the FP64 rounding
  // of the bounding-box distance
  const bool noprune = ldu(&J->half_noprune) != 0;
  const double rcut2 = noprune ? __builtin_inf() : S.rc2 * (1.0 + 1e-9);
  for (int ti = t0; ti < t1; ++ti) {
    // the previous tile's plane updates are visible to every lane
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const Tile tl = ldu(&tiles[ti]);
    const int count = tl.count;
    const int cx0 = tl.cx0, cx1 = tl.cx1;
    const bool active = lane < count;
    S.tstart = tl.start;
    const uint32_t i = tl.start + (uint32_t)(active ? lane : count - 1);
    const int span = cx1 - cx0 + 1;
    if constexpr (sizeof(T) == 4) {
      S.lo = ldu(&J->half_lo[span]);
      S.hi = ldu(&J->half_hi[span]);
    } else {
      S.lo = ldu(&J->half_lo64);
      S.hi = ldu(&J->half_hi64);
    }
    // the bounding boxes of the tile's halves (half_boxes_kernel; an empty
    // half B has lo = +inf, hi = -inf); their centres are the origins of the
    // sweep's coordinates
    const int countA = min(count, 32), countB = count - countA;
    double blA[3] = {0.0, 0.0, 0.0}, bhA[3] = {0.0, 0.0, 0.0};
    double blB[3] = {0.0, 0.0, 0.0}, bhB[3] = {0.0, 0.0, 0.0};
    {
      const double4 r = J->r64_x[i];
      const double ri[3] = {r.x, r.y, r.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) S.RI[lane * 3 + a] = ri[a];  // for queued pairs
      const double* bx = A.boxes + (size_t)ti * 12;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S.OA[a] = 0.0;
        S.OB[a] = 0.0;
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        blA[a] = ldu(&bx[a]);
        bhA[a] = ldu(&bx[3 + a]);
        blB[a] = ldu(&bx[6 + a]);
        bhB[a] = ldu(&bx[9 + a]);
        S.OA[a] = 0.5 * (blA[a] + bhA[a]);
        S.OB[a] = countB > 0 ? 0.5 * (blB[a] + bhB[a]) : S.OA[a];
      }
      const bool hb = lane >= 32;
      S.xi[0] = active ? (T)((ri[0] - (hb ? S.OB[0] : S.OA[0])) * S.inv_sig) : T(1e18);
      S.xi[1] = active ? (T)((ri[1] - (hb ? S.OB[1] : S.OA[1])) * S.inv_sig) : T(1e18);
      S.xi[2] = DIM == 3 ? (active ? (T)((ri[2] - (hb ? S.OB[2] : S.OA[2])) * S.inv_sig) : T(1e18)) : T(0);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.Fi[a] = 0.0;
      S.GA[lane * 3 + a] = 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    S.lhA = 0;
    S.ltA = 0;
    S.lhB = 0;
    S.ltB = 0;
    // pieces of the visited cell range [xlo, xhi] of row r: px = -1, 0, +1
    const int xlo = SELF ? cx0 : cx0 - lx, xhi = cx1 + lx;
    for (int px = -1; px <= 1; ++px) {
      int a0 = xlo, a1 = xhi;
      if (px < 0) { a1 = min(a1, -1); }
      else if (px == 0) { a0 = max(a0, 0); a1 = min(a1, nx - 1); }
      else { a0 = max(a0, nx); }
      if (a0 > a1) continue;
      const int c0 = a0 - px * nx, c1 = a1 - px * nx;  // wrapped cell indices
      uint32_t jb = ldu(&off[rbase + c0]);
      const uint32_t je = ldu(&off[rbase + c1 + 1]);
      if (SELF && px == 0) jb = tl.start;  // pairs j > i: from the tile's first particle on
      const int kc = kcode(px, py, pz);
      const double t[3] = {ldu(&J->tK[kc * 4 + 0]), ldu(&J->tK[kc * 4 + 1]), ldu(&J->tK[kc * 4 + 2])};
      for (uint32_t cb = jb; cb < je; cb += kWave) {
        // keep, in the list of each half, the candidates within the cutoff
        // of that half's bounding box
        const uint32_t j = cb + (uint32_t)lane;
        bool keepA = false, keepB = false;
        if (j < je) {
          const double4 r = J->r64_x[j];
          const double q[3] = {r.x + t[0], r.y + t[1], r.z + t[2]};
          double ddA = 0.0, ddB = 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            const double eA = fmax(0.0, fmax(blA[a] - q[a], q[a] - bhA[a]));
            const double eB = fmax(0.0, fmax(blB[a] - q[a], q[a] - bhB[a]));
            ddA += eA * eA;
            ddB += eB * eB;
          }
          keepA = ddA <= rcut2;
          // home row: half B pairs only with j after its first particle
          keepB = ddB <= rcut2 && !(SELF && px == 0 && !noprune && j <= tl.start + 32u);
        }
        const unsigned long long kmA = __builtin_amdgcn_ballot_w64(keepA);
        const unsigned long long kmB = __builtin_amdgcn_ballot_w64(keepB);
        S.ntested += (unsigned long long)count * min(je - cb, (uint32_t)kWave);
        S.nkept += (unsigned long long)countA * (unsigned long long)__popcll(kmA) +
                   (unsigned long long)countB * (unsigned long long)__popcll(kmB);
        const uint2 ent = make_uint2(j, (uint32_t)kc);
        if (keepA) S.LST[(S.ltA + (uint32_t)lane_rank(kmA)) & (uint32_t)(kHLCap - 1)] = ent;
        if (keepB) S.LST[kHLCap + ((S.ltB + (uint32_t)lane_rank(kmB)) & (uint32_t)(kHLCap - 1))] = ent;
        S.ltA += (uint32_t)__popcll(kmA);
        S.ltB += (uint32_t)__popcll(kmB);
        __builtin_amdgcn_wave_barrier();
        S.template run_full<SELF>(pjA, pjB, npad);
      }
    }
    S.template run_tail<SELF>(pjA, pjB, npad);
    // the tile's i-side sums (plane 3 rho, one writer per particle)
#pragma unroll
    for (int a = 0; a < DIM; ++a) S.Fi[a] += S.GA[lane * 3 + a];
    if (active) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) part_i[(size_t)a * npad + i] = (T)S.Fi[a];
    }
  }
}

}  // namespace

template <int DIM, bool VIR, typename T>
__device__ __forceinline__ void half_lj_body(const JobDesc* __restrict__ jobs, const HalfArgs& A,
                                             uint32_t* sQ, uint2* sL, uint2* sBC, double* sGA, double* sGJ,
                                             double* sR) {
  const int lane = (int)__lane_id();
  const int NR = A.NR;
  const int nrows = A.nitems / NR;
  // Launch order: each XCD (block index mod 8) takes a contiguous range of
  // rows (neighbouring rows share its L2) and runs its items rank by rank of
  // the row-offset order, the offsets with the most candidates first, so
  // that the cheapest items end the launch.
  int r0 = 0, nr = nrows, k = (int)blockIdx.x;
  if (nrows >= 8) {
    const int x = k & 7;
    r0 = (x * nrows) >> 3;
    nr = (((x + 1) * nrows) >> 3) - r0;
    k >>= 3;
  }
  if (k >= nr * NR) return;
  const int rank = k / nr;
  const int h = uniform(r0 + (k - rank * nr));
  const int rho = uniform((int)A.rho_order[rank]);
  const int item = h * NR + rho;
  const JobDesc* J = &jobs[0];

  Half<DIM, VIR, T> S;
  S.J = J;
  S.lane = lane;
  S.Q = sQ;
  S.LST = sL;
  S.BC = sBC;
  S.GA = sGA;
  S.GJ = sGJ;
  S.RI = sR;
  S.RJ = sR + kWave * 3;
  S.rc2 = ldu(&J->rc2);
  S.s2 = ldu(&J->s2);
  S.inv_sig = 1.0 / sqrt(S.s2);
  S.near2f = (T)ldu(&J->half_near2);
  S.E64 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) S.B[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) S.W[k] = 0.0;
  S.qband = 0;
  S.qnear = 0;
  S.cnt = 0;
  S.ntested = 0;
  S.nkept = 0;
  S.qtail = 0;
  S.key = 0x7fffffff;

  const int nx = ldu(&J->n[0]), ny = ldu(&J->n[1]), nz = ldu(&J->n[2]), l = ldu(&J->lcell);
  const int cy = h % ny, cz = DIM == 3 ? h / ny : 0;
  int dy, dz;
  row_offset(l, rho, &dy, &dz);
  int uy = cy + dy, uz = cz + dz, py = 0, pz = 0;
  if (uy >= ny) { uy -= ny; py = 1; } else if (uy < 0) { uy += ny; py = -1; }
  if (DIM == 3) {
    if (uz >= nz) { uz -= nz; pz = 1; }
  }
  const uint32_t* off = ldu(&J->off_x);
  const int rbase = (uy + ny * uz) * nx;
  const size_t npad = A.npad;
  T* part_i = (T*)A.part + (size_t)(3 * rho) * 3 * npad;
  T* pjA = (T*)A.part + (size_t)(3 * rho + 1) * 3 * npad;
  T* pjB = (T*)A.part + (size_t)(3 * rho + 2) * 3 * npad;
  {  // this item owns the two j-side planes over row r: clear them
    const uint32_t r0 = ldu(&off[rbase]), r1 = ldu(&off[rbase + nx]);
    for (uint32_t j = r0 + (uint32_t)lane; j < r1; j += kWave) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        pjA[(size_t)a * npad + j] = T(0);
        pjB[(size_t)a * npad + j] = T(0);
      }
    }
  }
  if (rho == 0)
    run_tiles<DIM, VIR, T, true>(S, A, h, py, pz, rbase, part_i, pjA, pjB);
  else
    run_tiles<DIM, VIR, T, false>(S, A, h, py, pz, rbase, part_i, pjA, pjB);

  // ---- item partials
  const unsigned long long cnt = S.cnt;
  const double e = wave_sum_d(S.E64);
  double* Pp = A.partials + (size_t)item * kPartialD;
  if (lane == 0) {
    A.pcount[item] = cnt;
    Pp[P_SUM] = e;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double bsum = wave_sum_d(S.B[k]);
    if (lane == 0) Pp[P_BOX + k] = bsum;
  }
  {
    constexpr int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    double ws[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) ws[k] = VIR ? wave_sum_d(S.W[k]) : 0.0;
    if (lane == 0) {
#pragma unroll
      for (int m = 0; m < 9; ++m) Pp[P_VIR + m] = ws[map[m]];
    }
  }
  const unsigned long long gb = wave_sum_u64(S.qband), gn = wave_sum_u64(S.qnear);
  if (lane == 0) {
    unsigned long long* g = ldu(&J->guard);
    if (gb | gn) {
      atomicAdd(&g[0], gb);
      atomicAdd(&g[1], gn);
    }
    atomicAdd(&g[2], S.ntested);
    atomicAdd(&g[3], S.nkept);
  }
}

// FP32 + FP64-guard form: 128 registers (four waves per SIMD).
template <int DIM, bool VIR>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
half_lj_kernel(const JobDesc* __restrict__ jobs, const HalfArgs A) {
  __shared__ uint32_t sQ[kHQCap];
  __shared__ uint2 sL[2 * kHLCap];
  __shared__ uint2 sBC[kWave];
  __shared__ double sGA[kWave * 3];
  __shared__ double sGJ[kWave * 3];
  __shared__ double sR[kWave * 6];
  half_lj_body<DIM, VIR, float>(jobs, A, sQ, sL, sBC, sGA, sGJ, sR);
}

// Plain FP64 form: the same sweep with FP64 coordinates, sums and force
// planes; twice the registers.
template <int DIM, bool VIR>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
half_lj64_kernel(const JobDesc* __restrict__ jobs, const HalfArgs A) {
  __shared__ uint32_t sQ[kHQCap];
  __shared__ uint2 sL[2 * kHLCap];
  __shared__ uint2 sBC[kWave];
  __shared__ double sGA[kWave * 3];
  __shared__ double sGJ[kWave * 3];
  __shared__ double sR[kWave * 6];
  half_lj_body<DIM, VIR, double>(jobs, A, sQ, sL, sBC, sGA, sGJ, sR);
}

// Bounding boxes of the wrapped positions of each tile's two halves (its
// first 32 particles, then the others; one wave per tile): the sweep reads
// them once per (tile, neighbour row) instead of reducing them.
__global__ void __launch_bounds__(256) half_boxes_kernel(const JobDesc* __restrict__ jobs, const HalfArgs A) {
  const JobDesc* J = &jobs[0];
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int t = (int)(blockIdx.x * 4 + threadIdx.x / kWave);
  const int ntiles = min((int)ldu(&A.row_off[A.nitems / A.NR]), A.max_tiles);
  if (t >= ntiles) return;
  const Tile tl = A.tiles[t];
  const int count = tl.count;
  const bool act = lane < count;
  const uint32_t i = tl.start + (uint32_t)(act ? lane : count - 1);
  const double4 r = J->r64_x[i];
  const double ri[3] = {r.x, r.y, r.z};
  double* bx = A.boxes + (size_t)t * 12;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // per 32-lane half; a half without particles gets lo = +inf, hi = -inf
    double lo = act ? ri[a] : __builtin_inf(), hi = act ? ri[a] : -__builtin_inf();
#pragma unroll
    for (int d = 16; d > 0; d >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, d, 64));
      hi = fmax(hi, __shfl_xor(hi, d, 64));
    }
    if ((lane & 31) == 0) {
      bx[(lane >> 5) * 6 + a] = lo;
      bx[(lane >> 5) * 6 + 3 + a] = hi;
    }
  }
}

hipError_t launch_half_boxes(const JobDesc* jobs, const HalfArgs& A, hipStream_t s) {
  const unsigned nb = (unsigned)((A.max_tiles + 3) / 4);
  if (nb > 0) half_boxes_kernel<<<nb, 256, 0, s>>>(jobs, A);
  return hipGetLastError();
}

// Sum of the 3 NR planes of each particle (fixed order), forces in original
// order, and the wrap term of the box gradient, sum over particles of
// G_p w_p^T (block partials after the item partials).
template <int DIM, typename T>
__global__ void __launch_bounds__(256) half_gather_kernel(const JobDesc* __restrict__ jobs, const HalfArgs A,
                                                          int n) {
  const JobDesc& J = jobs[0];
  __shared__ double red[4][9];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = blockIdx.x * 256 + tid;
  double G[3] = {0.0, 0.0, 0.0};
  double Bl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (p < n) {
    const size_t npad = A.npad;
    for (int q = 0; q < 3 * A.NR; ++q) {
      const T* pl = (const T*)A.part + (size_t)q * 3 * npad;
#pragma unroll
      for (int a = 0; a < DIM; ++a) G[a] += (double)pl[(size_t)a * npad + p];
    }
    const double mult = J.upstream ? *J.upstream : J.scale;
    const double sc = mult * 24.0 * J.eps;
    const uint32_t io = J.idx_x[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) J.forces[(size_t)io * DIM + a] = sc * G[a];
    const int4 wv = J.wrap_x[p];
    const int wa[3] = {wv.x, wv.y, wv.z};
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = 0; b < DIM; ++b) Bl[a * 3 + b] = G[a] * (double)wa[b];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double s = wave_sum_d(Bl[k]);
    if (lane == 0) red[w][k] = s;
  }
  __syncthreads();
  const size_t slot = (size_t)A.nitems + blockIdx.x;
  if (tid < kPartialD) {
    double v = 0.0;
    if (tid >= P_BOX && tid < P_BOX + 9) {
      const int k = tid - P_BOX;
      v = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
    A.partials[slot * kPartialD + tid] = v;
  }
  if (tid == 0) A.pcount[slot] = 0ull;
}

hipError_t launch_half_lj(int dim, bool virial, bool fp64, const JobDesc* jobs, const HalfArgs& A,
                          hipStream_t s) {
  if (A.nitems > 0) {
    // blocks beyond an XCD's rows return at once (half_lj_body)
    const int nrows = A.nitems / A.NR;
    const unsigned g = nrows >= 8 ? (unsigned)(8 * ((nrows + 7) / 8) * A.NR) : (unsigned)A.nitems;
    if (fp64) {
      if (dim == 3)
        virial ? half_lj64_kernel<3, true><<<g, 64, 0, s>>>(jobs, A) : half_lj64_kernel<3, false><<<g, 64, 0, s>>>(jobs, A);
      else
        virial ? half_lj64_kernel<2, true><<<g, 64, 0, s>>>(jobs, A) : half_lj64_kernel<2, false><<<g, 64, 0, s>>>(jobs, A);
    } else {
      if (dim == 3)
        virial ? half_lj_kernel<3, true><<<g, 64, 0, s>>>(jobs, A) : half_lj_kernel<3, false><<<g, 64, 0, s>>>(jobs, A);
      else
        virial ? half_lj_kernel<2, true><<<g, 64, 0, s>>>(jobs, A) : half_lj_kernel<2, false><<<g, 64, 0, s>>>(jobs, A);
    }
  }
  return hipGetLastError();
}

hipError_t launch_half_gather(int dim, bool fp64, const JobDesc* jobs, const HalfArgs& A, int n,
                              hipStream_t s) {
  const int nb = (n + 255) / 256;
  if (nb > 0) {
    if (fp64)
      dim == 3 ? half_gather_kernel<3, double><<<nb, 256, 0, s>>>(jobs, A, n)
               : half_gather_kernel<2, double><<<nb, 256, 0, s>>>(jobs, A, n);
    else
      dim == 3 ? half_gather_kernel<3, float><<<nb, 256, 0, s>>>(jobs, A, n)
               : half_gather_kernel<2, float><<<nb, 256, 0, s>>>(jobs, A, n);
  }
  return hipGetLastError();
}

}  // namespace clm
