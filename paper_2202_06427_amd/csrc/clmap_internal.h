// clmap_internal.h -- device-side data structures of libclmap (gfx950).
//
// Data layout in HBM after a build (n = particles of one set, sorted by cell,
// cells linearised x-fastest: c = cx + nx*(cy + ny*cz)):
//   pos   float4[n]   FP32 offset of the wrapped position from its cell origin
//                     (x, y, z[, unused]); used by the FP32 sweep (16 B, one
//                     scalar-cache line holds 4 particles)
//   r64   double4[n]  FP64 wrapped position r' (canonical, see clmap.h)
//   idx   uint32[n]   original index of each sorted slot
//   wrap  int4[n]     wrap integers w (r' = r - H w)
//   off   uint32[ncells+1] exclusive prefix of the cell occupancies
// plus the tile list (work units of <= 64 consecutive sorted particles of one
// cell row) and per-tile FP64 partials.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clm {

constexpr int kWave = 64;        // CDNA wavefront
constexpr int kTileMax = 64;     // particles per tile: one per lane
constexpr int kMaxSpan = 16;     // most cells a tile may span along x
constexpr int kBlock = 256;      // register budget of the sweep: up to 4 waves per block
constexpr int kSweepWaves = 1;   // waves (tiles) per launched sweep block: each wave
                                 // frees its slot as soon as its tile is done
constexpr int kNLStage = 256;    // per-wave LDS staging slots for neighbour pairs
constexpr int kPartialD = 20;    // doubles per tile partial
constexpr int kMaxBins = 1000;  // keeps 4 waves of private histograms within 64 KiB LDS

// Per-tile partial slots (doubles).
enum : int {
  P_SUM = 0,      // energy / sum of d / sum of 1/d (unscaled)
  P_VIR = 1,      // 9: virial (unscaled)
  P_BOX = 10,     // 9: box-gradient accumulator B (unscaled); dE/dH = -24 eps B
  P_FREE = 19
};

enum Kind : int {
  K_COUNT = 0, K_SUM_D = 1, K_SUM_INV_D = 2, K_LJ_E = 3, K_LJ_F = 4, K_LJ_FV = 5,
  K_HIST_DIST = 6, K_HIST_REL = 7, K_NL = 8,
  K_SUM_W = 9,     // sum of w_i w_j / d (weights in the 4th component of pos / r64)
  K_HIST_DV = 10   // distance histogram with per-bin sums of |v_j - v_i|
};

struct Tile {
  uint32_t start;   // first sorted index (x set)
  uint32_t row;     // cy + ny*cz
  uint16_t count;   // particles, 1..64
  uint16_t cx0;     // first cell (x) of the tile
  uint16_t cx1;     // last non-empty cell (x) of the tile
  uint16_t job;     // job descriptor index
};
static_assert(sizeof(Tile) == 16, "tile is 16 bytes");

// Everything the sweep needs about one job, resident in device memory and
// read through the scalar cache (all fields are wave-uniform).
struct JobDesc {
  // geometry
  int dim, lcell, full_shell, cross;
  int lcell_x, pad_lx;       // neighbour reach in cells along the row axis
  int n[3];
  int ncells;
  int nx, ny;            // particles of x and y (y == x for a single set)
  int pad0;
  double H[9];           // row-major, stride 3 (2D uses the 2x2 top-left)
  double Hn[9];          // H[a][b] / n[b]: cell-origin matrix (origin of cell u = Hn u)
  double tK[27 * 4];     // canonical image shifts H K, K in {-1,0,1}^3, index
                         // (Kx+1) + 3 (Ky+1) + 9 (Kz+1), 4 doubles per entry
  double rc2;
  double band;           // absolute band on FP32 squared distances
  float lo32, hi32;      // FP32 membership thresholds rc2 -+ band (rounded outwards)
  // sorted data
  const float4* pos_x; const double4* r64_x; const uint32_t* idx_x; const int4* wrap_x;
  const uint32_t* off_x;
  const float4* pos_y; const double4* r64_y; const uint32_t* idx_y; const int4* wrap_y;
  const uint32_t* off_y;
  // map
  int kind;
  int nbins;
  double s2;             // sigma^2
  float s2f, near2f;     // sigma^2 and (near_factor sigma)^2 in FP32
  double eps;
  const double* upstream;    // LJ adjoint: g (device), NULL -> scale
  double scale;              // multiplier of dE/dr when upstream == NULL
  int want_virial, want_sums, with_dist, pad1;
  double hist_hi;
  float inv_h, pad2;
  const double* E64;         // nbins+1 edges (squared), canonical
  const float* E32;          // the same rounded to FP32
  double* bandq;             // relative-speed band (device scalar, set by the prep kernel)
  const float4* vel32_x;     // sorted FP32 velocities
  const float4* vel32_y;
  const double* vel64_x;     // raw FP64 velocities (original order)
  const double* vel64_y;
  // outputs
  double* partials;          // per tile kPartialD
  unsigned long long* guard; // [2] FP32 form: band re-tests, other FP64 re-evaluations
  unsigned long long* pcount;// per tile pair count
  double* forces;            // n_x*dim, original order
  unsigned long long* hist;  // nbins+1
  double* hist_sums;         // nbins
  int32_t* pairs;
  double* dist;
  unsigned long long* nl_counter;
  // output offset of each work item (tile * G + g) from a counting pass, or
  // NULL: items then reserve output slots from nl_counter
  const unsigned long long* nl_offsets;
  long long capacity;
  int tile_begin, tile_end;  // this job's tiles in the launched tile list
  // the job's own tile list (built by its cell list)
  const Tile* own_tiles;
  const uint32_t* own_ntiles;  // device count
  int own_max_tiles;
  int pad3;
  // half-shell LJ sweep (coordinates in units of sigma): FP32 membership
  // thresholds on d^2 / sigma^2 per tile span (1..kMaxSpan cells along x) and
  // the near threshold near_factor^2
  float half_lo[kMaxSpan + 1], half_hi[kMaxSpan + 1];
  double half_lo64, half_hi64;  // the same for the FP64 form (any span)
  float half_near2;
  int half_noprune;          // 1: keep every candidate (no bounding-box pruning)
};

// Dynamic LDS bytes per wave of the sweep.  The FP32 form keeps a ring
// queue of candidates to re-evaluate in FP64 (kQueueCap entries of 8 bytes)
// and, for LJ forces, per-lane FP64 force accumulators fed by that queue.
// Histogram kinds add private histograms (nbins+1 u32 each) and per-bin FP64
// sums; the neighbour list adds a staging area.
constexpr int kQueueCap = 512;  // power of two
__host__ __device__ inline size_t sweep_lds_queue_bytes(int kind, bool fp32) {
  if (!fp32) return 0;
  size_t b = (size_t)kQueueCap * 8;
  if (kind == K_LJ_F || kind == K_LJ_FV) b += (size_t)kWave * 3 * 8;
  return b;
}
// Copies of a wave's private histogram: lane l adds to copy l % C (copies
// of nbins+1 counters, then copies of nbins sums, one after the other), so
// fewer lanes of one LDS atomic meet at one address.  C
// is the largest power of two up to 64 whose counters (and per-bin FP64
// sums) fit in kHistPrivBytes.
constexpr size_t kHistPrivBytes = 2048;
constexpr int kHistMaxCopies = 16;
// FP32 bin edges read from a per-wave LDS table (true) or formed in registers
constexpr bool kHistEdgeTable = false;
__host__ __device__ constexpr bool hist_has_sums(int kind) { return kind == K_HIST_REL || kind == K_HIST_DV; }
__host__ __device__ inline int hist_copies(int kind, int nbins) {
  const size_t per = (size_t)(nbins + 1) * 4 + (hist_has_sums(kind) ? (size_t)nbins * 8 : 0);
  int c = 1;
  while (c < kHistMaxCopies && (size_t)(2 * c) * per <= kHistPrivBytes) c *= 2;
  return c;
}
__host__ __device__ inline size_t sweep_lds_per_wave(int kind, int nbins, bool fp32) {
  size_t b = sweep_lds_queue_bytes(kind, fp32);
  if (kind == K_HIST_DIST || kind == K_HIST_REL || kind == K_HIST_DV) {
    const size_t C = (size_t)hist_copies(kind, nbins);
    b += C * (size_t)(nbins + 1) * 4 + 8 + (hist_has_sums(kind) ? C * (size_t)nbins * 8 : 0);
    if (kHistEdgeTable) b += (size_t)(nbins + 1) * 4;
  } else if (kind == K_NL)
    b += (size_t)kNLStage * 16 + 16;
  return (b + 15) & ~(size_t)15;
}

__host__ __device__ inline int kcode(int px, int py, int pz) {
  return (px + 1) + 3 * (py + 1) + 9 * (pz + 1);
}

// ---------------------------------------------------------------- launch parameters
struct BuildGeom {
  int dim;
  int n[3];
  double H[9];     // row-major stride 3
  double Hinv[9];  // row-major stride 3 (canonical adjugate / determinant)
};

struct TileGeom {
  int n[3];
  int smax;
  int nrows;
  int job;
  uint32_t max_tiles;
};

struct BruteArgs {
  int dim, n_x, n_y, cross, kind;
  double H[9], Hinv[9], w[3];
  double rc, rc2;
  double reach;   // min(rc, half the sum of lattice-vector lengths) (1 + 1e-6)
};

// ---------------------------------------------------------------- row split
// When a sweep has few tiles (small or sparse sets, cross sets with a small
// x), the neighbour rows of a tile are spread over G waves: work item
// tile * G + g visits the rows r (counted in visiting order) with r % G == g
// and owns partial slot tile * G + g.  G is derived on the device from the
// tile count, identically by the sweep and by the finalize.
constexpr int kSplitTarget = 16384;  // work items aimed at (about 4 per SIMD slot)
__host__ __device__ inline int sweep_split(int ntiles, int cap, int rows) {
  if (rows <= 1 || ntiles <= 0) return 1;
  int g = kSplitTarget / ntiles;
  g = g < rows ? g : rows;
  const int c = cap / ntiles;
  g = g < c ? g : c;
  return g > 1 ? g : 1;
}

// Rows a tile of a single-job sweep visits, or 1 when its rows must stay in
// one wave: maps with per-particle outputs (LJ forces, the adjoint) write
// each particle's result from the wave that holds it.
inline int sweep_split_rows(int kind, int dim, int lcell, bool full) {
  if (kind == K_LJ_F || kind == K_LJ_FV) return 1;
  const int side = 2 * lcell + 1;
  const int rows = dim == 3 ? side * side : side;
  return full ? rows : (rows + 1) / 2;
}

// Half-shell LJ force sweep (sweep_half.hip): one wave per (cell row,
// half-shell row offset) item; FP32 force planes indexed by sorted slot,
// 2 NR planes of 3 components (stride npad floats): plane 2 rho holds the
// i-side sums of offset rho, plane 2 rho + 1 the j-side sums.
// Half-shell row offsets including the home row: 2 l^2 + 2 l + 1 in 3D, l + 1 in 2D.
__host__ __device__ inline constexpr int half_rows(int dim, int l) { return dim == 3 ? 2 * l * l + 2 * l + 1 : l + 1; }
constexpr int kMaxHalfRows = 152;  // >= half_rows(3, 8), the largest lcell
static_assert(half_rows(3, 8) <= kMaxHalfRows, "row-offset order table too small");

struct HalfArgs {
  void* part;                  // 3 NR force planes of 3 components (float, or double in the FP64 form)
  size_t npad;
  double* partials;            // nitems + gather blocks, kPartialD each
  unsigned long long* pcount;  // nitems + gather blocks
  const uint32_t* row_off;     // tiles of row h: [row_off[h], row_off[h + 1])
  const Tile* tiles;
  double* boxes;               // per tile: bounding boxes of its two 32-particle halves' wrapped
                               // positions (lo xyz, hi xyz of half A, then of half B)
  int max_tiles;               // entries of tiles (and boxes)
  int nitems, NR;
  // launch order of the row offsets: rho_order[k] is the k-th (most
  // candidates first); items of one rank are launched before the next's
  uint8_t rho_order[kMaxHalfRows];
};

struct FinalArgs {
  int nparts;                      // used when nparts_dev is NULL
  const uint32_t* nparts_dev;      // device count of partials (tiles)
  int split_rows;                  // > 1: the sweep split rows (partials = tiles * G)
  int kind, dim, want_virial;
  int halve_count;                 // full-shell sweep: every pair was counted from both ends
  double eps;
  const double* upstream;          // LJ adjoint: g
  double box_mult;                 // when upstream is NULL
  double* energy;
  double* virial;
  double* grad_box;
  unsigned long long* count;
};

// ---------------------------------------------------------------- molecular dynamics
constexpr int kMdBlock = 256;  // threads per block of the per-particle / per-row kernels
constexpr int kMdPart = 8;     // doubles per block partial
constexpr int kDriftBlocks = 512;  // most blocks of the displacement check
constexpr int kBuildBlocks = 8192; // most blocks of the pair-list build
constexpr int kBuildWaves = 4;     // waves per block of the pair-list build
enum : int { MP_E = 0, MP_W = 1 /* 6: xx xy xz yy yz zz */, MP_KE = 7 };

// Device counters of a Verlet list (one per list, in its workspace).
struct VlFlags {
  unsigned long long maxd2;     // largest squared displacement of this step (double bits)
  unsigned long long updates, rebuilds, entries;
  uint32_t gate;                // 1: the list is rebuilt in this step
  uint32_t force;               // 1: the next update rebuilds regardless of displacements
  uint32_t overflow;            // sticky: a row exceeded its capacity at a rebuild
  uint32_t max_row;             // most partners of one particle at the last rebuild
};

struct VlRefresh {
  int n, dim;
  double H[9], Hinv[9];         // row-major stride 3
  const double* x;              // caller order
  const uint32_t* idx;          // sorted slot -> caller index
  const int4* wrap;             // wrap integers of the last rebuild (sorted)
  double4* pf;                  // frame positions (sorted)
  double* xref;                 // positions at the last rebuild (caller order)
  const uint32_t* gate;
};

struct VlBuild {
  int n[3];
  int l, lx, cap, max_tiles;
  int P, lgP;                   // lanes per row of the force kernel (list layout)
  int split, pad;               // 1: one wave per (tile, neighbour row), else per tile
  double rl2;                   // list threshold on the squared distance
  double tK[27 * 4];            // canonical image shifts H K
  const Tile* tiles;
  const uint32_t* ntiles;
  const uint32_t* off;
  const double4* r64;
  uint32_t* list;
  uint32_t* cnt;
  VlFlags* fl;
  const uint32_t* gate;
};

struct VlForce {
  int n, cap;
  double rc2, s2, eps, h;
  double tK[27 * 4];
  const uint32_t* list;
  const uint32_t* cnt;
  const double4* pf;
  const uint32_t* idx;
  double* forces;
  double* v;                    // fused second half-kick (KICK kernels only)
  double* part;
  unsigned long long* pcount;
};

struct MdFinal {
  int nb, dim;
  const double* part;
  const unsigned long long* pcount;   // NULL: no pair count
  double eps, mass;
  double* energy;
  double* virial;
  unsigned long long* count;
  double* ke;                   // caller's copy (may be NULL)
  double* ke_keep;              // the integrator's copy (NULL: no kinetic energy)
};

// ---------------------------------------------------------------- k closest pairs
struct KcRecord {            // a candidate pair: canonical d2 (bits), caller indices
  unsigned long long key;
  uint32_t i, j;
};
static_assert(sizeof(KcRecord) == 16, "record is 16 bytes");
constexpr int kKcLdsRecords = 2048;  // records sorted in LDS by one block
constexpr int kKcLdsThreads = 1024;

struct KcKeys {
  int dim, cross, cap, npow2;
  double tK[27 * 4];
  const int32_t* pairs;                 // candidate pairs (caller indices)
  const unsigned long long* count;      // number of candidates (device)
  const double4* r64_x;
  const double4* r64_y;
  const uint32_t* inv_x;
  const uint32_t* inv_y;
  KcRecord* rec;
};

// ---------------------------------------------------------------- launchers
// Host wrappers (defined next to their kernels); all enqueue on `s`.  The
// build launchers take an optional device gate: their kernels return at once
// when it reads 0 (NULL: always run).
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s,
                           const uint32_t* gate = nullptr);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s,
                           const uint32_t* gate = nullptr);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s,
                           const uint32_t* gate = nullptr);
// Binning plan: cells per bucket, buckets, particles per thread and blocks
// of the count and bucket passes (host-side, from the sizes only).
constexpr int kBinThreads = 1024;
constexpr int kMaxBuckets = 16384;
constexpr int kMaxBucketCells = 1024;  // with kMaxBuckets: up to 2^24 cells
constexpr int kPlaceCap = 2048;        // particles of a bucket assembled in LDS
constexpr int kPlaceTarget = 1280;     // mean particles per bucket aimed at
constexpr int kSortCell = 64;          // placement: cells up to this size are ordered by x within the cell
static_assert((int64_t)kMaxBuckets * kMaxBucketCells >= (int64_t(1) << 24), "cell cap");
struct BinPlan {
  int cpb, nbk, per, nblk;
};
struct alignas(32) BinRec {
  double x, y, z;   // position as given (z = 0 in 2D)
  uint32_t i, cell;
};
BinPlan bin_plan(int64_t ncells, int64_t n);
// Bin n particles: key (n), hist (nbk * nblk + 1, scanned in place), rec
// (n) are scratch; off (ncells + 1) and the sorted records are the result.
hipError_t launch_bin(const double* x, int n, const BuildGeom& g, int ncells, const BinPlan& P,
                      uint32_t* key, uint32_t* hist, uint32_t* scan_scratch, BinRec* rec, uint32_t* off,
                      float4* pos, double4* r64, uint32_t* idx, int4* wrap, hipStream_t s,
                      const uint32_t* gate = nullptr);
hipError_t launch_scan(const uint32_t* in, int n, uint32_t* sums_scratch, uint32_t* out,
                       hipStream_t s, const uint32_t* gate = nullptr);
size_t scan_scratch_elems(int n);
hipError_t launch_tiles(const uint32_t* off, const TileGeom& g, uint32_t* row_tiles,
                        uint32_t* row_off, uint32_t* scan_scratch, Tile* tiles, hipStream_t s,
                        const uint32_t* gate = nullptr);
constexpr int kExtremaBlocks = 512;
int extrema_blocks(int64_t n);
// lo (3) and hi (3) of the coordinates into out[0..5]; part: kExtremaBlocks * 6 doubles
hipError_t launch_extrema(const double* x, int64_t n, int dim, double* part, double* out, hipStream_t s);
hipError_t launch_gather_vel(const double* v, int dim, const uint32_t* idx, int n, float4* v32,
                             unsigned int* vmax_bits, hipStream_t s);
// Per-particle weights of a weighted map into the sorted records: pos[s].w =
// (float) w[idx[s]], r64[s].w = w[idx[s]].
hipError_t launch_gather_weights(const double* w, const uint32_t* idx, int n, float4* pos, double4* r64,
                                 hipStream_t s);
hipError_t launch_set_job(const JobDesc& jd, JobDesc* dst, hipStream_t s);
hipError_t launch_hist_edges(double* E64, float* E32, int nbins, double hi, int force_last,
                             double rc2, hipStream_t s);
hipError_t launch_relspeed_band(const unsigned int* vmax_bits, double hi, int dim, double* bandq,
                                hipStream_t s);
// Exclusive prefix sums of the per-item pair counts of a counting sweep
// (pcount, tiles * G items with G from sweep_split) into offsets.
hipError_t launch_nl_offsets(const unsigned long long* pcount, const uint32_t* ntiles_dev, int max_tiles,
                             int split_rows, unsigned long long* offsets, hipStream_t s);
// split_rows: rows a tile visits when its rows may be spread over waves
// (sweep_split), 1 to keep one wave per tile (maps with per-particle outputs,
// batches).
hipError_t launch_sweep(int dim, bool fp32, int kind, const JobDesc* jobs, const Tile* tiles,
                        const uint32_t* ntiles_dev, int max_tiles, int nbins, hipStream_t s,
                        int split_rows = 1);
// Brute-force path: j chunks per 64 particles (enough waves to fill the chip
// for a few thousand particles); partial rows = ceil(n_x / 64) * chunks.
__host__ __device__ inline int brute_chunks(int64_t ny) {
  int64_t c = (ny + 127) / 128;
  return (int)(c < 1 ? 1 : (c > 32 ? 32 : c));
}
hipError_t launch_brute(const JobDesc* jobs, const BruteArgs& A, double* FB, int* nparts_out,
                        hipStream_t s);
hipError_t launch_half_lj(int dim, bool virial, bool fp64, const JobDesc* jobs, const HalfArgs& A,
                          hipStream_t s);
hipError_t launch_half_boxes(const JobDesc* jobs, const HalfArgs& A, hipStream_t s);
hipError_t launch_half_gather(int dim, bool fp64, const JobDesc* jobs, const HalfArgs& A, int n,
                              hipStream_t s);
hipError_t launch_finalize(const JobDesc* jobs, const FinalArgs& F, double* scratch,
                           unsigned long long* scratch_count, hipStream_t s);
constexpr int kFinalBlocks = 128;  // first-level blocks of the two-level finalize
hipError_t launch_gather_tiles(JobDesc* jobs, int njobs, Tile* tiles, uint32_t* total,
                              hipStream_t s);
hipError_t launch_finalize_batch(const JobDesc* jobs, const FinalArgs* F, int njobs, hipStream_t s);
hipError_t launch_md_kick_drift(double* x, double* v, const double* f, int64_t ncomp, double h,
                                double dt, double target_ke, const double* ke, hipStream_t s);
hipError_t launch_md_kick(double* v, const double* f, int n, int dim, double h, double* part,
                          hipStream_t s);
hipError_t launch_md_rescale(double* v, int64_t ncomp, double target_ke, const double* ke,
                             hipStream_t s);
hipError_t launch_md_finalize(const MdFinal& F, hipStream_t s);
int vl_drift_blocks(int64_t n);
hipError_t launch_vl_drift(const double* x, const double* xref, int n, int dim, double lim2,
                           double* bmax, VlFlags* fl, hipStream_t s);
hipError_t launch_vl_rowstats(uint32_t* cnt, int n, int cap, VlFlags* fl, const uint32_t* gate,
                              hipStream_t s);
int vl_rows_per_lane_group(int64_t n);
hipError_t launch_vl_refresh(const VlRefresh& A, hipStream_t s);
hipError_t launch_vl_build(int dim, const VlBuild& A, hipStream_t s);
hipError_t launch_vl_lj(int dim, bool kick, bool vir, int P, const VlForce& A, hipStream_t s);
hipError_t launch_kc_inverse(const uint32_t* idx, int n, uint32_t* inv, hipStream_t s);
hipError_t launch_kc_keys(const KcKeys& A, hipStream_t s);
hipError_t launch_kc_sort(KcRecord* rec, int n, hipStream_t s);
hipError_t launch_kc_output(const KcRecord* rec, int k, int found, int32_t* io, int32_t* jo, double* d2o,
                            hipStream_t s);
hipError_t launch_candidates(const JobDesc* jobs, int ncells, int full, unsigned long long* out,
                             hipStream_t s);

// ---------------------------------------------------------------- calibration
// Microbenchmarks of the device's attainable FMA rate and copy bandwidth.
constexpr int kCalibThreads = 256;
constexpr int kCalibBlocks = 4096;      // 16 blocks per CU
constexpr int kCalibChains = 8;         // independent FMA chains per thread
constexpr int kCalibCopyBlocks = 8192;
// FMA chains of FP32 (fp64 = 0) or FP64; out holds kCalibBlocks * kCalibThreads values.
hipError_t launch_calib_fma(int fp64, void* out, int iters, hipStream_t s);
// dst[0..n16) = src[0..n16) in 16-byte vectors.
hipError_t launch_calib_copy(const void* src, void* dst, int64_t n16, hipStream_t s);


}  // namespace clm
