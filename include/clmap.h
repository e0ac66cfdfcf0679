/*
 * clmap.h -- C-ABI of libclmap.so: cell-list pair mapping on AMD MI355X
 * (gfx950), after "CellListMap.jl" (Martinez, arXiv 2202.06427).
 *
 * The calls follow the paper's statement of the problem (section 2.1):
 *   1. the pair function  -> a map kind chosen from a fixed set (clm_map_kind),
 *                            because a C ABI cannot take a closure
 *                            (the paper's user function, sections 2.3 and 2.7);
 *   2. geometry and cutoff -> clm_box_create (the paper's Box, section 2.5);
 *   3. the cell lists      -> clm_celllist_create + clm_celllist_build
 *                            (the paper's CellList, section 2.6);
 *   4. the mapping         -> clm_map, which always returns the reduced
 *                            result (map_pairwise, sections 2.3 and 2.7).
 *
 * Conventions
 *  - Every function returns clm_status (0 = CLM_OK).  None throws, exits or
 *    prints.  On an error the outputs are untouched and clm_last_error()
 *    returns a thread-local message.
 *  - Pointers named *_dev are device pointers on the context's device.  The
 *    caller owns every device buffer, including the workspace; the library
 *    never allocates device memory.  The library owns only the small host
 *    handles (context, box, cell list).
 *  - Device work is enqueued on the context's stream and the calls return
 *    before it completes (clm_celllist_build, clm_map); results are valid
 *    after clm_synchronize or any later stream-ordered event.
 *  - Box matrices are row-major dim x dim: H[a*dim+b] is Cartesian component
 *    a of lattice vector b, i.e. the lattice vectors are the COLUMNS of H
 *    (the paper prints the unit cell this way, Code 3).  An orthorhombic box
 *    is a diagonal H.
 *  - Coordinates are row-major n x dim FP64 (the paper's (N,M) coordinate
 *    matrices, section 2.4, stored particle by particle).  Indices in all
 *    outputs are 0-based (the paper's listings are 1-based).
 *  - The pair set is defined exactly (section 2.8 and the "minimum-image
 *    convention" of section 2.3): particle positions are first wrapped into
 *    the primary cell, s = Hinv r, w = floor(s), f = s - w (f = 0, w += 1 if
 *    the subtraction rounds to 1), r' = H f; a pair's displacement for an
 *    integer image K is D = (r'_j - r'_i) + H K, its squared distance
 *    d2 = (D0*D0 + D1*D1) + D2*D2, every operation rounded on its own in
 *    FP64 (no fused multiply-add; sums and products in the order written,
 *    Hinv = adjugate / determinant).  A pair is in the set when the minimum
 *    over K of d2 is <= rc2 = rc*rc.  Single set: unordered pairs i<j once;
 *    cross set: every (i in x, j in y).  Both precisions return exactly this
 *    set and these integer results.
 */
#ifndef CLMAP_H
#define CLMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLMAP_VERSION_MAJOR 0
#define CLMAP_VERSION_MINOR 1

typedef enum clm_status {
  CLM_OK = 0,
  CLM_E_INVALID_ARG = 1,  /* null pointer, bad size, bad enum value, ... */
  CLM_E_BAD_BOX = 2,      /* dim not 2/3, non-finite H, det H <= 0, cell flatter than 1:64 */
  CLM_E_BAD_CUTOFF = 3,   /* rc <= 0 or non-finite, lcell < 1 */
  CLM_E_CAPACITY = 4,     /* a neighbour list with check_capacity has more pairs than its
                             capacity (count_dev holds the true count), or a request needs
                             more than a fixed library buffer (clm_map_static) */
  CLM_E_WORKSPACE = 5,    /* workspace missing, too small or misaligned */
  CLM_E_DEVICE = 6,       /* a HIP call failed (message from the runtime) */
  CLM_E_UNSUPPORTED = 7   /* valid request this library does not serve */
} clm_status;

typedef enum clm_precision {
  CLM_FP64 = 0,       /* plain method: every distance in FP64, canonical */
  CLM_FP32_GUARD = 1  /* FP32 coordinates and distances, FP64 accumulation;
                         pairs whose FP32 squared distance lies within a
                         rigorous error band of the cutoff (or of a histogram
                         edge) are re-tested in canonical FP64, so the pair
                         set and every integer output equal the FP64 ones. */
} clm_precision;

typedef enum clm_map_kind {
  CLM_MAP_COUNT = 0,          /* number of pairs (paper section 2.8) */
  CLM_MAP_SUM_D = 1,          /* sum of d (Code 1) */
  CLM_MAP_SUM_INV_D = 2,      /* sum of 1/d (Code 5) */
  CLM_MAP_LJ_E = 3,           /* Lennard-Jones energy u = 4 eps ((s/d)^12 - (s/d)^6) (Code 6) */
  CLM_MAP_LJ_EF = 4,          /* LJ energy + forces (= -dE/dr, Code 7) + dE/dH [+ virial] */
  CLM_MAP_LJ_ADJOINT = 5,     /* g * dE/dr and g * dE/dH for an upstream g (differentiation, section 3.3) */
  CLM_MAP_HIST_DIST = 6,      /* histogram of d on (0, hi], right-closed bins (Code 10's rule) */
  CLM_MAP_HIST_RELSPEED = 7,  /* histogram of |v_j - v_i| on (0, hi] + per-bin sums (Code 10) */
  CLM_MAP_NEIGHBOR_LIST = 8,  /* compacted list of pairs (i, j[, d]) (section 4.1) */
  CLM_MAP_SUM_W_INV_D = 9,    /* sum of w_i w_j / d with per-particle weights (Code 5, masses) */
  CLM_MAP_HIST_DIST_VEL = 10  /* histogram of d on (0, hi] (Code 10's bins) with the per-bin sum
                                 of |v_j - v_i| in hist_sums_dev: the mean relative speed
                                 per distance bin is sums / counts (Code 10) */
} clm_map_kind;

typedef struct clm_context clm_context;
typedef struct clm_box clm_box;
typedef struct clm_celllist clm_celllist;

typedef struct clm_box_info {
  int dim;
  int lcell_requested;
  int lcell;            /* effective: largest l <= requested with >= 2l+1 cells per axis */
  int small_box;        /* 1: fewer than 3 cells on some axis -> brute-force minimum image */
  int grid[3];          /* cells per fractional axis (1 on unused axes) */
  int64_t ncells;
  double H[9];          /* row-major dim x dim (stride dim) */
  double Hinv[9];
  double widths[3];     /* perpendicular widths of the cell (distance between opposite faces) */
  double volume;
  double cutoff;
  double rc2;           /* fl(cutoff * cutoff), the membership threshold */
  double guard_band;    /* absolute band on FP32 squared distances, see clm_precision */
  int lcell_x;          /* effective neighbour reach in cells along the row (first) axis */
  int pad;
} clm_box_info;

typedef struct clm_celllist_info {
  int64_t n_x, n_y;
  int64_t ncells;
  int64_t ntiles;          /* work units of <= 64 particles */
  int64_t nonempty_cells;  /* cells holding particles of x */
  int64_t max_occupancy;   /* most particles in one cell (x or y) */
  int64_t candidate_pairs; /* pairs of the cell method on this grid: the particles
                              of each cell times those of its half-shell stencil
                              (lcell_x cells on along the row, the full reach of
                              the rows with (dz, dy) > (0, 0)), plus the pairs
                              within the cell; cross sets: the full stencil */
  int64_t guard_retests;   /* last map, FP32_GUARD: candidates within the band of rc^2
                              decided in FP64 */
  int64_t near_evaluations;/* last map, FP32_GUARD: other FP64 re-evaluations (LJ pairs
                              closer than near_factor*sigma, histogram values near an edge) */
  int64_t half_pairs_tested;/* last map, half-shell force sweep: (tile particle, candidate)
                              pairs before pruning by the tile's bounding box */
  int64_t half_pairs_kept;  /* the same after pruning: the pairs the sweep evaluates */
} clm_celllist_info;

typedef struct clm_map_params {
  double sigma, epsilon;        /* LJ_* */
  double near_factor;           /* FP32_GUARD LJ: pairs with d < near_factor*sigma are evaluated
                                   in FP64 (0 -> 1.0; the repulsive wall loses FP32 accuracy) */
  int want_virial;              /* LJ_EF: also the virial sum f_s D (x) D (costs ~6 FMAs/pair) */
  const double* upstream_dev;   /* LJ_ADJOINT: device pointer to the upstream gradient g (1 double) */
  int nbins;                    /* HIST_*: number of bins (1..1000) */
  double hist_hi;               /* HIST_*: upper edge of the last bin */
  const double* vel_x_dev;      /* HIST_RELSPEED, HIST_DIST_VEL: velocities of x, n_x*dim FP64 */
  const double* vel_y_dev;      /* the same, cross set: velocities of y */
  int want_sums;                /* HIST_RELSPEED: per-bin FP64 sum of |v_j - v_i| */
  int64_t capacity;             /* NEIGHBOR_LIST: pair slots available in pairs_dev */
  int with_distances;           /* NEIGHBOR_LIST: also write d (FP64) */
  double cutoff;                /* every kind: membership cutoff of this map, 0 < cutoff <=
                                   the box cutoff (0: the box cutoff).  The cell grid stays
                                   the box's; pairs are those with min-image d <= cutoff. */
  const double* weights_x_dev;  /* SUM_W_INV_D: n_x FP64 weights (caller order); the map copies
                                   them into the cell list's sorted records */
  const double* weights_y_dev;  /* SUM_W_INV_D, cross set: n_y weights */
  void* scratch_dev;            /* NEIGHBOR_LIST with sorted: caller-owned device scratch of at least
                                   clm_pairs_sort_workspace_bytes(capacity, with_distances) bytes
                                   (256-byte aligned).
                                   LJ_EF / LJ_ADJOINT, single set, either precision: caller-owned
                                   device scratch of at least clm_map_scratch_bytes bytes
                                   (256-byte aligned) enables the half-shell force sweep, which
                                   evaluates every pair once and keeps both particles' force sums
                                   in planes (FP32 in the FP32_GUARD form, FP64 in the FP64 form;
                                   one writer per slot) summed per particle in FP64.  NULL: the
                                   full-shell gather, which evaluates every pair from both ends.
                                   Both meet the form's tolerances; their force values differ in
                                   rounding.  A non-NULL scratch that is too small or misaligned
                                   is CLM_E_WORKSPACE; other kinds and cross sets ignore it. */
  size_t scratch_bytes;
  int no_prune;                 /* half-shell force sweep: 1 keeps every candidate of the visited
                                   cells (no pruning by the distance to the tile's bounding box;
                                   same results, for comparison) */
  int sorted;                   /* NEIGHBOR_LIST: 1 puts the written pairs in canonical order on the
                                   device (ascending i, then ascending j; distances moved along),
                                   as clm_pairs_sort does; needs scratch_dev */
  int check_capacity;           /* NEIGHBOR_LIST: 1 synchronizes the stream after the map and
                                   returns CLM_E_CAPACITY when the list has more pairs than
                                   capacity (count_dev holds the true count; re-call with a
                                   larger buffer).  0: the call stays asynchronous and overflow
                                   shows only in *count_dev. */
  int half_shell;               /* LJ_EF / LJ_ADJOINT with a map scratch: 0 runs the half-shell sweep
                                   when the grid gives at least 4096 (cell row, neighbour row)
                                   work items, or when a cell row holds no more 64-particle tiles
                                   (on average) than a gather tile visits rows, (2l+1)^(dim-1);
                                   otherwise the full-shell gather (one half-shell wave works
                                   through a whole row: long rows with few items leave the device
                                   idle); 1 runs the half-shell sweep whenever it applies; -1 never. */
} clm_map_params;

typedef struct clm_map_out {
  double* energy_dev;      /* [1] LJ energy; SUM_D / SUM_INV_D: the sum (FP64) */
  double* forces_dev;      /* LJ_EF: -dE/dr, LJ_ADJOINT: g*dE/dr; n_x*dim FP64, original order */
  double* virial_dev;      /* LJ_EF with want_virial: dim*dim FP64 */
  double* grad_box_dev;    /* LJ_EF: dE/dH, LJ_ADJOINT: g*dE/dH (fixed Cartesian r); dim*dim */
  uint64_t* hist_dev;      /* HIST_*: nbins+1 counts, the last slot counts values above hist_hi */
  double* hist_sums_dev;   /* HIST_RELSPEED with want_sums, HIST_DIST_VEL: nbins FP64 */
  int32_t* pairs_dev;      /* NEIGHBOR_LIST: capacity x 2 (i, j); single set i < j;
                              cross set i indexes x and j indexes y.  Order: clm_map on
                              a cell list with at least 2*lcell+1 cells per axis writes
                              the pairs in an order fixed by the built cell list (a
                              counting sweep first gives every work item its output
                              offset), so repeated calls give the same list, also in
                              clm_map_batch; small boxes take slots from a shared
                              counter (order unspecified).  With params->sorted:
                              ascending i, then j, on every path. */
  double* dist_dev;        /* NEIGHBOR_LIST with with_distances: capacity FP64 */
  uint64_t* count_dev;     /* [1] REQUIRED for every kind: number of pairs in the set.
                              NEIGHBOR_LIST: if *count_dev > capacity only the first
                              capacity pairs were written; re-call with a larger buffer. */
} clm_map_out;

/* Context: a device and the caller's stream (hipStream_t; NULL = default). */
clm_status clm_context_create(int hip_device, void* hip_stream, clm_context** out);
clm_status clm_context_set_stream(clm_context* ctx, void* hip_stream);
clm_status clm_context_destroy(clm_context* ctx);

/* Box (host only, no device work): H as above, cutoff rc > 0, lcell >= 1
 * (cell side ~ rc/lcell, the paper's lcell, section 2.8). */
clm_status clm_box_create(int dim, const double* H, double cutoff, int lcell, clm_box** out);
/* The same with a separate reach along the row (first fractional) axis:
 * cells there are ~ rc/lcell_x thick, on the other axes ~ rc/lcell
 * (lcell_x = 0: lcell).  Any lcell_x >= 1 gives the same pair set; a finer
 * row axis packs more particles into each work tile of whole cells. */
clm_status clm_box_create_ex(int dim, const double* H, double cutoff, int lcell, int lcell_x,
                             clm_box** out);
/* Bounding box of a NON-periodic computation (paper section 4.1: the
 * extrema of the points set a box large enough to avoid periodic
 * interactions within the cutoff): orthorhombic, side (hi[a] - lo[a]) +
 * 1.000001 * cutoff along each axis a, with lo/hi the coordinate extrema over
 * every set (clm_extrema).  Every periodic image of a displacement between
 * points inside [lo, hi] is then farther than the cutoff, so the canonical
 * pair set of this box is the set of pairs whose Euclidean distance is
 * <= cutoff.  Errors: CLM_E_BAD_BOX (non-finite or lo > hi), as clm_box_create. */
clm_status clm_box_nonperiodic(int dim, const double* lo, const double* hi, double cutoff, int lcell,
                               clm_box** out);
/* Coordinate extrema of n >= 1 points (n x dim FP64, device): lo[a] = min,
 * hi[a] = max over the points (host arrays of dim doubles).  Synchronizes
 * the context's stream.  Workspace: clm_extrema_workspace_bytes. */
clm_status clm_extrema_workspace_bytes(int64_t n, size_t* bytes);
clm_status clm_extrema(clm_context* ctx, int dim, const double* x_dev, int64_t n, void* workspace_dev,
                       size_t workspace_bytes, double* lo, double* hi);
/* Triclinic box from lengths (a, b, c) and angles in degrees (alpha =
 * angle(b,c), beta = angle(a,c), gamma = angle(a,b)); a along x, b in xy. */
clm_status clm_box_from_lengths_angles(const double* lengths, const double* angles_deg,
                                       double cutoff, int lcell, clm_box** out);
clm_status clm_box_info_get(const clm_box* box, clm_box_info* out);
clm_status clm_box_destroy(clm_box* box);

/* Cell list over n_x particles (and, for a cross set, n_y more; n_y = 0 for
 * a single set).  The workspace (device memory, 256-byte aligned) holds the
 * cell-sorted coordinates, the cell offsets, the work tiles and the map
 * partials; query its size first. */
clm_status clm_celllist_workspace_bytes(const clm_box* box, int64_t n_x, int64_t n_y,
                                        clm_precision precision, size_t* bytes);
clm_status clm_celllist_create(clm_context* ctx, const clm_box* box, int64_t n_x, int64_t n_y,
                               clm_precision precision, void* workspace_dev,
                               size_t workspace_bytes, clm_celllist** out);
/* Bin the particles (async).  x_dev: n_x*dim FP64; y_dev: n_y*dim FP64 or
 * NULL for a single set.  The inputs may be freed after the build. */
clm_status clm_celllist_build(clm_celllist* cl, const double* x_dev, const double* y_dev);
/* Bytes of map scratch (clm_map_params.scratch_dev) that make LJ_EF and
 * LJ_ADJOINT use the half-shell force sweep on this cell list (paper
 * section 2.8's half shell; 0 where that sweep does not apply: cross sets,
 * boxes with fewer than 2*lcell+1 cells per axis, other kinds).  About
 * 26 x 12 bytes per particle at lcell 2 in 3D (2 (2 l^2 + 2 l + 1) planes of
 * 3 FP32 components), twice that in the FP64 form. */
clm_status clm_map_scratch_bytes(const clm_celllist* cl, clm_map_kind kind, size_t* bytes);
/* Map one kind over the pair set and reduce it (async). */
clm_status clm_map(clm_celllist* cl, clm_map_kind kind, const clm_map_params* params,
                   const clm_map_out* out);
/* Batched map (serving): one sweep launch covers the tiles of every job.
 * All cell lists must share the context, dim and precision and be built;
 * params[k] / outs[k] are job k's arguments as for clm_map (histograms of a
 * batch share nbins).  Jobs whose box has fewer than 3 cells per axis run as
 * separate brute-force launches.  Each job's results equal those of
 * clm_map on that job alone (sums up to FP64 summation order).  The batch
 * workspace (device, 256-byte aligned, caller-owned) holds the job
 * descriptors and the concatenated tile list; it may be reused after the
 * batch has run. */
clm_status clm_map_batch_workspace_bytes(int njobs, clm_celllist* const* cls, size_t* bytes);
clm_status clm_map_batch(int njobs, clm_celllist* const* cls, clm_map_kind kind,
                         const clm_map_params* params, const clm_map_out* outs, void* workspace_dev,
                         size_t workspace_bytes);

/* Canonical order of a neighbour list (section 4.1's list of pairs within
 * the cutoff): the first min(*count_dev, capacity) pairs of pairs_dev
 * (int32 (i, j), 8-byte aligned, i < n_i, j < n_j) are put in ascending
 * order of i, then j, in place, with dist_dev (FP64, may be NULL) moved
 * along.  Asynchronous on the context's stream (the count is read on the
 * device).  The workspace (256-byte aligned, clm_pairs_sort_workspace_bytes
 * bytes) holds a second key buffer, a second distance buffer and the digit
 * table of the radix sort.  Errors: CLM_E_INVALID_ARG (index ranges outside
 * 1..2^31, capacity outside 0..2^31 - 2^20, misaligned pairs),
 * CLM_E_WORKSPACE. */
clm_status clm_pairs_sort_workspace_bytes(int64_t capacity, int with_distances, size_t* bytes);
clm_status clm_pairs_sort(clm_context* ctx, int64_t n_i, int64_t n_j, int32_t* pairs_dev,
                          double* dist_dev, const uint64_t* count_dev, int64_t capacity,
                          void* workspace_dev, size_t workspace_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bin and
 * map in one call with no workspace argument and no allocation.  The cell
 * list is placed in a static device array of the library (its size from
 * clm_map_static_max_bytes: 64 MiB, held on every device the library runs
 * on until the process ends).  Arguments as clm_celllist_create +
 * clm_celllist_build + clm_map with x_dev / y_dev (n_x*dim and n_y*dim FP64,
 * y_dev NULL and n_y = 0 for a single set); results, order of neighbour
 * lists included, equal theirs.  Asynchronous on the context's stream; the
 * inputs may be freed once the call's work has run.  Errors: as those calls,
 * plus CLM_E_CAPACITY (synchronously, before any launch) when the cell list
 * needs more than the static array (clm_celllist_workspace_bytes).  Every
 * call on one device shares that device's array: calls that overlap on one
 * device (different streams or host threads) race.  Timing events
 * (clm_context_set_timing) are not recorded for these calls. */
clm_status clm_map_static_max_bytes(size_t* bytes);
clm_status clm_map_static(clm_context* ctx, const clm_box* box, const double* x_dev, int64_t n_x,
                          const double* y_dev, int64_t n_y, clm_precision precision,
                          clm_map_kind kind, const clm_map_params* params, const clm_map_out* out);

/* Host-side counters of the last build (synchronizes the stream). */
clm_status clm_celllist_info_get(clm_celllist* cl, clm_celllist_info* out);
clm_status clm_celllist_destroy(clm_celllist* cl);

clm_status clm_synchronize(clm_context* ctx);

/* Kernel timing (tracing aid).  When enabled, the library records HIP events
 * on the context's stream around every build (bin + scan + tiles + scatter)
 * and around every sweep kernel of clm_map.  clm_stats_get synchronizes,
 * returns the accumulated times and counts, and clears them when reset != 0.
 * Events are host-side runtime objects; no device memory is allocated. */
typedef struct clm_stats {
  int64_t builds;
  int64_t sweeps;
  double build_ms;   /* sum of build durations */
  double sweep_ms;   /* sum of sweep-kernel durations */
  double last_sweep_ms;
} clm_stats;
clm_status clm_context_set_timing(clm_context* ctx, int enable);
clm_status clm_stats_get(clm_context* ctx, clm_stats* out, int reset);
const char* clm_last_error(void);
const char* clm_status_string(clm_status s);

#ifdef __cplusplus
}
#endif

#endif /* CLMAP_H */
