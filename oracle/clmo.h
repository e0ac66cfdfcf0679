/*
 * clmo.h -- plain, slow FP64 CPU oracle for the cell-list pair map of
 * "CellListMap.jl" (Martinez, arXiv 2202.06427).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; both sides implement the
 * same written definitions (below) independently.
 *
 * What it computes (paper sections 2.3 and 2.8): for a periodic box with
 * unit-cell matrix H (columns = lattice vectors, section 2.5 / Code 3), a
 * cutoff rc and particle positions, the set of particle pairs whose
 * minimum-image distance is within the cutoff, and a map reduced over that
 * set (sum of 1/d, LJ energy and its gradient, histograms, neighbour list).
 *
 * Canonical definitions (FP64, round-to-nearest, every operation rounded on
 * its own, never fused; the GPU library follows the same definitions):
 *
 *  H is given row-major: H[a*dim+b] is Cartesian component a of lattice
 *  vector b.  Hinv is the adjugate divided by the determinant:
 *     2D: det = H00*H11 - H01*H10; Hinv = [H11, -H01; -H10, H00] / det
 *     3D: C_ab are the cofactors written as one difference of two products,
 *         C00 = H11*H22 - H12*H21, C01 = H12*H20 - H10*H22,
 *         C02 = H10*H21 - H11*H20, C10 = H02*H21 - H01*H22,
 *         C11 = H00*H22 - H02*H20, C12 = H01*H20 - H00*H21,
 *         C20 = H01*H12 - H02*H11, C21 = H02*H10 - H00*H12,
 *         C22 = H00*H11 - H01*H10,
 *         det = (H00*C00 + H01*C01) + H02*C02,  Hinv_ab = C_ba / det.
 *  Wrap (the paper maps every particle into the primary cell before the
 *  pair loop, section 2.6): s_a = (Hinv_a0*r0 + Hinv_a1*r1) + Hinv_a2*r2
 *  (summed left to right), w_a = floor(s_a), f_a = s_a - w_a, and if
 *  f_a >= 1 then f_a = 0, w_a += 1.  The wrapped position is
 *  r'_a = (H_a0*f0 + H_a1*f1) + H_a2*f2.
 *  Image shift for an integer vector K: t_a = (H_a0*K0 + H_a1*K1) + H_a2*K2.
 *  Pair displacement and squared distance for image K:
 *     D_a = (r'_j,a - r'_i,a) + t_a,   d2 = (D0*D0 + D1*D1) + D2*D2.
 *  Minimum image: d2(i,j) = min over all K of d2(i,j,K).
 *  Membership: d2 <= rc2 with rc2 = rc*rc; self pairs excluded; single set:
 *  unordered pairs i<j once; cross set: every (i in x, j in y).
 *  Frame (positions kept in the wrap of an earlier step, as between
 *  rebuilds of a list reused over molecular-dynamics steps): given integer
 *  vectors w''_i, the frame position is r''_a = (H_a0*f0 + H_a1*f1) + H_a2*f2
 *  with f_a = s_a - w''_a (no floor).  Displacements, the minimum image and
 *  membership are then the definitions above with r'' in place of r'.  With
 *  w'' equal to the canonical w this is the canonical computation (except
 *  for s within one rounding below an integer, where the canonical wrap
 *  rounds f up to 1 and resets it to 0).
 *  Histogram edges: h = hi/nb, e_k = k*h, E_k = e_k*e_k (k = 0..nb); for a
 *  distance histogram with hi == rc, E_nb = rc2.  A value v goes to the
 *  first bin k (0-based) with v <= E_{k+1} (v = 0 goes to bin 0); values
 *  above E_nb go to the overflow slot nb.
 */
#ifndef CLMO_H
#define CLMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLMO_OK 0
#define CLMO_EINVAL 1

/* what to compute (bit mask for clmo_request.want) */
#define CLMO_W_COUNT 1
#define CLMO_W_SUM_D 2
#define CLMO_W_SUM_INV_D 4
#define CLMO_W_LJ 8          /* LJ energy, virial, dE/dH (and gradient if lj_grad) */
#define CLMO_W_HIST_DIST 16  /* distance histogram */
#define CLMO_W_HIST_REL 32   /* relative-speed histogram (+ per-bin sums) */
#define CLMO_W_NL 64         /* neighbour list (sorted) */
#define CLMO_W_SUM_W_INV_D 128    /* sum of w_i w_j / d (Code 5, masses) */
#define CLMO_W_HIST_DIST_VEL 256  /* distance histogram with per-bin sum of |v_j - v_i| (Code 10) */

#define CLMO_METHOD_AUTO (-1)
#define CLMO_METHOD_BRUTE 0
#define CLMO_METHOD_CELLS 1

typedef struct clmo_request {
  int want;        /* CLMO_W_* bits */
  int method;      /* CLMO_METHOD_* */
  int nthreads;    /* OpenMP threads, 0 = runtime default */
  double sigma, epsilon;          /* LJ: u = 4 eps ((s^2/d2)^6 - (s^2/d2)^3) */
  int hist_nbins; double hist_hi; /* distance histogram on (0, hi] */
  int rel_nbins; double rel_hi;   /* relative-speed histogram on (0, hi] */
  const double* vel_x;            /* nx*dim velocities (relative speed) */
  const double* vel_y;            /* ny*dim velocities of the cross set */
  int64_t nl_capacity;            /* entries available in nl_i/nl_j/nl_d */
  const int64_t* frame_x;         /* nx*dim frame integers w'' (single set), or NULL */
  const double* weights_x;        /* nx weights (SUM_W_INV_D) */
  const double* weights_y;        /* ny weights of the cross set */
  int dv_nbins; double dv_hi;     /* HIST_DIST_VEL: distance bins on (0, dv_hi], velocities vel_x/y */
} clmo_request;

typedef struct clmo_result {
  uint64_t count;          /* pairs within the cutoff */
  double sum_d, sum_inv_d; /* sum of d and of 1/d over the pairs */
  double lj_energy;
  double virial[9];        /* sum over pairs of f_s D (x) D, row-major dim x dim */
  double dEdH[9];          /* dE/dH at fixed Cartesian positions, row-major */
  double* lj_grad;         /* caller-owned nx*dim, dE/dr (single set), or NULL */
  uint64_t* hist;          /* caller-owned hist_nbins+1 (last = overflow) */
  uint64_t* rel_hist;      /* caller-owned rel_nbins+1 (last = overflow) */
  double* rel_sum;         /* caller-owned rel_nbins: per-bin sum of |v_j - v_i| */
  int64_t* nl_i;           /* caller-owned nl_capacity */
  int64_t* nl_j;
  double* nl_d;            /* may be NULL */
  uint64_t nl_count;       /* true number of pairs (may exceed capacity) */
  int method_used;
  double* nl_d2;           /* squared distances d2 of the listed pairs (may be NULL) */
  double sum_w_inv_d;      /* sum of w_i w_j / d */
  uint64_t* dv_hist;       /* caller-owned dv_nbins+1: pairs per distance bin (last = overflow) */
  double* dv_sum;          /* caller-owned dv_nbins: per distance bin, sum of |v_j - v_i| */
  double* lj_fabs;         /* caller-owned nx (with lj_grad): per particle, the sum over its
                              pairs of the pair-force magnitude |f_s| d (scale of force errors) */
} clmo_result;

/* Box geometry per the definitions above.  widths = perpendicular widths
 * (volume / area of the opposite face), volume = |det H|. */
int clmo_box_inverse(int dim, const double* H, double* Hinv);
int clmo_box_widths(int dim, const double* H, double* widths, double* volume);

/* Triclinic H from lengths (a,b,c) and angles (alpha = angle(b,c),
 * beta = angle(a,c), gamma = angle(a,b)) in degrees; a along x, b in xy. */
int clmo_box_from_lengths_angles(const double* len, const double* deg, double* H);

/* Canonical wrap of n positions: xw = wrapped positions (n*dim), frac =
 * wrapped fractional coordinates (n*dim, may be NULL), wrap = integer
 * w (n*dim, may be NULL). */
int clmo_wrap(int dim, const double* H, int64_t n, const double* x,
              double* xw, double* frac, int64_t* wrap);

/* Minimum-image squared distance of one pair of raw positions; K_out
 * (dim ints, may be NULL) receives the image of j relative to i in terms
 * of the raw positions (D = x_j - x_i + H K).  Searches every image whose
 * projection bound allows a distance up to `reach` (> 0); returns +inf if
 * none is within reach. */
double clmo_pair_d2(int dim, const double* H, const double* xi,
                    const double* xj, double reach, int* K_out);

/* Full computation over a single set (y == NULL) or a cross set. */
int clmo_compute(int dim, const double* H, double cutoff,
                 const double* x, int64_t nx, const double* y, int64_t ny,
                 const clmo_request* req, clmo_result* res);

/* For each sampled particle i (single set): E_i = sum over j != i within
 * the cutoff of u(d_ij) and g_i = dE/dr_i, by brute force over all j. */
int clmo_lj_sample(int dim, const double* H, double cutoff, const double* x,
                   int64_t n, const int64_t* sample, int64_t ns, double sigma,
                   double epsilon, int nthreads, double* energy_i, double* grad_i);

/* Neighbours of particle i (brute force): j indices and their images K
 * in terms of the raw positions (D = x_j - x_i + H K).  Returns the true
 * count in *count; writes at most cap entries. */
int clmo_neighbors_of(int dim, const double* H, double cutoff, const double* x,
                      int64_t n, int64_t i, int64_t cap, int64_t* js, int* Ks,
                      int64_t* count);

/* The paper's own computing-cell grid convention (Code 3), informational:
 * orthorhombic: n_d = floor(L_d/(rc/lcell)) + 2*lcell;
 * triclinic: n_d = ceil(extent_d/(rc/lcell)) + 2*lcell, where extent_d is
 * the extent of the unit cell along Cartesian axis d.  sizes_out gets the
 * computing-cell side per axis. */
int clmo_paper_ghost_grid(int dim, const double* H, double cutoff, int lcell,
                          int* ncells_out, double* sizes_out);

#ifdef __cplusplus
}
#endif

#endif /* CLMO_H */
