/*
 * clmap_md.h -- molecular-dynamics steps on top of libclmap.so: a
 * velocity-Verlet integrator and a Verlet pair list reused across steps
 * (after "CellListMap.jl", Martinez, arXiv 2202.06427, section 4.2: a Neon
 * fluid with Lennard-Jones interactions only, velocity-Verlet propagation with
 * a fixed time step and velocity rescaling every few steps; the paper notes
 * that production codes do not rebuild their pair lists at every step).
 *
 * Conventions are those of clmap.h (status codes, caller-owned device
 * memory, asynchronous work on the context's stream, row-major n x dim FP64
 * arrays in the caller's particle order).  No call here synchronizes the
 * stream except clm_vlist_info_get.  Nothing here allocates device memory:
 * workspaces are sized by the *_workspace_bytes calls and owned by the caller
 * (256-byte aligned, untouched by the caller while the handle lives).
 *
 * Velocity Verlet, with h = (dt / 2) / mass (FP64, computed once):
 *   kick+drift   v = lambda v + h F;  x = x + dt v
 *   forces       F = -dE/dx at the new x
 *   kick         v = v + h F;  KE = mass / 2 * sum_i |v_i|^2
 * lambda is 1, or sqrt(target_ke / KE) of the last kick when a rescale is
 * requested (the paper rescales velocities every 10 steps; applying the
 * factor at the start of the next step is the same arithmetic as applying it
 * at the end of the last one).  Positions are never wrapped by these calls.
 *
 * Verlet pair list: the cell list of `cl` is built with the LIST cutoff
 * rl = the box cutoff, and the interactions use a cutoff rc <= rl; the skin
 * is rl - rc.  The list holds, for every particle, every partner within rl
 * at the last rebuild (both directions) with its periodic image.  Each step
 * the largest displacement since the last rebuild is measured on the device;
 * when some particle has moved by more than skin / 2 (|x - x_ref|^2 >
 * (skin / 2)^2) the cell list and the pair list are rebuilt on the device,
 * without a host round trip (every rebuild kernel is launched each step and
 * returns at once when no rebuild is due).
 *
 * Pair distances between rebuilds are taken in the FRAME of the last
 * rebuild: the wrap integers w of that rebuild are kept and the position
 * used is r'' = H (Hinv x - w) (the wrap of clmap.h without the floor,
 * same operation order).  These are the same real distances as the
 * canonical wrap, rounded in another frame; at a rebuild step r'' is the
 * canonical r' (except for a coordinate s within one rounding below an
 * integer, where the wrap rounds f up to 1 and resets it to 0).  The pair
 * set of a step is every pair whose frame distance is <= rc, exactly, in
 * FP64 (the list kernel runs in FP64).
 */
#ifndef CLMAP_MD_H
#define CLMAP_MD_H

#include "clmap.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clm_md clm_md;        /* integrator (host handle) */
typedef struct clm_vlist clm_vlist;  /* Verlet pair list (host handle) */

/* ---------------------------------------------------------------- integrator */

/* Device workspace for an integrator of n particles. */
clm_status clm_md_workspace_bytes(int64_t n, size_t* bytes);

/* n particles of one mass (mass > 0), time step dt > 0, dim 2 or 3.
 * Errors: CLM_E_INVALID_ARG (sizes, mass, dt), CLM_E_WORKSPACE. */
clm_status clm_md_create(clm_context* ctx, int dim, int64_t n, double mass, double dt,
                         void* workspace_dev, size_t workspace_bytes, clm_md** out);

/* First half of a step: v = lambda v + h f, then x = x + dt v (x, v updated
 * in place; f = the forces of the previous step, n x dim).  rescale_target_ke
 * > 0 sets lambda = sqrt(rescale_target_ke / KE) with KE from the last kick
 * (clm_md_kick or clm_vlist_lj with an integrator); 0 means lambda = 1. */
clm_status clm_md_kick_drift(clm_md* md, double* x_dev, double* v_dev, const double* f_dev,
                             double rescale_target_ke);

/* Second half of a step: v = v + h f and KE = mass/2 sum |v|^2 (written to
 * ke_dev when not NULL, and kept for the next rescale). */
clm_status clm_md_kick(clm_md* md, double* v_dev, const double* f_dev, double* ke_dev);

/* Kinetic energy of velocities v alone: KE = mass/2 sum |v|^2, written to
 * ke_dev when not NULL and kept for the next rescale, as clm_md_kick computes
 * it (v is not changed).  The initial kinetic energy of a run (section 4.2
 * reports the kinetic energy of every step, the first included). */
clm_status clm_md_kinetic(clm_md* md, const double* v_dev, double* ke_dev);

/* v = sqrt(target_ke / KE) v in place, KE the one kept by the last
 * clm_md_kick, clm_vlist_lj with an integrator, or clm_md_kinetic: the
 * velocity rescaling of section 4.2 applied at the end of a run (within a run
 * clm_md_kick_drift applies it at the start of the next step).  target_ke > 0.
 * Errors: CLM_E_INVALID_ARG. */
clm_status clm_md_rescale(clm_md* md, double* v_dev, double target_ke);

clm_status clm_md_destroy(clm_md* md);

/* ---------------------------------------------------------------- Verlet list */

typedef struct clm_vlist_info {
  int64_t updates;       /* clm_vlist_update calls so far */
  int64_t rebuilds;      /* list builds so far (the first one included) */
  int64_t entries;       /* entries of the current list (each pair twice) */
  int64_t max_row;       /* most partners of one particle at the last rebuild */
  int64_t row_capacity;
  double skin;           /* box cutoff - interaction cutoff */
  int overflow;          /* 1: some row needed more than row_capacity entries at
                            a rebuild since creation; every result computed
                            from that list on is invalid */
  int pad;
} clm_vlist_info;

/* Workspace for a list over the single-set cell list `cl` with at most
 * row_capacity partners per particle (the row capacity bounds the partners
 * within the LIST cutoff; about 1.3 times the mean plus a margin is
 * typical). */
clm_status clm_vlist_workspace_bytes(const clm_celllist* cl, int64_t row_capacity, size_t* bytes);

/* A Verlet list for the particles of `cl` (single set, FP32 or FP64 cell
 * list, not a small box: the box must give >= 2 lcell + 1 cells per axis),
 * interaction cutoff 0 < cutoff < the box cutoff.  The list borrows the
 * cell list: clm_vlist_update rebuilds it, and the caller must not build it
 * otherwise while the list lives.  The first update always rebuilds.
 * Errors: CLM_E_INVALID_ARG, CLM_E_BAD_CUTOFF, CLM_E_UNSUPPORTED (cross
 * set, small box, n >= 2^27), CLM_E_WORKSPACE. */
clm_status clm_vlist_create(clm_celllist* cl, double cutoff, int64_t row_capacity,
                            void* workspace_dev, size_t workspace_bytes, clm_vlist** out);

/* One step's list maintenance for positions x (n x dim, caller order):
 * displacement check, rebuild when due (cell list + pair list), and the
 * frame positions of this step. */
clm_status clm_vlist_update(clm_vlist* vl, const double* x_dev);

/* Lennard-Jones over the pairs within the interaction cutoff at the last
 * update's positions: u(d) = 4 eps ((s/d)^12 - (s/d)^6) (paper Code 6),
 * forces = -dE/dx (n x dim, caller order, overwritten), energy_dev (1
 * double), virial_dev (dim x dim, sum over pairs of f_s D (x) D with
 * f_s = 24 eps (2 (s/d)^12 - (s/d)^6) / d^2, may be NULL), count_dev (pairs,
 * may be NULL).  With md != NULL the second half-kick of the step is fused:
 * v = v + h F and KE (ke_dev may be NULL) as in clm_md_kick. */
clm_status clm_vlist_lj(clm_vlist* vl, double sigma, double epsilon, double* forces_dev,
                        double* energy_dev, double* virial_dev, unsigned long long* count_dev,
                        clm_md* md, double* v_dev, double* ke_dev);

/* Counters of the list (synchronizes the context's stream). */
clm_status clm_vlist_info_get(clm_vlist* vl, clm_vlist_info* out);

clm_status clm_vlist_destroy(clm_vlist* vl);

#ifdef __cplusplus
}
#endif

#endif /* CLMAP_MD_H */
