/*
 * clmap_kclosest.h -- the k closest pairs of a cell list (libclmap.so), after
 * "CellListMap.jl" (Martinez, arXiv 2202.06427), section 3.2 and Code 8: the
 * closest pairs between two sets of particles within the cutoff, which the
 * paper computes with per-thread lists merged by a custom reduction that
 * keeps the smallest distances.
 *
 * Conventions are those of clmap.h.  The result is the k pairs with the
 * smallest squared distance d2 (the canonical d2 of clmap.h) among the pairs
 * within the box cutoff, in ascending (d2, i, j) order (equal distances are
 * ordered by index, so the result is unique); cross set: i in x, j in y;
 * single set: i < j.  With fewer than k pairs within the cutoff, every pair
 * is returned and the remaining slots hold (-1, -1, +inf).
 *
 * Method (all device work in the library's kernels, host decisions between
 * steps): an exact 1000-bin distance histogram of the pairs within a cutoff
 * r finds the bin that holds the k-th smallest distance; while the pairs up
 * to that bin's upper edge exceed `capacity`, the histogram is repeated with
 * r = that edge; then a neighbour-list map at the final edge collects the
 * candidates, their canonical d2 is recomputed from the cell list's FP64
 * positions (minimum over the images K in {-1,0,1}^dim), and a bitonic sort
 * orders them.  The call reads histograms back, so it synchronizes the
 * context's stream.
 */
#ifndef CLMAP_KCLOSEST_H
#define CLMAP_KCLOSEST_H

#include "clmap.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace for clm_kclosest on `cl` with up to `capacity` candidate pairs
 * (capacity >= k; 8192 or a few times k is typical). */
clm_status clm_kclosest_workspace_bytes(const clm_celllist* cl, int64_t k, int64_t capacity,
                                        size_t* bytes);

/* The k closest pairs of the built cell list `cl` (single or cross set, FP32
 * or FP64 form; not a small box).  Outputs i_dev, j_dev (int32, k each) and
 * d2_dev (FP64, k) in ascending (d2, i, j) order; *found (host) receives the
 * number of real pairs written (min(k, pairs within the cutoff)).
 * Errors: CLM_E_INVALID_ARG (k < 1, capacity < k, NULL outputs, cell list
 * not built), CLM_E_UNSUPPORTED (small box), CLM_E_WORKSPACE, CLM_E_CAPACITY
 * (more than `capacity` pairs share the distances up to the k-th one even
 * after refinement, e.g. many exactly equal distances: *found then receives
 * the number of candidates needed, and nothing is written). */
clm_status clm_kclosest(clm_celllist* cl, int64_t k, int64_t capacity, void* workspace_dev,
                        size_t workspace_bytes, int32_t* i_dev, int32_t* j_dev, double* d2_dev,
                        int64_t* found);

#ifdef __cplusplus
}
#endif

#endif /* CLMAP_KCLOSEST_H */
