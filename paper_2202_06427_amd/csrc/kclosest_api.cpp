// kclosest_api.cpp -- the C-ABI of the k-closest-pairs call of libclmap.so
// (declared in include/clmap_kclosest.h; paper section 3.2, Code 8).
//
// Host orchestration of device steps: exact distance histograms (clm_map)
// narrow a threshold until the candidates fit, a neighbour-list map collects
// them, and the kernels of kclosest_kernels.hip key and sort them.  Every
// device buffer belongs to the caller.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/clmap_kclosest.h"
#include "clmap_state.h"

namespace {

constexpr int kKcBins = 1000;     // histogram bins per refinement level
constexpr int kKcLevels = 12;     // refinement levels before giving up on ties

int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct KcLayout {
  size_t hist, hcount, pairs, ncount, inv_x, inv_y, rec, total;
};

KcLayout kc_layout(int64_t nx, int64_t ny, int64_t cap) {
  Carve c;
  KcLayout L;
  L.hist = c.take(sizeof(uint64_t) * (kKcBins + 1));
  L.hcount = c.take(sizeof(uint64_t));
  L.pairs = c.take(sizeof(int32_t) * 2 * (size_t)cap);
  L.ncount = c.take(sizeof(uint64_t));
  L.inv_x = c.take(sizeof(uint32_t) * (size_t)std::max<int64_t>(nx, 1));
  L.inv_y = c.take(sizeof(uint32_t) * (size_t)std::max<int64_t>(ny, 1));
  L.rec = c.take(sizeof(KcRecord) * (size_t)pow2_at_least(cap));
  L.total = c.off;
  return L;
}

clm_status kc_check(const clm_celllist* cl, int64_t k, int64_t cap) {
  if (!cl) return fail(CLM_E_INVALID_ARG, "cell list is NULL");
  if (cl->box.small)
    return fail(CLM_E_UNSUPPORTED, "k closest pairs need a box with at least 2 lcell + 1 cells per axis");
  if (k < 1 || k > (int64_t(1) << 24)) return fail(CLM_E_INVALID_ARG, "k must be in 1..2^24");
  if (cap < k || cap > (int64_t(1) << 26))
    return fail(CLM_E_INVALID_ARG, "capacity must be in k..2^26 (got %lld)", (long long)cap);
  return CLM_OK;
}

// Host copy of a device buffer on the context's stream (synchronizes).
clm_status fetch(clm_context* ctx, void* dst, const void* src, size_t bytes) {
  CLM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
  CLM_HIP(hipStreamSynchronize(ctx->stream));
  return CLM_OK;
}

}  // namespace

extern "C" {

clm_status clm_kclosest_workspace_bytes(const clm_celllist* cl, int64_t k, int64_t cap, size_t* bytes) {
  clm_status s = kc_check(cl, k, cap);
  if (s != CLM_OK) return s;
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  *bytes = kc_layout(cl->nx, cl->cross ? cl->ny : 0, cap).total;
  return CLM_OK;
}

clm_status clm_kclosest(clm_celllist* cl, int64_t k, int64_t cap, void* ws, size_t ws_bytes,
                        int32_t* io, int32_t* jo, double* d2o, int64_t* found) {
  clm_status s = kc_check(cl, k, cap);
  if (s != CLM_OK) return s;
  if (!io || !jo || !d2o || !found) return fail(CLM_E_INVALID_ARG, "an output is NULL");
  if (!cl->built) return fail(CLM_E_INVALID_ARG, "the cell list is not built");
  const KcLayout L = kc_layout(cl->nx, cl->cross ? cl->ny : 0, cap);
  if (!ws) return fail(CLM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(CLM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(CLM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  char* base = (char*)ws;
  uint64_t* hist = (uint64_t*)(base + L.hist);
  uint64_t* hcount = (uint64_t*)(base + L.hcount);
  int32_t* pairs = (int32_t*)(base + L.pairs);
  uint64_t* ncount = (uint64_t*)(base + L.ncount);
  uint32_t* inv_x = (uint32_t*)(base + L.inv_x);
  uint32_t* inv_y = (uint32_t*)(base + L.inv_y);
  KcRecord* rec = (KcRecord*)(base + L.rec);
  clm_context* ctx = cl->ctx;
  CLM_HIP(hipSetDevice(ctx->device));

  // 1. threshold: the smallest histogram edge with >= k pairs up to it,
  //    refined while the pairs up to it exceed the capacity
  double hi = cl->box.rc;
  double thr = hi;
  uint64_t C = 0;
  bool fits = false;
  std::vector<uint64_t> h(kKcBins + 1);
  for (int level = 0; level < kKcLevels && !fits; ++level) {
    clm_map_params P;
    std::memset(&P, 0, sizeof P);
    P.nbins = kKcBins;
    P.hist_hi = hi;
    P.cutoff = hi;
    clm_map_out O;
    std::memset(&O, 0, sizeof O);
    O.hist_dev = hist;
    O.count_dev = hcount;
    s = clm_map(cl, CLM_MAP_HIST_DIST, &P, &O);
    if (s != CLM_OK) return s;
    s = fetch(ctx, h.data(), hist, sizeof(uint64_t) * (kKcBins + 1));
    if (s != CLM_OK) return s;
    uint64_t total = 0;
    for (int b = 0; b < kKcBins; ++b) total += h[b];
    if (total <= (uint64_t)cap) {  // every pair up to hi fits
      thr = hi;
      C = total;
      fits = true;
      break;
    }
    // first bin m with >= k pairs up to its upper edge e_{m+1} = (m + 1) h
    uint64_t cum = 0;
    int m = 0;
    for (; m < kKcBins; ++m) {
      cum += h[m];
      if (cum >= (uint64_t)k) break;
    }
    const double hw = hi / (double)kKcBins;
    const double e = m + 1 < kKcBins ? (double)(m + 1) * hw : hi;
    if (cum <= (uint64_t)cap) {
      thr = e;
      C = cum;
      fits = true;
      break;
    }
    if (!(e < hi)) {  // the k-th distance sits in the last bin: no narrower edge
      C = cum;
      break;
    }
    hi = e;
    C = cum;
  }
  if (!fits) {
    *found = (int64_t)C;
    return fail(CLM_E_CAPACITY,
                "%llu candidate pairs share the distances up to the k-th one (capacity %lld)",
                (unsigned long long)C, (long long)cap);
  }

  // 2. candidates: every pair within the threshold
  {
    clm_map_params P;
    std::memset(&P, 0, sizeof P);
    P.capacity = cap;
    P.cutoff = thr;
    clm_map_out O;
    std::memset(&O, 0, sizeof O);
    O.pairs_dev = pairs;
    O.count_dev = ncount;
    // up to 2^20 candidates the shared output counter is not contended: one
    // sweep instead of a counting sweep and the list sweep
    s = map_one(cl, CLM_MAP_NEIGHBOR_LIST, &P, &O, C > (uint64_t(1) << 20));
    if (s != CLM_OK) return s;
    uint64_t got = 0;
    s = fetch(ctx, &got, ncount, sizeof got);
    if (s != CLM_OK) return s;
    if (got != C)
      return fail(CLM_E_DEVICE, "neighbour list found %llu pairs, the histogram %llu",
                  (unsigned long long)got, (unsigned long long)C);
  }

  // 3. canonical keys, order, output
  hipStream_t st = ctx->stream;
  CLM_HIP(launch_kc_inverse(cl->X.idx, (int)cl->nx, inv_x, st));
  if (cl->cross) CLM_HIP(launch_kc_inverse(cl->Y.idx, (int)cl->ny, inv_y, st));
  KcKeys A;
  std::memset(&A, 0, sizeof A);
  A.dim = cl->box.dim;
  A.cross = cl->cross;
  A.cap = (int)cap;
  A.npow2 = (int)pow2_at_least(std::max<int64_t>((int64_t)C, 1));
  for (int q = 0; q < 27 * 4; ++q) A.tK[q] = cl->box.tK[q];
  A.pairs = pairs;
  A.count = (const unsigned long long*)ncount;
  A.r64_x = cl->X.r64;
  A.r64_y = cl->cross ? cl->Y.r64 : cl->X.r64;
  A.inv_x = inv_x;
  A.inv_y = cl->cross ? inv_y : inv_x;
  A.rec = rec;
  CLM_HIP(launch_kc_keys(A, st));
  CLM_HIP(launch_kc_sort(rec, A.npow2, st));
  const int64_t nf = std::min<int64_t>(k, (int64_t)C);
  CLM_HIP(launch_kc_output(rec, (int)k, (int)nf, io, jo, d2o, st));
  *found = nf;
  return CLM_OK;
}

}  // extern "C"
