// md_api.cpp -- the C-ABI of the molecular-dynamics calls of libclmap.so
// (declared in include/clmap_md.h): velocity Verlet and the Verlet pair list.
//
// Host side only: validation, workspace carving and launches on the
// context's stream.  Every device buffer belongs to the caller.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/clmap_md.h"
#include "clmap_state.h"

struct clm_md {
  clm_context* ctx;
  int dim;
  int64_t n;
  double mass, dt, h;
  double* part;      // per-block partials of the kick
  double* ke_keep;   // KE of the last kick
};

struct clm_vlist {
  clm_celllist* cl;
  int dim;
  int64_t n;
  int64_t cap;       // row capacity, a multiple of P
  int P, lgP;        // lanes per row in the force kernel (list layout)
  double rc, rc2;    // interaction cutoff
  double rl2;        // list threshold: (box cutoff)^2 with a relative margin
  double lim2;       // rebuild when a squared displacement exceeds (skin / 2)^2
  uint32_t* list;
  uint32_t* cnt;
  double4* pf;
  double* xref;
  VlFlags* fl;
  double* bmax;      // per-block maxima of the displacement check
  double* part;
  unsigned long long* pcount;
};

static int64_t md_blocks(int64_t n) { return (n + kMdBlock - 1) / kMdBlock; }

static void md_layout(int64_t n, char* base, size_t* total, clm_md* md) {
  Carve c;
  const size_t o_part = c.take(sizeof(double) * kMdPart * (size_t)std::max<int64_t>(md_blocks(n), 1));
  const size_t o_ke = c.take(sizeof(double));
  if (base && md) {
    md->part = (double*)(base + o_part);
    md->ke_keep = (double*)(base + o_ke);
  }
  *total = c.off;
}

static void vl_layout(int64_t n, int64_t cap, char* base, size_t* total, clm_vlist* vl) {
  // the force kernel runs up to 16 lanes per row: up to 16 n threads of block partials
  Carve c;
  const int64_t slices = (n + kWave - 1) / kWave;
  const size_t o_list = c.take(sizeof(uint32_t) * (size_t)slices * (size_t)cap * kWave);
  const size_t o_cnt = c.take(sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1));
  const size_t o_pf = c.take(sizeof(double4) * (size_t)std::max<int64_t>(n, 1));
  const size_t o_xref = c.take(sizeof(double) * 3 * (size_t)std::max<int64_t>(n, 1));
  const size_t o_fl = c.take(sizeof(VlFlags));
  const size_t o_bmax = c.take(sizeof(double) * kDriftBlocks);
  const int64_t nb = std::max<int64_t>(md_blocks(16 * n), 1);
  const size_t o_part = c.take(sizeof(double) * kMdPart * (size_t)nb);
  const size_t o_pc = c.take(sizeof(unsigned long long) * (size_t)nb);
  if (base && vl) {
    vl->list = (uint32_t*)(base + o_list);
    vl->cnt = (uint32_t*)(base + o_cnt);
    vl->pf = (double4*)(base + o_pf);
    vl->xref = (double*)(base + o_xref);
    vl->fl = (VlFlags*)(base + o_fl);
    vl->bmax = (double*)(base + o_bmax);
    vl->part = (double*)(base + o_part);
    vl->pcount = (unsigned long long*)(base + o_pc);
  }
  *total = c.off;
}

static clm_status check_ws(void* ws, size_t have, size_t need) {
  if (!ws) return fail(CLM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(CLM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (have < need)
    return fail(CLM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
  return CLM_OK;
}

extern "C" {

// ---------------------------------------------------------------- integrator
clm_status clm_md_workspace_bytes(int64_t n, size_t* bytes) {
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  if (n < 0 || n > (int64_t(1) << 31) - 1) return fail(CLM_E_INVALID_ARG, "n out of range");
  md_layout(n, nullptr, bytes, nullptr);
  return CLM_OK;
}

clm_status clm_md_create(clm_context* ctx, int dim, int64_t n, double mass, double dt, void* ws,
                         size_t ws_bytes, clm_md** out) {
  if (!ctx || !out) return fail(CLM_E_INVALID_ARG, "ctx or out is NULL");
  if (dim != 2 && dim != 3) return fail(CLM_E_INVALID_ARG, "dim must be 2 or 3");
  if (n < 0 || n > (int64_t(1) << 31) - 1) return fail(CLM_E_INVALID_ARG, "n out of range");
  if (!(mass > 0.0) || !std::isfinite(mass)) return fail(CLM_E_INVALID_ARG, "mass must be > 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CLM_E_INVALID_ARG, "dt must be > 0");
  size_t need = 0;
  md_layout(n, nullptr, &need, nullptr);
  clm_status s = check_ws(ws, ws_bytes, need);
  if (s != CLM_OK) return s;
  clm_md* md = new (std::nothrow) clm_md();
  if (!md) return fail(CLM_E_INVALID_ARG, "out of host memory");
  md->ctx = ctx;
  md->dim = dim;
  md->n = n;
  md->mass = mass;
  md->dt = dt;
  md->h = (0.5 * dt) / mass;
  md_layout(n, (char*)ws, &need, md);
  *out = md;
  return CLM_OK;
}

clm_status clm_md_kick_drift(clm_md* md, double* x, double* v, const double* f, double target_ke) {
  if (!md) return fail(CLM_E_INVALID_ARG, "md is NULL");
  if (md->n > 0 && (!x || !v || !f)) return fail(CLM_E_INVALID_ARG, "x, v or f is NULL");
  if (target_ke < 0.0 || !std::isfinite(target_ke))
    return fail(CLM_E_INVALID_ARG, "rescale_target_ke must be >= 0");
  CLM_HIP(hipSetDevice(md->ctx->device));
  CLM_HIP(launch_md_kick_drift(x, v, f, md->n * md->dim, md->h, md->dt, target_ke, md->ke_keep,
                               md->ctx->stream));
  return CLM_OK;
}

// Second half-kick (f != NULL) or kinetic energy alone (f == NULL).
static clm_status md_kick_or_ke(clm_md* md, double* v, const double* f, double* ke) {
  CLM_HIP(hipSetDevice(md->ctx->device));
  hipStream_t st = md->ctx->stream;
  if (md->n > 0) CLM_HIP(launch_md_kick(v, f, (int)md->n, md->dim, md->h, md->part, st));
  MdFinal F;
  std::memset(&F, 0, sizeof F);
  F.nb = (int)md_blocks(md->n);
  F.dim = md->dim;
  F.part = md->part;
  F.mass = md->mass;
  F.ke = ke;
  F.ke_keep = md->ke_keep;
  CLM_HIP(launch_md_finalize(F, st));
  return CLM_OK;
}

clm_status clm_md_kick(clm_md* md, double* v, const double* f, double* ke) {
  if (!md) return fail(CLM_E_INVALID_ARG, "md is NULL");
  if (md->n > 0 && (!v || !f)) return fail(CLM_E_INVALID_ARG, "v or f is NULL");
  return md_kick_or_ke(md, v, f, ke);
}

clm_status clm_md_kinetic(clm_md* md, const double* v, double* ke) {
  if (!md) return fail(CLM_E_INVALID_ARG, "md is NULL");
  if (md->n > 0 && !v) return fail(CLM_E_INVALID_ARG, "v is NULL");
  return md_kick_or_ke(md, const_cast<double*>(v), nullptr, ke);
}

clm_status clm_md_rescale(clm_md* md, double* v, double target_ke) {
  if (!md) return fail(CLM_E_INVALID_ARG, "md is NULL");
  if (md->n > 0 && !v) return fail(CLM_E_INVALID_ARG, "v is NULL");
  if (!(target_ke > 0.0) || !std::isfinite(target_ke))
    return fail(CLM_E_INVALID_ARG, "target_ke must be > 0");
  CLM_HIP(hipSetDevice(md->ctx->device));
  CLM_HIP(launch_md_rescale(v, md->n * md->dim, target_ke, md->ke_keep, md->ctx->stream));
  return CLM_OK;
}

clm_status clm_md_destroy(clm_md* md) {
  delete md;
  return CLM_OK;
}

// ---------------------------------------------------------------- Verlet list
static clm_status vl_check_cl(const clm_celllist* cl) {
  if (!cl) return fail(CLM_E_INVALID_ARG, "cell list is NULL");
  if (cl->cross) return fail(CLM_E_UNSUPPORTED, "a Verlet list needs a single-set cell list");
  if (cl->box.small)
    return fail(CLM_E_UNSUPPORTED,
                "a Verlet list needs a box with at least 2 lcell + 1 cells per axis");
  if (cl->nx >= (int64_t(1) << 27))
    return fail(CLM_E_UNSUPPORTED, "a Verlet list holds fewer than 2^27 particles");
  return CLM_OK;
}

clm_status clm_vlist_workspace_bytes(const clm_celllist* cl, int64_t cap, size_t* bytes) {
  clm_status s = vl_check_cl(cl);
  if (s != CLM_OK) return s;
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  if (cap < 1 || cap > (int64_t(1) << 20)) return fail(CLM_E_INVALID_ARG, "row_capacity must be in 1..2^20");
  const int64_t P = vl_rows_per_lane_group(cl->nx);
  vl_layout(cl->nx, (cap + P - 1) / P * P, nullptr, bytes, nullptr);
  return CLM_OK;
}

clm_status clm_vlist_create(clm_celllist* cl, double cutoff, int64_t cap, void* ws, size_t ws_bytes,
                            clm_vlist** out) {
  clm_status s = vl_check_cl(cl);
  if (s != CLM_OK) return s;
  if (!out) return fail(CLM_E_INVALID_ARG, "out is NULL");
  if (cap < 1 || cap > (int64_t(1) << 20)) return fail(CLM_E_INVALID_ARG, "row_capacity must be in 1..2^20");
  const double rl = cl->box.rc;
  if (!(cutoff > 0.0) || !std::isfinite(cutoff) || !(cutoff < rl))
    return fail(CLM_E_BAD_CUTOFF, "cutoff must be in (0, box cutoff %g) (got %g)", rl, cutoff);
  const int P = vl_rows_per_lane_group(cl->nx);
  cap = (cap + P - 1) / P * P;
  size_t need = 0;
  vl_layout(cl->nx, cap, nullptr, &need, nullptr);
  s = check_ws(ws, ws_bytes, need);
  if (s != CLM_OK) return s;
  clm_vlist* vl = new (std::nothrow) clm_vlist();
  if (!vl) return fail(CLM_E_INVALID_ARG, "out of host memory");
  vl->cl = cl;
  vl->dim = cl->box.dim;
  vl->n = cl->nx;
  vl->cap = cap;
  vl->P = P;
  vl->lgP = 0;
  while ((1 << vl->lgP) < P) ++vl->lgP;
  vl->rc = cutoff;
  vl->rc2 = cutoff * cutoff;
  // Partners within rl at the rebuild are listed with a relative margin far
  // above rounding, so every pair that can come within rc before the next
  // rebuild (each particle moves at most skin / 2) is in the list.
  vl->rl2 = (rl * rl) * (1.0 + 1e-9);
  const double hs = 0.5 * (rl - cutoff);
  vl->lim2 = hs * hs;
  vl_layout(cl->nx, cap, (char*)ws, &need, vl);
  CLM_HIP(hipSetDevice(cl->ctx->device));
  hipStream_t st = cl->ctx->stream;
  // counters zero, the first update rebuilds
  CLM_HIP(launch_fill_u32((uint32_t*)vl->fl, sizeof(VlFlags) / 4, 0u, st));
  CLM_HIP(launch_fill_u32(&vl->fl->force, 1, 1u, st));
  CLM_HIP(launch_fill_u32(vl->cnt, (size_t)vl->n, 0u, st));
  *out = vl;
  return CLM_OK;
}

clm_status clm_vlist_update(clm_vlist* vl, const double* x) {
  if (!vl) return fail(CLM_E_INVALID_ARG, "list is NULL");
  if (vl->n > 0 && !x) return fail(CLM_E_INVALID_ARG, "x is NULL");
  clm_celllist* cl = vl->cl;
  CLM_HIP(hipSetDevice(cl->ctx->device));
  hipStream_t st = cl->ctx->stream;
  const int n = (int)vl->n;
  CLM_HIP(launch_vl_drift(x, vl->xref, n, vl->dim, vl->lim2, vl->bmax, vl->fl, st));
  const uint32_t* gate = &vl->fl->gate;
  clm_status s = celllist_build_gated(cl, x, nullptr, gate);
  if (s != CLM_OK) return s;
  CLM_HIP(launch_fill_u32(vl->cnt, (size_t)vl->n, 0u, st, gate));
  VlBuild B;
  std::memset(&B, 0, sizeof B);
  for (int d = 0; d < 3; ++d) B.n[d] = cl->box.n[d];
  B.l = cl->box.lcell;
  B.lx = cl->box.lcx;
  B.cap = (int)vl->cap;
  B.P = vl->P;
  B.lgP = vl->lgP;
  // few tiles: spread each tile over its neighbour rows to fill the chip
  B.split = cl->nx < 400000 ? 1 : 0;
  B.max_tiles = cl->max_tiles;
  B.rl2 = vl->rl2;
  for (int k = 0; k < 27 * 4; ++k) B.tK[k] = cl->box.tK[k];
  B.tiles = cl->tiles;
  B.ntiles = &cl->row_off[cl->nrows];
  B.off = cl->X.off;
  B.r64 = cl->X.r64;
  B.list = vl->list;
  B.cnt = vl->cnt;
  B.fl = vl->fl;
  B.gate = gate;
  CLM_HIP(launch_vl_build(vl->dim, B, st));
  CLM_HIP(launch_vl_rowstats(vl->cnt, n, (int)vl->cap, vl->fl, gate, st));
  VlRefresh R;
  std::memset(&R, 0, sizeof R);
  R.n = n;
  R.dim = vl->dim;
  for (int k = 0; k < 9; ++k) {
    R.H[k] = cl->box.H[k];
    R.Hinv[k] = cl->box.Hinv[k];
  }
  R.x = x;
  R.idx = cl->X.idx;
  R.wrap = cl->X.wrap;
  R.pf = vl->pf;
  R.xref = vl->xref;
  R.gate = gate;
  CLM_HIP(launch_vl_refresh(R, st));
  return CLM_OK;
}

clm_status clm_vlist_lj(clm_vlist* vl, double sigma, double eps, double* forces, double* energy,
                        double* virial, unsigned long long* count, clm_md* md, double* v,
                        double* ke) {
  if (!vl) return fail(CLM_E_INVALID_ARG, "list is NULL");
  if (!(sigma > 0.0) || !std::isfinite(sigma) || !std::isfinite(eps))
    return fail(CLM_E_INVALID_ARG, "sigma must be > 0 and epsilon finite");
  if (vl->n > 0 && !forces) return fail(CLM_E_INVALID_ARG, "forces is NULL");
  if (!energy) return fail(CLM_E_INVALID_ARG, "energy is NULL");
  if (md) {
    if (md->n != vl->n || md->dim != vl->dim)
      return fail(CLM_E_INVALID_ARG, "integrator and list sizes differ");
    if (vl->n > 0 && !v) return fail(CLM_E_INVALID_ARG, "v is NULL");
  }
  clm_celllist* cl = vl->cl;
  CLM_HIP(hipSetDevice(cl->ctx->device));
  hipStream_t st = cl->ctx->stream;
  VlForce A;
  std::memset(&A, 0, sizeof A);
  A.n = (int)vl->n;
  A.cap = (int)vl->cap;
  A.rc2 = vl->rc2;
  A.s2 = sigma * sigma;
  A.eps = eps;
  A.h = md ? md->h : 0.0;
  for (int k = 0; k < 27 * 4; ++k) A.tK[k] = cl->box.tK[k];
  A.list = vl->list;
  A.cnt = vl->cnt;
  A.pf = vl->pf;
  A.idx = cl->X.idx;
  A.forces = forces;
  A.v = md ? v : nullptr;
  A.part = vl->part;
  A.pcount = vl->pcount;
  if (vl->n > 0) CLM_HIP(launch_vl_lj(vl->dim, md != nullptr, virial != nullptr, vl->P, A, st));
  MdFinal F;
  std::memset(&F, 0, sizeof F);
  F.nb = vl->n > 0 ? (int)md_blocks(vl->n * vl->P) : 0;
  F.dim = vl->dim;
  F.part = vl->part;
  F.pcount = vl->pcount;
  F.eps = eps;
  F.mass = md ? md->mass : 0.0;
  F.energy = energy;
  F.virial = virial;
  F.count = count;
  F.ke = md ? ke : nullptr;
  F.ke_keep = md ? md->ke_keep : nullptr;
  CLM_HIP(launch_md_finalize(F, st));
  return CLM_OK;
}

clm_status clm_vlist_info_get(clm_vlist* vl, clm_vlist_info* o) {
  if (!vl || !o) return fail(CLM_E_INVALID_ARG, "list or out is NULL");
  CLM_HIP(hipSetDevice(vl->cl->ctx->device));
  VlFlags f;
  CLM_HIP(hipMemcpyAsync(&f, vl->fl, sizeof f, hipMemcpyDeviceToHost, vl->cl->ctx->stream));
  CLM_HIP(hipStreamSynchronize(vl->cl->ctx->stream));
  std::memset(o, 0, sizeof *o);
  o->updates = (int64_t)f.updates;
  o->rebuilds = (int64_t)f.rebuilds;
  o->entries = (int64_t)f.entries;
  o->max_row = (int64_t)f.max_row;
  o->row_capacity = vl->cap;
  o->skin = vl->cl->box.rc - vl->rc;
  o->overflow = f.overflow != 0u ? 1 : 0;
  return CLM_OK;
}

clm_status clm_vlist_destroy(clm_vlist* vl) {
  delete vl;
  return CLM_OK;
}

}  // extern "C"
