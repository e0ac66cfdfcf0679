// clmap_api.cpp -- the C-ABI of libclmap.so (declared in include/clmap.h).
//
// Host side only: argument validation, FP64 box geometry, workspace carving
// and kernel launches on the caller's stream.  Every device buffer belongs
// to the caller; this file never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "clmap_state.h"

// ---------------------------------------------------------------- geometry
// Canonical inverse: adjugate / determinant, every operation rounded on its
// own in the order written (the same definition the CPU oracle implements).
static int box_inverse(int dim, const double* H, double* Hi /* stride 3 */) {
  if (dim == 2) {
    const double H00 = H[0], H01 = H[1], H10 = H[3], H11 = H[4];
    double det = H00 * H11 - H01 * H10;
    if (!(det > 0.0) || !std::isfinite(det)) return 0;
    Hi[0] = H11 / det;
    Hi[1] = -H01 / det;
    Hi[3] = -H10 / det;
    Hi[4] = H00 / det;
    return 1;
  }
  const double H00 = H[0], H01 = H[1], H02 = H[2];
  const double H10 = H[3], H11 = H[4], H12 = H[5];
  const double H20 = H[6], H21 = H[7], H22 = H[8];
  const double C00 = H11 * H22 - H12 * H21;
  const double C01 = H12 * H20 - H10 * H22;
  const double C02 = H10 * H21 - H11 * H20;
  const double C10 = H02 * H21 - H01 * H22;
  const double C11 = H00 * H22 - H02 * H20;
  const double C12 = H01 * H20 - H00 * H21;
  const double C20 = H01 * H12 - H02 * H11;
  const double C21 = H02 * H10 - H00 * H12;
  const double C22 = H00 * H11 - H01 * H10;
  double det = (H00 * C00 + H01 * C01) + H02 * C02;
  if (!(det > 0.0) || !std::isfinite(det)) return 0;
  Hi[0] = C00 / det; Hi[1] = C10 / det; Hi[2] = C20 / det;
  Hi[3] = C01 / det; Hi[4] = C11 / det; Hi[5] = C21 / det;
  Hi[6] = C02 / det; Hi[7] = C12 / det; Hi[8] = C22 / det;
  return 1;
}

static float round_down_f(double v) {
  float f = (float)v;
  if ((double)f > v) f = std::nextafter(f, -INFINITY);
  return f;
}
static float round_up_f(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

static constexpr int64_t kMaxCells = int64_t(1) << 24;

// FP32 error band for membership at cutoff rc (<= the box cutoff: the grid's
// cells are fixed by the box).  The FP32 displacement is D32 = fl32(o_j - q_i)
// with o_j = fl32(offset of j from its cell origin, |o_j,a| <= C_a, the
// Cartesian extent of one cell along a) and q_i = fl32(r'_i - O_u) (one
// rounding of an FP64 value with |q_a| <= C_a + |D_a|).  Three roundings of
// relative size u = 2^-24 give, per component,
//   |D32_a - D_a| <= u (2 C_a + 2 |D_a|) + e64,
// e64 covering the FP64 roundings of r', of the cell origins and of the
// canonical d2 itself.  Near any threshold X <= rc^2 a candidate has
// |D| <= 1.01 rc (a farther one has d2_32 > rc^2 whatever the rounding), so
// |d2_32 - d2| <= 2 (1.01 rc) |E| + |E|^2 + 4 u (1.02 rc^2) for the FMA chain
// of three roundings.  The band is twice that bound.
// M scales the cell extent per fractional axis: the i coordinates of the
// half-shell LJ sweep are offsets from the centre of the tile's bounding box,
// within M_b cells along axis b (C_a = sum_b |H_ab| M_b / n_b), and the j
// coordinates from the same origin are at most |D_a| + C_a, which the same
// bound covers.
static void map_band(const clm_box& B, double rc, double* band, float* lo32, float* hi32,
                     const double* M = nullptr) {
  const int dim = B.dim;
  const double rc2 = rc * rc;
  const double u = std::ldexp(1.0, -24);
  double E2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    double C = 0.0, Hs = 0.0;
    for (int b = 0; b < dim; ++b) {
      C += std::fabs(B.H[a * 3 + b]) / (double)B.n[b] * (M ? M[b] : 1.0);
      Hs += std::fabs(B.H[a * 3 + b]);
    }
    double e64 = 64.0 * std::ldexp(1.0, -53) * (4.0 * Hs + 4.0 * rc);
    double Ea = u * (2.0 * C + 2.02 * rc) * (1.0 + 1e-6) + e64;
    E2 += Ea * Ea;
  }
  const double E = std::sqrt(E2);
  const double b0 = 2.02 * rc * E + E2 + 4.08 * u * rc2 + 1e-12 * rc2;
  *band = 2.0 * b0;
  *lo32 = round_down_f(rc2 - *band);
  *hi32 = round_up_f(rc2 + *band);
}

static clm_status box_setup(int dim, const double* Hin, double cutoff, int lcell, int lcell_x,
                            clm_box* B) {
  if (dim != 2 && dim != 3) return fail(CLM_E_BAD_BOX, "dim must be 2 or 3 (got %d)", dim);
  if (!Hin) return fail(CLM_E_INVALID_ARG, "H is NULL");
  if (!(cutoff > 0.0) || !std::isfinite(cutoff))
    return fail(CLM_E_BAD_CUTOFF, "cutoff must be finite and > 0");
  if (lcell < 1 || lcell > 8) return fail(CLM_E_BAD_CUTOFF, "lcell must be in 1..8 (got %d)", lcell);
  if (lcell_x == 0) lcell_x = lcell;
  if (lcell_x < 1 || lcell_x > 8)
    return fail(CLM_E_BAD_CUTOFF, "lcell_x must be 0 or in 1..8 (got %d)", lcell_x);
  std::memset(B, 0, sizeof *B);
  B->dim = dim;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) {
      double v = Hin[a * dim + b];
      if (!std::isfinite(v)) return fail(CLM_E_BAD_BOX, "H has a non-finite entry");
      B->H[a * 3 + b] = v;
    }
  if (!box_inverse(dim, B->H, B->Hinv))
    return fail(CLM_E_BAD_BOX, "det H must be > 0 (right-handed, non-degenerate cell)");
  // sum of the lattice-vector lengths: bounds every minimum-image distance
  // by half of it; cells flatter than 1:64 are rejected
  double sum_len = 0.0;
  for (int b = 0; b < dim; ++b) {
    double s2 = 0.0;
    for (int a = 0; a < dim; ++a) s2 += B->H[a * 3 + b] * B->H[a * 3 + b];
    sum_len += std::sqrt(s2);
  }
  B->sum_len = sum_len;
  // perpendicular widths: 1 / |row d of Hinv| (distance between the faces
  // spanned by the other lattice vectors); volume |det H|
  for (int d = 0; d < dim; ++d) {
    double s = 0.0;
    for (int b = 0; b < dim; ++b) s += B->Hinv[d * 3 + b] * B->Hinv[d * 3 + b];
    B->w[d] = 1.0 / std::sqrt(s);
  }
  {
    double wmin = B->w[0];
    for (int d = 1; d < dim; ++d) wmin = std::min(wmin, B->w[d]);
    if (!(sum_len <= 64.0 * wmin))
      return fail(CLM_E_BAD_BOX, "cell too flat or skewed (sum of edge lengths > 64 x smallest width)");
  }
  if (dim == 2)
    B->V = std::fabs(B->H[0] * B->H[4] - B->H[1] * B->H[3]);
  else {
    const double* H = B->H;
    B->V = std::fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                     H[2] * (H[3] * H[7] - H[4] * H[6]));
  }
  B->rc = cutoff;
  B->rc2 = cutoff * cutoff;
  B->lcell_req = lcell;
  B->lcx_req = lcell_x;
  for (int a = 0; a < 3; ++a) B->n[a] = 1;
  // grid: cells of fractional width 1/n_d with w_d / n_d >= (rc / l_d)(1 + 1e-9),
  // at least 2 l_d + 1 cells per axis (so the +-l_d neighbours are distinct
  // cells).  l_d = lcell on the cross-row axes; the row axis may use a finer
  // lcell_x (more, thinner cells per row: fuller tiles).  When an axis is too
  // short both levels step down together.
  B->small = 1;
  for (int l = lcell, lx = lcell_x; l >= 1 && lx >= 1; --l, --lx) {
    int n[3] = {1, 1, 1};
    int ld[3] = {lx, l, l};
    bool ok = true;
    double prod = 1.0;
    for (int d = 0; d < dim; ++d) {
      double m = std::floor(B->w[d] * (double)ld[d] / cutoff / (1.0 + 1e-9));
      if (!(m >= 2.0 * ld[d] + 1.0)) { ok = false; break; }
      if (m > 65535.0) m = 65535.0;
      n[d] = (int)m;
      prod *= m;
    }
    if (!ok) {
      if (l == 1 && lx > 1) l = 2;  // keep lcell 1 on the cross-row axes, refine x less
      else if (lx == 1 && l > 1) lx = 2;
      continue;
    }
    if (prod > (double)kMaxCells) {  // coarser cells stay correct (side >= rc/l)
      double f = std::pow((double)kMaxCells / prod, 1.0 / dim);
      prod = 1.0;
      for (int d = 0; d < dim; ++d) {
        n[d] = std::max(2 * ld[d] + 1, (int)std::floor(n[d] * f));
        prod *= n[d];
      }
      if (prod > (double)kMaxCells) continue;
    }
    B->lcell = l;
    B->lcx = lx;
    B->small = 0;
    for (int d = 0; d < dim; ++d) B->n[d] = n[d];
    break;
  }
  if (B->small) B->lcell = B->lcx = 1;
  B->ncells = (int64_t)B->n[0] * B->n[1] * B->n[2];
  B->smax = std::max(1, std::min(kMaxSpan, B->n[0] - 2 * B->lcx));
  // canonical image shifts t = H K for K in {-1,0,1}^3
  for (int kz = -1; kz <= 1; ++kz)
    for (int ky = -1; ky <= 1; ++ky)
      for (int kx = -1; kx <= 1; ++kx) {
        const double K[3] = {(double)kx, (double)ky, (double)kz};
        double* t = &B->tK[kcode(kx, ky, kz) * 4];
        for (int a = 0; a < 3; ++a) {
          if (a >= dim) { t[a] = 0.0; continue; }
          double acc = B->H[a * 3 + 0] * K[0];
          acc = acc + B->H[a * 3 + 1] * K[1];
          if (dim == 3) acc = acc + B->H[a * 3 + 2] * K[2];
          t[a] = acc;
        }
        t[3] = 0.0;
      }
  map_band(*B, cutoff, &B->band, &B->lo32, &B->hi32);
  return CLM_OK;
}

// ---------------------------------------------------------------- workspace
static const int kPadParticles = 64;

static int64_t max_tiles_for(const clm_box& B, int64_t n) {
  int64_t nrows = (int64_t)B.n[1] * B.n[2];
  int64_t t = 5 * ((n + 63) / 64) + nrows * ((B.n[0] + B.smax - 1) / B.smax + 2) + 4;
  return (t + 3) & ~(int64_t)3;
}

static void layout(clm_celllist* cl, char* base, size_t* total) {
  const clm_box& B = cl->box;
  Carve c;
  int64_t hist_max = 1;
  auto set = [&](SetBufs& S, int64_t n) {
    const BinPlan P = bin_plan(B.ncells, n);
    const int64_t nh = (int64_t)P.nbk * P.nblk;
    hist_max = std::max(hist_max, nh);
    size_t o_hist = c.take(sizeof(uint32_t) * (nh + 1));
    size_t o_off = c.take(sizeof(uint32_t) * (B.ncells + 1));
    size_t o_key = c.take(sizeof(uint32_t) * std::max<int64_t>(n, 1));
    size_t o_rec = c.take(sizeof(BinRec) * std::max<int64_t>(n, 1));
    size_t o_pos = c.take(sizeof(float4) * (n + kPadParticles));
    size_t o_r64 = c.take(sizeof(double4) * (n + kPadParticles));
    size_t o_idx = c.take(sizeof(uint32_t) * (n + kPadParticles));
    size_t o_wrap = c.take(sizeof(int4) * (n + kPadParticles));
    size_t o_vel = c.take(sizeof(float4) * (n + kPadParticles));
    if (base) {
      S.hist = (uint32_t*)(base + o_hist);
      S.off = (uint32_t*)(base + o_off);
      S.key = (uint32_t*)(base + o_key);
      S.rec = (BinRec*)(base + o_rec);
      S.pos = (float4*)(base + o_pos);
      S.r64 = (double4*)(base + o_r64);
      S.idx = (uint32_t*)(base + o_idx);
      S.wrap = (int4*)(base + o_wrap);
      S.vel32 = (float4*)(base + o_vel);
    }
  };
  set(cl->X, cl->nx);
  if (cl->cross) set(cl->Y, cl->ny);
  const int nrows = (int)(B.n[1] * B.n[2]);
  const int64_t maxt = max_tiles_for(B, cl->nx);
  // brute-force path (small boxes): partial rows per (64 particles, j chunk)
  // and per-chunk force rows
  const int64_t nyb = cl->cross ? cl->ny : cl->nx;
  const int64_t brute_rows =
      B.small ? std::max<int64_t>(1, (cl->nx + kWave - 1) / kWave) * brute_chunks(nyb) : 1;
  const int64_t parts = std::max<int64_t>(maxt, brute_rows);
  const size_t scan_elems =
      std::max(scan_scratch_elems((int)hist_max), scan_scratch_elems(nrows));
  size_t o_scan = c.take(sizeof(uint32_t) * scan_elems);
  size_t o_rt = c.take(sizeof(uint32_t) * (nrows + 1));
  size_t o_ro = c.take(sizeof(uint32_t) * (nrows + 1));
  size_t o_tiles = c.take(sizeof(Tile) * maxt);
  size_t o_job = c.take(sizeof(JobDesc));
  size_t o_part = c.take(sizeof(double) * kPartialD * parts);
  size_t o_pc = c.take(sizeof(unsigned long long) * parts);
  size_t o_nlo = c.take(sizeof(unsigned long long) * parts);
  size_t o_E64 = c.take(sizeof(double) * (kMaxBins + 1));
  size_t o_E32 = c.take(sizeof(float) * (kMaxBins + 1));
  size_t o_bq = c.take(sizeof(double) * 2);
  size_t o_vm = c.take(sizeof(unsigned int) * 2);
  size_t o_nlc = c.take(sizeof(unsigned long long) * 2);
  size_t o_cand = c.take(sizeof(unsigned long long) * maxt);
  size_t o_guard = c.take(sizeof(unsigned long long) * 4);
  size_t o_fin = c.take(sizeof(double) * kPartialD * kFinalBlocks);
  size_t o_finc = c.take(sizeof(unsigned long long) * kFinalBlocks);
  size_t o_fb = B.small ? c.take(sizeof(double) * 3 * (size_t)brute_chunks(nyb) * (size_t)cl->nx) : 0;
  if (base) {
    cl->scan_scratch = (uint32_t*)(base + o_scan);
    cl->row_tiles = (uint32_t*)(base + o_rt);
    cl->row_off = (uint32_t*)(base + o_ro);
    cl->tiles = (Tile*)(base + o_tiles);
    cl->job_dev = (JobDesc*)(base + o_job);
    cl->partials = (double*)(base + o_part);
    cl->pcount = (unsigned long long*)(base + o_pc);
    cl->nl_off = (unsigned long long*)(base + o_nlo);
    cl->E64 = (double*)(base + o_E64);
    cl->E32 = (float*)(base + o_E32);
    cl->bandq = (double*)(base + o_bq);
    cl->vmax_bits = (unsigned int*)(base + o_vm);
    cl->nl_counter = (unsigned long long*)(base + o_nlc);
    cl->cand = (unsigned long long*)(base + o_cand);
    cl->guard = (unsigned long long*)(base + o_guard);
    cl->fin_scratch = (double*)(base + o_fin);
    cl->fin_count = (unsigned long long*)(base + o_finc);
    cl->brute_fb = B.small ? (double*)(base + o_fb) : nullptr;
    cl->max_tiles = (int)maxt;
    cl->max_parts = (int)parts;
    cl->nrows = nrows;
  }
  *total = c.off;
}

// ---------------------------------------------------------------- API
extern "C" {

const char* clm_last_error(void) { return g_err.c_str(); }

const char* clm_status_string(clm_status s) {
  switch (s) {
    case CLM_OK: return "CLM_OK";
    case CLM_E_INVALID_ARG: return "CLM_E_INVALID_ARG";
    case CLM_E_BAD_BOX: return "CLM_E_BAD_BOX";
    case CLM_E_BAD_CUTOFF: return "CLM_E_BAD_CUTOFF";
    case CLM_E_CAPACITY: return "CLM_E_CAPACITY";
    case CLM_E_WORKSPACE: return "CLM_E_WORKSPACE";
    case CLM_E_DEVICE: return "CLM_E_DEVICE";
    case CLM_E_UNSUPPORTED: return "CLM_E_UNSUPPORTED";
  }
  return "unknown status";
}

clm_status clm_context_create(int hip_device, void* hip_stream, clm_context** out) {
  if (!out) return fail(CLM_E_INVALID_ARG, "out is NULL");
  int ndev = 0;
  CLM_HIP(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev)
    return fail(CLM_E_INVALID_ARG, "device %d out of range (%d devices)", hip_device, ndev);
  auto* c = new (std::nothrow) clm_context;
  if (!c) return fail(CLM_E_INVALID_ARG, "out of host memory");
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return CLM_OK;
}

clm_status clm_context_set_stream(clm_context* ctx, void* hip_stream) {
  if (!ctx) return fail(CLM_E_INVALID_ARG, "ctx is NULL");
  ctx->stream = (hipStream_t)hip_stream;
  return CLM_OK;
}

clm_status clm_context_destroy(clm_context* ctx) {
  if (!ctx) return CLM_OK;
  for (auto* v : {&ctx->pool, &ctx->build_ev, &ctx->sweep_ev})
    for (auto& e : *v) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
  delete ctx;
  return CLM_OK;
}

clm_status clm_context_set_timing(clm_context* ctx, int enable) {
  if (!ctx) return fail(CLM_E_INVALID_ARG, "ctx is NULL");
  ctx->timing = enable != 0;
  return CLM_OK;
}

clm_status clm_stats_get(clm_context* ctx, clm_stats* out, int reset) {
  if (!ctx || !out) return fail(CLM_E_INVALID_ARG, "NULL argument");
  CLM_HIP(hipSetDevice(ctx->device));
  std::memset(out, 0, sizeof *out);
  auto sum = [&](std::vector<EventPair>& v, double* total, double* last) -> clm_status {
    for (auto& e : v) {
      CLM_HIP(hipEventSynchronize(e.b));
      float ms = 0.0f;
      CLM_HIP(hipEventElapsedTime(&ms, e.a, e.b));
      *total += ms;
      if (last) *last = ms;
    }
    return CLM_OK;
  };
  clm_status s = sum(ctx->build_ev, &out->build_ms, nullptr);
  if (s != CLM_OK) return s;
  s = sum(ctx->sweep_ev, &out->sweep_ms, &out->last_sweep_ms);
  if (s != CLM_OK) return s;
  out->builds = (int64_t)ctx->build_ev.size();
  out->sweeps = (int64_t)ctx->sweep_ev.size();
  if (reset) {
    for (auto& e : ctx->build_ev) ctx->pool.push_back(e);
    for (auto& e : ctx->sweep_ev) ctx->pool.push_back(e);
    ctx->build_ev.clear();
    ctx->sweep_ev.clear();
  }
  return CLM_OK;
}

clm_status clm_box_create_ex(int dim, const double* H, double cutoff, int lcell, int lcell_x,
                             clm_box** out) {
  if (!out) return fail(CLM_E_INVALID_ARG, "out is NULL");
  clm_box tmp;
  clm_status s = box_setup(dim, H, cutoff, lcell, lcell_x, &tmp);
  if (s != CLM_OK) return s;
  auto* b = new (std::nothrow) clm_box(tmp);
  if (!b) return fail(CLM_E_INVALID_ARG, "out of host memory");
  *out = b;
  return CLM_OK;
}

clm_status clm_box_create(int dim, const double* H, double cutoff, int lcell, clm_box** out) {
  return clm_box_create_ex(dim, H, cutoff, lcell, 0, out);
}

clm_status clm_box_from_lengths_angles(const double* len, const double* deg, double cutoff,
                                       int lcell, clm_box** out) {
  if (!len || !deg || !out) return fail(CLM_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (!(len[k] > 0.0) || !std::isfinite(len[k]) || !(deg[k] > 0.0) || !(deg[k] < 180.0))
      return fail(CLM_E_BAD_BOX, "lengths must be > 0 and angles in (0, 180)");
  const double pi = 3.14159265358979323846;
  const double ca = std::cos(deg[0] * pi / 180.0), cb = std::cos(deg[1] * pi / 180.0);
  const double cg = std::cos(deg[2] * pi / 180.0), sg = std::sin(deg[2] * pi / 180.0);
  const double cy = (ca - cb * cg) / sg;
  const double cz2 = 1.0 - cb * cb - cy * cy;
  if (!(cz2 > 0.0)) return fail(CLM_E_BAD_BOX, "angles do not form a cell");
  const double a[3] = {len[0], 0.0, 0.0};
  const double b[3] = {len[1] * cg, len[1] * sg, 0.0};
  const double c[3] = {len[2] * cb, len[2] * cy, len[2] * std::sqrt(cz2)};
  double H[9];
  for (int r = 0; r < 3; ++r) {
    H[r * 3 + 0] = a[r];
    H[r * 3 + 1] = b[r];
    H[r * 3 + 2] = c[r];
  }
  return clm_box_create(3, H, cutoff, lcell, out);
}

clm_status clm_box_nonperiodic(int dim, const double* lo, const double* hi, double cutoff, int lcell,
                               clm_box** out) {
  if (dim != 2 && dim != 3) return fail(CLM_E_BAD_BOX, "dim must be 2 or 3 (got %d)", dim);
  if (!lo || !hi || !out) return fail(CLM_E_INVALID_ARG, "lo, hi or out is NULL");
  if (!(cutoff > 0.0) || !std::isfinite(cutoff))
    return fail(CLM_E_BAD_CUTOFF, "cutoff must be finite and > 0");
  double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < dim; ++a) {
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(lo[a] <= hi[a]))
      return fail(CLM_E_BAD_BOX, "extrema must be finite with lo <= hi (axis %d)", a);
    // every periodic image of a displacement is then farther than the cutoff
    H[a * dim + a] = (hi[a] - lo[a]) + 1.000001 * cutoff;
  }
  return clm_box_create(dim, H, cutoff, lcell, out);
}

clm_status clm_extrema_workspace_bytes(int64_t n, size_t* bytes) {
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  if (n < 1) return fail(CLM_E_INVALID_ARG, "n must be >= 1");
  *bytes = sizeof(double) * (6 * (size_t)kExtremaBlocks + 8);
  return CLM_OK;
}

clm_status clm_extrema(clm_context* ctx, int dim, const double* x, int64_t n, void* ws, size_t ws_bytes,
                       double* lo, double* hi) {
  if (!ctx || !x || !lo || !hi) return fail(CLM_E_INVALID_ARG, "an argument is NULL");
  if (dim != 2 && dim != 3) return fail(CLM_E_INVALID_ARG, "dim must be 2 or 3");
  if (n < 1) return fail(CLM_E_INVALID_ARG, "n must be >= 1");
  const size_t need = sizeof(double) * (6 * (size_t)kExtremaBlocks + 8);
  if (!ws || ws_bytes < need) return fail(CLM_E_WORKSPACE, "workspace needs %zu bytes", need);
  if (((uintptr_t)ws & 255u) != 0) return fail(CLM_E_WORKSPACE, "workspace must be 256-byte aligned");
  CLM_HIP(hipSetDevice(ctx->device));
  double* part = (double*)ws;
  double* res = part + 6 * kExtremaBlocks;
  CLM_HIP(launch_extrema(x, n, dim, part, res, ctx->stream));
  double h[6];
  CLM_HIP(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  CLM_HIP(hipStreamSynchronize(ctx->stream));
  for (int a = 0; a < dim; ++a) {
    lo[a] = h[a];
    hi[a] = h[3 + a];
  }
  return CLM_OK;
}

clm_status clm_box_info_get(const clm_box* B, clm_box_info* o) {
  if (!B || !o) return fail(CLM_E_INVALID_ARG, "NULL argument");
  std::memset(o, 0, sizeof *o);
  o->dim = B->dim;
  o->lcell_requested = B->lcell_req;
  o->lcell = B->lcell;
  o->lcell_x = B->lcx;
  o->small_box = B->small;
  for (int d = 0; d < 3; ++d) o->grid[d] = B->n[d];
  o->ncells = B->ncells;
  for (int a = 0; a < B->dim; ++a)
    for (int b = 0; b < B->dim; ++b) {
      o->H[a * B->dim + b] = B->H[a * 3 + b];
      o->Hinv[a * B->dim + b] = B->Hinv[a * 3 + b];
    }
  for (int d = 0; d < 3; ++d) o->widths[d] = d < B->dim ? B->w[d] : 0.0;
  o->volume = B->V;
  o->cutoff = B->rc;
  o->rc2 = B->rc2;
  o->guard_band = B->band;
  return CLM_OK;
}

clm_status clm_box_destroy(clm_box* b) {
  delete b;
  return CLM_OK;
}

static clm_status check_sizes(const clm_box* box, int64_t n_x, int64_t n_y, clm_precision p) {
  if (!box) return fail(CLM_E_INVALID_ARG, "box is NULL");
  if (p != CLM_FP64 && p != CLM_FP32_GUARD) return fail(CLM_E_INVALID_ARG, "bad precision %d", (int)p);
  const int64_t kMaxN = (int64_t)1 << 30;
  if (n_x < 0 || n_y < 0 || n_x > kMaxN || n_y > kMaxN)
    return fail(CLM_E_INVALID_ARG, "particle counts must be in [0, 2^30]");
  return CLM_OK;
}

clm_status clm_celllist_workspace_bytes(const clm_box* box, int64_t n_x, int64_t n_y,
                                        clm_precision precision, size_t* bytes) {
  clm_status s = check_sizes(box, n_x, n_y, precision);
  if (s != CLM_OK) return s;
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  clm_celllist tmp;
  std::memset(&tmp, 0, sizeof tmp);
  tmp.box = *box;
  tmp.nx = n_x;
  tmp.ny = n_y;
  tmp.cross = n_y > 0;
  layout(&tmp, nullptr, bytes);
  return CLM_OK;
}

clm_status clm_celllist_create(clm_context* ctx, const clm_box* box, int64_t n_x, int64_t n_y,
                               clm_precision precision, void* ws, size_t ws_bytes,
                               clm_celllist** out) {
  if (!ctx || !out) return fail(CLM_E_INVALID_ARG, "NULL argument");
  clm_status s = check_sizes(box, n_x, n_y, precision);
  if (s != CLM_OK) return s;
  auto* cl = new (std::nothrow) clm_celllist;
  if (!cl) return fail(CLM_E_INVALID_ARG, "out of host memory");
  s = celllist_init(cl, ctx, box, n_x, n_y, precision, ws, ws_bytes);
  if (s != CLM_OK) {
    delete cl;
    return s;
  }
  *out = cl;
  return CLM_OK;
}

}  // extern "C"

clm_status celllist_init(clm_celllist* cl, clm_context* ctx, const clm_box* box, int64_t n_x,
                         int64_t n_y, clm_precision precision, void* ws, size_t ws_bytes) {
  if (!ctx || !cl) return fail(CLM_E_INVALID_ARG, "NULL argument");
  clm_status s = check_sizes(box, n_x, n_y, precision);
  if (s != CLM_OK) return s;
  size_t need = 0;
  clm_celllist_workspace_bytes(box, n_x, n_y, precision, &need);
  if (!ws) return fail(CLM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(CLM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(CLM_E_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
  std::memset(cl, 0, sizeof *cl);
  cl->ctx = ctx;
  cl->box = *box;
  cl->nx = n_x;
  cl->ny = n_y;
  cl->cross = n_y > 0;
  cl->prec = precision;
  cl->ws = (char*)ws;
  cl->ws_bytes = ws_bytes;
  size_t tot = 0;
  layout(cl, (char*)ws, &tot);
  if (!cl->cross) cl->Y = cl->X;
  return CLM_OK;
}

static clm_status build_set(clm_celllist* cl, const double* x, int64_t n, SetBufs& S,
                            const uint32_t* gate) {
  hipStream_t st = cl->ctx->stream;
  const BuildGeom g = geom_of(cl->box);
  const int nc = (int)cl->box.ncells;
  const BinPlan P = bin_plan(nc, n);
  CLM_HIP(launch_bin(x, (int)n, g, nc, P, S.key, S.hist, cl->scan_scratch, S.rec, S.off, S.pos, S.r64,
                     S.idx, S.wrap, st, gate));
  return CLM_OK;
}

clm_status celllist_build_gated(clm_celllist* cl, const double* x, const double* y,
                                const uint32_t* gate) {
  if (!cl) return fail(CLM_E_INVALID_ARG, "cell list is NULL");
  if (cl->nx > 0 && !x) return fail(CLM_E_INVALID_ARG, "x is NULL");
  if (cl->cross && cl->ny > 0 && !y) return fail(CLM_E_INVALID_ARG, "y is NULL for a cross set");
  if (!cl->cross && y) return fail(CLM_E_INVALID_ARG, "y given but the cell list has n_y = 0");
  CLM_HIP(hipSetDevice(cl->ctx->device));
  Timed tb(cl->untimed ? nullptr : cl->ctx, &cl->ctx->build_ev);
  clm_status s = tb.start();
  if (s != CLM_OK) return s;
  s = build_set(cl, x, cl->nx, cl->X, gate);
  if (s != CLM_OK) return s;
  if (cl->cross) {
    s = build_set(cl, y, cl->ny, cl->Y, gate);
    if (s != CLM_OK) return s;
  }
  if (!cl->box.small) {
    TileGeom tg;
    for (int d = 0; d < 3; ++d) tg.n[d] = cl->box.n[d];
    tg.smax = cl->box.smax;
    tg.nrows = cl->nrows;
    tg.job = 0;
    tg.max_tiles = (uint32_t)cl->max_tiles;
    CLM_HIP(launch_tiles(cl->X.off, tg, cl->row_tiles, cl->row_off, cl->scan_scratch, cl->tiles,
                         cl->ctx->stream, gate));
  }
  CLM_HIP(launch_fill_u64(cl->guard, 4, 0ull, cl->ctx->stream, gate));
  s = tb.stop();
  if (s != CLM_OK) return s;
  cl->built = 1;
  return CLM_OK;
}

extern "C" {

clm_status clm_celllist_build(clm_celllist* cl, const double* x, const double* y) {
  return celllist_build_gated(cl, x, y, nullptr);
}

static int internal_kind(clm_map_kind k) {
  switch (k) {
    case CLM_MAP_COUNT: return K_COUNT;
    case CLM_MAP_SUM_D: return K_SUM_D;
    case CLM_MAP_SUM_INV_D: return K_SUM_INV_D;
    case CLM_MAP_LJ_E: return K_LJ_E;
    case CLM_MAP_LJ_EF: return K_LJ_F;
    case CLM_MAP_LJ_ADJOINT: return K_LJ_F;
    case CLM_MAP_HIST_DIST: return K_HIST_DIST;
    case CLM_MAP_HIST_RELSPEED: return K_HIST_REL;
    case CLM_MAP_NEIGHBOR_LIST: return K_NL;
    case CLM_MAP_SUM_W_INV_D: return K_SUM_W;
    case CLM_MAP_HIST_DIST_VEL: return K_HIST_DV;
  }
  return -1;
}

static JobDesc base_job(const clm_celllist* cl) {
  JobDesc jd;
  std::memset(&jd, 0, sizeof jd);
  const clm_box& B = cl->box;
  jd.dim = B.dim;
  jd.lcell = B.lcell;
  jd.lcell_x = B.lcx;
  jd.cross = cl->cross;
  for (int d = 0; d < 3; ++d) jd.n[d] = B.n[d];
  jd.ncells = (int)B.ncells;
  jd.nx = (int)cl->nx;
  jd.ny = (int)(cl->cross ? cl->ny : cl->nx);
  for (int k = 0; k < 9; ++k) jd.H[k] = B.H[k];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) jd.Hn[a * 3 + b] = B.H[a * 3 + b] / (double)B.n[b];
  for (int k = 0; k < 27 * 4; ++k) jd.tK[k] = B.tK[k];
  jd.rc2 = B.rc2;
  jd.band = B.band;
  jd.lo32 = B.lo32;
  jd.hi32 = B.hi32;
  jd.pos_x = cl->X.pos; jd.r64_x = cl->X.r64; jd.idx_x = cl->X.idx; jd.wrap_x = cl->X.wrap;
  jd.off_x = cl->X.off;
  jd.pos_y = cl->Y.pos; jd.r64_y = cl->Y.r64; jd.idx_y = cl->Y.idx; jd.wrap_y = cl->Y.wrap;
  jd.off_y = cl->Y.off;
  jd.vel32_x = cl->X.vel32;
  jd.vel32_y = cl->Y.vel32;
  jd.partials = cl->partials;
  jd.pcount = cl->pcount;
  jd.bandq = cl->bandq;
  jd.E64 = cl->E64;
  jd.E32 = cl->E32;
  jd.nl_counter = cl->nl_counter;
  jd.guard = cl->guard;
  jd.tile_begin = 0;
  jd.tile_end = cl->max_tiles;
  return jd;
}

// Validates one map request, enqueues its per-job preparation kernels
// (histogram edges, zeroed outputs, sorted velocities) and fills the job
// descriptor and finalize arguments.
static clm_status prepare_job(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P,
                              const clm_map_out* O, JobDesc* jdo, FinalArgs* Fo, int* k_launch_out) {
  if (!cl || !P || !O) return fail(CLM_E_INVALID_ARG, "NULL argument");
  if (!cl->built) return fail(CLM_E_INVALID_ARG, "cell list not built");
  const int k = internal_kind(kind);
  if (k < 0) return fail(CLM_E_INVALID_ARG, "unknown map kind %d", (int)kind);
  if (!O->count_dev) return fail(CLM_E_INVALID_ARG, "out->count_dev is required");
  const clm_box& B = cl->box;
  const int dim = B.dim;
  const bool lj = kind == CLM_MAP_LJ_E || kind == CLM_MAP_LJ_EF || kind == CLM_MAP_LJ_ADJOINT;
  const bool ljf = k == K_LJ_F;
  if (lj && (!(P->sigma > 0.0) || !std::isfinite(P->sigma) || !std::isfinite(P->epsilon)))
    return fail(CLM_E_INVALID_ARG, "LJ needs sigma > 0 and finite epsilon");
  if (ljf && cl->cross) return fail(CLM_E_UNSUPPORTED, "LJ forces need a single set");
  if (ljf && !O->forces_dev) return fail(CLM_E_INVALID_ARG, "out->forces_dev is required");
  if (kind == CLM_MAP_LJ_ADJOINT && !P->upstream_dev)
    return fail(CLM_E_INVALID_ARG, "params->upstream_dev is required for LJ_ADJOINT");
  if (ljf && P->want_virial && !O->virial_dev)
    return fail(CLM_E_INVALID_ARG, "want_virial needs out->virial_dev");
  if ((kind == CLM_MAP_SUM_D || kind == CLM_MAP_SUM_INV_D || kind == CLM_MAP_SUM_W_INV_D || lj) &&
      !O->energy_dev)
    return fail(CLM_E_INVALID_ARG, "out->energy_dev is required");
  if (k == K_SUM_W && (!P->weights_x_dev || (cl->cross && !P->weights_y_dev)))
    return fail(CLM_E_INVALID_ARG, "SUM_W_INV_D needs weights_x_dev (and weights_y_dev for a cross set)");
  const bool hist = k == K_HIST_DIST || k == K_HIST_REL || k == K_HIST_DV;
  if (hist) {
    if (P->nbins < 1 || P->nbins > kMaxBins)
      return fail(CLM_E_INVALID_ARG, "nbins must be in 1..%d", kMaxBins);
    if (!(P->hist_hi > 0.0) || !std::isfinite(P->hist_hi))
      return fail(CLM_E_INVALID_ARG, "hist_hi must be finite and > 0");
    if (!O->hist_dev) return fail(CLM_E_INVALID_ARG, "out->hist_dev is required");
  }
  if (k == K_HIST_DV) {
    if (!P->vel_x_dev || (cl->cross && !P->vel_y_dev))
      return fail(CLM_E_INVALID_ARG, "HIST_DIST_VEL needs velocities");
    if (!O->hist_sums_dev) return fail(CLM_E_INVALID_ARG, "HIST_DIST_VEL needs hist_sums_dev");
  }
  if (k == K_HIST_REL) {
    if (!P->vel_x_dev || (cl->cross && !P->vel_y_dev))
      return fail(CLM_E_INVALID_ARG, "relative-speed histogram needs velocities");
    if (P->want_sums && !O->hist_sums_dev) return fail(CLM_E_INVALID_ARG, "want_sums needs hist_sums_dev");
  }
  if (k == K_NL) {
    if (P->capacity < 0) return fail(CLM_E_INVALID_ARG, "capacity must be >= 0");
    if (P->capacity > 0 && !O->pairs_dev) return fail(CLM_E_INVALID_ARG, "pairs_dev is NULL");
    if (P->capacity > 0 && P->with_distances && !O->dist_dev)
      return fail(CLM_E_INVALID_ARG, "with_distances needs dist_dev");
    if (P->sorted && P->capacity > 0 && cl->nx > 0 && (!cl->cross || cl->ny > 0)) {
      clm_status s = sort_pairs_check(cl->nx, cl->cross ? cl->ny : cl->nx, O->pairs_dev, P->capacity,
                                      P->with_distances != 0, P->scratch_dev, P->scratch_bytes);
      if (s != CLM_OK) return s;
    }
  }
  // membership cutoff of this map (the grid stays the box's)
  double rcm = B.rc;
  if (P->cutoff != 0.0) {
    if (!(P->cutoff > 0.0) || !std::isfinite(P->cutoff) || P->cutoff > B.rc)
      return fail(CLM_E_BAD_CUTOFF, "params->cutoff must be in (0, box cutoff %g] (got %g)", B.rc,
                  P->cutoff);
    rcm = P->cutoff;
  }
  hipStream_t st = cl->ctx->stream;
  CLM_HIP(hipSetDevice(cl->ctx->device));

  JobDesc jd = base_job(cl);
  if (rcm != B.rc) {
    jd.rc2 = rcm * rcm;
    map_band(B, rcm, &jd.band, &jd.lo32, &jd.hi32);
  }
  if (ljf) {  // half-shell LJ sweep: thresholds per tile span, in units of sigma^2
    const double s2 = P->sigma * P->sigma;
    for (int sp = 0; sp <= kMaxSpan; ++sp) {
      const double M[3] = {(double)std::max(sp, 1), 1.0, 1.0};
      double bd;
      float lo, hi;
      map_band(B, rcm, &bd, &lo, &hi, M);
      jd.half_lo[sp] = round_down_f((rcm * rcm - bd) / s2);
      jd.half_hi[sp] = round_up_f((rcm * rcm + bd) / s2);
    }
    {
      // FP64 form: the sweep's d^2 (sigma units about the tile's centre)
      // differs from the canonical one by a few roundings of coordinates of
      // at most a few box lengths; a band of 2^-40 (rc + sum of the box's
      // lattice-vector lengths)^2 covers that many times over
      const double ext = rcm + B.sum_len;
      const double bd = std::ldexp(ext * ext, -40);
      jd.half_lo64 = std::nextafter((rcm * rcm - bd) / s2, 0.0);
      jd.half_hi64 = std::nextafter((rcm * rcm + bd) / s2, HUGE_VAL);
    }
    const double nf = P->near_factor > 0.0 ? P->near_factor : 1.0;
    jd.half_near2 = round_up_f(nf * nf);
    jd.half_noprune = P->no_prune ? 1 : 0;
  }
  const int k_launch = (ljf && P->want_virial) ? K_LJ_FV : k;
  jd.kind = k_launch;
  jd.full_shell = ljf ? 1 : 0;
  if (lj) {
    jd.s2 = P->sigma * P->sigma;
    jd.s2f = (float)jd.s2;
    const double nf = P->near_factor > 0.0 ? P->near_factor : 1.0;
    const double near = nf * P->sigma;
    jd.near2f = round_up_f(near * near);
    jd.eps = P->epsilon;
    jd.upstream = kind == CLM_MAP_LJ_ADJOINT ? P->upstream_dev : nullptr;
    jd.scale = kind == CLM_MAP_LJ_EF ? -1.0 : 1.0;
    jd.want_virial = ljf && P->want_virial ? 1 : 0;
    jd.forces = O->forces_dev;
  }
  if (hist) {
    jd.nbins = P->nbins;
    jd.hist_hi = P->hist_hi;
    jd.inv_h = (float)((double)P->nbins / P->hist_hi);
    jd.hist = (unsigned long long*)O->hist_dev;
    jd.hist_sums = O->hist_sums_dev;
    jd.want_sums = ((k == K_HIST_REL && P->want_sums) || k == K_HIST_DV) ? 1 : 0;
    jd.vel64_x = P->vel_x_dev;
    jd.vel64_y = cl->cross ? P->vel_y_dev : P->vel_x_dev;
  }
  if (k == K_NL) {
    jd.pairs = O->pairs_dev;
    jd.dist = P->with_distances ? O->dist_dev : nullptr;
    jd.with_dist = P->with_distances && O->dist_dev ? 1 : 0;
    jd.capacity = P->capacity;
  }
  if (hist) {
    const int force_last = ((k == K_HIST_DIST || k == K_HIST_DV) && P->hist_hi == rcm) ? 1 : 0;
    CLM_HIP(launch_hist_edges(cl->E64, cl->E32, P->nbins, P->hist_hi, force_last, jd.rc2, st));
    CLM_HIP(launch_fill_u64((unsigned long long*)O->hist_dev, (size_t)P->nbins + 1, 0ull, st));
    if (jd.want_sums) CLM_HIP(launch_fill_f64(O->hist_sums_dev, (size_t)P->nbins, 0.0, st));
  }
  if (k == K_HIST_REL) {
    CLM_HIP(launch_fill_u32(cl->vmax_bits, 1, 0u, st));
    CLM_HIP(launch_gather_vel(P->vel_x_dev, dim, cl->X.idx, (int)cl->nx, cl->X.vel32, cl->vmax_bits, st));
    if (cl->cross)
      CLM_HIP(launch_gather_vel(P->vel_y_dev, dim, cl->Y.idx, (int)cl->ny, cl->Y.vel32, cl->vmax_bits, st));
    CLM_HIP(launch_relspeed_band(cl->vmax_bits, P->hist_hi, dim, cl->bandq, st));
  }
  if (k == K_HIST_DV) {
    CLM_HIP(launch_gather_vel(P->vel_x_dev, dim, cl->X.idx, (int)cl->nx, cl->X.vel32, cl->vmax_bits, st));
    if (cl->cross)
      CLM_HIP(launch_gather_vel(P->vel_y_dev, dim, cl->Y.idx, (int)cl->ny, cl->Y.vel32, cl->vmax_bits, st));
  }
  if (k == K_SUM_W) {
    CLM_HIP(launch_gather_weights(P->weights_x_dev, cl->X.idx, (int)cl->nx, cl->X.pos, cl->X.r64, st));
    if (cl->cross)
      CLM_HIP(launch_gather_weights(P->weights_y_dev, cl->Y.idx, (int)cl->ny, cl->Y.pos, cl->Y.r64, st));
  }
  if (k == K_NL) CLM_HIP(launch_fill_u64(cl->nl_counter, 1, 0ull, st));
  CLM_HIP(launch_fill_u64(cl->guard, 4, 0ull, st));

  FinalArgs F;
  std::memset(&F, 0, sizeof F);
  F.kind = k_launch;
  F.dim = dim;
  F.want_virial = jd.want_virial;
  F.eps = lj ? P->epsilon : 0.0;
  F.upstream = jd.upstream;
  F.box_mult = 1.0;
  F.energy = O->energy_dev;
  F.virial = jd.want_virial ? O->virial_dev : nullptr;
  F.grad_box = ljf ? O->grad_box_dev : nullptr;
  F.count = (unsigned long long*)O->count_dev;
  F.halve_count = (ljf && !cl->cross && !B.small) ? 1 : 0;
  *jdo = jd;
  *Fo = F;
  *k_launch_out = k_launch;
  return CLM_OK;
}

clm_status clm_map(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P,
                   const clm_map_out* O) {
  return map_one(cl, kind, P, O, true);
}

// ---------------------------------------------------------------- half-shell LJ scratch
// The automatic choice between the half-shell sweep and the full-shell
// gather.  With at least kHalfMinItems (cell row, neighbour row) items the
// half shell fills the device.  With fewer, both sweeps are bound by their
// longest wave: an item works through the tiles of a row against one
// neighbour row, a gather tile through the (2l+1)^(dim-1) rows of its
// stencil, so the half shell is taken while a row holds no more tiles than
// that (its waves are then no longer, and it evaluates half the pairs).
// Long rows with few items take the gather (a 2D clustered set of 2*10^6
// points, 600 items of 156 tiles a row: 93 against 9 ms; 10^6 particles at
// lcell 1: 4.5 against 3.9 ms), short ones the half shell (10^4 Neon atoms,
// 637 items of 3 tiles a row: 0.12 against 0.58 ms).
static constexpr int kHalfMinItems = 4096;

static bool half_auto(const clm_celllist* cl, int nitems) {
  if (nitems >= kHalfMinItems) return true;
  const int l = cl->box.lcell;
  const int reach = cl->box.dim == 3 ? (2 * l + 1) * (2 * l + 1) : 2 * l + 1;
  const double tiles_per_row = (double)cl->nx / ((double)kTileMax * std::max(cl->nrows, 1));
  return tiles_per_row <= (double)reach;
}

static bool half_applies(const clm_celllist* cl, int k) {
  return k == K_LJ_F && !cl->box.small && !cl->cross && cl->nx > 0;
}

struct HalfLayout {
  int NR, nitems, ngather;
  size_t npad, o_part, o_parts, o_pc, o_boxes, total;
};

static HalfLayout half_layout(const clm_celllist* cl) {
  HalfLayout L;
  L.NR = half_rows(cl->box.dim, cl->box.lcell);
  L.nitems = cl->nrows * L.NR;
  L.ngather = (int)((cl->nx + 255) / 256);
  L.npad = (size_t)((cl->nx + 63) / 64) * 64;
  Carve c;
  const size_t esz = cl->prec == CLM_FP64 ? sizeof(double) : sizeof(float);
  L.o_part = c.take(esz * 3 * (size_t)L.NR * 3 * L.npad);
  L.o_parts = c.take(sizeof(double) * kPartialD * (size_t)(L.nitems + L.ngather));
  L.o_pc = c.take(sizeof(unsigned long long) * (size_t)(L.nitems + L.ngather));
  L.o_boxes = c.take(sizeof(double) * 12 * (size_t)std::max<int64_t>(cl->max_tiles, 1));
  L.total = c.off;
  return L;
}

// Launch order of the half-shell row offsets, by the distance between the
// cross-sections (perpendicular to the rows) of the home row's cell and the
// neighbour row's: the closest rows hold the most candidates within the
// cutoff of a tile, so their items start first.  The home row (about half of
// an adjacent row's work) comes after the adjacent rows.
static void half_rho_order(const clm_box& B, int NR, uint8_t* order) {
  const int dim = B.dim, l = B.lcell;
  std::vector<double> key(NR, 0.0);
  // the lattice vectors a1 (along the rows), a2 / ny, a3 / nz
  double a1[3], u[3], v[3];
  for (int r = 0; r < 3; ++r) {
    a1[r] = B.H[r * 3 + 0];
    u[r] = dim > 1 ? B.H[r * 3 + 1] / B.n[1] : 0.0;
    v[r] = dim > 2 ? B.H[r * 3 + 2] / B.n[2] : 0.0;
  }
  const double a1n = std::sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
  auto perp = [&](const double* p, double* q) {  // component perpendicular to a1
    const double t = (p[0] * a1[0] + p[1] * a1[1] + p[2] * a1[2]) / (a1n * a1n);
    for (int r = 0; r < 3; ++r) q[r] = p[r] - t * a1[r];
  };
  double pu[3], pv[3];
  perp(u, pu);
  perp(v, pv);
  auto norm = [](const double* p) { return std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]); };
  for (int rho = 1; rho < NR; ++rho) {
    int dy, dz;
    if (rho <= l) { dy = rho; dz = 0; }
    else { const int q = rho - l - 1; dz = 1 + q / (2 * l + 1); dy = q % (2 * l + 1) - l; }
    // distance from 0 to {(dy + s) pu + (dz + t) pv : |s|, |t| <= 1}: the
    // smallest over a grid of the parallelogram's points (close enough for
    // an ordering)
    double best = 1e300;
    for (int i = 0; i <= 32; ++i)
      for (int j = 0; j <= (dim > 2 ? 32 : 0); ++j) {
        const double s = dy - 1.0 + i / 16.0, t = dim > 2 ? dz - 1.0 + j / 16.0 : 0.0;
        double p[3];
        for (int r = 0; r < 3; ++r) p[r] = s * pu[r] + t * pv[r];
        best = std::min(best, norm(p));
      }
    key[rho] = best;
  }
  std::vector<int> ix(NR);
  for (int r = 0; r < NR; ++r) ix[r] = r;
  // home row: after every row at distance 0
  std::stable_sort(ix.begin(), ix.end(), [&](int a, int b) {
    const double ka = a == 0 ? 1e-300 : key[a], kb = b == 0 ? 1e-300 : key[b];
    return ka < kb;
  });
  for (int r = 0; r < NR; ++r) order[r] = (uint8_t)ix[r];
}

clm_status clm_map_scratch_bytes(const clm_celllist* cl, clm_map_kind kind, size_t* bytes) {
  if (!cl || !bytes) return fail(CLM_E_INVALID_ARG, "NULL argument");
  const int k = internal_kind(kind);
  if (k < 0) return fail(CLM_E_INVALID_ARG, "unknown map kind %d", (int)kind);
  *bytes = half_applies(cl, k) ? half_layout(cl).total : 0;
  return CLM_OK;
}

}  // extern "C"

// Neighbour lists after the map: the device sort into canonical order
// (params->sorted), then the synchronous capacity check (params->check_capacity).
static clm_status nl_sort_after(clm_celllist* cl, const clm_map_params* P, const clm_map_out* O) {
  if (!P->sorted || P->capacity == 0 || cl->nx == 0 || (cl->cross && cl->ny == 0)) return CLM_OK;
  return sort_pairs(cl->ctx->stream, cl->nx, cl->cross ? cl->ny : cl->nx, O->pairs_dev,
                    P->with_distances ? O->dist_dev : nullptr, (const unsigned long long*)O->count_dev,
                    P->capacity, P->scratch_dev);
}

static clm_status nl_capacity_after(clm_celllist* cl, const clm_map_params* P, const clm_map_out* O) {
  if (!P->check_capacity) return CLM_OK;
  uint64_t c = 0;
  hipStream_t st = cl->ctx->stream;
  CLM_HIP(hipMemcpyAsync(&c, O->count_dev, sizeof c, hipMemcpyDeviceToHost, st));
  CLM_HIP(hipStreamSynchronize(st));
  if (c > (uint64_t)P->capacity)
    return fail(CLM_E_CAPACITY, "the neighbour list has %llu pairs and capacity %lld: only the first "
                "capacity pairs were written (count_dev holds the total)", (unsigned long long)c,
                (long long)P->capacity);
  return CLM_OK;
}

static clm_status map_one_inner(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P,
                                const clm_map_out* O, bool nl_two_pass_ok);

clm_status map_one(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P, const clm_map_out* O,
                   bool nl_two_pass_ok) {
  clm_status s = map_one_inner(cl, kind, P, O, nl_two_pass_ok);
  if (s != CLM_OK || kind != CLM_MAP_NEIGHBOR_LIST) return s;
  s = nl_sort_after(cl, P, O);
  if (s != CLM_OK) return s;
  return nl_capacity_after(cl, P, O);
}

static clm_status map_one_inner(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P,
                                const clm_map_out* O, bool nl_two_pass_ok) {
  // a map scratch given for the half-shell sweep is checked whether or not
  // the sweep is chosen, before any launch
  const bool half_ok = P && half_applies(cl, internal_kind(kind)) && P->scratch_dev && P->half_shell >= 0;
  if (half_ok) {
    const HalfLayout HL = half_layout(cl);
    if (((uintptr_t)P->scratch_dev & 255) != 0)
      return fail(CLM_E_WORKSPACE, "map scratch must be 256-byte aligned");
    if (P->scratch_bytes < HL.total)
      return fail(CLM_E_WORKSPACE, "map scratch too small: %zu bytes given, %zu needed", P->scratch_bytes,
                  HL.total);
  }
  JobDesc jd;
  FinalArgs F;
  int k_launch = 0;
  clm_status s = prepare_job(cl, kind, P, O, &jd, &F, &k_launch);
  if (s != CLM_OK) return s;
  const clm_box& B = cl->box;
  hipStream_t st = cl->ctx->stream;
  if (half_ok && (P->half_shell > 0 || half_auto(cl, half_layout(cl).nitems))) {
    // half-shell LJ sweep: every pair once, force planes in the map scratch
    const HalfLayout HL = half_layout(cl);
    char* base = (char*)P->scratch_dev;
    HalfArgs A;
    A.part = (void*)(base + HL.o_part);
    A.npad = HL.npad;
    A.partials = (double*)(base + HL.o_parts);
    A.pcount = (unsigned long long*)(base + HL.o_pc);
    A.row_off = cl->row_off;
    A.tiles = cl->tiles;
    A.boxes = (double*)(base + HL.o_boxes);
    A.max_tiles = cl->max_tiles;
    A.nitems = HL.nitems;
    A.NR = HL.NR;
    half_rho_order(B, HL.NR, A.rho_order);
    jd.partials = A.partials;  // the finalize reads the item and gather partials
    jd.pcount = A.pcount;
    CLM_HIP(launch_set_job(jd, cl->job_dev, st));
    const bool fp64 = cl->prec == CLM_FP64;
    CLM_HIP(launch_half_boxes(cl->job_dev, A, st));
    // the sweep's timed region holds the sweep kernel alone
    Timed ts(cl->untimed ? nullptr : cl->ctx, &cl->ctx->sweep_ev);
    s = ts.start();
    if (s != CLM_OK) return s;
    CLM_HIP(launch_half_lj(B.dim, k_launch == K_LJ_FV, fp64, cl->job_dev, A, st));
    s = ts.stop();
    if (s != CLM_OK) return s;
    CLM_HIP(launch_half_gather(B.dim, fp64, cl->job_dev, A, (int)cl->nx, st));
    F.nparts = HL.nitems + HL.ngather;
    F.nparts_dev = nullptr;
    F.split_rows = 0;
    F.halve_count = 0;
    CLM_HIP(launch_finalize(cl->job_dev, F, cl->fin_scratch, cl->fin_count, st));
    return CLM_OK;
  }
  // neighbour lists: a counting sweep gives every work item its output
  // offset, so the list sweep writes without a shared counter
  const bool nl_two_pass = nl_two_pass_ok && k_launch == K_NL && !B.small;
  if (nl_two_pass) jd.nl_offsets = cl->nl_off;
  CLM_HIP(launch_set_job(jd, cl->job_dev, st));
  Timed ts(cl->untimed ? nullptr : cl->ctx, &cl->ctx->sweep_ev);
  s = ts.start();
  if (s != CLM_OK) return s;
  if (B.small) {
    BruteArgs A;
    std::memset(&A, 0, sizeof A);
    A.dim = B.dim;
    A.n_x = (int)cl->nx;
    A.n_y = (int)(cl->cross ? cl->ny : cl->nx);
    A.cross = cl->cross;
    A.kind = internal_kind(kind);
    for (int q = 0; q < 9; ++q) {
      A.H[q] = B.H[q];
      A.Hinv[q] = B.Hinv[q];
    }
    for (int d = 0; d < 3; ++d) A.w[d] = B.w[d];
    A.rc = P->cutoff != 0.0 ? P->cutoff : B.rc;
    A.rc2 = A.rc * A.rc;
    A.reach = std::min(A.rc, 0.5 * B.sum_len) * (1.0 + 1e-6);
    const double pairs = (double)A.n_x * (double)(cl->cross ? A.n_y : A.n_x);
    if (pairs > 4.0e9)
      return fail(CLM_E_UNSUPPORTED,
                  "box has fewer than 3 cells per axis and %.3g candidate pairs: the brute-force "
                  "minimum-image path serves at most 4e9", pairs);
    int nblocks = 0;
    CLM_HIP(launch_brute(cl->job_dev, A, cl->brute_fb, &nblocks, st));
    F.nparts = nblocks;
    F.nparts_dev = nullptr;
  } else {
    const bool hist = k_launch == K_HIST_DIST || k_launch == K_HIST_REL || k_launch == K_HIST_DV;
    const int split = sweep_split_rows(k_launch, B.dim, B.lcell, jd.full_shell || cl->cross);
    if (nl_two_pass) {
      CLM_HIP(launch_sweep(B.dim, cl->prec == CLM_FP32_GUARD, K_COUNT, cl->job_dev, cl->tiles,
                           &cl->row_off[cl->nrows], cl->max_tiles, 0, st, split));
      CLM_HIP(launch_nl_offsets(cl->pcount, &cl->row_off[cl->nrows], cl->max_tiles, split, cl->nl_off, st));
      CLM_HIP(launch_fill_u64(cl->guard, 4, 0ull, st));  // count the list pass's re-tests only
    }
    CLM_HIP(launch_sweep(B.dim, cl->prec == CLM_FP32_GUARD, k_launch, cl->job_dev, cl->tiles,
                         &cl->row_off[cl->nrows], cl->max_tiles, hist ? P->nbins : 0, st, split));
    F.nparts = cl->max_tiles;
    F.nparts_dev = &cl->row_off[cl->nrows];
    F.split_rows = split;
  }
  s = ts.stop();
  if (s != CLM_OK) return s;
  CLM_HIP(launch_finalize(cl->job_dev, F, cl->fin_scratch, cl->fin_count, st));
  return CLM_OK;
}

extern "C" {

// ---------------------------------------------------------------- batched maps
static size_t batch_layout(int njobs, int64_t tiles, size_t* o_jobs, size_t* o_fin, size_t* o_tiles,
                           size_t* o_total) {
  Carve c;
  *o_jobs = c.take(sizeof(JobDesc) * njobs);
  *o_fin = c.take(sizeof(FinalArgs) * njobs);
  *o_tiles = c.take(sizeof(Tile) * (size_t)std::max<int64_t>(tiles, 4));
  *o_total = c.take(sizeof(uint32_t) * 4);
  return c.off;
}

static int64_t batch_tiles(int njobs, clm_celllist* const* cls) {
  int64_t t = 0;
  for (int k = 0; k < njobs; ++k)
    if (cls[k] && !cls[k]->box.small) t += cls[k]->max_tiles;
  return (t + 3) & ~(int64_t)3;
}

clm_status clm_map_batch_workspace_bytes(int njobs, clm_celllist* const* cls, size_t* bytes) {
  if (njobs < 1 || njobs > 4096 || !cls || !bytes)
    return fail(CLM_E_INVALID_ARG, "njobs must be in 1..4096 with non-NULL arrays");
  size_t a, b, c, d;
  *bytes = batch_layout(njobs, batch_tiles(njobs, cls), &a, &b, &c, &d);
  return CLM_OK;
}

clm_status clm_map_batch(int njobs, clm_celllist* const* cls, clm_map_kind kind,
                         const clm_map_params* P, const clm_map_out* O, void* ws, size_t ws_bytes) {
  if (njobs < 1 || njobs > 4096 || !cls || !P || !O)
    return fail(CLM_E_INVALID_ARG, "njobs must be in 1..4096 with non-NULL arrays");
  for (int k = 0; k < njobs; ++k)
    if (!cls[k]) return fail(CLM_E_INVALID_ARG, "cell list %d is NULL", k);
  clm_context* ctx = cls[0]->ctx;
  const int dim = cls[0]->box.dim;
  const clm_precision prec = cls[0]->prec;
  for (int k = 1; k < njobs; ++k) {
    if (cls[k]->ctx != ctx) return fail(CLM_E_INVALID_ARG, "all cell lists must share one context");
    if (cls[k]->box.dim != dim || cls[k]->prec != prec)
      return fail(CLM_E_INVALID_ARG, "all cell lists of a batch need the same dim and precision");
    if ((kind == CLM_MAP_HIST_DIST || kind == CLM_MAP_HIST_RELSPEED || kind == CLM_MAP_HIST_DIST_VEL) &&
        P[k].nbins != P[0].nbins)
      return fail(CLM_E_INVALID_ARG, "all histograms of a batch need the same nbins");
  }
  size_t need = 0, o_jobs, o_fin, o_tiles, o_total;
  need = batch_layout(njobs, batch_tiles(njobs, cls), &o_jobs, &o_fin, &o_tiles, &o_total);
  if (!ws || ((uintptr_t)ws & 255) != 0 || ws_bytes < need)
    return fail(CLM_E_WORKSPACE, "batch workspace: %zu bytes (256-aligned) needed, %zu given", need,
                ws_bytes);
  char* base = (char*)ws;
  JobDesc* jobs_dev = (JobDesc*)(base + o_jobs);
  FinalArgs* fin_dev = (FinalArgs*)(base + o_fin);
  Tile* tiles_dev = (Tile*)(base + o_tiles);
  uint32_t* total_dev = (uint32_t*)(base + o_total);
  std::vector<JobDesc> jds;
  std::vector<FinalArgs> fas;
  std::vector<clm_celllist*> bcl;  // the batched (not small-box) jobs' cell lists
  jds.reserve(njobs);
  fas.reserve(njobs);
  bcl.reserve(njobs);
  int k_launch = -1, nbins = 0;
  for (int k = 0; k < njobs; ++k) {
    if (cls[k]->box.small) {  // brute-force minimum image: a job of its own
      clm_status s = clm_map(cls[k], kind, &P[k], &O[k]);
      if (s != CLM_OK) return s;
      continue;
    }
    JobDesc jd;
    FinalArgs F;
    int kl = 0;
    clm_status s = prepare_job(cls[k], kind, &P[k], &O[k], &jd, &F, &kl);
    if (s != CLM_OK) return s;
    if (k_launch >= 0 && kl != k_launch)
      return fail(CLM_E_INVALID_ARG, "all jobs of a batch must launch the same map (virial flags differ)");
    k_launch = kl;
    nbins = jd.nbins;
    if (kl == K_NL) jd.nl_offsets = cls[k]->nl_off;  // two passes, as in clm_map
    bcl.push_back(cls[k]);
    jd.own_tiles = cls[k]->tiles;
    jd.own_ntiles = &cls[k]->row_off[cls[k]->nrows];
    jd.own_max_tiles = cls[k]->max_tiles;
    jds.push_back(jd);
    fas.push_back(F);
  }
  if (jds.empty()) return CLM_OK;
  const int nb = (int)jds.size();
  hipStream_t st = ctx->stream;
  CLM_HIP(hipSetDevice(ctx->device));
  // pageable host -> device: the runtime stages the data before returning
  CLM_HIP(hipMemcpyAsync(jobs_dev, jds.data(), sizeof(JobDesc) * nb, hipMemcpyHostToDevice, st));
  CLM_HIP(hipMemcpyAsync(fin_dev, fas.data(), sizeof(FinalArgs) * nb, hipMemcpyHostToDevice, st));
  CLM_HIP(launch_gather_tiles(jobs_dev, nb, tiles_dev, total_dev, st));
  int64_t maxt = 0;
  for (const JobDesc& jd : jds) maxt += jd.own_max_tiles;
  maxt = (maxt + 3) & ~(int64_t)3;
  Timed ts(ctx, &ctx->sweep_ev);
  clm_status s = ts.start();
  if (s != CLM_OK) return s;
  if (k_launch == K_NL) {  // counting sweep, then each job's per-tile output offsets
    CLM_HIP(launch_sweep(dim, prec == CLM_FP32_GUARD, K_COUNT, jobs_dev, tiles_dev, total_dev,
                         (int)std::min<int64_t>(maxt, INT32_MAX), 0, st));
    for (clm_celllist* c : bcl) {
      CLM_HIP(launch_nl_offsets(c->pcount, &c->row_off[c->nrows], c->max_tiles, 1, c->nl_off, st));
      CLM_HIP(launch_fill_u64(c->guard, 4, 0ull, st));
    }
  }
  CLM_HIP(launch_sweep(dim, prec == CLM_FP32_GUARD, k_launch, jobs_dev, tiles_dev, total_dev,
                       (int)std::min<int64_t>(maxt, INT32_MAX), nbins, st));
  s = ts.stop();
  if (s != CLM_OK) return s;
  CLM_HIP(launch_finalize_batch(jobs_dev, fin_dev, nb, st));
  if (kind == CLM_MAP_NEIGHBOR_LIST) {  // small-box jobs were finished by clm_map above
    for (int k = 0; k < njobs; ++k) {
      if (cls[k]->box.small) continue;
      clm_status s = nl_sort_after(cls[k], &P[k], &O[k]);
      if (s != CLM_OK) return s;
    }
    for (int k = 0; k < njobs; ++k) {
      if (cls[k]->box.small) continue;
      clm_status s = nl_capacity_after(cls[k], &P[k], &O[k]);
      if (s != CLM_OK) return s;
    }
  }
  return CLM_OK;
}

clm_status clm_celllist_info_get(clm_celllist* cl, clm_celllist_info* o) {
  if (!cl || !o) return fail(CLM_E_INVALID_ARG, "NULL argument");
  if (!cl->built) return fail(CLM_E_INVALID_ARG, "cell list not built");
  std::memset(o, 0, sizeof *o);
  hipStream_t st = cl->ctx->stream;
  CLM_HIP(hipSetDevice(cl->ctx->device));
  o->n_x = cl->nx;
  o->n_y = cl->ny;
  o->ncells = cl->box.ncells;
  const int nc = (int)cl->box.ncells;
  uint32_t* hoff = new (std::nothrow) uint32_t[nc + 1];
  if (!hoff) return fail(CLM_E_INVALID_ARG, "out of host memory");
  CLM_HIP(hipMemcpyAsync(hoff, cl->X.off, sizeof(uint32_t) * (nc + 1), hipMemcpyDeviceToHost, st));
  CLM_HIP(hipStreamSynchronize(st));
  int64_t ne = 0, mo = 0;
  for (int c = 0; c < nc; ++c) {
    int64_t m = hoff[c + 1] - hoff[c];
    ne += m > 0;
    mo = std::max(mo, m);
  }
  if (cl->cross) {
    CLM_HIP(hipMemcpyAsync(hoff, cl->Y.off, sizeof(uint32_t) * (nc + 1), hipMemcpyDeviceToHost, st));
    CLM_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < nc; ++c) mo = std::max<int64_t>(mo, hoff[c + 1] - hoff[c]);
  }
  delete[] hoff;
  o->nonempty_cells = ne;
  o->max_occupancy = mo;
  {
    unsigned long long g[4] = {0, 0, 0, 0};
    CLM_HIP(hipMemcpyAsync(g, cl->guard, sizeof g, hipMemcpyDeviceToHost, st));
    CLM_HIP(hipStreamSynchronize(st));
    o->guard_retests = (int64_t)g[0];
    o->near_evaluations = (int64_t)g[1];
    o->half_pairs_tested = (int64_t)g[2];
    o->half_pairs_kept = (int64_t)g[3];
  }
  if (cl->box.small) {
    o->ntiles = 0;
    o->candidate_pairs = cl->cross ? cl->nx * cl->ny : cl->nx * (cl->nx - 1) / 2;
    return CLM_OK;
  }
  uint32_t nt = 0;
  CLM_HIP(hipMemcpyAsync(&nt, &cl->row_off[cl->nrows], sizeof nt, hipMemcpyDeviceToHost, st));
  CLM_HIP(hipStreamSynchronize(st));
  if ((int64_t)nt > cl->max_tiles)
    return fail(CLM_E_DEVICE, "internal: %u tiles exceed the bound %d", nt, cl->max_tiles);
  o->ntiles = nt;
  // candidates: the grid's half-shell cell pairs (full stencil for cross sets)
  JobDesc jd = base_job(cl);
  CLM_HIP(launch_set_job(jd, cl->job_dev, st));
  CLM_HIP(launch_candidates(cl->job_dev, (int)cl->box.ncells, 0, cl->cand, st));
  unsigned long long tot = 0;
  CLM_HIP(hipMemcpyAsync(&tot, cl->cand, sizeof tot, hipMemcpyDeviceToHost, st));
  CLM_HIP(hipStreamSynchronize(st));
  o->candidate_pairs = (int64_t)tot;
  return CLM_OK;
}

clm_status clm_celllist_destroy(clm_celllist* cl) {
  delete cl;
  return CLM_OK;
}

clm_status clm_synchronize(clm_context* ctx) {
  if (!ctx) return fail(CLM_E_INVALID_ARG, "ctx is NULL");
  CLM_HIP(hipSetDevice(ctx->device));
  CLM_HIP(hipStreamSynchronize(ctx->stream));
  return CLM_OK;
}

}  // extern "C"
