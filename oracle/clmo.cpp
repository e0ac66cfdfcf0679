/*
 * clmo.cpp -- plain FP64 CPU oracle (test infrastructure only; see clmo.h).
 *
 * Two independent enumerations of the same pair set:
 *   - brute force over all pairs with an explicit minimum-image search;
 *   - a plain cell list (cells of side >= rc in fractional space, the full
 *     3x3(x3) neighbourhood of every cell, an i<j test), paper section 2.8.
 * No half shell, no LDS, no guard bands, no reduced precision.  Sums use
 * Neumaier compensation per home cell (or per particle for brute force) and
 * are combined in a fixed order, so results do not depend on thread count.
 *
 * Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math
 *        -shared -fPIC clmo.cpp -o liboracle.so
 */
#include "clmo.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

namespace {

/* Neumaier's improvement of Kahan summation. */
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

struct Box {
  int dim = 3;
  double H[9] = {0};   /* row-major dim x dim (stride dim) */
  double Hi[9] = {0};
  double w[3] = {0};   /* perpendicular widths */
  double V = 0;
  double rc = 0, rc2 = 0;
  double h(int a, int b) const { return H[a * dim + b]; }
  double hi(int a, int b) const { return Hi[a * dim + b]; }
};

int inverse(int dim, const double* H, double* Hi) {
  if (dim == 2) {
    double det = H[0] * H[3] - H[1] * H[2];
    if (!(det > 0.0) || !std::isfinite(det)) return CLMO_EINVAL;
    Hi[0] = H[3] / det;
    Hi[1] = -H[1] / det;
    Hi[2] = -H[2] / det;
    Hi[3] = H[0] / det;
    return CLMO_OK;
  }
  const double H00 = H[0], H01 = H[1], H02 = H[2];
  const double H10 = H[3], H11 = H[4], H12 = H[5];
  const double H20 = H[6], H21 = H[7], H22 = H[8];
  double C00 = H11 * H22 - H12 * H21, C01 = H12 * H20 - H10 * H22;
  double C02 = H10 * H21 - H11 * H20, C10 = H02 * H21 - H01 * H22;
  double C11 = H00 * H22 - H02 * H20, C12 = H01 * H20 - H00 * H21;
  double C20 = H01 * H12 - H02 * H11, C21 = H02 * H10 - H00 * H12;
  double C22 = H00 * H11 - H01 * H10;
  double det = (H00 * C00 + H01 * C01) + H02 * C02;
  if (!(det > 0.0) || !std::isfinite(det)) return CLMO_EINVAL;
  /* Hinv_ab = C_ba / det */
  Hi[0] = C00 / det; Hi[1] = C10 / det; Hi[2] = C20 / det;
  Hi[3] = C01 / det; Hi[4] = C11 / det; Hi[5] = C21 / det;
  Hi[6] = C02 / det; Hi[7] = C12 / det; Hi[8] = C22 / det;
  return CLMO_OK;
}

void cross3(const double* u, const double* v, double* out) {
  out[0] = u[1] * v[2] - u[2] * v[1];
  out[1] = u[2] * v[0] - u[0] * v[2];
  out[2] = u[0] * v[1] - u[1] * v[0];
}

int widths(int dim, const double* H, double* w, double* V) {
  if (dim == 2) {
    double A = std::fabs(H[0] * H[3] - H[1] * H[2]);
    double la = std::sqrt(H[0] * H[0] + H[2] * H[2]);  /* column 0 */
    double lb = std::sqrt(H[1] * H[1] + H[3] * H[3]);  /* column 1 */
    w[0] = A / lb;
    w[1] = A / la;
    *V = A;
    return CLMO_OK;
  }
  double col[3][3];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) col[b][a] = H[a * 3 + b];
  double bc[3], ca[3], ab[3];
  cross3(col[1], col[2], bc);
  cross3(col[2], col[0], ca);
  cross3(col[0], col[1], ab);
  double vol = std::fabs(col[0][0] * bc[0] + col[0][1] * bc[1] + col[0][2] * bc[2]);
  auto norm = [](const double* u) { return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); };
  w[0] = vol / norm(bc);
  w[1] = vol / norm(ca);
  w[2] = vol / norm(ab);
  *V = vol;
  return CLMO_OK;
}

int make_box(int dim, const double* H, double cutoff, Box* B) {
  if (dim != 2 && dim != 3) return CLMO_EINVAL;
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return CLMO_EINVAL;
  B->dim = dim;
  for (int k = 0; k < dim * dim; ++k) {
    if (!std::isfinite(H[k])) return CLMO_EINVAL;
    B->H[k] = H[k];
  }
  if (inverse(dim, H, B->Hi) != CLMO_OK) return CLMO_EINVAL;
  widths(dim, H, B->w, &B->V);
  B->rc = cutoff;
  B->rc2 = cutoff * cutoff;
  return CLMO_OK;
}

/* Canonical wrap of one position. */
void wrap_one(const Box& B, const double* r, double* rw, double* f, int64_t* w) {
  const int dim = B.dim;
  double s[3], fr[3];
  for (int a = 0; a < dim; ++a) {
    double acc = B.hi(a, 0) * r[0];
    for (int b = 1; b < dim; ++b) acc = acc + B.hi(a, b) * r[b];
    s[a] = acc;
  }
  for (int a = 0; a < dim; ++a) {
    double fl = std::floor(s[a]);
    double fa = s[a] - fl;
    if (fa >= 1.0) {
      fa = 0.0;
      fl = fl + 1.0;
    }
    fr[a] = fa;
    if (f) f[a] = fa;
    if (w) w[a] = (int64_t)fl;
  }
  for (int a = 0; a < dim; ++a) {
    double acc = B.h(a, 0) * fr[0];
    for (int b = 1; b < dim; ++b) acc = acc + B.h(a, b) * fr[b];
    rw[a] = acc;
  }
}

/* Frame position of one particle for given integers w'': f = s - w''. */
void frame_one(const Box& B, const double* r, const int64_t* wf, double* rw, double* f) {
  const int dim = B.dim;
  double s[3];
  for (int a = 0; a < dim; ++a) {
    double acc = B.hi(a, 0) * r[0];
    for (int b = 1; b < dim; ++b) acc = acc + B.hi(a, b) * r[b];
    s[a] = acc;
  }
  for (int a = 0; a < dim; ++a) f[a] = s[a] - (double)wf[a];
  for (int a = 0; a < dim; ++a) {
    double acc = B.h(a, 0) * f[0];
    for (int b = 1; b < dim; ++b) acc = acc + B.h(a, b) * f[b];
    rw[a] = acc;
  }
}

/* t = H K (canonical order). */
void shift(const Box& B, const int* K, double* t) {
  for (int a = 0; a < B.dim; ++a) {
    double acc = B.h(a, 0) * (double)K[0];
    for (int b = 1; b < B.dim; ++b) acc = acc + B.h(a, b) * (double)K[b];
    t[a] = acc;
  }
}

/* Canonical displacement and squared distance (wrapped positions). */
double pair_d2(const Box& B, const double* ri, const double* rj, const double* t, double* D) {
  for (int a = 0; a < B.dim; ++a) D[a] = (rj[a] - ri[a]) + t[a];
  double d2 = D[0] * D[0] + D[1] * D[1];
  if (B.dim == 3) d2 = d2 + D[2] * D[2];
  return d2;
}

/* Brute-force minimum image of a wrapped pair among every image K whose
 * distance could be <= reach.  Geometric fact used to bound the search:
 * for image K, the component of D along the unit normal of the face pair d
 * has length |fs_d + K_d| * w_d, where fs = f_j - f_i; so |D| <= reach
 * requires |fs_d + K_d| <= reach / w_d.  A relative slack of 1e-6 covers
 * rounding.  Returns +inf when no image is within reach. */
double min_image(const Box& B, const double* ri, const double* fi, const double* rj,
                 const double* fj, double reach, double* Dbest, int* Kbest) {
  const int dim = B.dim;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    double fs = fj[d] - fi[d];
    double R = reach / B.w[d] * (1.0 + 1e-6) + 1e-12;
    lo[d] = (int)std::ceil(-fs - R);
    hi[d] = (int)std::floor(-fs + R);
  }
  double best = std::numeric_limits<double>::infinity();
  int K[3] = {0, 0, 0};
  double t[3], D[3];
  for (K[0] = lo[0]; K[0] <= hi[0]; ++K[0])
    for (K[1] = lo[1]; K[1] <= hi[1]; ++K[1])
      for (K[2] = (dim == 3 ? lo[2] : 0); K[2] <= (dim == 3 ? hi[2] : 0); ++K[2]) {
        shift(B, K, t);
        double d2 = pair_d2(B, ri, rj, t, D);
        /* strict '<' keeps the lexicographically smallest K on ties */
        if (d2 < best) {
          best = d2;
          for (int a = 0; a < dim; ++a) {
            Dbest[a] = D[a];
            Kbest[a] = K[a];
          }
        }
      }
  return best;
}

/* Histogram edges E_k (k = 0..nb), per the definitions in clmo.h. */
std::vector<double> edges(int nb, double hi, bool force_last, double rc2) {
  std::vector<double> E(nb + 1);
  double h = hi / (double)nb;
  for (int k = 0; k <= nb; ++k) {
    double e = (double)k * h;
    E[k] = e * e;
  }
  if (force_last) E[nb] = rc2;
  return E;
}

/* First m in [0, nb] with v <= E_m; bin = max(m-1, 0); overflow = nb. */
int bin_of(const std::vector<double>& E, double v) {
  int nb = (int)E.size() - 1;
  if (!(v <= E[nb])) return nb;
  int lo = 0, hi = nb; /* invariant: v <= E[hi] */
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (v <= E[mid])
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo == 0 ? 0 : lo - 1;
}

struct Pair {
  int64_t i, j;
  double d, d2;
};

/* Per-home-cell (or per-particle) partial results. */
struct Partial {
  uint64_t count = 0;
  Neumaier sum_d, sum_inv_d, lj, sum_w;
  Neumaier vir[9], dEdH[9];
};

struct Ctx {
  const Box* B;
  const clmo_request* req;
  bool cross;
  int64_t nx, ny;
  std::vector<double> xw, fx, yw, fy;   /* wrapped positions and fractions */
  std::vector<int64_t> wx, wy;          /* wrap integers (the frame's, when one is given) */
  std::vector<double> cfx;              /* canonical fractions (cell membership) */
  std::vector<int64_t> dwx;             /* canonical minus frame integers */
  const double* vx = nullptr;
  const double* vy = nullptr;
  std::vector<double> Ehist, Erel;
  /* per-thread integer and list outputs (order-independent or sorted) */
  std::vector<std::vector<uint64_t>> hist_t, rel_t, dv_t;
  std::vector<double> Edv;
  int nrel = 0;                         /* per-unit sums: [0, nrel) relative speed, then distance bins */
  std::vector<std::vector<Pair>> nl_t;
};

/* Accumulate one unordered within-cutoff pair (i from x, j from x or y),
 * with displacement D (j minus i) for image K of the wrapped positions. */
void accumulate(Ctx& C, Partial& P, std::vector<Neumaier>& rel_sum, int tid, int64_t i,
                int64_t j, double d2, const double* D, const int* K) {
  const clmo_request& q = *C.req;
  const int dim = C.B->dim;
  const int want = q.want;
  P.count += 1;
  if (want & (CLMO_W_SUM_D | CLMO_W_SUM_INV_D | CLMO_W_NL)) {
    double d = std::sqrt(d2);
    if (want & CLMO_W_SUM_D) P.sum_d.add(d);
    if (want & CLMO_W_SUM_INV_D) P.sum_inv_d.add(1.0 / d);
    if (want & CLMO_W_NL) C.nl_t[tid].push_back(Pair{i, j, d, d2});
  }
  if (want & CLMO_W_SUM_W_INV_D) {
    /* Code 5, second example: m_i m_j / d */
    const double wi = q.weights_x[i];
    const double wj = C.cross ? q.weights_y[j] : q.weights_x[j];
    P.sum_w.add((wi * wj) / std::sqrt(d2));
  }
  if (want & CLMO_W_LJ) {
    double x = (q.sigma * q.sigma) / d2;
    double x3 = x * x * x;
    double u = 4.0 * q.epsilon * (x3 * x3 - x3);
    double fs = 24.0 * q.epsilon * (2.0 * x3 * x3 - x3) / d2;
    P.lj.add(u);
    /* image in terms of the raw positions: K + w_i - w_j */
    const int64_t* wi = &C.wx[i * dim];
    const int64_t* wj = C.cross ? &C.wy[j * dim] : &C.wx[j * dim];
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b) {
        P.vir[a * dim + b].add(fs * D[a] * D[b]);
        double Ko = (double)((int64_t)K[b] + wi[b] - wj[b]);
        P.dEdH[a * dim + b].add(-fs * D[a] * Ko);
      }
  }
  if (want & CLMO_W_HIST_DIST) C.hist_t[tid][bin_of(C.Ehist, d2)] += 1;
  if (want & CLMO_W_HIST_REL) {
    const double* vi = &C.vx[i * dim];
    const double* vj = C.cross ? &C.vy[j * dim] : &C.vx[j * dim];
    double dv[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) dv[a] = vj[a] - vi[a];
    double qq = dv[0] * dv[0] + dv[1] * dv[1];
    if (dim == 3) qq = qq + dv[2] * dv[2];
    int b = bin_of(C.Erel, qq);
    C.rel_t[tid][b] += 1;
    if (b < q.rel_nbins) rel_sum[b].add(std::sqrt(qq));
  }
  if (want & CLMO_W_HIST_DIST_VEL) {
    /* Code 10: pairs binned by distance, |v_j - v_i| summed per bin */
    const double* vi = &C.vx[i * dim];
    const double* vj = C.cross ? &C.vy[j * dim] : &C.vx[j * dim];
    double dv[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) dv[a] = vj[a] - vi[a];
    double qq = dv[0] * dv[0] + dv[1] * dv[1];
    if (dim == 3) qq = qq + dv[2] * dv[2];
    int b = bin_of(C.Edv, d2);
    C.dv_t[tid][b] += 1;
    if (b < q.dv_nbins) rel_sum[C.nrel + b].add(std::sqrt(qq));
  }
}

/* dE/dr_i contribution of partner j (gather form): f_s * D_ij; and the
 * magnitude of that pair force, |f_s| d, into ga. */
inline void lj_grad_add(const clmo_request& q, int dim, double d2, const double* D, Neumaier* g,
                        Neumaier* ga) {
  double x = (q.sigma * q.sigma) / d2;
  double x3 = x * x * x;
  double fs = 24.0 * q.epsilon * (2.0 * x3 * x3 - x3) / d2;
  for (int a = 0; a < dim; ++a) g[a].add(fs * D[a]);
  ga->add(std::fabs(fs) * std::sqrt(d2));
}

int oracle_grid(const Box& B, int* n) {
  for (int d = 0; d < B.dim; ++d) {
    double m = std::floor(B.w[d] / B.rc * (1.0 - 1e-9));
    if (!(m >= 3.0)) return 0;
    n[d] = m > 4096.0 ? 4096 : (int)m;
  }
  return 1;
}

int cell_of(const double* f, const int* n, int dim) {
  int c[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    int k = (int)std::floor(f[d] * (double)n[d]);
    if (k < 0) k = 0;
    if (k >= n[d]) k = n[d] - 1;
    c[d] = k;
  }
  return dim == 3 ? c[0] + n[0] * (c[1] + n[1] * c[2]) : c[0] + n[0] * c[1];
}

}  // namespace

extern "C" {

int clmo_box_inverse(int dim, const double* H, double* Hinv) {
  if ((dim != 2 && dim != 3) || !H || !Hinv) return CLMO_EINVAL;
  return inverse(dim, H, Hinv);
}

int clmo_box_widths(int dim, const double* H, double* w, double* V) {
  if ((dim != 2 && dim != 3) || !H || !w || !V) return CLMO_EINVAL;
  return widths(dim, H, w, V);
}

int clmo_box_from_lengths_angles(const double* len, const double* deg, double* H) {
  if (!len || !deg || !H) return CLMO_EINVAL;
  const double pi = 3.14159265358979323846;
  double ca = std::cos(deg[0] * pi / 180.0), cb = std::cos(deg[1] * pi / 180.0);
  double cg = std::cos(deg[2] * pi / 180.0), sg = std::sin(deg[2] * pi / 180.0);
  double cy = (ca - cb * cg) / sg;
  double cz2 = 1.0 - cb * cb - cy * cy;
  if (!(cz2 > 0.0)) return CLMO_EINVAL;
  double a[3] = {len[0], 0.0, 0.0};
  double b[3] = {len[1] * cg, len[1] * sg, 0.0};
  double c[3] = {len[2] * cb, len[2] * cy, len[2] * std::sqrt(cz2)};
  for (int r = 0; r < 3; ++r) {
    H[r * 3 + 0] = a[r];
    H[r * 3 + 1] = b[r];
    H[r * 3 + 2] = c[r];
  }
  return CLMO_OK;
}

int clmo_wrap(int dim, const double* H, int64_t n, const double* x, double* xw,
              double* frac, int64_t* wrap) {
  Box B;
  if (make_box(dim, H, 1.0, &B) != CLMO_OK || n < 0 || (n > 0 && (!x || !xw))) return CLMO_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    wrap_one(B, &x[i * dim], &xw[i * dim], frac ? &frac[i * dim] : nullptr,
             wrap ? &wrap[i * dim] : nullptr);
  return CLMO_OK;
}

double clmo_pair_d2(int dim, const double* H, const double* xi, const double* xj, double reach,
                    int* K_out) {
  Box B;
  if (make_box(dim, H, 1.0, &B) != CLMO_OK || !xi || !xj || !(reach > 0.0))
    return std::numeric_limits<double>::quiet_NaN();
  double ri[3], rj[3], fi[3], fj[3], D[3];
  int64_t wi[3], wj[3];
  int K[3] = {0, 0, 0};
  wrap_one(B, xi, ri, fi, wi);
  wrap_one(B, xj, rj, fj, wj);
  double d2 = min_image(B, ri, fi, rj, fj, reach, D, K);
  if (K_out)
    for (int a = 0; a < dim; ++a) K_out[a] = (int)((int64_t)K[a] + wi[a] - wj[a]);
  return d2;
}

int clmo_compute(int dim, const double* H, double cutoff, const double* x, int64_t nx,
                 const double* y, int64_t ny, const clmo_request* req, clmo_result* res) {
  Box B;
  if (!req || !res || make_box(dim, H, cutoff, &B) != CLMO_OK) return CLMO_EINVAL;
  if (nx < 0 || (nx > 0 && !x)) return CLMO_EINVAL;
  const bool cross = (y != nullptr);
  if (cross && ny < 0) return CLMO_EINVAL;
  const int want = req->want;
  if ((want & CLMO_W_LJ) && res->lj_grad && cross) return CLMO_EINVAL;
  if (req->frame_x && cross) return CLMO_EINVAL;
  if ((want & CLMO_W_SUM_W_INV_D) && (!req->weights_x || (cross && !req->weights_y))) return CLMO_EINVAL;
  if ((want & CLMO_W_HIST_DIST_VEL) &&
      (req->dv_nbins < 1 || !(req->dv_hi > 0) || !res->dv_hist || !res->dv_sum || !req->vel_x ||
       (cross && !req->vel_y)))
    return CLMO_EINVAL;
  if ((want & CLMO_W_HIST_DIST) && (req->hist_nbins < 1 || !(req->hist_hi > 0) || !res->hist))
    return CLMO_EINVAL;
  if ((want & CLMO_W_HIST_REL) &&
      (req->rel_nbins < 1 || !(req->rel_hi > 0) || !res->rel_hist || !res->rel_sum ||
       !req->vel_x || (cross && !req->vel_y)))
    return CLMO_EINVAL;
  if ((want & CLMO_W_NL) && req->nl_capacity > 0 && (!res->nl_i || !res->nl_j)) return CLMO_EINVAL;

  int nthreads = req->nthreads > 0 ? req->nthreads : omp_get_max_threads();

  Ctx C;
  C.B = &B;
  C.req = req;
  C.cross = cross;
  C.nx = nx;
  C.ny = cross ? ny : nx;
  C.xw.resize(nx * dim);
  C.fx.resize(nx * dim);
  C.wx.resize(nx * dim);
  for (int64_t i = 0; i < nx; ++i) wrap_one(B, &x[i * dim], &C.xw[i * dim], &C.fx[i * dim], &C.wx[i * dim]);
  const bool framed = req->frame_x != nullptr;
  if (framed) {
    /* cells come from the canonical fractions; distances from the frame */
    C.cfx = C.fx;
    C.dwx.resize(nx * dim);
    for (int64_t i = 0; i < nx; ++i)
      frame_one(B, &x[i * dim], &req->frame_x[i * dim], &C.xw[i * dim], &C.fx[i * dim]);
    for (int64_t k = 0; k < nx * dim; ++k) {
      C.dwx[k] = C.wx[k] - req->frame_x[k];
      C.wx[k] = req->frame_x[k];
    }
  }
  if (cross) {
    C.yw.resize(ny * dim);
    C.fy.resize(ny * dim);
    C.wy.resize(ny * dim);
    for (int64_t j = 0; j < ny; ++j) wrap_one(B, &y[j * dim], &C.yw[j * dim], &C.fy[j * dim], &C.wy[j * dim]);
  }
  C.vx = req->vel_x;
  C.vy = req->vel_y;
  if (want & CLMO_W_HIST_DIST)
    C.Ehist = edges(req->hist_nbins, req->hist_hi, req->hist_hi == cutoff, B.rc2);
  if (want & CLMO_W_HIST_REL) C.Erel = edges(req->rel_nbins, req->rel_hi, false, 0.0);
  if (want & CLMO_W_HIST_DIST_VEL) C.Edv = edges(req->dv_nbins, req->dv_hi, req->dv_hi == cutoff, B.rc2);
  C.dv_t.assign(nthreads, std::vector<uint64_t>((want & CLMO_W_HIST_DIST_VEL) ? req->dv_nbins + 1 : 0, 0));
  C.hist_t.assign(nthreads, std::vector<uint64_t>((want & CLMO_W_HIST_DIST) ? req->hist_nbins + 1 : 0, 0));
  C.rel_t.assign(nthreads, std::vector<uint64_t>((want & CLMO_W_HIST_REL) ? req->rel_nbins + 1 : 0, 0));
  C.nl_t.assign(nthreads, std::vector<Pair>());

  const double* yw = cross ? C.yw.data() : C.xw.data();
  const double* fy = cross ? C.fy.data() : C.fx.data();
  const int64_t nyy = C.ny;
  C.nrel = (want & CLMO_W_HIST_REL) ? req->rel_nbins : 0;
  const int ndv = (want & CLMO_W_HIST_DIST_VEL) ? req->dv_nbins : 0;
  const int nrel = C.nrel + ndv;  /* per-unit FP64 sums of both histograms */
  double* grad = ((want & CLMO_W_LJ) && !cross) ? res->lj_grad : nullptr;
  if (grad) std::memset(grad, 0, sizeof(double) * nx * dim);

  int n[3] = {1, 1, 1};
  int method = req->method;
  if (method == CLMO_METHOD_AUTO) method = oracle_grid(B, n) ? CLMO_METHOD_CELLS : CLMO_METHOD_BRUTE;
  if (method == CLMO_METHOD_CELLS && !oracle_grid(B, n)) method = CLMO_METHOD_BRUTE;
  res->method_used = method;

  /* Units of work: one particle i (brute force) or one home cell. */
  std::vector<Partial> partial;
  std::vector<std::vector<Neumaier>> relsum_part;

  if (method == CLMO_METHOD_BRUTE) {
    /* The nearest image of any displacement lies within half the sum of the
     * lattice-vector lengths (round the fractional displacement), so no
     * image beyond that reach can be the minimum. */
    double sum_len = 0.0;
    for (int b = 0; b < dim; ++b) {
      double s2 = 0.0;
      for (int a = 0; a < dim; ++a) s2 += B.h(a, b) * B.h(a, b);
      sum_len += std::sqrt(s2);
    }
    const double reach = std::min(B.rc, 0.5 * sum_len * (1.0 + 1e-6));
    partial.assign(nx, Partial());
    relsum_part.assign(nx, std::vector<Neumaier>(nrel));
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t i = 0; i < nx; ++i) {
      int tid = omp_get_thread_num();
      double D[3];
      int K[3];
      Neumaier g[3], ga;
      for (int64_t j = 0; j < nyy; ++j) {
        if (!cross && j == i) continue;
        double d2 = min_image(B, &C.xw[i * dim], &C.fx[i * dim], &yw[j * dim], &fy[j * dim],
                              reach, D, K);
        if (!(d2 <= B.rc2)) continue;
        if (grad) lj_grad_add(*req, dim, d2, D, g, &ga);
        if (cross || i < j) accumulate(C, partial[i], relsum_part[i], tid, i, j, d2, D, K);
      }
      if (grad)
        for (int a = 0; a < dim; ++a) grad[i * dim + a] = g[a].value();
      if (grad && res->lj_fabs) res->lj_fabs[i] = ga.value();
    }
  } else {
    const int ncell = dim == 3 ? n[0] * n[1] * n[2] : n[0] * n[1];
    /* plain per-cell particle lists */
    std::vector<std::vector<int64_t>> xcells(ncell), ycells;
    const std::vector<double>& cf = framed ? C.cfx : C.fx;
    for (int64_t i = 0; i < nx; ++i) xcells[cell_of(&cf[i * dim], n, dim)].push_back(i);
    if (cross) {
      ycells.assign(ncell, std::vector<int64_t>());
      for (int64_t j = 0; j < ny; ++j) ycells[cell_of(&C.fy[j * dim], n, dim)].push_back(j);
    }
    const std::vector<std::vector<int64_t>>& jcells = cross ? ycells : xcells;
    partial.assign(ncell, Partial());
    relsum_part.assign(ncell, std::vector<Neumaier>(nrel));
    const int nz = dim == 3 ? n[2] : 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int c = 0; c < ncell; ++c) {
      int tid = omp_get_thread_num();
      int cx = c % n[0], cy = (c / n[0]) % n[1], cz = dim == 3 ? c / (n[0] * n[1]) : 0;
      for (int64_t i : xcells[c]) {
        Neumaier g[3], ga;
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int ux = cx + dx, uy = cy + dy, uz = cz + dz;
              int K[3] = {0, 0, 0};
              /* periodic wrap of the neighbour cell; K is its image */
              if (ux < 0) { ux += n[0]; K[0] = -1; } else if (ux >= n[0]) { ux -= n[0]; K[0] = 1; }
              if (uy < 0) { uy += n[1]; K[1] = -1; } else if (uy >= n[1]) { uy -= n[1]; K[1] = 1; }
              if (dim == 3) {
                if (uz < 0) { uz += nz; K[2] = -1; } else if (uz >= nz) { uz -= nz; K[2] = 1; }
              }
              int cn = dim == 3 ? ux + n[0] * (uy + n[1] * uz) : ux + n[0] * uy;
              double t[3], D[3];
              shift(B, K, t);
              for (int64_t j : jcells[cn]) {
                if (!cross && j == i) continue;
                int Kp[3] = {K[0], K[1], K[2]};
                double tp[3] = {t[0], t[1], t[2]};
                if (framed) {
                  /* the same real displacement in the frame: K - dw_j + dw_i */
                  for (int a = 0; a < dim; ++a)
                    Kp[a] = (int)((int64_t)K[a] - C.dwx[j * dim + a] + C.dwx[i * dim + a]);
                  shift(B, Kp, tp);
                }
                double d2 = pair_d2(B, &C.xw[i * dim], &yw[j * dim], tp, D);
                if (!(d2 <= B.rc2)) continue;
                if (grad) lj_grad_add(*req, dim, d2, D, g, &ga);
                if (cross || i < j) accumulate(C, partial[c], relsum_part[c], tid, i, j, d2, D, Kp);
              }
            }
        if (grad)
          for (int a = 0; a < dim; ++a) grad[i * dim + a] = g[a].value();
        if (grad && res->lj_fabs) res->lj_fabs[i] = ga.value();
      }
    }
  }

  /* fixed-order combination */
  uint64_t count = 0;
  Neumaier sd, sid, lj, sw, vir[9], dh[9];
  std::vector<Neumaier> rs(nrel);
  for (size_t u = 0; u < partial.size(); ++u) {
    const Partial& P = partial[u];
    count += P.count;
    sd.add(P.sum_d.value());
    sid.add(P.sum_inv_d.value());
    sw.add(P.sum_w.value());
    lj.add(P.lj.value());
    for (int k = 0; k < 9; ++k) {
      vir[k].add(P.vir[k].value());
      dh[k].add(P.dEdH[k].value());
    }
    for (int b = 0; b < nrel; ++b) rs[b].add(relsum_part[u][b].value());
  }
  res->count = count;
  res->sum_d = sd.value();
  res->sum_inv_d = sid.value();
  res->sum_w_inv_d = sw.value();
  res->lj_energy = lj.value();
  for (int k = 0; k < 9; ++k) {
    res->virial[k] = vir[k].value();
    res->dEdH[k] = dh[k].value();
  }
  if (want & CLMO_W_HIST_DIST) {
    for (int b = 0; b <= req->hist_nbins; ++b) {
      uint64_t s = 0;
      for (int t = 0; t < nthreads; ++t) s += C.hist_t[t][b];
      res->hist[b] = s;
    }
  }
  if (want & CLMO_W_HIST_REL) {
    for (int b = 0; b <= req->rel_nbins; ++b) {
      uint64_t s = 0;
      for (int t = 0; t < nthreads; ++t) s += C.rel_t[t][b];
      res->rel_hist[b] = s;
    }
    for (int b = 0; b < C.nrel; ++b) res->rel_sum[b] = rs[b].value();
  }
  if (want & CLMO_W_HIST_DIST_VEL) {
    for (int b = 0; b <= req->dv_nbins; ++b) {
      uint64_t s = 0;
      for (int t = 0; t < nthreads; ++t) s += C.dv_t[t][b];
      res->dv_hist[b] = s;
    }
    for (int b = 0; b < ndv; ++b) res->dv_sum[b] = rs[C.nrel + b].value();
  }
  res->nl_count = 0;
  if (want & CLMO_W_NL) {
    std::vector<Pair> all;
    for (auto& v : C.nl_t) all.insert(all.end(), v.begin(), v.end());
    std::sort(all.begin(), all.end(), [](const Pair& p, const Pair& q) {
      return p.i < q.i || (p.i == q.i && p.j < q.j);
    });
    res->nl_count = all.size();
    int64_t m = std::min<int64_t>((int64_t)all.size(), req->nl_capacity);
    for (int64_t k = 0; k < m; ++k) {
      res->nl_i[k] = all[k].i;
      res->nl_j[k] = all[k].j;
      if (res->nl_d) res->nl_d[k] = all[k].d;
      if (res->nl_d2) res->nl_d2[k] = all[k].d2;
    }
  }
  return CLMO_OK;
}

int clmo_lj_sample(int dim, const double* H, double cutoff, const double* x, int64_t n,
                   const int64_t* sample, int64_t ns, double sigma, double epsilon, int nthreads,
                   double* energy_i, double* grad_i) {
  Box B;
  if (make_box(dim, H, cutoff, &B) != CLMO_OK || n < 0 || ns < 0 || (ns > 0 && (!sample || !x)))
    return CLMO_EINVAL;
  for (int64_t k = 0; k < ns; ++k)
    if (sample[k] < 0 || sample[k] >= n) return CLMO_EINVAL;
  std::vector<double> xw(n * dim), fx(n * dim);
  for (int64_t i = 0; i < n; ++i) wrap_one(B, &x[i * dim], &xw[i * dim], &fx[i * dim], nullptr);
  clmo_request q;
  std::memset(&q, 0, sizeof(q));
  q.sigma = sigma;
  q.epsilon = epsilon;
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t k = 0; k < ns; ++k) {
    int64_t i = sample[k];
    Neumaier e;
    Neumaier g[3];
    double D[3];
    int K[3];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d2 = min_image(B, &xw[i * dim], &fx[i * dim], &xw[j * dim], &fx[j * dim], B.rc, D, K);
      if (!(d2 <= B.rc2)) continue;
      double xx = (sigma * sigma) / d2;
      double x3 = xx * xx * xx;
      e.add(4.0 * epsilon * (x3 * x3 - x3));
      double fs = 24.0 * epsilon * (2.0 * x3 * x3 - x3) / d2;
      for (int a = 0; a < dim; ++a) g[a].add(fs * D[a]);
    }
    if (energy_i) energy_i[k] = e.value();
    if (grad_i)
      for (int a = 0; a < dim; ++a) grad_i[k * dim + a] = g[a].value();
  }
  return CLMO_OK;
}

int clmo_neighbors_of(int dim, const double* H, double cutoff, const double* x, int64_t n,
                      int64_t i, int64_t cap, int64_t* js, int* Ks, int64_t* count) {
  Box B;
  if (make_box(dim, H, cutoff, &B) != CLMO_OK || i < 0 || i >= n || !x || !count) return CLMO_EINVAL;
  double ri[3], fi[3];
  int64_t wi[3];
  wrap_one(B, &x[i * dim], ri, fi, wi);
  int64_t m = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double rj[3], fj[3], D[3];
    int64_t wj[3];
    int K[3];
    wrap_one(B, &x[j * dim], rj, fj, wj);
    double d2 = min_image(B, ri, fi, rj, fj, B.rc, D, K);
    if (!(d2 <= B.rc2)) continue;
    if (m < cap) {
      js[m] = j;
      for (int a = 0; a < dim; ++a) Ks[m * dim + a] = (int)((int64_t)K[a] + wi[a] - wj[a]);
    }
    ++m;
  }
  *count = m;
  return CLMO_OK;
}

int clmo_paper_ghost_grid(int dim, const double* H, double cutoff, int lcell, int* ncells_out,
                          double* sizes_out) {
  if ((dim != 2 && dim != 3) || !H || !(cutoff > 0) || lcell != 1 || !ncells_out || !sizes_out)
    return CLMO_EINVAL;
  bool ortho = true;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b)
      if (a != b && H[a * dim + b] != 0.0) ortho = false;
  for (int d = 0; d < dim; ++d) {
    if (ortho) {
      double L = H[d * dim + d];
      double m = std::floor(L / cutoff);
      ncells_out[d] = (int)m + 2;
      sizes_out[d] = L / m;
    } else {
      double lo = 0.0, hi = 0.0; /* extent of the cell along Cartesian axis d */
      for (int b = 0; b < dim; ++b) {
        double v = H[d * dim + b];
        if (v < 0) lo += v; else hi += v;
      }
      ncells_out[d] = (int)std::ceil((hi - lo) / cutoff) + 2;
      sizes_out[d] = cutoff;
    }
  }
  return CLMO_OK;
}

}  // extern "C"
