// clmap_state.h -- host-side objects of libclmap shared by its C-ABI files
// (contexts, boxes, cell lists, error reporting).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/clmap.h"
#include "clmap_internal.h"

using namespace clm;

// ---------------------------------------------------------------- errors
inline thread_local std::string g_err;

inline clm_status fail(clm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline clm_status fail(clm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define CLM_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CLM_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

// ---------------------------------------------------------------- objects
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

struct clm_context {
  int device;
  hipStream_t stream;
  bool timing = false;
  std::vector<EventPair> pool;               // reusable events
  std::vector<EventPair> build_ev, sweep_ev; // recorded, not yet read
};

inline clm_status take_events(clm_context* c, EventPair* out) {
  if (!c->pool.empty()) {
    *out = c->pool.back();
    c->pool.pop_back();
    return CLM_OK;
  }
  CLM_HIP(hipEventCreate(&out->a));
  CLM_HIP(hipEventCreate(&out->b));
  return CLM_OK;
}

// Records a start event when timing is on; `stop` records the end.
struct Timed {
  clm_context* c;
  std::vector<EventPair>* dst;
  EventPair ev;
  bool on = false;
  Timed(clm_context* ctx, std::vector<EventPair>* d) : c(ctx), dst(d) {}
  clm_status start() {
    if (!c || !c->timing || dst->size() >= 4096) return CLM_OK;
    clm_status s = take_events(c, &ev);
    if (s != CLM_OK) return s;
    CLM_HIP(hipEventRecord(ev.a, c->stream));
    on = true;
    return CLM_OK;
  }
  clm_status stop() {
    if (!on) return CLM_OK;
    CLM_HIP(hipEventRecord(ev.b, c->stream));
    dst->push_back(ev);
    on = false;
    return CLM_OK;
  }
};

struct clm_box {
  int dim;
  int lcell_req, lcell;
  int lcx_req, lcx;  // along the first fractional axis (rows run along it)
  int small;
  int n[3];
  int64_t ncells;
  int smax;
  double H[9];     // stride 3
  double Hinv[9];  // stride 3
  double w[3];
  double V;
  double rc, rc2;
  double band;
  float lo32, hi32;
  double tK[27 * 4];
  double sum_len;   // sum of the lattice-vector lengths
};

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct SetBufs {
  uint32_t* hist = nullptr;   // binning: (bucket, block) table, nbk * nblk + 1
  uint32_t* off = nullptr;    // ncells + 1
  uint32_t* key = nullptr;    // binning: cell of every particle, n
  BinRec* rec = nullptr;      // binning: records in bucket order, n
  float4* pos = nullptr;      // n + pad
  double4* r64 = nullptr;
  uint32_t* idx = nullptr;
  int4* wrap = nullptr;
  float4* vel32 = nullptr;
};

struct clm_celllist {
  clm_context* ctx;
  clm_box box;
  int64_t nx, ny;
  int cross;
  clm_precision prec;
  char* ws;
  size_t ws_bytes;
  SetBufs X, Y;
  uint32_t* scan_scratch;
  uint32_t* row_tiles;
  uint32_t* row_off;      // nrows + 1; row_off[nrows] = number of tiles
  Tile* tiles;
  int max_tiles;
  int nrows;
  JobDesc* job_dev;
  double* partials;
  unsigned long long* pcount;
  unsigned long long* nl_off;  // neighbour lists: per-item output offsets
  int max_parts;
  double* E64;
  float* E32;
  double* bandq;
  unsigned int* vmax_bits;
  unsigned long long* nl_counter;
  unsigned long long* cand;
  unsigned long long* guard;  // [2] re-evaluation counts of the last map
  double* fin_scratch;
  unsigned long long* fin_count;
  double* brute_fb;       // small boxes: per-chunk LJ force rows
  int built;
  int untimed;            // never record timing events (no runtime objects created)
};

// ---------------------------------------------------------------- shared helpers
inline BuildGeom geom_of(const clm_box& B) {
  BuildGeom g;
  g.dim = B.dim;
  for (int d = 0; d < 3; ++d) g.n[d] = B.n[d];
  for (int k = 0; k < 9; ++k) {
    g.H[k] = B.H[k];
    g.Hinv[k] = B.Hinv[k];
  }
  return g;
}

// clm_map; a neighbour list is written in two passes (a counting sweep gives
// every work item its output offset) unless nl_two_pass_ok is false, when the
// work items reserve output slots from one shared counter (cheaper for short
// lists, where the counter is not contended).
clm_status map_one(clm_celllist* cl, clm_map_kind kind, const clm_map_params* P, const clm_map_out* O,
                   bool nl_two_pass_ok);
// Neighbour lists in canonical order (nl_sort.hip).
clm_status sort_pairs_check(int64_t n_i, int64_t n_j, const int32_t* pairs, int64_t capacity,
                            bool dist, const void* ws, size_t ws_bytes);
size_t sort_pairs_bytes(int64_t capacity, bool dist);
clm_status sort_pairs(hipStream_t st, int64_t n_i, int64_t n_j, int32_t* pairs, double* dist,
                      const unsigned long long* count, int64_t capacity, void* ws);

// Fills a caller-provided cell-list handle over workspace `ws` (the body of
// clm_celllist_create without the host allocation of the handle).
clm_status celllist_init(clm_celllist* cl, clm_context* ctx, const clm_box* box, int64_t n_x,
                         int64_t n_y, clm_precision precision, void* ws, size_t ws_bytes);

// Cell-list build whose kernels all return at once when `gate` (device
// uint32) reads 0; gate == NULL builds unconditionally.
clm_status celllist_build_gated(clm_celllist* cl, const double* x, const double* y,
                                const uint32_t* gate);
