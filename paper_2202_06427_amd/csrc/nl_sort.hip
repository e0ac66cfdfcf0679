// nl_sort.hip -- a neighbour list in canonical order on the device: pairs
// ascending in i, then in j (the order in which the pair set of the paper's
// neighbour-list map, section 4.1, is compared with other lists), with the
// distances moved along.
//
// Method: every pair (i, j) becomes the key i * 2^bj + j (bj bits hold the
// largest j), and the keys are put in order by a stable least-significant-
// digit radix sort with 8-bit digits: per pass, each block of 2048 keys
// counts its digits in LDS, one exclusive scan over the digit-major table
// (digit, block) gives every block its first slot per digit, and the block
// writes its keys to those slots in input order.  Input order within a digit
// is kept by ranking each chunk of 256 keys in LDS: a wave finds the lanes
// holding the same digit with eight ballots (one per bit), the lowest of
// them posts the group size, and each key's slot is the digit's running
// offset plus the keys of earlier waves and lower lanes.  Pairs are unique,
// so the result does not depend on the order the map wrote them in.
//
// The pair buffer doubles as one of the two key buffers (a pair of int32 is
// 8 bytes, as a key), so the workspace holds one key buffer, one distance
// buffer and the digit table.  Every kernel reads the true pair count from
// the device and sorts min(count, capacity) pairs.
#include <algorithm>
#include <cstdint>
#include <utility>

#include "clmap_state.h"
#include "device_util.h"

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortPer = 8;
constexpr int kSortChunk = kSortThreads * kSortPer;
constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;

struct SortPass {
  const unsigned long long* count;
  long long capacity;
  const uint64_t* kin;
  uint64_t* kout;
  const double* din;   // NULL: no distances
  double* dout;
  uint32_t* table;     // kDigits * nblocks (+1), digit-major
  int shift, nblocks;
};

__device__ __forceinline__ long long sort_len(const unsigned long long* count, long long cap) {
  const unsigned long long c = *count;
  return c < (unsigned long long)cap ? (long long)c : cap;
}

// (i, j) int32 pairs -> keys, in place.
__global__ void __launch_bounds__(kSortThreads) pack_keys_kernel(uint64_t* pk,
                                                                 const unsigned long long* count,
                                                                 long long cap, int bj) {
  const long long m = sort_len(count, cap);
  for (long long t = (long long)blockIdx.x * kSortThreads + threadIdx.x; t < m;
       t += (long long)gridDim.x * kSortThreads) {
    const uint64_t p = pk[t];
    const uint64_t i = (uint32_t)p, j = (uint32_t)(p >> 32);
    pk[t] = (i << bj) | j;
  }
}

// keys -> (i, j) int32 pairs (src may equal dst), distances copied when
// they sit in the other buffer.
__global__ void __launch_bounds__(kSortThreads) unpack_keys_kernel(const uint64_t* src, uint64_t* dst,
                                                                   const double* dsrc, double* ddst,
                                                                   const unsigned long long* count,
                                                                   long long cap, int bj) {
  const long long m = sort_len(count, cap);
  const uint64_t jmask = (uint64_t(1) << bj) - 1;
  for (long long t = (long long)blockIdx.x * kSortThreads + threadIdx.x; t < m;
       t += (long long)gridDim.x * kSortThreads) {
    const uint64_t k = src[t];
    dst[t] = (k >> bj) | ((k & jmask) << 32);
    if (dsrc != ddst) ddst[t] = dsrc[t];
  }
}

__global__ void __launch_bounds__(kSortThreads) digit_count_kernel(SortPass P) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const long long m = sort_len(P.count, P.capacity);
  const long long base = (long long)blockIdx.x * kSortChunk;
#pragma unroll
  for (int k = 0; k < kSortPer; ++k) {
    const long long t = base + k * kSortThreads + threadIdx.x;
    if (t < m) atomicAdd(&h[(P.kin[t] >> P.shift) & (kDigits - 1)], 1u);
  }
  __syncthreads();
  P.table[(size_t)threadIdx.x * P.nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) digit_scatter_kernel(SortPass P) {
  __shared__ uint32_t run[kDigits];
  __shared__ uint32_t wc[kSortThreads / kWave][kDigits];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const long long m = sort_len(P.count, P.capacity);
  const long long base = (long long)blockIdx.x * kSortChunk;
  if (base >= m) return;  // uniform over the block
  run[tid] = P.table[(size_t)tid * P.nblocks + blockIdx.x];
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int k = 0; k < kSortPer; ++k) {
#pragma unroll
    for (int v = 0; v < kSortThreads / kWave; ++v) wc[v][tid] = 0;
    __syncthreads();
    const long long t = base + k * kSortThreads + tid;
    const bool valid = t < m;
    const uint64_t key = valid ? P.kin[t] : 0;
    const uint32_t dig = (uint32_t)(key >> P.shift) & (kDigits - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t set = __ballot(bit);
      peers &= bit ? set : ~set;
    }
    const uint32_t r = (uint32_t)__popcll(peers & below);
    if (valid && r == 0) wc[w][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t slot = run[dig] + r;
      for (int v = 0; v < w; ++v) slot += wc[v][dig];
      P.kout[slot] = key;
      if (P.din) P.dout[slot] = P.din[t];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int v = 0; v < kSortThreads / kWave; ++v) add += wc[v][tid];
    run[tid] += add;
    __syncthreads();
  }
}

int bits_for(int64_t n) {  // bits of the largest index n - 1 (at least 1)
  int b = 1;
  while (b < 62 && (int64_t(1) << b) < n) ++b;
  return b;
}

struct SortLayout {
  int64_t nblocks;
  size_t o_keys, o_dist, o_table, o_sums, total;
};

SortLayout sort_layout(int64_t capacity, bool dist) {
  SortLayout L;
  L.nblocks = std::max<int64_t>((capacity + kSortChunk - 1) / kSortChunk, 1);
  const int64_t nt = kDigits * L.nblocks;
  Carve c;
  L.o_keys = c.take(sizeof(uint64_t) * (size_t)std::max<int64_t>(capacity, 1));
  L.o_dist = dist ? c.take(sizeof(double) * (size_t)std::max<int64_t>(capacity, 1)) : 0;
  L.o_table = c.take(sizeof(uint32_t) * (size_t)(nt + 1));
  L.o_sums = c.take(sizeof(uint32_t) * scan_scratch_elems((int)nt));
  L.total = c.off;
  return L;
}

// Largest capacity: the digit table is scanned as int-indexed u32 and slots
// are u32.
constexpr int64_t kSortMaxCapacity = (int64_t(1) << 31) - (int64_t(1) << 20);

}  // namespace

clm_status sort_pairs_check(int64_t n_i, int64_t n_j, const int32_t* pairs, int64_t capacity,
                            bool dist, const void* ws, size_t ws_bytes) {
  if (n_i < 1 || n_j < 1 || n_i > (int64_t(1) << 31) || n_j > (int64_t(1) << 31))
    return fail(CLM_E_INVALID_ARG, "index ranges must be 1..2^31");
  if (capacity < 0 || capacity > kSortMaxCapacity)
    return fail(CLM_E_INVALID_ARG, "capacity must be in 0..%lld", (long long)kSortMaxCapacity);
  if (capacity > 0 && (!pairs || ((uintptr_t)pairs & 7) != 0))
    return fail(CLM_E_INVALID_ARG, "pairs must be a non-NULL, 8-byte aligned (i, j) int32 array");
  const SortLayout L = sort_layout(capacity, dist);
  if (!ws) return fail(CLM_E_WORKSPACE, "sort workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(CLM_E_WORKSPACE, "sort workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(CLM_E_WORKSPACE, "sort workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  return CLM_OK;
}

size_t sort_pairs_bytes(int64_t capacity, bool dist) { return sort_layout(capacity, dist).total; }

// Enqueue the sort (arguments already checked by sort_pairs_check).
clm_status sort_pairs(hipStream_t st, int64_t n_i, int64_t n_j, int32_t* pairs, double* dist,
                      const unsigned long long* count, int64_t capacity, void* ws) {
  if (capacity == 0) return CLM_OK;
  const SortLayout L = sort_layout(capacity, dist != nullptr);
  char* base = (char*)ws;
  const int bj = bits_for(n_j);
  const int nbits = bits_for(n_i) + bj;
  const int passes = (nbits + kDigitBits - 1) / kDigitBits;
  uint64_t* a = (uint64_t*)pairs;
  uint64_t* b = (uint64_t*)(base + L.o_keys);
  double* da = dist;
  double* db = dist ? (double*)(base + L.o_dist) : nullptr;
  uint32_t* table = (uint32_t*)(base + L.o_table);
  uint32_t* sums = (uint32_t*)(base + L.o_sums);
  const int nb = (int)L.nblocks;
  const unsigned eg = (unsigned)std::min<int64_t>(L.nblocks * kSortPer, 65536);
  pack_keys_kernel<<<eg, kSortThreads, 0, st>>>(a, count, capacity, bj);
  CLM_HIP(hipGetLastError());
  for (int p = 0; p < passes; ++p) {
    SortPass P;
    P.count = count;
    P.capacity = capacity;
    P.kin = a;
    P.kout = b;
    P.din = da;
    P.dout = db;
    P.table = table;
    P.shift = p * kDigitBits;
    P.nblocks = nb;
    digit_count_kernel<<<nb, kSortThreads, 0, st>>>(P);
    CLM_HIP(hipGetLastError());
    CLM_HIP(launch_scan(table, kDigits * nb, sums, table, st));
    digit_scatter_kernel<<<nb, kSortThreads, 0, st>>>(P);
    CLM_HIP(hipGetLastError());
    std::swap(a, b);
    std::swap(da, db);
  }
  unpack_keys_kernel<<<eg, kSortThreads, 0, st>>>(a, (uint64_t*)pairs, da, dist, count, capacity, bj);
  CLM_HIP(hipGetLastError());
  return CLM_OK;
}

extern "C" {

clm_status clm_pairs_sort_workspace_bytes(int64_t capacity, int with_distances, size_t* bytes) {
  if (!bytes) return fail(CLM_E_INVALID_ARG, "bytes is NULL");
  if (capacity < 0 || capacity > kSortMaxCapacity)
    return fail(CLM_E_INVALID_ARG, "capacity must be in 0..%lld", (long long)kSortMaxCapacity);
  *bytes = sort_pairs_bytes(capacity, with_distances != 0);
  return CLM_OK;
}

clm_status clm_pairs_sort(clm_context* ctx, int64_t n_i, int64_t n_j, int32_t* pairs_dev,
                          double* dist_dev, const uint64_t* count_dev, int64_t capacity,
                          void* workspace_dev, size_t workspace_bytes) {
  if (!ctx || !count_dev) return fail(CLM_E_INVALID_ARG, "ctx or count_dev is NULL");
  clm_status s = sort_pairs_check(n_i, n_j, pairs_dev, capacity, dist_dev != nullptr, workspace_dev,
                                  workspace_bytes);
  if (s != CLM_OK) return s;
  CLM_HIP(hipSetDevice(ctx->device));
  return sort_pairs(ctx->stream, n_i, n_j, pairs_dev, dist_dev, (const unsigned long long*)count_dev,
                    capacity, workspace_dev);
}

}  // extern "C"
