// k-nearest-neighbour graph of points (Section 5.1 builds its kNN graphs
// from Euclidean distances), union-symmetrised, with the Gaussian weights
// w_ij = exp(-d_ij^2 / sigma^2), sigma = the median k-th neighbour distance.
//
// Exact by construction:
//   - d^2 is summed over the coordinates in order, each difference squared
//     by a plain product (no fused multiply-add), so d^2(i, j) = d^2(j, i)
//     bit for bit and equals a sequential reference;
//   - every point scans every other point in increasing index order and
//     keeps the k smallest d^2, an equal d^2 never displacing an earlier
//     (smaller) index: ties go to the smaller index;
//   - sigma is selected exactly (radix select on the FP64 bit patterns of
//     the k-th d^2, which order like the values since they are >= 0).
// Pipeline: check -> brute-force top-k (candidate tiles in LDS, the top-k
// list in registers) -> sigma -> each row's list sorted by index -> reverse
// lists (count, scan, scatter, sort) -> union per row (count, scan, write
// with weights).
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.h"

namespace me {

namespace {

constexpr int kKnnThreads = 256;  // queries per workgroup = candidates per LDS tile
constexpr int kKnnMaxK = 32;
constexpr int kKnnMaxDim = 64;

__device__ __forceinline__ double sqd_add(double acc, double a, double b) {
  const double t = __dsub_rn(a, b);
  return __dadd_rn(acc, __dmul_rn(t, t));
}

__global__ void k_knn_check(int64_t count, const double* x, int* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count && !isfinite(x[i])) atomicOr(flag, 1);
}

// Inserts (d, j) into the sorted list (bd, bi) at the first entry with a
// larger d (after every equal one: candidates arrive in increasing j, so an
// equal distance keeps the smaller index first) and shifts the rest down by
// one, the last entry dropping out.
template <int KMAX>
__device__ __forceinline__ void insert_top(double (&bd)[KMAX], int32_t (&bi)[KMAX], double d,
                                           int32_t j) {
  bool moving = false;
#pragma unroll
  for (int u = 0; u < KMAX; ++u) {
    if (moving || d < bd[u]) {
      const double td = bd[u];
      const int32_t ti = bi[u];
      bd[u] = d;
      bi[u] = j;
      d = td;
      j = ti;
      moving = true;
    }
  }
}

// One query per thread; DIM > 0 fixes the dimension at compile time,
// DIM = 0 takes `dim` (<= kKnnMaxDim) at run time.  The list keeps the KMAX
// best (d^2, j) in increasing order; its first k entries are the answer.
template <int KMAX, int DIM>
__global__ void __launch_bounds__(kKnnThreads) k_knn_brute(int64_t n, int dim, int k,
                                                           const double* __restrict__ x,
                                                           int32_t* __restrict__ nbr,
                                                           double* __restrict__ kth, int* flag) {
  __shared__ double tile[kKnnThreads * (DIM > 0 ? DIM : 1)];
  const int D = DIM > 0 ? DIM : dim;
  const int64_t i = blockIdx.x * (int64_t)kKnnThreads + threadIdx.x;
  const bool live = i < n;
  double xi[DIM > 0 ? DIM : 1];
  if constexpr (DIM > 0) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = live ? x[i * DIM + d] : 0.0;
  }
  double bd[KMAX];
  int32_t bi[KMAX];
#pragma unroll
  for (int u = 0; u < KMAX; ++u) {
    bd[u] = INFINITY;
    bi[u] = INT32_MAX;
  }
  for (int64_t j0 = 0; j0 < n; j0 += kKnnThreads) {
    const int64_t jn = min<int64_t>(kKnnThreads, n - j0);
    if constexpr (DIM > 0) {
      __syncthreads();
      for (int t = threadIdx.x; t < jn * DIM; t += kKnnThreads) tile[t] = x[j0 * DIM + t];
      __syncthreads();
      if (live) {
        for (int t = 0; t < jn; ++t) {
          double acc = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) acc = sqd_add(acc, xi[d], tile[t * DIM + d]);
          const int32_t j = (int32_t)(j0 + t);
          if (acc < bd[KMAX - 1] && j != i) insert_top<KMAX>(bd, bi, acc, j);
        }
      }
    } else {
      // run-time dimension: coordinates straight from global memory (the
      // general form; the common dimensions have their own instances)
      if (live) {
        for (int t = 0; t < jn; ++t) {
          const int64_t j = j0 + t;
          double s = 0.0;
          for (int d = 0; d < D; ++d) s = sqd_add(s, x[i * D + d], x[j * D + d]);
          if (s < bd[KMAX - 1] && j != i) insert_top<KMAX>(bd, bi, s, (int32_t)j);
        }
      }
    }
  }
  if (!live) return;
  bool full = true;
#pragma unroll
  for (int u = 0; u < KMAX; ++u) {
    if (u < k) {
      // a d^2 that overflows to infinity never enters the list
      full = full && bi[u] != INT32_MAX;
      nbr[i * k + u] = bi[u] != INT32_MAX ? bi[u] : (int32_t)i;
    }
    if (u == k - 1) kth[i] = bd[u];
  }
  if (!full) atomicOr(flag, 2);
}

// ---- exact selection of an order statistic of non-negative doubles ----
// Eight passes over 8-bit digits of the bit pattern, most significant first.
// st[0] = prefix bits, st[1] = mask of fixed bits, st[2] = rank still to
// skip inside the prefix; hist: 256 counters.
__global__ void k_sel_init(uint64_t* st, int64_t rank) {
  st[0] = 0;
  st[1] = 0;
  st[2] = (uint64_t)rank;
}

__global__ void __launch_bounds__(256) k_sel_hist(int64_t n, const double* v, const uint64_t* st,
                                                  int shift, unsigned int* hist) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t pre = st[0], mask = st[1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t b = (uint64_t)__double_as_longlong(v[i]);
    if ((b & mask) == pre) atomicAdd(&h[(b >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_sel_pick(uint64_t* st, int shift, unsigned int* hist) {
  uint64_t r = st[2];
  int b = 0;
  for (; b < 255; ++b) {
    if (r < hist[b]) break;
    r -= hist[b];
  }
  st[0] |= (uint64_t)b << shift;
  st[1] |= (uint64_t)0xff << shift;
  st[2] = r;
  for (int q = 0; q < 256; ++q) hist[q] = 0;
}

// sigma = median of sqrt(kth): the middle value, or the mean of the two
// middle ones (sel[0] = key of rank floor((n-1)/2), sel[1] = of rank n/2).
__global__ void k_sigma(const uint64_t* lo, const uint64_t* hi, int64_t n, double* sigma) {
  const double a = __dsqrt_rn(__longlong_as_double((long long)lo[0]));
  const double b = __dsqrt_rn(__longlong_as_double((long long)hi[0]));
  *sigma = (n & 1) ? a : __ddiv_rn(__dadd_rn(a, b), 2.0);
}

// Each row's k neighbours in increasing index (and its count of reverse
// edges).
__global__ void k_knn_sort_rows(int64_t n, int k, int32_t* nbr, int32_t* rcnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t* r = nbr + i * k;
  for (int a = 1; a < k; ++a) {
    const int32_t v = r[a];
    int b = a - 1;
    while (b >= 0 && r[b] > v) {
      r[b + 1] = r[b];
      --b;
    }
    r[b + 1] = v;
  }
  for (int a = 0; a < k; ++a) atomicAdd(&rcnt[r[a]], 1);
}

// Reverse lists: for every edge i -> j, i is appended to j's list.
__global__ void k_knn_scatter(int64_t n, int k, const int32_t* nbr, const int64_t* roff,
                              int32_t* rcur, int32_t* rlist) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int32_t j = nbr[e];
  const int32_t i = (int32_t)(e / k);
  rlist[roff[j] + atomicAdd(&rcur[j], 1)] = i;
}

// Sorts each reverse list (insertion sort; a list holds the points that
// have j among their k nearest, a few times k on sampled manifolds).
__global__ void k_knn_sort_rev(int64_t n, const int64_t* roff, int32_t* rlist) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  int32_t* r = rlist + roff[j];
  const int64_t m = roff[j + 1] - roff[j];
  for (int64_t a = 1; a < m; ++a) {
    const int32_t v = r[a];
    int64_t b = a - 1;
    while (b >= 0 && r[b] > v) {
      r[b + 1] = r[b];
      --b;
    }
    r[b + 1] = v;
  }
}

// Union of row i's own list and its reverse list (both sorted): WRITE = 0
// counts the distinct neighbours, WRITE = 1 writes them with their weights.
template <bool WRITE>
__global__ void k_knn_union(int64_t n, int dim, int k, const double* __restrict__ x,
                            const int32_t* __restrict__ nbr, const int64_t* __restrict__ roff,
                            const int32_t* __restrict__ rlist, int32_t* cnt,
                            const int64_t* __restrict__ rowptr, int32_t* col, double* val,
                            const double* sigma) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t* a = nbr + i * k;
  const int32_t* b = rlist + roff[i];
  const int64_t nb = roff[i + 1] - roff[i];
  double s2 = 0.0;
  int64_t out = 0;
  if constexpr (WRITE) {
    s2 = __dmul_rn(*sigma, *sigma);
    out = rowptr[i];
  }
  int64_t pa = 0, pb = 0, c = 0;
  while (pa < k || pb < nb) {
    int32_t j;
    if (pb >= nb || (pa < k && a[pa] < b[pb])) {
      j = a[pa++];
    } else if (pa >= k || b[pb] < a[pa]) {
      j = b[pb++];
    } else {
      j = a[pa++];
      ++pb;
    }
    if constexpr (WRITE) {
      double d2 = 0.0;
      for (int d = 0; d < dim; ++d) d2 = sqd_add(d2, x[i * dim + d], x[(int64_t)j * dim + d]);
      double w = exp(__ddiv_rn(-d2, s2));
      if (!(w >= DBL_MIN)) w = DBL_MIN;  // underflow: the smallest normal weight
      col[out + c] = j;
      val[out + c] = w;
    }
    ++c;
  }
  if constexpr (!WRITE) cnt[i] = (int32_t)c;
}

__global__ void k_zero_i32(int64_t n, int32_t* a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ void k_zero_u32(int64_t n, unsigned int* a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

int kmax_for(int k) { return k <= 8 ? 8 : (k <= 16 ? 16 : 32); }

template <int KMAX>
void launch_brute(int64_t n, int dim, int k, const double* x, int32_t* nbr, double* kth,
                  int* flag, hipStream_t s) {
  const dim3 g((unsigned)ceil_div(n, kKnnThreads)), b(kKnnThreads);
  switch (dim) {
    case 1: k_knn_brute<KMAX, 1><<<g, b, 0, s>>>(n, dim, k, x, nbr, kth, flag); break;
    case 2: k_knn_brute<KMAX, 2><<<g, b, 0, s>>>(n, dim, k, x, nbr, kth, flag); break;
    case 3: k_knn_brute<KMAX, 3><<<g, b, 0, s>>>(n, dim, k, x, nbr, kth, flag); break;
    default: k_knn_brute<KMAX, 0><<<g, b, 0, s>>>(n, dim, k, x, nbr, kth, flag); break;
  }
}

struct KnnScratch {
  int32_t *nbr, *rcnt, *rcur, *rlist, *cnt;
  double *kth, *sigma;
  int64_t *roff, *tmp;
  uint64_t* sel;  // two selection states of 4 words
  unsigned int* hist;
  int* flag;
};

size_t knn_scratch_bytes(int64_t n, int k, KnnScratch* out, char* base) {
  Arena a{base, (size_t)-1, 0};
  KnnScratch sc{};
  sc.nbr = a.take<int32_t>((size_t)n * k);
  sc.rlist = a.take<int32_t>((size_t)n * k);
  sc.rcnt = a.take<int32_t>(n);
  sc.rcur = a.take<int32_t>(n);
  sc.cnt = a.take<int32_t>(n);
  sc.kth = a.take<double>(n);
  sc.sigma = a.take<double>(1);
  sc.roff = a.take<int64_t>(n + 1);
  sc.tmp = a.take<int64_t>(scan_tmp_count(n));
  sc.sel = a.take<uint64_t>(8);
  sc.hist = a.take<unsigned int>(256);
  sc.flag = a.take<int>(1);
  if (out) *out = sc;
  return a.used;
}

int select_rank(int64_t n, const double* v, int64_t rank, uint64_t* st, unsigned int* hist,
                hipStream_t s) {
  k_sel_init<<<1, 1, 0, s>>>(st, rank);
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 256), 1), 1024);
  for (int shift = 56; shift >= 0; shift -= 8) {
    k_sel_hist<<<grid, 256, 0, s>>>(n, v, st, shift, hist);
    k_sel_pick<<<1, 1, 0, s>>>(st, shift, hist);
  }
  return ME_OK;
}

}  // namespace

size_t knn_workspace_bytes(int64_t n, int k) {
  return kHeapAlign + DevHeap::round(knn_scratch_bytes(n, k, nullptr, nullptr));
}

int knn_graph(const double* x, int64_t n, int dim, int k, void* ws, size_t ws_bytes,
              int64_t* rowptr, int32_t* col, double* val, int64_t* nnz, double* sigma_out,
              hipStream_t s) {
  if (!x || !rowptr || !col || !val || !nnz || n < 2 || n >= (int64_t)INT32_MAX || dim < 1 ||
      dim > kKnnMaxDim)
    return ME_ERR_INVALID_ARG;
  if (k < 1 || k > kKnnMaxK || k >= n) return ME_ERR_K_RANGE;
  if (ws && ws_bytes < knn_workspace_bytes(n, k)) return ME_ERR_WORKSPACE;
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  void* mem = nullptr;
  const size_t bytes = knn_scratch_bytes(n, k, nullptr, nullptr);
  ME_TRY_STATUS(heap.alloc(&mem, bytes, s));
  struct Free {
    DevHeap& h;
    void* p;
    hipStream_t s;
    ~Free() {
      (void)hipStreamSynchronize(s);
      h.release(p, s);
    }
  } release{heap, mem, s};
  KnnScratch sc;
  knn_scratch_bytes(n, k, &sc, (char*)mem);
  const int64_t nb = ceil_div(n, kBlock);
  // finite coordinates
  k_zero_i32<<<1, 1, 0, s>>>(1, sc.flag);
  k_knn_check<<<ceil_div(n * dim, kBlock), kBlock, 0, s>>>(n * dim, x, sc.flag);
  int hflag = 0;
  ME_TRY(hipMemcpyAsync(&hflag, sc.flag, 4, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (hflag) return ME_ERR_INVALID_ARG;
  // the k nearest of every point
  switch (kmax_for(k)) {
    case 8: launch_brute<8>(n, dim, k, x, sc.nbr, sc.kth, sc.flag, s); break;
    case 16: launch_brute<16>(n, dim, k, x, sc.nbr, sc.kth, sc.flag, s); break;
    default: launch_brute<32>(n, dim, k, x, sc.nbr, sc.kth, sc.flag, s); break;
  }
  ME_TRY(hipMemcpyAsync(&hflag, sc.flag, 4, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (hflag) return ME_ERR_INVALID_ARG;  // squared distances overflow
  // sigma
  k_zero_u32<<<1, 256, 0, s>>>(256, sc.hist);
  select_rank(n, sc.kth, (n - 1) / 2, sc.sel, sc.hist, s);
  select_rank(n, sc.kth, n / 2, sc.sel + 4, sc.hist, s);
  k_sigma<<<1, 1, 0, s>>>(sc.sel, sc.sel + 4, n, sc.sigma);
  double sigma = 0.0;
  ME_TRY(hipMemcpyAsync(&sigma, sc.sigma, 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (!(sigma > 0.0)) return ME_ERR_BAD_WEIGHT;  // every weight would be undefined
  // reverse lists
  k_zero_i32<<<nb, kBlock, 0, s>>>(n, sc.rcnt);
  k_zero_i32<<<nb, kBlock, 0, s>>>(n, sc.rcur);
  k_knn_sort_rows<<<nb, kBlock, 0, s>>>(n, k, sc.nbr, sc.rcnt);
  scan_counts(n, sc.rcnt, sc.roff, sc.tmp, s);
  k_knn_scatter<<<ceil_div(n * k, kBlock), kBlock, 0, s>>>(n, k, sc.nbr, sc.roff, sc.rcur,
                                                           sc.rlist);
  k_knn_sort_rev<<<nb, kBlock, 0, s>>>(n, sc.roff, sc.rlist);
  // union rows
  k_knn_union<false><<<nb, kBlock, 0, s>>>(n, dim, k, x, sc.nbr, sc.roff, sc.rlist, sc.cnt,
                                           nullptr, nullptr, nullptr, nullptr);
  scan_counts(n, sc.cnt, rowptr, sc.tmp, s);
  k_knn_union<true><<<nb, kBlock, 0, s>>>(n, dim, k, x, sc.nbr, sc.roff, sc.rlist, nullptr,
                                          rowptr, col, val, sc.sigma);
  int64_t total = 0;
  ME_TRY(hipMemcpyAsync(&total, rowptr + n, 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  *nnz = total;
  if (sigma_out) *sigma_out = sigma;
  return ME_OK;
}

}  // namespace me

extern "C" {

size_t me_knn_workspace_bytes(int64_t n, int dim, int k) {
  if (n < 2 || dim < 1 || k < 1) return 0;
  return me::knn_workspace_bytes(n, k);
}

int me_knn_graph(const double* points, int64_t n, int dim, int k, void* ws, size_t ws_bytes,
                 int64_t* rowptr, int32_t* col, double* val, int64_t* nnz, double* sigma,
                 void* stream) {
  return me::knn_graph(points, n, dim, k, ws, ws_bytes, rowptr, col, val, nnz, sigma,
                       (hipStream_t)stream);
}

}  // extern "C"
