// Betweenness centrality of every node and its variance (VBC), the check of
// Section 3.3 that accepts a graph as a manifold graph (eq. (3), Table 1):
//   C_B(i) = sum over ordered pairs (s, t), s != t, s != i, t != i, of
//            sigma_st(i) / sigma_st,
// shortest paths counted in edges.  Brandes' accumulation, one source per
// workgroup at a time:
//   - breadth-first levels from s with path counts sigma (an edge adds the
//     count of its upper end; the counts are integers, exact in FP64 below
//     2^53, so their sums do not depend on the order of the additions);
//   - from the deepest level up, every node v pulls
//     delta(v) = sigma(v) * sum over neighbours w one level below of
//                (1 + delta(w)) / sigma(w),
//     its neighbours visited in row order (no atomics: the same sums on
//     every run);
//   - each workgroup adds delta to a row of partial sums of its own; the
//     rows are added in workgroup order at the end.
// VBC = the mean of (C_B - mean C_B)^2 over the nodes.
#include <algorithm>

#include "common.h"

namespace me {

namespace {

constexpr int kBrThreads = 256;
constexpr int kBrMaxGroups = 256;  // sources in flight

// dist and sigma change through atomics, which are performed in L2: every
// read of them is an agent-scope atomic load, so that no stale L1 copy is used.
__device__ __forceinline__ int32_t ld_l2(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_l2(const double* p) {
  return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const long long*>(p),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Structure of W: row pointers from 0 to nnz and non-decreasing, columns in
// range, strictly increasing in each row, no self loop, symmetric.
__global__ void k_br_check(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                           int* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == 0 && rp[0] != 0) atomicOr(flag, 1);
  if (i == n) {
    if (rp[n] != nnz) atomicOr(flag, 1);
    return;
  }
  const int64_t a = rp[i], b = rp[i + 1];
  if (a > b || a < 0 || b > nnz) {
    atomicOr(flag, 1);
    return;
  }
  for (int64_t e = a; e < b; ++e) {
    const int32_t j = col[e];
    if (j < 0 || j >= n || j == i || (e > a && col[e - 1] >= j)) {
      atomicOr(flag, 1);
      return;
    }
  }
}

__global__ void k_br_symmetric(int64_t n, const int64_t* rp, const int32_t* col, int* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int32_t j = col[e];
    int64_t lo = rp[j], hi = rp[j + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (col[mid] < i) lo = mid + 1; else hi = mid;
    }
    if (lo >= rp[j + 1] || col[lo] != i) {
      atomicOr(flag, 1);
      return;
    }
  }
}

// One source per workgroup pass.  Scratch per workgroup: dist (int32 n),
// order (int32 n, the visit order by levels), levoff (int32 n + 1, where
// each level starts in order), sigma and delta (double n), part (double n,
// this workgroup's sums of delta).
__global__ void __launch_bounds__(kBrThreads) k_brandes(int64_t n, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        int32_t* dist_all, int32_t* order_all,
                                                        int32_t* levoff_all, double* sigma_all,
                                                        double* delta_all, double* part_all) {
  int32_t* dist = dist_all + blockIdx.x * n;
  int32_t* order = order_all + blockIdx.x * n;
  int32_t* levoff = levoff_all + blockIdx.x * (n + 1);
  double* sigma = sigma_all + blockIdx.x * n;
  double* delta = delta_all + blockIdx.x * n;
  double* part = part_all + blockIdx.x * n;
  __shared__ int32_t s_cnt;
  __shared__ int32_t s_lvl[2];  // start of the current level in order, its end
  const int tid = threadIdx.x;
  for (int64_t v = tid; v < n; v += kBrThreads) part[v] = 0.0;
  for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
    for (int64_t v = tid; v < n; v += kBrThreads) {
      dist[v] = -1;
      sigma[v] = 0.0;
      delta[v] = 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      dist[s] = 0;
      sigma[s] = 1.0;
      order[0] = (int32_t)s;
      s_cnt = 1;
      s_lvl[0] = 0;
      s_lvl[1] = 1;
    }
    __syncthreads();
    // levels with path counts
    int32_t lev = 0;
    for (;;) {
      const int32_t a = s_lvl[0], b = s_lvl[1];
      if (tid == 0) levoff[lev] = a;  // level lev starts at a (ends the levels if empty)
      if (a == b) break;
      for (int32_t q = a + tid; q < b; q += kBrThreads) {
        const int32_t u = order[q];
        const double su = ld_l2(&sigma[u]);
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
          const int32_t v = col[e];
          int32_t dv = ld_l2(&dist[v]);
          if (dv < 0) {
            const int32_t old = atomicCAS(&dist[v], -1, lev + 1);
            if (old == -1) order[atomicAdd(&s_cnt, 1)] = v;
            dv = old == -1 ? lev + 1 : old;
          }
          if (dv == lev + 1) atomicAdd(&sigma[v], su);
        }
      }
      __syncthreads();
      if (tid == 0) {
        s_lvl[0] = b;
        s_lvl[1] = s_cnt;
      }
      ++lev;
      __syncthreads();
    }
    __syncthreads();
    // accumulation from the deepest level up (level l is order[levoff[l],
    // levoff[l + 1]))
    for (int32_t l = lev - 1; l >= 0; --l) {
      const int32_t lo = levoff[l], hi = levoff[l + 1];
      for (int32_t q = lo + tid; q < hi; q += kBrThreads) {
        const int32_t v = order[q];
        double acc = 0.0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
          const int32_t w = col[e];
          if (ld_l2(&dist[w]) == l + 1) acc += (1.0 + delta[w]) / ld_l2(&sigma[w]);
        }
        delta[v] = ld_l2(&sigma[v]) * acc;
        if (v != s) part[v] += delta[v];
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

// cb[v] = sum over workgroups g (in order) of part[g][v].
__global__ void k_br_sum(int64_t n, int groups, const double* part, double* cb) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * n + v];
  cb[v] = s;
}

// Sum and sum of squares about a shift, one workgroup, fixed order.
__global__ void __launch_bounds__(256) k_br_moments(int64_t n, const double* cb, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t v = threadIdx.x; v < n; v += 256) s += cb[v];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double mean = sh[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t v = threadIdx.x; v < n; v += 256) {
    const double d = cb[v] - mean;
    q += d * d;
  }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = mean;
    out[1] = sh[0] / (double)n;
  }
}

int br_groups(int64_t n) { return (int)std::min<int64_t>(n, kBrMaxGroups); }

const int kZero = 0;

}  // namespace

size_t betweenness_workspace_bytes(int64_t n) {
  const size_t g = (size_t)br_groups(n);
  return kHeapAlign +
         DevHeap::round(g * n * (4 + 4 + 8 + 8 + 8) + g * (n + 1) * 4 + 64 * 8 + 7 * kHeapAlign);
}

int betweenness(const me_csr* W, void* ws, size_t ws_bytes, double* cb, double* vbc,
                hipStream_t s) {
  if (!W || !cb || W->n < 1 || W->nnz < 0 || !W->rowptr || (W->nnz > 0 && !W->col) ||
      W->n >= (int64_t)INT32_MAX)
    return ME_ERR_INVALID_ARG;
  const int64_t n = W->n;
  if (ws && ws_bytes < betweenness_workspace_bytes(n)) return ME_ERR_WORKSPACE;
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  const int G = br_groups(n);
  void* mem = nullptr;
  const size_t bytes = betweenness_workspace_bytes(n) - kHeapAlign;
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
  Arena a{(char*)mem, bytes, 0};
  int32_t* dist = a.take<int32_t>((size_t)G * n);
  int32_t* order = a.take<int32_t>((size_t)G * n);
  int32_t* levoff = a.take<int32_t>((size_t)G * (n + 1));
  double* sigma = a.take<double>((size_t)G * n);
  double* delta = a.take<double>((size_t)G * n);
  double* part = a.take<double>((size_t)G * n);
  double* mom = a.take<double>(2);
  int* flag = a.take<int>(1);
  if (!flag) return ME_ERR_WORKSPACE;
  ME_TRY(hipMemcpyAsync(flag, &kZero, 4, hipMemcpyHostToDevice, s));
  k_br_check<<<ceil_div(n + 1, kBlock), kBlock, 0, s>>>(n, W->nnz, W->rowptr, W->col, flag);
  int h = 0;
  ME_TRY(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (h) return ME_ERR_INVALID_ARG;
  k_br_symmetric<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, W->rowptr, W->col, flag);
  ME_TRY(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (h) return ME_ERR_NOT_SYMMETRIC;
  k_brandes<<<G, kBrThreads, 0, s>>>(n, W->rowptr, W->col, dist, order, levoff, sigma, delta,
                                     part);
  k_br_sum<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, G, part, cb);
  k_br_moments<<<1, 256, 0, s>>>(n, cb, mom);
  double hm[2] = {0, 0};
  ME_TRY(hipMemcpyAsync(hm, mom, 16, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (vbc) *vbc = hm[1];
  return ME_OK;
}

}  // namespace me

extern "C" {

size_t me_betweenness_workspace_bytes(int64_t n) {
  return n < 1 ? 0 : me::betweenness_workspace_bytes(n);
}

int me_betweenness(const me_csr* W, void* ws, size_t ws_bytes, double* cb, double* vbc,
                   void* stream) {
  return me::betweenness(W, ws, ws_bytes, cb, vbc, (hipStream_t)stream);
}

}  // extern "C"
