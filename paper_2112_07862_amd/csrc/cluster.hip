// Clustering of the embedding and its criteria (Section 5.1, Table 3): the
// rows of the N x K embedding are clustered into C clusters by k-means and
// by a Gaussian mixture model, and a clustering is scored against known
// classes by the Rand index, Precision, Purity and NMI.
//
// k-means: k-means++ seeds from caller-given uniforms (the first seed is
// point floor(u_0 n); seed t is the first point whose running sum of D^2,
// the squared distance to the nearest seed so far, exceeds u_t times the
// total), then Lloyd iterations: every point joins its nearest centre (ties
// to the lower index), every centre becomes its points' mean (an empty
// cluster keeps its centre), until no point moves.
// GMM: full covariances, EM from a partition, each covariance regularised
// by reg I (reg = 1e-6 times the mean per-coordinate variance of the data),
// stopping when the log-likelihood changes by at most tol of its magnitude.
// Squared distances are summed over the coordinates in order with plain
// products, as everywhere in the library.  Every reduction has a fixed
// order (per-thread runs, a fixed tree, blocks added in order), so results
// repeat bit for bit.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace me {

namespace {

constexpr int kClMaxK = 16;   // embedding dimensions
constexpr int kClMaxC = 64;   // clusters
constexpr int kClThreads = 256;
constexpr int kClBlocks = 256;  // blocks of the fixed-order reductions
constexpr int kMom = 1 + kClMaxK + kClMaxK * (kClMaxK + 1) / 2;  // weight, first, second moments

__device__ __forceinline__ double sqd(double acc, double a, double b) {
  const double t = __dsub_rn(a, b);
  return __dadd_rn(acc, __dmul_rn(t, t));
}

// ---- fixed-order FP64 inclusive scan (k-means++ seeding) -------------------
constexpr int kScanEl = 4;
constexpr int kScanBlk = kClThreads * kScanEl;

__device__ double block_scan_f64(double v, double* sh, double* total) {
  // inclusive scan over the workgroup, Hillis-Steele in LDS (fixed order)
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kClThreads; o <<= 1) {
    const double a = t >= o ? sh[t - o] : 0.0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const double r = sh[t];
  *total = sh[kClThreads - 1];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kClThreads) k_scan_f64_tiles(int64_t n, const double* in,
                                                               double* out, double* tiles) {
  __shared__ double sh[kClThreads];
  const int64_t base = blockIdx.x * (int64_t)kScanBlk + threadIdx.x * kScanEl;
  double v[kScanEl];
  double run = 0.0;
  for (int q = 0; q < kScanEl; ++q) {
    v[q] = base + q < n ? in[base + q] : 0.0;
    run += v[q];
  }
  double tot;
  (void)block_scan_f64(run, sh, &tot);
  // the runs of the threads before this one, then this thread's elements
  double acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
  for (int q = 0; q < kScanEl; ++q) {
    acc += v[q];
    if (base + q < n) out[base + q] = acc;
  }
  if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

__global__ void k_scan_f64_carry(int64_t ntiles, double* tiles) {
  double c = 0.0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const double v = tiles[t];
    tiles[t] = c;
    c += v;
  }
}

__global__ void k_scan_f64_add(int64_t n, double* out, const double* tiles) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += tiles[i / kScanBlk];
}

// ---- k-means++ -------------------------------------------------------------
__global__ void k_pp_dist(int64_t n, int K, const double* x, const int32_t* seed, double* d2,
                          int first) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = *seed;
  double a = 0.0;
  for (int k = 0; k < K; ++k) a = sqd(a, x[i * K + k], x[s * K + k]);
  d2[i] = first ? a : fmin(d2[i], a);
}

// The first point whose running sum exceeds u times the total (one
// workgroup; the running sums are non-decreasing).
__global__ void __launch_bounds__(kClThreads) k_pp_pick(int64_t n, const double* cs, double u,
                                                        int32_t* seed) {
  __shared__ int64_t s_first;
  if (threadIdx.x == 0) s_first = n - 1;
  __syncthreads();
  const double target = u * cs[n - 1];
  // binary search by one thread
  if (threadIdx.x == 0) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (cs[mid] > target) hi = mid; else lo = mid + 1;
    }
    s_first = lo < n ? lo : n - 1;
    *seed = (int32_t)s_first;
  }
}

__global__ void k_gather_rows(int C, int K, const double* x, const int32_t* idx, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < C * K) out[t] = x[(int64_t)idx[t / K] * K + t % K];
}

// ---- Lloyd ------------------------------------------------------------------
__global__ void __launch_bounds__(kClThreads) k_assign(int64_t n, int K, int C, const double* x,
                                                       const double* cen, int32_t* labels,
                                                       int* changed, int first) {
  __shared__ double sc[kClMaxC * kClMaxK];
  for (int t = threadIdx.x; t < C * K; t += kClThreads) sc[t] = cen[t];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)kClThreads + threadIdx.x;
  if (i >= n) return;
  double xi[kClMaxK];
  for (int k = 0; k < K; ++k) xi[k] = x[i * K + k];
  double best = INFINITY;
  int bc = 0;
  for (int c = 0; c < C; ++c) {
    double a = 0.0;
    for (int k = 0; k < K; ++k) a = sqd(a, xi[k], sc[c * K + k]);
    if (a < best) {
      best = a;
      bc = c;
    }
  }
  if (!first && labels[i] != bc) atomicAdd(changed, 1);
  labels[i] = bc;
}

// Fixed-order moments per cluster: block b, cluster blockIdx.y sums its
// points of a strided run per thread, then a tree in LDS.  mode 0: count
// and sums of x; mode 1: also sums of (x - m)(x - m)^T (upper triangle) about
// m = mean[c]; weights w (n x C, may be null: hard labels).
__global__ void __launch_bounds__(kClThreads) k_moments(int64_t n, int K, int C, const double* x,
                                                        const int32_t* labels, const double* w,
                                                        const double* mean, int mode,
                                                        double* part) {
  const int c = blockIdx.y;
  const int M = 1 + K + (mode ? K * (K + 1) / 2 : 0);
  double acc[kMom];
  for (int q = 0; q < M; ++q) acc[q] = 0.0;
  double m[kClMaxK];
  if (mode)
    for (int k = 0; k < K; ++k) m[k] = mean[c * K + k];
  for (int64_t i = blockIdx.x * (int64_t)kClThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kClThreads) {
    double r;
    if (w) r = w[i * C + c];
    else r = labels[i] == c ? 1.0 : 0.0;
    if (r == 0.0) continue;
    acc[0] += r;
    double xi[kClMaxK];
    for (int k = 0; k < K; ++k) {
      xi[k] = x[i * K + k];
      acc[1 + k] += r * xi[k];
    }
    if (mode) {
      int q = 1 + K;
      for (int a = 0; a < K; ++a) {
        const double da = xi[a] - m[a];
        for (int b = a; b < K; ++b) acc[q++] += r * da * (xi[b] - m[b]);
      }
    }
  }
  __shared__ double sh[kClThreads];
  for (int q = 0; q < M; ++q) {
    sh[threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = kClThreads / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)c * gridDim.x + blockIdx.x) * kMom + q] = sh[0];
    __syncthreads();
  }
}

// mom[c][q] = sum over blocks (in order) of part[c][b][q].
__global__ void k_moments_sum(int C, int blocks, int M, const double* part, double* mom) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C * M) return;
  const int c = t / M, q = t % M;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += part[((int64_t)c * blocks + b) * kMom + q];
  mom[c * kMom + q] = s;
}

// centres from the moments; an empty cluster keeps its centre.
__global__ void k_centres(int C, int K, const double* mom, double* cen) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C * K) return;
  const int c = t / K, k = t % K;
  const double cnt = mom[c * kMom];
  if (cnt > 0.0) cen[t] = mom[c * kMom + 1 + k] / cnt;
}

// ---- GMM ----------------------------------------------------------------------
// per-coordinate mean and population variance of the data -> reg (one
// workgroup per coordinate, fixed order)
__global__ void __launch_bounds__(kClThreads) k_col_var(int64_t n, int K, const double* x,
                                                        double* var) {
  __shared__ double sh[kClThreads];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kClThreads) s += x[i * K + k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kClThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double mean = sh[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kClThreads) {
    const double d = x[i * K + k] - mean;
    q += d * d;
  }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int o = kClThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) var[k] = sh[0] / (double)n;
}

// Parameters from the moments (mode 1 moments about the new means):
// weights, means, covariances + reg I, and each covariance's Cholesky
// factor and log-determinant.  One thread per component.  init: from a
// partition (hard moments, divisor max(count, 1), the data mean for an
// empty cluster); otherwise the M-step (components with no weight keep
// their parameters).
__global__ void k_gmm_params(int C, int K, int64_t n, const double* mom_cov, const double* var,
                             int init, double* wts, double* cov, double* chol, double* logdet,
                             int* bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double reg = 0.0;
  for (int k = 0; k < K; ++k) reg += var[k];
  reg = 1e-6 * (reg / (double)K);
  const double nk = mom_cov[c * kMom];
  const bool have = nk > 0.0;
  wts[c] = fmax(nk / (double)n, 1e-300);
  if (init || have) {
    const double div = init ? fmax(nk, 1.0) : nk;
    int q = 1 + K;
    for (int a = 0; a < K; ++a)
      for (int b = a; b < K; ++b) {
        const double v = mom_cov[c * kMom + q++] / div + (a == b ? reg : 0.0);
        cov[(c * K + a) * K + b] = v;
        cov[(c * K + b) * K + a] = v;
      }
  }
  // Cholesky, lower, in the component's chol block
  double* L = chol + (int64_t)c * K * K;
  const double* S = cov + (int64_t)c * K * K;
  double ld = 0.0;
  for (int j = 0; j < K; ++j) {
    double d = S[j * K + j];
    for (int p = 0; p < j; ++p) d -= L[j * K + p] * L[j * K + p];
    if (!(d > 0.0)) {
      atomicOr(bad, 1);
      d = 1e-300;
    }
    const double ljj = sqrt(d);
    L[j * K + j] = ljj;
    ld += log(ljj);
    for (int i = j + 1; i < K; ++i) {
      double v = S[i * K + j];
      for (int p = 0; p < j; ++p) v -= L[i * K + p] * L[j * K + p];
      L[i * K + j] = v / ljj;
    }
    for (int i = 0; i < j; ++i) L[i * K + j] = 0.0;
  }
  logdet[c] = 2.0 * ld;
}

__global__ void k_gmm_means(int C, int K, const double* mom, const double* datamean, int init,
                            double* mu) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C * K) return;
  const int c = t / K, k = t % K;
  const double nk = mom[c * kMom];
  if (nk > 0.0) mu[t] = mom[c * kMom + 1 + k] / nk;
  else if (init) mu[t] = datamean[k];
}

// E-step: responsibilities r (n x C), each point's log-sum-exp s, the most
// responsible component.
__global__ void __launch_bounds__(kClThreads) k_gmm_estep(int64_t n, int K, int C, const double* x,
                                                          const double* wts, const double* mu,
                                                          const double* chol,
                                                          const double* logdet, double* r,
                                                          double* s_out, int32_t* labels) {
  const int64_t i = blockIdx.x * (int64_t)kClThreads + threadIdx.x;
  if (i >= n) return;
  double xi[kClMaxK];
  for (int k = 0; k < K; ++k) xi[k] = x[i * K + k];
  const double l2pi = log(2.0 * M_PI);
  double lg[kClMaxC];
  double mx = -INFINITY;
  int arg = 0;
  for (int c = 0; c < C; ++c) {
    const double* L = chol + (int64_t)c * K * K;
    double y[kClMaxK];
    double q = 0.0;
    for (int a = 0; a < K; ++a) {
      double v = xi[a] - mu[c * K + a];
      for (int p = 0; p < a; ++p) v -= L[a * K + p] * y[p];
      y[a] = v / L[a * K + a];
      q += y[a] * y[a];
    }
    const double g = -0.5 * ((double)K * l2pi + logdet[c] + q) + log(wts[c]);
    lg[c] = g;
    if (g > mx) {
      mx = g;
      arg = c;
    }
  }
  double se = 0.0;
  for (int c = 0; c < C; ++c) se += exp(lg[c] - mx);
  const double s = log(se) + mx;
  for (int c = 0; c < C; ++c) r[i * C + c] = exp(lg[c] - s);
  s_out[i] = s;
  labels[i] = arg;
}

__global__ void __launch_bounds__(kClThreads) k_sum_f64(int64_t n, const double* v, double* out) {
  __shared__ double sh[kClThreads];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kClThreads) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kClThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_fill_i32(int64_t n, int32_t* a, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---- criteria -------------------------------------------------------------------
constexpr int kClMaxLabels = 256;
__global__ void k_contingency(int64_t n, const int32_t* a, const int32_t* b, int nb,
                              unsigned long long* t, int* bad, int na) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t u = a[i], v = b[i];
  if (u < 0 || u >= na || v < 0 || v >= nb) {
    atomicOr(bad, 1);
    return;
  }
  atomicAdd(&t[(int64_t)u * nb + v], 1ull);
}

__global__ void k_criteria(int na, int nb, int64_t n, const unsigned long long* t, double* out) {
  auto pairs = [](double v) { return v * (v - 1.0) / 2.0; };
  double as[kClMaxLabels], bs[kClMaxLabels];
  double tp = 0.0, ppred = 0.0, ptrue = 0.0, purity = 0.0, mi = 0.0, ha = 0.0, hb = 0.0;
  const double dn = (double)n;
  for (int j = 0; j < nb; ++j) bs[j] = 0.0;
  for (int i = 0; i < na; ++i) {
    double ai = 0.0;
    for (int j = 0; j < nb; ++j) {
      const double v = (double)t[i * nb + j];
      ai += v;
      bs[j] += v;
      tp += pairs(v);
    }
    as[i] = ai;
    ptrue += pairs(ai);
    if (ai > 0) ha -= (ai / dn) * log(ai / dn);
  }
  for (int j = 0; j < nb; ++j) {
    double mx = 0.0;
    for (int i = 0; i < na; ++i) mx = fmax(mx, (double)t[i * nb + j]);
    ppred += pairs(bs[j]);
    purity += mx;
    if (bs[j] > 0) hb -= (bs[j] / dn) * log(bs[j] / dn);
  }
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      const double v = (double)t[i * nb + j];
      if (v <= 0) continue;
      const double pij = v / dn;
      mi += pij * log(pij / ((as[i] / dn) * (bs[j] / dn)));
    }
  const double tot = pairs(dn);
  out[0] = (tot - ppred - ptrue + 2.0 * tp) / tot;
  out[1] = ppred > 0 ? tp / ppred : 0.0;
  out[2] = purity / dn;
  out[3] = (ha == 0.0 && hb == 0.0) ? 1.0 : ((ha == 0.0 || hb == 0.0) ? 0.0 : mi / sqrt(ha * hb));
}

struct ClScratch {
  double *d2, *cs, *tiles, *cen0, *part, *mom, *mom2, *var, *dmean, *r, *s, *ll, *chol, *logdet;
  int32_t *seeds, *lab;
  int* flag;
};

size_t cl_scratch(int64_t n, int K, int C, ClScratch* out, char* base) {
  Arena a{base, (size_t)-1, 0};
  ClScratch sc{};
  sc.d2 = a.take<double>(n);
  sc.cs = a.take<double>(n);
  sc.tiles = a.take<double>(ceil_div(n, kScanBlk) + 1);
  sc.cen0 = a.take<double>((size_t)C * K);
  sc.part = a.take<double>((size_t)C * kClBlocks * kMom);
  sc.mom = a.take<double>((size_t)C * kMom);
  sc.mom2 = a.take<double>((size_t)C * kMom);
  sc.var = a.take<double>(kClMaxK);
  sc.dmean = a.take<double>(kClMaxK);
  sc.r = a.take<double>((size_t)n * C);
  sc.s = a.take<double>(n);
  sc.ll = a.take<double>(1);
  sc.chol = a.take<double>((size_t)C * K * K);
  sc.logdet = a.take<double>(C);
  sc.seeds = a.take<int32_t>(C);
  sc.lab = a.take<int32_t>(n);
  sc.flag = a.take<int>(4);
  if (out) *out = sc;
  return a.used;
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kClThreads)); }

void moments(int64_t n, int K, int C, const double* x, const int32_t* lab, const double* w,
             const double* mean, int mode, const ClScratch& sc, double* mom, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(kClBlocks, std::max<int64_t>(1, ceil_div(n, kClThreads)));
  k_moments<<<dim3(blocks, C), kClThreads, 0, s>>>(n, K, C, x, lab, w, mean, mode, sc.part);
  const int M = 1 + K + (mode ? K * (K + 1) / 2 : 0);
  k_moments_sum<<<(unsigned)ceil_div(C * M, 256), 256, 0, s>>>(C, blocks, M, sc.part, mom);
}

const int kZeroI = 0;

}  // namespace

size_t cluster_workspace_bytes(int64_t n, int K, int C) {
  return kHeapAlign + DevHeap::round(cl_scratch(n, K, C, nullptr, nullptr));
}

static int cl_args(const double* x, int64_t n, int K, int C) {
  if (!x || n < 2 || n >= (int64_t)INT32_MAX || K < 1 || K > kClMaxK || C < 1 || C > kClMaxC ||
      C > n)
    return ME_ERR_INVALID_ARG;
  return ME_OK;
}

int kmeans(const double* x, int64_t n, int K, int C, const double* u, int max_iter, void* ws,
           size_t ws_bytes, int32_t* labels, double* centres, int* iters, hipStream_t s) {
  ME_TRY_STATUS(cl_args(x, n, K, C));
  if (!u || !labels || !centres || max_iter < 1) return ME_ERR_INVALID_ARG;
  for (int t = 0; t < C; ++t)
    if (!(u[t] >= 0.0 && u[t] < 1.0)) return ME_ERR_INVALID_ARG;
  if (ws && ws_bytes < cluster_workspace_bytes(n, K, C)) return ME_ERR_WORKSPACE;
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  const size_t bytes = cl_scratch(n, K, C, nullptr, nullptr);
  void* mem = nullptr;
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
  ClScratch sc;
  cl_scratch(n, K, C, &sc, (char*)mem);
  // k-means++ seeds
  const int32_t first = (int32_t)std::min<int64_t>((int64_t)std::floor(u[0] * (double)n), n - 1);
  ME_TRY(hipMemcpyAsync(sc.seeds, &first, 4, hipMemcpyHostToDevice, s));
  k_pp_dist<<<grid_of(n), kClThreads, 0, s>>>(n, K, x, sc.seeds, sc.d2, 1);
  const int64_t nt = ceil_div(n, kScanBlk);
  for (int t = 1; t < C; ++t) {
    k_scan_f64_tiles<<<(unsigned)nt, kClThreads, 0, s>>>(n, sc.d2, sc.cs, sc.tiles);
    k_scan_f64_carry<<<1, 1, 0, s>>>(nt, sc.tiles);
    k_scan_f64_add<<<grid_of(n), kClThreads, 0, s>>>(n, sc.cs, sc.tiles);
    k_pp_pick<<<1, kClThreads, 0, s>>>(n, sc.cs, u[t], sc.seeds + t);
    k_pp_dist<<<grid_of(n), kClThreads, 0, s>>>(n, K, x, sc.seeds + t, sc.d2, 0);
  }
  k_gather_rows<<<(unsigned)ceil_div(C * K, 256), 256, 0, s>>>(C, K, x, sc.seeds, centres);
  // Lloyd
  k_assign<<<grid_of(n), kClThreads, 0, s>>>(n, K, C, x, centres, labels, sc.flag, 1);
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    moments(n, K, C, x, labels, nullptr, nullptr, 0, sc, sc.mom, s);
    k_centres<<<(unsigned)ceil_div(C * K, 256), 256, 0, s>>>(C, K, sc.mom, centres);
    ME_TRY(hipMemcpyAsync(sc.flag, &kZeroI, 4, hipMemcpyHostToDevice, s));
    k_assign<<<grid_of(n), kClThreads, 0, s>>>(n, K, C, x, centres, labels, sc.flag, 0);
    int changed = 0;
    ME_TRY(hipMemcpyAsync(&changed, sc.flag, 4, hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
    if (changed == 0) break;
  }
  if (iters) *iters = std::min(it, max_iter);
  return ME_OK;
}

int gmm(const double* x, int64_t n, int K, int C, const int32_t* labels0, int max_iter, double tol,
        void* ws, size_t ws_bytes, int32_t* labels, double* wts, double* mu, double* cov,
        double* loglik, int* iters, hipStream_t s) {
  ME_TRY_STATUS(cl_args(x, n, K, C));
  if (!labels0 || !labels || !wts || !mu || !cov || max_iter < 1 || !(tol >= 0.0))
    return ME_ERR_INVALID_ARG;
  if (ws && ws_bytes < cluster_workspace_bytes(n, K, C)) return ME_ERR_WORKSPACE;
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  const size_t bytes = cl_scratch(n, K, C, nullptr, nullptr);
  void* mem = nullptr;
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
  ClScratch sc;
  cl_scratch(n, K, C, &sc, (char*)mem);
  ME_TRY(hipMemcpyAsync(sc.flag, &kZeroI, 4, hipMemcpyHostToDevice, s));
  // data mean and variance (reg), the partition's parameters
  k_col_var<<<K, kClThreads, 0, s>>>(n, K, x, sc.var);
  // the data mean (for an empty cluster of the partition): the moments of
  // one cluster holding every point
  k_fill_i32<<<grid_of(n), kClThreads, 0, s>>>(n, sc.lab, 0);
  moments(n, K, 1, x, sc.lab, nullptr, nullptr, 0, sc, sc.mom2, s);
  k_centres<<<1, 256, 0, s>>>(1, K, sc.mom2, sc.dmean);
  moments(n, K, C, x, labels0, nullptr, nullptr, 0, sc, sc.mom, s);
  k_gmm_means<<<(unsigned)ceil_div(C * K, 256), 256, 0, s>>>(C, K, sc.mom, sc.dmean, 1, mu);
  moments(n, K, C, x, labels0, nullptr, mu, 1, sc, sc.mom2, s);
  k_gmm_params<<<1, kClMaxC, 0, s>>>(C, K, n, sc.mom2, sc.var, 1, wts, cov, sc.chol, sc.logdet,
                                     sc.flag);
  double prev = 0.0, ll = -INFINITY;
  bool have_prev = false;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    k_gmm_estep<<<grid_of(n), kClThreads, 0, s>>>(n, K, C, x, wts, mu, sc.chol, sc.logdet, sc.r,
                                                  sc.s, labels);
    k_sum_f64<<<1, kClThreads, 0, s>>>(n, sc.s, sc.ll);
    int bad = 0;
    ME_TRY(hipMemcpyAsync(&ll, sc.ll, 8, hipMemcpyDeviceToHost, s));
    ME_TRY(hipMemcpyAsync(&bad, sc.flag, 4, hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
    if (bad || !std::isfinite(ll)) return ME_ERR_BREAKDOWN;
    if (have_prev && std::fabs(ll - prev) <= tol * std::fabs(ll)) break;
    prev = ll;
    have_prev = true;
    // M-step: weights and means, then covariances about the new means
    moments(n, K, C, x, nullptr, sc.r, nullptr, 0, sc, sc.mom, s);
    k_gmm_means<<<(unsigned)ceil_div(C * K, 256), 256, 0, s>>>(C, K, sc.mom, sc.dmean, 0, mu);
    moments(n, K, C, x, nullptr, sc.r, mu, 1, sc, sc.mom2, s);
    k_gmm_params<<<1, kClMaxC, 0, s>>>(C, K, n, sc.mom2, sc.var, 0, wts, cov, sc.chol,
                                       sc.logdet, sc.flag);
  }
  if (it > max_iter) {
    // out of iterations: the labels of the last parameters
    k_gmm_estep<<<grid_of(n), kClThreads, 0, s>>>(n, K, C, x, wts, mu, sc.chol, sc.logdet, sc.r,
                                                  sc.s, labels);
    it = max_iter;
  }
  ME_TRY(hipStreamSynchronize(s));
  if (loglik) *loglik = ll;
  if (iters) *iters = it;
  return ME_OK;
}

int cluster_scores(const int32_t* classes, const int32_t* clusters, int64_t n, int na, int nb,
                   void* ws, size_t ws_bytes, double* scores, hipStream_t s) {
  if (!classes || !clusters || !scores || n < 2 || na < 1 || nb < 1 || na > kClMaxLabels ||
      nb > kClMaxLabels)
    return ME_ERR_INVALID_ARG;
  const size_t bytes = (size_t)na * nb * 8 + 64;
  if (ws && ws_bytes < kHeapAlign + DevHeap::round(bytes)) return ME_ERR_WORKSPACE;
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  void* mem = nullptr;
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
  auto* t = (unsigned long long*)mem;
  int* bad = (int*)((char*)mem + (size_t)na * nb * 8);
  double* out = (double*)((char*)mem + (size_t)na * nb * 8 + 16);
  std::vector<unsigned long long> z((size_t)na * nb, 0ull);
  ME_TRY(hipMemcpyAsync(t, z.data(), z.size() * 8, hipMemcpyHostToDevice, s));
  ME_TRY(hipMemcpyAsync(bad, &kZeroI, 4, hipMemcpyHostToDevice, s));
  k_contingency<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, classes, clusters, nb, t, bad, na);
  k_criteria<<<1, 1, 0, s>>>(na, nb, n, t, out);
  int hb = 0;
  ME_TRY(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, s));
  ME_TRY(hipMemcpyAsync(scores, out, 32, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (hb) return ME_ERR_INVALID_ARG;
  return ME_OK;
}

}  // namespace me

extern "C" {

size_t me_cluster_workspace_bytes(int64_t n, int K, int C) {
  if (n < 2 || K < 1 || C < 1) return 0;
  // also covers me_cluster_scores with up to 256 classes and clusters
  return std::max(me::cluster_workspace_bytes(n, K, C),
                  me::kHeapAlign + me::DevHeap::round((size_t)256 * 256 * 8 + 64));
}

int me_kmeans(const double* X, int64_t n, int K, int C, const double* u, int max_iter, void* ws,
              size_t ws_bytes, int32_t* labels, double* centres, int* iters, void* stream) {
  return me::kmeans(X, n, K, C, u, max_iter, ws, ws_bytes, labels, centres, iters,
                    (hipStream_t)stream);
}

int me_gmm(const double* X, int64_t n, int K, int C, const int32_t* labels0, int max_iter,
           double tol, void* ws, size_t ws_bytes, int32_t* labels, double* weights, double* means,
           double* covs, double* loglik, int* iters, void* stream) {
  return me::gmm(X, n, K, C, labels0, max_iter, tol, ws, ws_bytes, labels, weights, means, covs,
                 loglik, iters, (hipStream_t)stream);
}

int me_cluster_scores(const int32_t* classes, const int32_t* clusters, int64_t n, int n_classes,
                      int n_clusters, void* ws, size_t ws_bytes, double* scores, void* stream) {
  return me::cluster_scores(classes, clusters, n, n_classes, n_clusters, ws, ws_bytes, scores,
                            (hipStream_t)stream);
}

}  // extern "C"
