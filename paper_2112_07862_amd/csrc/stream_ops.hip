// N-length (HBM-bound) kernels of the LOBPCG iteration.
//
// Blocks X, W, P, AX, AW, AP are row-major n x kb (kb in {4, 8, 16}).  A
// group of LPR = kb / VEC lanes owns one row, each lane VEC consecutive
// columns loaded as one 16-byte vector (VEC = 2 doubles or 4 floats), so a
// wave reads whole rows with fully coalesced 16-byte accesses.
//
// Difference-form operator (eq. (obj2) with the Laplacian identity of
// Section 3.1): with the merged row [W columns | T columns],
//   (A x)_i = sum_{j in N(i)} w_ij (x_i - x_j)
//             - mu sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j) + eps x_i
//   (Q x)_i = sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j)
// The diagonal is never stored; the differences x_i - x_j keep the rounding
// error proportional to the local variation of x rather than to |A| |x|.
#include <cmath>

#include "common.h"

namespace me {

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

template <typename T, int KB>
struct Lay {
  static constexpr int VEC = (16 / (int)sizeof(T)) < KB ? (16 / (int)sizeof(T)) : KB;
  static constexpr int LPR = KB / VEC;  // lanes per row
  using Vec = VecT<T, VEC>;
};

template <typename T, int V>
__device__ inline VecT<T, V> ldv(const T* p) {
  return *reinterpret_cast<const VecT<T, V>*>(p);
}
template <typename T, int V>
__device__ inline void stv(T* p, const VecT<T, V>& v) {
  *reinterpret_cast<VecT<T, V>*>(p) = v;
}

#define ME_DISPATCH_KB(kb, ...)                       \
  switch (kb) {                                       \
    case 4: { constexpr int KB = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int KB = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int KB = 16; __VA_ARGS__; } break; \
    default: break;                                   \
  }

// ---------------------------------------------------------------------------
// SpMM: Y = Op X in difference form
// ---------------------------------------------------------------------------

// Row i of the product, without the diagonal term.  A group of G
// consecutive lanes owns one row and splits the row's entries: lane q takes
// entries q, q + G, q + 2G, ..., loads their columns and weights (coalesced
// over the group), gathers the neighbour rows x_j whole (KB values, 16-byte
// loads) UNR at a time, and accumulates the full row; a butterfly over the
// group leaves the sum in every lane.  Entries before a_split are W entries
// (weight w_ij), the rest T entries (weight c_t (1/T_i + 1/T_j)).  All
// lanes of the wave must call it (shuffles).
template <typename T, int KB>
struct RowCfg {
  static constexpr int G = 8;                                  // lanes per row
  static constexpr int UNR = (KB * sizeof(T) >= 128) ? 2 : 4;  // entries in flight per lane
  static constexpr int V16 = 16 / sizeof(T);                   // values per 16-byte load
  static constexpr int NLD = KB * sizeof(T) / 16;              // 16-byte loads per row
};

template <typename T, int KB>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[KB]) {
  using C = RowCfg<T, KB>;
#pragma unroll
  for (int l = 0; l < C::NLD; ++l) {
    const auto t = ldv<T, C::V16>(p + l * C::V16);
#pragma unroll
    for (int q = 0; q < C::V16; ++q) v[l * C::V16 + q] = t.v[q];
  }
}

template <typename T, int KB>
__device__ __forceinline__ void spmm_row(bool live, int64_t row, int q,
                                         const int32_t* __restrict__ a_rp,
                                         const int32_t* __restrict__ a_split,
                                         const int32_t* __restrict__ a_col,
                                         const T* __restrict__ a_w, const T* __restrict__ invt,
                                         T c_t, int skip_w, const T* __restrict__ x,
                                         const T (&xi)[KB], T (&acc)[KB]) {
  using C = RowCfg<T, KB>;
  constexpr int G = C::G, UNR = C::UNR;
  int32_t s = 0, sp = 0, e = 0;
  T ti = 0;
  if (live) {
    s = skip_w ? a_split[row] : a_rp[row];
    sp = a_split[row];
    e = a_rp[row + 1];
    ti = invt[row];
  }
#pragma unroll
  for (int v = 0; v < KB; ++v) acc[v] = 0;
  // steps of G entries; loop to the wave's longest row
  int32_t steps = (e - s + G - 1) / G;
  for (int o = kWave / 2; o > 0; o >>= 1) steps = max(steps, __shfl_xor(steps, o));
  for (int32_t st = 0; st < steps; st += UNR) {
    int32_t c[UNR];
    T cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = s + (st + u) * G + q;
      const bool ok = k < e;
      c[u] = ok ? a_col[k] : -1;
      cf[u] = (ok && k < sp) ? a_w[k] : (T)0;
    }
    T xj[UNR][KB];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = s + (st + u) * G + q;
      if (c[u] >= 0) {
        load_row<T, KB>(x + (int64_t)c[u] * KB, xj[u]);
        if (k >= sp) cf[u] = c_t * (ti + invt[c[u]]);
      } else {
#pragma unroll
        for (int v = 0; v < KB; ++v) xj[u][v] = xi[v];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int v = 0; v < KB; ++v) acc[v] += cf[u] * (xi[v] - xj[u][v]);
  }
#pragma unroll
  for (int v = 0; v < KB; ++v)
    for (int o = G / 2; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
}

// Y = Op X: G lanes per row; lane q < KB / V16 writes the q-th 16-byte
// slice of the row.
template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_spmm(int64_t n, const int32_t* __restrict__ a_rp,
                                                 const int32_t* __restrict__ a_split,
                                                 const int32_t* __restrict__ a_col,
                                                 const T* __restrict__ a_w,
                                                 const T* __restrict__ invt, T c_t, T s_diag,
                                                 int skip_w, const T* __restrict__ x,
                                                 T* __restrict__ y, const int* done) {
  using C = RowCfg<T, KB>;
  if (done && *done) return;
  const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t row = gt / C::G;
  const int q = (int)(gt % C::G);
  const bool live = row < n;
  T xi[KB];
#pragma unroll
  for (int v = 0; v < KB; ++v) xi[v] = 0;
  if (live) load_row<T, KB>(x + row * KB, xi);
  T acc[KB];
  spmm_row<T, KB>(live, row, q, a_rp, a_split, a_col, a_w, invt, c_t, skip_w, x, xi, acc);
  if (!live) return;
#pragma unroll
  for (int l = 0; l < C::NLD; ++l) {
    if (q == l) {
      VecT<T, C::V16> out;
#pragma unroll
      for (int v = 0; v < C::V16; ++v) out.v[v] = acc[l * C::V16 + v] + s_diag * xi[l * C::V16 + v];
      stv<T, C::V16>(y + row * KB + l * C::V16, out);
    }
  }
}

// Chebyshev iteration for Op y = R with diagonal scaling D (spectrum of
// D^-1 Op in [a, b], theta = (a + b) / 2): y_1 = D^-1 R / theta = dd_1, then
// y_{k+1} = y_k + dd_{k+1}, dd_{k+1} = alpha_k dd_k + beta_k D^-1 (R - Op y_k).
template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_cheb_first(int64_t n, const T* __restrict__ r,
                                                       const T* __restrict__ dinv,
                                                       const Ctrl* ctrl, T* __restrict__ y,
                                                       T* __restrict__ dd) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR;
  if (ctrl->done) return;
  const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t row = gt / LPR;
  const int sub = (int)(gt % LPR);
  if (row >= n) return;
  const T sc = (T)(1.0 / ctrl->cheb_theta) * dinv[row];
  auto v = ldv<T, VEC>(r + row * KB + sub * VEC);
#pragma unroll
  for (int q = 0; q < VEC; ++q) v.v[q] *= sc;
  stv<T, VEC>(y + row * KB + sub * VEC, v);
  stv<T, VEC>(dd + row * KB + sub * VEC, v);
}

template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_cheb_step(
    int64_t n, const int32_t* __restrict__ a_rp, const int32_t* __restrict__ a_split,
    const int32_t* __restrict__ a_col, const T* __restrict__ a_w, const T* __restrict__ invt,
    T c_t, T s_diag, int skip_w, const T* __restrict__ r, const T* __restrict__ dinv, int k,
    const Ctrl* ctrl, const T* __restrict__ yin, T* __restrict__ yout, T* __restrict__ dd) {
  using C = RowCfg<T, KB>;
  if (ctrl->done) return;
  const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t row = gt / C::G;
  const int q = (int)(gt % C::G);
  const bool live = row < n;
  T yi[KB];
#pragma unroll
  for (int v = 0; v < KB; ++v) yi[v] = 0;
  if (live) load_row<T, KB>(yin + row * KB, yi);
  T acc[KB];
  spmm_row<T, KB>(live, row, q, a_rp, a_split, a_col, a_w, invt, c_t, skip_w, yin, yi, acc);
  if (!live || q >= C::NLD) return;
  const T alpha = (T)ctrl->cheb_alpha[k], beta = (T)ctrl->cheb_beta[k] * dinv[row];
#pragma unroll
  for (int l = 0; l < C::NLD; ++l) {
    if (q == l) {
      const int64_t o = row * KB + l * C::V16;
      const auto ri = ldv<T, C::V16>(r + o);
      auto di = ldv<T, C::V16>(dd + o);
      VecT<T, C::V16> yo;
#pragma unroll
      for (int v = 0; v < C::V16; ++v) {
        const int c = l * C::V16 + v;
        const T res = ri.v[v] - (acc[c] + s_diag * yi[c]);
        di.v[v] = alpha * di.v[v] + beta * res;
        yo.v[v] = yi[c] + di.v[v];
      }
      stv<T, C::V16>(dd + o, di);
      stv<T, C::V16>(yout + o, yo);
    }
  }
}

template <typename T>
struct OpArrays;
template <>
struct OpArrays<double> {
  static const double* w(const GraphOps& g) { return g.a_w; }
  static const double* invt(const GraphOps& g) { return g.invt_s; }
};
template <>
struct OpArrays<float> {
  static const float* w(const GraphOps& g) { return g.a_w32; }
  static const float* invt(const GraphOps& g) { return g.invt32_s; }
};

template <typename T>
void launch_spmm(const GraphOps& g, int kb, OpKind op, const T* x, T* y, const int* done,
                 hipStream_t s) {
  const T c_t = op == OP_A ? (T)(-g.mu) : (T)1;
  const T s_diag = op == OP_A ? (T)g.eps : (T)0;
  const int skip_w = op == OP_Q;
  ME_DISPATCH_KB(kb, {
    const int64_t grid = ceil_div(g.n * RowCfg<T, KB>::G, kBlock);
    k_spmm<T, KB><<<grid, kBlock, 0, s>>>(g.n, g.a_rp, g.a_split, g.a_col, OpArrays<T>::w(g),
                                          OpArrays<T>::invt(g), c_t, s_diag, skip_w, x, y, done);
  });
}
template void launch_spmm<double>(const GraphOps&, int, OpKind, const double*, double*,
                                  const int*, hipStream_t);

// Chebyshev preconditioner steps (see k_cheb_first / k_cheb_step).
template <typename T>
void launch_cheb_first(const GraphOps& g, int kb, const T* r, const T* dinv, const Ctrl* ctrl,
                       T* y, T* dd, hipStream_t s) {
  ME_DISPATCH_KB(kb, {
    constexpr int LPR = Lay<T, KB>::LPR;
    k_cheb_first<T, KB><<<ceil_div(g.n * LPR, kBlock), kBlock, 0, s>>>(g.n, r, dinv, ctrl, y, dd);
  });
}
template <typename T>
void launch_cheb_step(const GraphOps& g, int kb, OpKind op, int k, const T* r, const T* dinv,
                      const Ctrl* ctrl, const T* yin, T* yout, T* dd, hipStream_t s) {
  const T c_t = op == OP_A ? (T)(-g.mu) : (T)1;
  const T s_diag = op == OP_A ? (T)g.eps : (T)0;
  const int skip_w = op == OP_Q;
  ME_DISPATCH_KB(kb, {
    k_cheb_step<T, KB><<<ceil_div(g.n * RowCfg<T, KB>::G, kBlock), kBlock, 0, s>>>(
        g.n, g.a_rp, g.a_split, g.a_col, OpArrays<T>::w(g), OpArrays<T>::invt(g), c_t, s_diag,
        skip_w, r, dinv, k, ctrl, yin, yout, dd);
  });
}
template void launch_cheb_first<double>(const GraphOps&, int, const double*, const double*,
                                        const Ctrl*, double*, double*, hipStream_t);
template void launch_cheb_first<float>(const GraphOps&, int, const float*, const float*,
                                       const Ctrl*, float*, float*, hipStream_t);
template void launch_cheb_step<double>(const GraphOps&, int, OpKind, int, const double*,
                                       const double*, const Ctrl*, const double*, double*,
                                       double*, hipStream_t);
template void launch_cheb_step<float>(const GraphOps&, int, OpKind, int, const float*,
                                      const float*, const Ctrl*, const float*, float*, float*,
                                      hipStream_t);
template void launch_spmm<float>(const GraphOps&, int, OpKind, const float*, float*, const int*,
                                 hipStream_t);

// ---------------------------------------------------------------------------
// Residual R = AX - B X Lambda; W = R (precond 0) or W = D^-1 R (precond 1,
// Jacobi); per block: column sums of |r|^2, |B x|^2 and x^T D x (double)
// (partials: 3 kb entries per block).
// ---------------------------------------------------------------------------

template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_resid(int64_t n, const T* __restrict__ x,
                                                  const T* __restrict__ ax,
                                                  const T* __restrict__ bdiag,
                                                  const T* __restrict__ dinv, int precond,
                                                  const double* __restrict__ lam, T* w,
                                                  double* partials, const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR;
  constexpr int NE = 3 * KB;
  __shared__ double sh[kBlock / kWave][NE];
  if (done && *done) return;
  const int tid = threadIdx.x;
  const int sub = tid % LPR;
  double r2[VEC], b2[VEC], xd[VEC];
  T lm[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) { r2[v] = 0; b2[v] = 0; xd[v] = 0; lm[v] = (T)lam[sub * VEC + v]; }
  const int64_t total = n * LPR;
  for (int64_t g = blockIdx.x * (int64_t)kBlock + tid; g < total;
       g += (int64_t)gridDim.x * kBlock) {
    const int64_t row = g / LPR;
    const auto xi = ldv<T, VEC>(x + row * KB + sub * VEC);
    const auto ai = ldv<T, VEC>(ax + row * KB + sub * VEC);
    const T bi = bdiag ? bdiag[row] : (T)1;
    const T dv = dinv[row];
    const T di = precond == 1 ? dv : (T)1;
    const double rdv = 1.0 / (double)dv;
    typename L::Vec wv;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const T bx = bi * xi.v[v];
      const T r = ai.v[v] - lm[v] * bx;
      r2[v] += (double)r * (double)r;
      b2[v] += (double)bx * (double)bx;
      xd[v] += (double)xi.v[v] * (double)xi.v[v] * rdv;
      wv.v[v] = di * r;
    }
    if (w) stv<T, VEC>(w + row * KB + sub * VEC, wv);
  }
  // lanes with equal `sub` hold the same columns: reduce over the other bits
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    for (int off = kWave / 2; off >= LPR; off >>= 1) {
      r2[v] += __shfl_xor(r2[v], off);
      b2[v] += __shfl_xor(b2[v], off);
      xd[v] += __shfl_xor(xd[v], off);
    }
  }
  const int lane = tid % kWave, wv_ = tid / kWave;
  if (lane < LPR) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      sh[wv_][lane * VEC + v] = r2[v];
      sh[wv_][KB + lane * VEC + v] = b2[v];
      sh[wv_][2 * KB + lane * VEC + v] = xd[v];
    }
  }
  __syncthreads();
  if (tid < NE) {
    double acc = 0;
    for (int q = 0; q < kBlock / kWave; ++q) acc += sh[q][tid];
    partials[blockIdx.x * NE + tid] = acc;
  }
}

template <typename T>
void launch_resid(int64_t n, int kb, const T* x, const T* ax, const T* bdiag, const T* dinv,
                  int precond, const double* lam, T* w, double* partials, int nparts,
                  const int* done, hipStream_t s) {
  ME_DISPATCH_KB(kb, {
    k_resid<T, KB><<<nparts, kBlock, 0, s>>>(n, x, ax, bdiag, dinv, precond, lam, w, partials,
                                             done);
  });
}
template void launch_resid<double>(int64_t, int, const double*, const double*, const double*,
                                   const double*, int, const double*, double*, double*, int,
                                   const int*, hipStream_t);
template void launch_resid<float>(int64_t, int, const float*, const float*, const float*,
                                  const float*, int, const double*, float*, double*, int,
                                  const int*, hipStream_t);

// rho_j = |r_j| / (|lambda_j| |B x_j|), with |lambda_j| replaced by the
// operator scale when it is below the zero threshold; convergence
// bookkeeping; Chebyshev interval and coefficients for this iteration.
// One wave: lane l sums partials l, l + 64, ...; then a fixed xor tree.
template <int KB>
__global__ void __launch_bounds__(kWave) k_resid_finalize(const double* partials, int nparts,
                                                          const double* lam, Ctrl* ctrl,
                                                          int final_pass) {
  constexpr int NE = 3 * KB;
  __shared__ double tot[NE];
  if (!final_pass && ctrl->done) return;
  const int lane = threadIdx.x;
  double acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) acc[e] = 0.0;
  for (int p = lane; p < nparts; p += kWave) {
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] += partials[p * NE + e];
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    double v = acc[e];
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) tot[e] = v;
  }
  __syncthreads();
  int conv = 0, bad = 0;
  if (lane < KB) {
    const double al = fabs(lam[lane]);
    const double den = (al >= ctrl->lam_floor ? al : ctrl->lam_scale) * sqrt(tot[KB + lane]);
    const double rho = sqrt(tot[lane]) / den;
    ctrl->rho[lane] = rho;
    conv = (lane < ctrl->need) && (rho <= ctrl->tol);
    bad = !isfinite(rho);
  }
  const int nc = __popcll(__ballot(conv));
  const int nb = __popcll(__ballot(bad));
  if (lane == 0) {
    ctrl->nconv = nc;
    if (nb) ctrl->nonfinite = 1;
    if (!final_pass) {
      if (nc >= ctrl->need || nb || ctrl->iter >= ctrl->max_iter) ctrl->done = 1;
      else ctrl->iter += 1;
    }
  }
  const int deg = ctrl->cheb_deg;
  if (final_pass || deg < 2) return;
  // [a, b]: a = afac * (x_j^T A x_j) / (x_j^T D x_j) with x_j^T B x_j = 1
  const double b = ctrl->cheb_b;
  // leading Ritz pair with a nonzero value (the eps = 0 case has lambda_1 = 0)
  double a = -1.0;
  for (int j = 0; j < KB; ++j) {
    if (fabs(lam[j]) >= ctrl->lam_floor) {
      a = ctrl->cheb_afac * fabs(lam[j]) / tot[2 * KB + j];
      break;
    }
  }
  if (!(a > 0.0) || !isfinite(a)) a = 1e-3 * b;
  a = fmin(fmax(a, 1e-9 * b), 0.5 * b);
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
  const double phi = acosh(theta / delta);
  // rho_k = T_k(sigma) / T_{k+1}(sigma) = cosh(k phi) / cosh((k+1) phi)
  for (int k = lane + 1; k < deg; k += kWave) {
    const double rk = cosh(k * phi) / cosh((k + 1) * phi);
    const double rkm = cosh((k - 1) * phi) / cosh(k * phi);
    ctrl->cheb_alpha[k] = rk * rkm;
    ctrl->cheb_beta[k] = 2.0 * rk / delta;
  }
  if (lane == 0) {
    ctrl->cheb_a = a;
    ctrl->cheb_theta = theta;
  }
}

void launch_resid_finalize(int kb, const double* partials, int nparts, const double* lam,
                           Ctrl* ctrl, int final_pass, hipStream_t s) {
  ME_DISPATCH_KB(kb, {
    k_resid_finalize<KB><<<1, kWave, 0, s>>>(partials, nparts, lam, ctrl, final_pass);
  });
}

// ---------------------------------------------------------------------------
// Tall-skinny Gram products on MFMA:
//   G1 = U^T diag(wd) V   ((nu kb) x (nv kb)),   G2 = U^T V2  ((nu kb) x (nv2 kb))
// U, V, V2 are lists of n x kb blocks.  Contraction over rows: each
// 16x16x4 MFMA step consumes 4 rows; lane l supplies U[row0 + l/16][16a + l%16]
// (A operand) and V[row0 + l/16][16b + l%16] (B operand).  Each block writes
// its partial result; a second kernel sums the partials in a fixed order.
// ---------------------------------------------------------------------------

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Accumulator layout of a 16x16 tile: lane l, element q holds D[i][l % 16]
// with i = row(l / 16, q): 4 (l / 16) + q for the f32 instruction and
// 4 q + l / 16 for the f64 one.
template <>
struct Mfma<double> {
  using Acc = dx4;
  static __device__ inline Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int q) { return 4 * q + lk; }
};
template <>
struct Mfma<float> {
  using Acc = fx4;
  static __device__ inline Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int q) { return 4 * lk + q; }
};

template <typename T>
struct BlockList {
  const T* p[3];
};

template <typename T, int KB>
__device__ inline T load_cat(const BlockList<T>& bl, int nblk, int64_t row, int col, int64_t n) {
  const int blk = col / KB;
  if (row >= n || blk >= nblk) return (T)0;
  return bl.p[blk][row * KB + (col % KB)];
}

template <typename T, int KB, int NU, int NV, int NV2>
__global__ void __launch_bounds__(kBlock) k_gram(int64_t n, BlockList<T> u, BlockList<T> v,
                                                 const T* __restrict__ wd, BlockList<T> v2,
                                                 double* partials, const int* done) {
  constexpr int MU = NU * KB, MV = NV * KB, MV2 = NV2 * KB;
  constexpr int TU = (MU + 15) / 16, TV = (MV + 15) / 16, TV2 = (MV2 + 15) / 16;
  constexpr int E1 = MU * MV, E2 = MU * MV2;
  using Acc = typename Mfma<T>::Acc;
  __shared__ double sh[E1 + E2];
  if (done && *done) return;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  Acc acc1[TU][TV > 0 ? TV : 1];
  Acc acc2[TU][TV2 > 0 ? TV2 : 1];
#pragma unroll
  for (int a = 0; a < TU; ++a) {
#pragma unroll
    for (int b = 0; b < TV; ++b) acc1[a][b] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < TV2; ++b) acc2[a][b] = Acc{0, 0, 0, 0};
  }
  // contiguous row range of this block; each wave takes 16 rows (4 MFMA
  // k-steps) per pass and issues all their loads before the MFMAs
  const int64_t per = ((ceil_div(n, gridDim.x) + 15) / 16) * 16;
  const int64_t r0 = blockIdx.x * per;
  const int64_t r1 = (r0 + per < n) ? r0 + per : n;
  const int li = lane % 16, lk = lane / 16;
  constexpr int NW = kBlock / kWave;
  for (int64_t base = r0 + 16 * wave; base < r1; base += 16 * NW) {
    T ua[4][TU], vb[4][TV > 0 ? TV : 1], v2b[4][TV2 > 0 ? TV2 : 1];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int64_t row = base + 4 * ks + lk;
      const bool ok = row < r1;
#pragma unroll
      for (int a = 0; a < TU; ++a) ua[ks][a] = ok ? load_cat<T, KB>(u, NU, row, 16 * a + li, n) : (T)0;
      const T wr = (ok && TV > 0) ? (wd ? wd[row] : (T)1) : (T)0;
#pragma unroll
      for (int b = 0; b < TV; ++b) vb[ks][b] = ok ? wr * load_cat<T, KB>(v, NV, row, 16 * b + li, n) : (T)0;
#pragma unroll
      for (int b = 0; b < TV2; ++b) v2b[ks][b] = ok ? load_cat<T, KB>(v2, NV2, row, 16 * b + li, n) : (T)0;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
      for (int a = 0; a < TU; ++a) {
#pragma unroll
        for (int b = 0; b < TV; ++b) acc1[a][b] = Mfma<T>::step(ua[ks][a], vb[ks][b], acc1[a][b]);
#pragma unroll
        for (int b = 0; b < TV2; ++b) acc2[a][b] = Mfma<T>::step(ua[ks][a], v2b[ks][b], acc2[a][b]);
      }
    }
  }
  for (int wv = 0; wv < kBlock / kWave; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int a = 0; a < TU; ++a) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * a + Mfma<T>::row(lk, q);
          if (i >= MU) continue;
#pragma unroll
          for (int b = 0; b < TV; ++b) {
            const int j = 16 * b + li;
            if (j < MV) {
              const double val = (double)acc1[a][b][q];
              if (wv == 0) sh[i * MV + j] = val; else sh[i * MV + j] += val;
            }
          }
#pragma unroll
          for (int b = 0; b < TV2; ++b) {
            const int j = 16 * b + li;
            if (j < MV2) {
              const double val = (double)acc2[a][b][q];
              if (wv == 0) sh[E1 + i * MV2 + j] = val; else sh[E1 + i * MV2 + j] += val;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < E1 + E2; e += kBlock) partials[blockIdx.x * (int64_t)(E1 + E2) + e] = sh[e];
}

template <typename T>
static BlockList<T> mk_list(int nb, const T* const* p) {
  BlockList<T> bl{{nullptr, nullptr, nullptr}};
  for (int i = 0; i < nb && i < 3; ++i) bl.p[i] = p[i];
  return bl;
}

template <typename T>
void launch_gram(int64_t n, int kb, int nu, const T* const* u, int nv, const T* const* v,
                 const T* wdiag, int nv2, const T* const* v2, double* partials, int nparts,
                 const int* done, hipStream_t s) {
  const auto bu = mk_list<T>(nu, u), bv = mk_list<T>(nv, v), bv2 = mk_list<T>(nv2, v2);
#define ME_GRAM(NU_, NV_, NV2_)                                                              \
  if (nu == NU_ && nv == NV_ && nv2 == NV2_) {                                               \
    ME_DISPATCH_KB(kb, {                                                                      \
      k_gram<T, KB, NU_, NV_, NV2_><<<nparts, kBlock, 0, s>>>(n, bu, bv, wdiag, bv2, partials, \
                                                              done);                          \
    });                                                                                       \
    return;                                                                                   \
  }
  ME_GRAM(2, 1, 0)  // [X W]^T B W
  ME_GRAM(1, 1, 1)  // X^T B X, X^T AX
  ME_GRAM(2, 2, 2)  // [X W] pair
  ME_GRAM(3, 3, 3)  // [X W P] pair
  ME_GRAM(1, 1, 0)  // X^T B X
#undef ME_GRAM
}
template void launch_gram<double>(int64_t, int, int, const double* const*, int,
                                  const double* const*, const double*, int, const double* const*,
                                  double*, int, const int*, hipStream_t);
template void launch_gram<float>(int64_t, int, int, const float* const*, int, const float* const*,
                                 const float*, int, const float* const*, double*, int, const int*,
                                 hipStream_t);

// out[e] = sum_p partials[p][e], p ascending (deterministic).
__global__ void __launch_bounds__(kBlock) k_reduce_partials(int nparts, int nent,
                                                            const double* partials, double* out,
                                                            const int* done) {
  __shared__ double sh[8][33];
  if (done && *done) return;
  const int el = threadIdx.x % 32, pl = threadIdx.x / 32;
  const int e = blockIdx.x * 32 + el;
  double s = 0;
  if (e < nent) {
#pragma unroll 8
    for (int p = pl; p < nparts; p += 8) s += partials[(int64_t)p * nent + e];
  }
  sh[pl][el] = s;
  __syncthreads();
  if (pl == 0 && e < nent) {
    double t = 0;
    for (int q = 0; q < 8; ++q) t += sh[q][el];
    out[e] = t;
  }
}

void launch_reduce_partials(int nparts, int nent, const double* partials, double* out,
                            const int* done, hipStream_t s) {
  k_reduce_partials<<<ceil_div(nent, 32), kBlock, 0, s>>>(nparts, nent, partials, out, done);
}

// ---------------------------------------------------------------------------
// Block combination: out_o = sum_s in_s coef_o[s]  (coef_o is (nin kb) x kb,
// all outputs' coefficients stacked).  Each block stages its rows in LDS
// (coalesced), then every lane forms VEC output columns.  Outputs may alias
// inputs: a block reads all of its rows before writing any.
// ---------------------------------------------------------------------------

template <typename T>
struct OutList {
  T* p[2];
};

// ngroup groups share the coefficients: group g maps in[g] (nin blocks) to
// out[g] (nout blocks).
template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_combine(int64_t n, int nin, int ngroup,
                                                    BlockList<T> in0, BlockList<T> in1, int nout,
                                                    OutList<T> out0, OutList<T> out1,
                                                    const double* coef, const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR, RB = kBlock / LPR;
  __shared__ T rows[2][RB][3 * KB + 1];
  __shared__ T cf[2][3 * KB][KB];
  if (done && *done) return;
  const int tid = threadIdx.x;
  const int m = nin * KB;
  for (int u = tid; u < nout * m * KB; u += kBlock) {
    const int o = u / (m * KB), rem = u % (m * KB);
    cf[o][rem / KB][rem % KB] = (T)coef[u];
  }
  const int rloc = tid / LPR, sub = tid % LPR;
  const int64_t row = blockIdx.x * (int64_t)RB + rloc;
  if (row < n) {
    for (int g = 0; g < ngroup; ++g) {
      const BlockList<T>& in = g == 0 ? in0 : in1;
      for (int sidx = 0; sidx < nin; ++sidx) {
        const auto v = ldv<T, VEC>(in.p[sidx] + row * KB + sub * VEC);
#pragma unroll
        for (int q = 0; q < VEC; ++q) rows[g][rloc][sidx * KB + sub * VEC + q] = v.v[q];
      }
    }
  }
  __syncthreads();
  if (row >= n) return;
  for (int g = 0; g < ngroup; ++g) {
    const OutList<T>& out = g == 0 ? out0 : out1;
    for (int o = 0; o < nout; ++o) {
      T acc[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] = 0;
      for (int k = 0; k < m; ++k) {
        const T a = rows[g][rloc][k];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] += a * cf[o][k][sub * VEC + q];
      }
      typename L::Vec ov;
#pragma unroll
      for (int q = 0; q < VEC; ++q) ov.v[q] = acc[q];
      stv<T, VEC>(out.p[o] + row * KB + sub * VEC, ov);
    }
  }
}

template <typename T>
void launch_combine2(int64_t n, int kb, int nin, int ngroup, const T* const* in0,
                     const T* const* in1, int nout, T* const* out0, T* const* out1,
                     const double* coef, const int* done, hipStream_t s) {
  const auto b0 = mk_list<T>(nin, in0);
  const auto b1 = mk_list<T>(ngroup > 1 ? nin : 0, in1);
  OutList<T> o0{{out0[0], nout > 1 ? out0[1] : nullptr}};
  OutList<T> o1{{ngroup > 1 ? out1[0] : nullptr, (ngroup > 1 && nout > 1) ? out1[1] : nullptr}};
  ME_DISPATCH_KB(kb, {
    constexpr int RB = kBlock / Lay<T, KB>::LPR;
    k_combine<T, KB><<<ceil_div(n, RB), kBlock, 0, s>>>(n, nin, ngroup, b0, b1, nout, o0, o1,
                                                        coef, done);
  });
}
template void launch_combine2<double>(int64_t, int, int, int, const double* const*,
                                      const double* const*, int, double* const*, double* const*,
                                      const double*, const int*, hipStream_t);
template void launch_combine2<float>(int64_t, int, int, int, const float* const*,
                                     const float* const*, int, float* const*, float* const*,
                                     const double*, const int*, hipStream_t);

template <typename T>
void launch_combine(int64_t n, int kb, int nin, const T* const* in, int nout, T* const* out,
                    const double* coef, const int* done, hipStream_t s) {
  launch_combine2<T>(n, kb, nin, 1, in, nullptr, nout, out, nullptr, coef, done, s);
}
template void launch_combine<double>(int64_t, int, int, const double* const*, int,
                                     double* const*, const double*, const int*, hipStream_t);
template void launch_combine<float>(int64_t, int, int, const float* const*, int, float* const*,
                                    const double*, const int*, hipStream_t);

// ---------------------------------------------------------------------------
// Column sums (for deflating the constant vector) and subtraction of the mean
// ---------------------------------------------------------------------------

template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_colsum(int64_t n, const T* __restrict__ x,
                                                   double* partials, const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR;
  __shared__ double sh[kBlock / kWave][KB];
  if (done && *done) return;
  const int tid = threadIdx.x, sub = tid % LPR;
  double acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  for (int64_t g = blockIdx.x * (int64_t)kBlock + tid; g < n * LPR;
       g += (int64_t)gridDim.x * kBlock) {
    const auto xv = ldv<T, VEC>(x + (g / LPR) * KB + sub * VEC);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += (double)xv.v[v];
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v)
    for (int off = kWave / 2; off >= LPR; off >>= 1) acc[v] += __shfl_xor(acc[v], off);
  const int lane = tid % kWave, wv = tid / kWave;
  if (lane < LPR)
#pragma unroll
    for (int v = 0; v < VEC; ++v) sh[wv][lane * VEC + v] = acc[v];
  __syncthreads();
  if (tid < KB) {
    double s = 0;
    for (int q = 0; q < kBlock / kWave; ++q) s += sh[q][tid];
    partials[blockIdx.x * KB + tid] = s;
  }
}

template <typename T, int KB>
__global__ void k_sub_mean(int64_t n, T* x, const double* sums, const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR;
  if (done && *done) return;
  const int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (g >= n * LPR) return;
  const int sub = (int)(g % LPR);
  T* p = x + (g / LPR) * KB + sub * VEC;
  auto xv = ldv<T, VEC>(p);
#pragma unroll
  for (int v = 0; v < VEC; ++v) xv.v[v] -= (T)(sums[sub * VEC + v] / (double)n);
  stv<T, VEC>(p, xv);
}

template <typename T>
void launch_deflate_ones(int64_t n, int kb, T* x, double* partials, int nparts, double* sums,
                         const int* done, hipStream_t s) {
  ME_DISPATCH_KB(kb, {
    constexpr int LPR = Lay<T, KB>::LPR;
    k_colsum<T, KB><<<nparts, kBlock, 0, s>>>(n, x, partials, done);
    launch_reduce_partials(nparts, KB, partials, sums, done, s);
    k_sub_mean<T, KB><<<ceil_div(n * LPR, kBlock), kBlock, 0, s>>>(n, x, sums, done);
  });
}
template void launch_deflate_ones<double>(int64_t, int, double*, double*, int, double*,
                                          const int*, hipStream_t);
template void launch_deflate_ones<float>(int64_t, int, float*, double*, int, double*, const int*,
                                         hipStream_t);

// ---------------------------------------------------------------------------
// Starting block: copies x0 (n x kcopy) and fills the remaining columns with
// a counter-based generator (SplitMix64 of seed and element index, Steele,
// Lea & Flood 2014), uniform in [-1, 1).
// ---------------------------------------------------------------------------

__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Solver row i' holds user row u = perm[i'] (perm may be null: identity);
// values depend only on (seed, u, j), so the start is independent of the
// solver's node order.
__global__ void k_fill_start(int64_t n, int kb, int kcopy, const double* x0, uint64_t seed,
                             const int32_t* perm, double* x) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * kb) return;
  const int64_t i = g / kb;
  const int j = (int)(g % kb);
  const int64_t u = perm ? perm[i] : i;
  double v;
  if (x0 && j < kcopy) {
    v = x0[u * kcopy + j];
  } else {
    const uint64_t h = splitmix64(seed * 0x2545F4914F6CDD1Dull + (uint64_t)(u * kb + j));
    v = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  x[g] = v;
}

void launch_fill_random(int64_t n, int kb, int kcopy, const double* x0, uint64_t seed,
                        const int32_t* perm, double* x, hipStream_t s) {
  k_fill_start<<<ceil_div(n * kb, kBlock), kBlock, 0, s>>>(n, kb, kcopy, x0, seed, perm, x);
}

// ---------------------------------------------------------------------------
// Output: sign convention (largest |x| of each column positive, lowest row on
// ties) and the copy of the first k columns.
// ---------------------------------------------------------------------------

// Per column: largest |x| and the lowest user row holding it (user row of
// solver row i is perm[i], or i when perm is null).
__global__ void __launch_bounds__(kBlock) k_col_argmax(int64_t n, int kb, const double* x,
                                                       const int32_t* perm, double* pval,
                                                       int64_t* pidx) {
  __shared__ double sv[kBlock];
  __shared__ int64_t si[kBlock];
  for (int j = 0; j < kb; ++j) {
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
      const double a = fabs(x[i * kb + j]);
      const int64_t u = perm ? perm[i] : i;
      if (a > best || (a == best && u < bi)) { best = a; bi = u; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) {
        const double ov = sv[threadIdx.x + st];
        const int64_t oi = si[threadIdx.x + st];
        if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
          sv[threadIdx.x] = ov;
          si[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      pval[blockIdx.x * kb + j] = sv[0];
      pidx[blockIdx.x * kb + j] = si[0];
    }
    __syncthreads();
  }
}

// out[u][j] = sign_j * x[iperm[u]][j] for j < k (user order), sign_j making
// the largest-magnitude entry positive.
__global__ void k_signed_copy(int64_t n, int kb, int k, const double* x, const int32_t* iperm,
                              const double* pval, const int64_t* pidx, int nparts, double* out,
                              const double* lam, double* lam_out) {
  __shared__ double sgn[kMaxBasis];
  if (threadIdx.x < (unsigned)k) {
    const int j = threadIdx.x;
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int p = 0; p < nparts; ++p) {
      const double v = pval[p * kb + j];
      const int64_t ii = pidx[p * kb + j];
      if (v > best || (v == best && ii < bi)) { best = v; bi = ii; }
    }
    double val = 1.0;
    if (bi < n) val = x[(iperm ? (int64_t)iperm[bi] : bi) * kb + j];
    sgn[j] = val < 0.0 ? -1.0 : 1.0;
    if (blockIdx.x == 0) lam_out[j] = lam[j];
  }
  __syncthreads();
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * k) return;
  const int64_t u = g / k;
  const int j = (int)(g % k);
  const int64_t i = iperm ? iperm[u] : u;
  out[g] = sgn[j] * x[i * kb + j];
}

void launch_sign_fix_and_copy(int64_t n, int kb, int k, const double* x, double* out,
                              const double* lam, double* lam_out, double* scratch,
                              const int32_t* perm, const int32_t* iperm, hipStream_t s) {
  const int nparts = (int)std::min<int64_t>(ceil_div(n, kBlock), 64);
  double* pval = scratch;
  int64_t* pidx = reinterpret_cast<int64_t*>(scratch + nparts * kb);
  k_col_argmax<<<nparts, kBlock, 0, s>>>(n, kb, x, perm, pval, pidx);
  k_signed_copy<<<ceil_div(n * k, kBlock), kBlock, 0, s>>>(n, kb, k, x, iperm, pval, pidx, nparts,
                                                           out, lam, lam_out);
}

// ---------------------------------------------------------------------------
// Misc
// ---------------------------------------------------------------------------

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t count, const Tin* in, Tout* out) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < count) out[g] = (Tout)in[g];
}

template <typename Tin, typename Tout>
void launch_convert(int64_t count, const Tin* in, Tout* out, hipStream_t s) {
  k_convert<Tin, Tout><<<ceil_div(count, kBlock), kBlock, 0, s>>>(count, in, out);
}
template void launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);
template void launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);
template void launch_convert<double, double>(int64_t, const double*, double*, hipStream_t);

__global__ void k_scale_rows(int64_t n, int k, const double* b, const double* x, double* y) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n * k) y[g] = b[g / k] * x[g];
}

void launch_scale_rows(int64_t n, int k, const double* b, const double* x, double* y,
                       hipStream_t s) {
  k_scale_rows<<<ceil_div(n * k, kBlock), kBlock, 0, s>>>(n, k, b, x, y);
}

// Dense n x n operator (graphs with n <= 48): which 0 = A, 1 = Q; also B.
__global__ void k_dense_ops(int64_t n, const int64_t* w_rp, const int32_t* w_col,
                            const double* w_val, const int64_t* t_rp, const int32_t* t_col,
                            const double* invt, const double* d, const double* qdiag,
                            const double* b, double mu, double eps, int which, double* out,
                            double* bmat) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t j = 0; j < n; ++j) {
    out[i * n + j] = 0.0;
    bmat[i * n + j] = 0.0;
  }
  if (which == 0) {
    for (int64_t t = w_rp[i]; t < w_rp[i + 1]; ++t) out[i * n + w_col[t]] = -w_val[t];
    for (int64_t t = t_rp[i]; t < t_rp[i + 1]; ++t)
      out[i * n + t_col[t]] = mu * (invt[i] + invt[t_col[t]]);
    out[i * n + i] = d[i] - mu * qdiag[i] + eps;
    bmat[i * n + i] = b[i];
  } else {
    for (int64_t t = t_rp[i]; t < t_rp[i + 1]; ++t)
      out[i * n + t_col[t]] = -(invt[i] + invt[t_col[t]]);
    out[i * n + i] = qdiag[i];
    bmat[i * n + i] = 1.0;
  }
}

void launch_dense_ops(const GraphOps& g, int which, double* out, double* bmat, hipStream_t s) {
  k_dense_ops<<<1, kDenseMaxN > 64 ? 128 : 64, 0, s>>>(g.n, g.w_rp, g.w_col, g.w_val, g.t_rp,
                                                       g.t_col, g.invt, g.d, g.qdiag, g.b, g.mu,
                                                       g.eps, which, out, bmat);
}

// dst[i][j] = src[map ? map[i] : i][j] for j < kcopy
__global__ void k_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const int32_t* map,
                            const double* src, double* dst) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * kcopy) return;
  const int64_t i = g / kcopy;
  const int j = (int)(g % kcopy);
  const int64_t r = map ? map[i] : i;
  dst[i * kdst + j] = src[r * ksrc + j];
}

void launch_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const int32_t* map,
                      const double* src, double* dst, hipStream_t s) {
  if (n * kcopy == 0) return;
  k_copy_cols<<<ceil_div(n * kcopy, kBlock), kBlock, 0, s>>>(n, ksrc, kdst, kcopy, map, src, dst);
}

}  // namespace me
