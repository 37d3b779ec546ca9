// Whole-graph kernels outside the LOBPCG engine: the operator product for
// the test hook me_apply, the dense path for graphs of at most 48 nodes
// (operator assembly, sign convention and output copy), and small copies.
//
// Difference-form operator (eq. (obj2) with the Laplacian identity of
// Section 3.1): with a row's W entries and T entries,
//   (A x)_i = sum_{j in N(i)} w_ij (x_i - x_j)
//             - mu sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j) + eps x_i
//   (Q x)_i = sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j)
// The diagonal is never stored; the differences x_i - x_j keep the rounding
// error proportional to the local variation of x rather than to |A| |x|.
#include <cmath>

#include "common.h"
#include "rowops.h"

namespace me {

// ---------------------------------------------------------------------------
// SpMM: Y = Op X in difference form
// ---------------------------------------------------------------------------

// Y = Op X: G lanes per row; lane q < KB / V16 writes the q-th 16-byte
// slice of the row.
template <typename T, int KB>
__global__ void __launch_bounds__((RowCfg<T, KB>::THREADS)) k_spmm(int64_t n, const int32_t* __restrict__ a_rp,
                                                 const int32_t* __restrict__ a_tp,
                                                 const int32_t* __restrict__ a_col,
                                                 const T* __restrict__ a_w, T c_t, T s_diag,
                                                 int skip_w, const T* __restrict__ x,
                                                 T* __restrict__ y, const int* done) {
  using C = RowCfg<T, KB>;
  if (done && *done) return;
  const int64_t blk = xcd_block(ceil_div(n, C::ROWS));
  if (blk * C::ROWS >= n) return;
  const int64_t gt = blk * C::THREADS + threadIdx.x;
  const int64_t row = gt / C::G;
  const int q = (int)(gt % C::G);
  const bool live = row < n;
  const int ch = q % C::NCH;
  T xi[C::V16], acc[C::V16];
  load_chunk<T, C::V16>(x + (live ? row : 0) * KB + ch * C::V16, xi);
  spmm_row<T, KB>(live, row, q, a_rp, a_tp, a_col, a_w, c_t, skip_w ? kRangeT : kRangeAll, x,
                  xi, acc);
  if (!live || q >= C::NCH) return;
  VecT<T, C::V16> o;
#pragma unroll
  for (int v = 0; v < C::V16; ++v) o.v[v] = fmaT(s_diag, xi[v], acc[v]);
  stv<T, C::V16>(y + row * KB + q * C::V16, o);
}

template <typename T>
struct OpArrays;
template <>
struct OpArrays<double> {
  static const double* w(const GraphOps& g) { return g.a_w; }
};
template <>
struct OpArrays<float> {
  static const float* w(const GraphOps& g) { return g.a_w32; }
};

template <typename T>
void launch_spmm(const GraphOps& g, int kb, OpKind op, const T* x, T* y, const int* done,
                 hipStream_t s) {
  const T c_t = op == OP_A ? (T)(-g.mu) : (T)1;
  const T s_diag = op == OP_A ? (T)g.eps : (T)0;
  const int skip_w = op == OP_Q;
  ME_DISPATCH_KB(kb, {
    const int64_t grid = xcd_grid(ceil_div(g.n, RowCfg<T, KB>::ROWS));
    k_spmm<T, KB><<<grid, RowCfg<T, KB>::THREADS, 0, s>>>(g.n, g.a_rp, g.a_tp, g.a_col, OpArrays<T>::w(g),
                                          c_t, s_diag, skip_w, x, y, done);
  });
}
template void launch_spmm<double>(const GraphOps&, int, OpKind, const double*, double*,
                                  const int*, hipStream_t);

template void launch_spmm<float>(const GraphOps&, int, OpKind, const float*, float*, const int*,
                                 hipStream_t);

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
