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

template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_spmm(int64_t n, const int32_t* __restrict__ a_rp,
                                                 const int32_t* __restrict__ a_split,
                                                 const int32_t* __restrict__ a_col,
                                                 const T* __restrict__ a_w,
                                                 const T* __restrict__ invt, T c_t, T s_diag,
                                                 int skip_w, const T* __restrict__ x,
                                                 T* __restrict__ y, const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR;
  if (done && *done) return;
  const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t row = gt / LPR;
  const int sub = (int)(gt % LPR);
  if (row >= n) return;
  const auto xi = ldv<T, VEC>(x + row * KB + sub * VEC);
  T acc[VEC], acc2[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) { acc[v] = 0; acc2[v] = 0; }
  const int32_t s = a_rp[row], sp = a_split[row], e = a_rp[row + 1];
  if (!skip_w) {
#pragma unroll 4
    for (int32_t k = s; k < sp; ++k) {
      const int32_t c = a_col[k];
      const T w = a_w[k];
      const auto xj = ldv<T, VEC>(x + (int64_t)c * KB + sub * VEC);
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += w * (xi.v[v] - xj.v[v]);
    }
  }
  const T ti = invt[row];
#pragma unroll 4
  for (int32_t k = sp; k < e; ++k) {
    const int32_t c = a_col[k];
    const T q = ti + invt[c];
    const auto xj = ldv<T, VEC>(x + (int64_t)c * KB + sub * VEC);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc2[v] += q * (xi.v[v] - xj.v[v]);
  }
  typename L::Vec out;
#pragma unroll
  for (int v = 0; v < VEC; ++v) out.v[v] = acc[v] + c_t * acc2[v] + s_diag * xi.v[v];
  stv<T, VEC>(y + row * KB + sub * VEC, out);
}

template <typename T>
struct OpArrays;
template <>
struct OpArrays<double> {
  static const double* w(const GraphOps& g) { return g.a_w; }
  static const double* invt(const GraphOps& g) { return g.invt; }
};
template <>
struct OpArrays<float> {
  static const float* w(const GraphOps& g) { return g.a_w32; }
  static const float* invt(const GraphOps& g) { return g.invt32; }
};

template <typename T>
void launch_spmm(const GraphOps& g, int kb, OpKind op, const T* x, T* y, const int* done,
                 hipStream_t s) {
  const T c_t = op == OP_A ? (T)(-g.mu) : (T)1;
  const T s_diag = op == OP_A ? (T)g.eps : (T)0;
  const int skip_w = op == OP_Q;
  ME_DISPATCH_KB(kb, {
    constexpr int LPR = Lay<T, KB>::LPR;
    const int64_t grid = ceil_div(g.n * LPR, kBlock);
    k_spmm<T, KB><<<grid, kBlock, 0, s>>>(g.n, g.a_rp, g.a_split, g.a_col, OpArrays<T>::w(g),
                                          OpArrays<T>::invt(g), c_t, s_diag, skip_w, x, y, done);
  });
}
template void launch_spmm<double>(const GraphOps&, int, OpKind, const double*, double*,
                                  const int*, hipStream_t);
template void launch_spmm<float>(const GraphOps&, int, OpKind, const float*, float*, const int*,
                                 hipStream_t);

// ---------------------------------------------------------------------------
// Residual R = AX - B X Lambda, preconditioned W = T R, column sums of
// |r|^2 and |B x|^2 per block (double).  precond: 0 none, 1 multiply by
// dinv[i], 2 divide by dinv[i] (used with Q's diagonal).
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
  __shared__ double sh[kBlock / kWave][2 * KB];
  if (done && *done) return;
  const int tid = threadIdx.x;
  const int sub = tid % LPR;
  double r2[VEC], b2[VEC];
  T lm[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) { r2[v] = 0; b2[v] = 0; lm[v] = (T)lam[sub * VEC + v]; }
  const int64_t total = n * LPR;
  for (int64_t g = blockIdx.x * (int64_t)kBlock + tid; g < total;
       g += (int64_t)gridDim.x * kBlock) {
    const int64_t row = g / LPR;
    const auto xi = ldv<T, VEC>(x + row * KB + sub * VEC);
    const auto ai = ldv<T, VEC>(ax + row * KB + sub * VEC);
    const T bi = bdiag ? bdiag[row] : (T)1;
    T di = (T)1;
    if (precond == 1) di = dinv[row];
    else if (precond == 2) di = (T)1 / dinv[row];
    typename L::Vec wv;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const T bx = bi * xi.v[v];
      const T r = ai.v[v] - lm[v] * bx;
      r2[v] += (double)r * (double)r;
      b2[v] += (double)bx * (double)bx;
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
    }
  }
  const int lane = tid % kWave, wv_ = tid / kWave;
  if (lane < LPR) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      sh[wv_][lane * VEC + v] = r2[v];
      sh[wv_][KB + lane * VEC + v] = b2[v];
    }
  }
  __syncthreads();
  if (tid < 2 * KB) {
    double s = 0;
    for (int q = 0; q < kBlock / kWave; ++q) s += sh[q][tid];
    partials[blockIdx.x * (2 * KB) + tid] = s;
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
// operator scale when it is below the zero threshold; convergence bookkeeping.
__global__ void k_resid_finalize(int kb, const double* partials, int nparts, const double* lam,
                                 Ctrl* ctrl, int final_pass) {
  __shared__ int conv[kMaxBlockCols];
  __shared__ int bad[kMaxBlockCols];
  if (!final_pass && ctrl->done) return;
  const int j = threadIdx.x;
  if (j < kb) {
    double r2 = 0, b2 = 0;
    for (int p = 0; p < nparts; ++p) {
      r2 += partials[p * 2 * kb + j];
      b2 += partials[p * 2 * kb + kb + j];
    }
    const double al = fabs(lam[j]);
    const double den = (al >= ctrl->lam_floor ? al : ctrl->lam_scale) * sqrt(b2);
    const double rho = sqrt(r2) / den;
    ctrl->rho[j] = rho;
    conv[j] = (j < ctrl->need) && (rho <= ctrl->tol);
    bad[j] = !isfinite(rho);
  }
  __syncthreads();
  if (j == 0) {
    int nc = 0, nb = 0;
    for (int q = 0; q < kb; ++q) { nc += conv[q]; nb += bad[q]; }
    ctrl->nconv = nc;
    if (nb) ctrl->nonfinite = 1;
    if (!final_pass) {
      if (nc >= ctrl->need || nb || ctrl->iter >= ctrl->max_iter) ctrl->done = 1;
      else ctrl->iter += 1;
    }
  }
}

void launch_resid_finalize(int kb, const double* partials, int nparts, const double* lam,
                           Ctrl* ctrl, int final_pass, hipStream_t s) {
  k_resid_finalize<<<1, kWave, 0, s>>>(kb, partials, nparts, lam, ctrl, final_pass);
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
  // contiguous row range of this block, split in 4-row steps across waves
  const int64_t per = ((ceil_div(n, gridDim.x) + 15) / 16) * 16;
  const int64_t r0 = blockIdx.x * per;
  const int64_t r1 = (r0 + per < n) ? r0 + per : n;
  const int li = lane % 16, lk = lane / 16;
  for (int64_t base = r0 + 4 * wave; base < r1; base += 16) {
    const int64_t row = base + lk;
    const bool ok = row < r1;
    T ua[TU];
#pragma unroll
    for (int a = 0; a < TU; ++a) ua[a] = ok ? load_cat<T, KB>(u, NU, row, 16 * a + li, n) : (T)0;
    if (TV > 0) {
      const T wr = ok ? (wd ? wd[row] : (T)1) : (T)0;
#pragma unroll
      for (int b = 0; b < TV; ++b) {
        const T vb = ok ? wr * load_cat<T, KB>(v, NV, row, 16 * b + li, n) : (T)0;
#pragma unroll
        for (int a = 0; a < TU; ++a) acc1[a][b] = Mfma<T>::step(ua[a], vb, acc1[a][b]);
      }
    }
#pragma unroll
    for (int b = 0; b < TV2; ++b) {
      const T vb = ok ? load_cat<T, KB>(v2, NV2, row, 16 * b + li, n) : (T)0;
#pragma unroll
      for (int a = 0; a < TU; ++a) acc2[a][b] = Mfma<T>::step(ua[a], vb, acc2[a][b]);
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
  if (e < nent)
    for (int p = pl; p < nparts; p += 8) s += partials[(int64_t)p * nent + e];
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

template <typename T, int KB>
__global__ void __launch_bounds__(kBlock) k_combine(int64_t n, int nin, BlockList<T> in, int nout,
                                                    T* out0, T* out1, const double* coef,
                                                    const int* done) {
  using L = Lay<T, KB>;
  constexpr int VEC = L::VEC, LPR = L::LPR, RB = kBlock / LPR;
  __shared__ T rows[RB][3 * KB + 1];
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
    for (int sidx = 0; sidx < nin; ++sidx) {
      const auto v = ldv<T, VEC>(in.p[sidx] + row * KB + sub * VEC);
#pragma unroll
      for (int q = 0; q < VEC; ++q) rows[rloc][sidx * KB + sub * VEC + q] = v.v[q];
    }
  }
  __syncthreads();
  if (row >= n) return;
  for (int o = 0; o < nout; ++o) {
    T acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = 0;
    for (int k = 0; k < m; ++k) {
      const T a = rows[rloc][k];
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] += a * cf[o][k][sub * VEC + q];
    }
    typename L::Vec ov;
#pragma unroll
    for (int q = 0; q < VEC; ++q) ov.v[q] = acc[q];
    stv<T, VEC>((o == 0 ? out0 : out1) + row * KB + sub * VEC, ov);
  }
}

template <typename T>
void launch_combine(int64_t n, int kb, int nin, const T* const* in, int nout, T* const* out,
                    const double* coef, const int* done, hipStream_t s) {
  const auto bl = mk_list<T>(nin, in);
  ME_DISPATCH_KB(kb, {
    constexpr int RB = kBlock / Lay<T, KB>::LPR;
    k_combine<T, KB><<<ceil_div(n, RB), kBlock, 0, s>>>(n, nin, bl, nout, out[0],
                                                        nout > 1 ? out[1] : nullptr, coef, done);
  });
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

__global__ void k_fill_start(int64_t n, int kb, int kcopy, const double* x0, uint64_t seed,
                             double* x) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * kb) return;
  const int64_t i = g / kb;
  const int j = (int)(g % kb);
  double v;
  if (x0 && j < kcopy) {
    v = x0[i * kcopy + j];
  } else {
    const uint64_t h = splitmix64(seed * 0x2545F4914F6CDD1Dull + (uint64_t)g);
    v = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  x[g] = v;
}

void launch_fill_random(int64_t n, int kb, int kcopy, const double* x0, uint64_t seed, double* x,
                        hipStream_t s) {
  k_fill_start<<<ceil_div(n * kb, kBlock), kBlock, 0, s>>>(n, kb, kcopy, x0, seed, x);
}

// ---------------------------------------------------------------------------
// Output: sign convention (largest |x| of each column positive, lowest row on
// ties) and the copy of the first k columns.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_col_argmax(int64_t n, int kb, const double* x,
                                                       double* pval, int64_t* pidx) {
  __shared__ double sv[kBlock];
  __shared__ int64_t si[kBlock];
  for (int j = 0; j < kb; ++j) {
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
      const double a = fabs(x[i * kb + j]);
      if (a > best) { best = a; bi = i; }  // i ascending per thread: keeps the lowest on ties
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

__global__ void k_signed_copy(int64_t n, int kb, int k, const double* x, const double* pval,
                              const int64_t* pidx, int nparts, double* out, const double* lam,
                              double* lam_out) {
  __shared__ double sgn[kMaxBlockCols];
  if (threadIdx.x < (unsigned)k) {
    const int j = threadIdx.x;
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int p = 0; p < nparts; ++p) {
      const double v = pval[p * kb + j];
      const int64_t ii = pidx[p * kb + j];
      if (v > best || (v == best && ii < bi)) { best = v; bi = ii; }
    }
    sgn[j] = (bi < n && x[bi * kb + j] < 0.0) ? -1.0 : 1.0;
    if (blockIdx.x == 0) lam_out[j] = lam[j];
  }
  __syncthreads();
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * k) return;
  const int64_t i = g / k;
  const int j = (int)(g % k);
  out[g] = sgn[j] * x[i * kb + j];
}

void launch_sign_fix_and_copy(int64_t n, int kb, int k, const double* x, double* out,
                              const double* lam, double* lam_out, double* scratch,
                              hipStream_t s) {
  const int nparts = (int)std::min<int64_t>(ceil_div(n, kBlock), 64);
  double* pval = scratch;
  int64_t* pidx = reinterpret_cast<int64_t*>(scratch + nparts * kb);
  k_col_argmax<<<nparts, kBlock, 0, s>>>(n, kb, x, pval, pidx);
  k_signed_copy<<<ceil_div(n * k, kBlock), kBlock, 0, s>>>(n, kb, k, x, pval, pidx, nparts, out,
                                                           lam, lam_out);
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

__global__ void k_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const double* src,
                            double* dst) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n * kcopy) return;
  const int64_t i = g / kcopy;
  const int j = (int)(g % kcopy);
  dst[i * kdst + j] = src[i * ksrc + j];
}

void launch_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const double* src, double* dst,
                      hipStream_t s) {
  if (n * kcopy == 0) return;
  k_copy_cols<<<ceil_div(n * kcopy, kBlock), kBlock, 0, s>>>(n, ksrc, kdst, kcopy, src, dst);
}

}  // namespace me
