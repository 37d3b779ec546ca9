// Small dense FP64 solves on one workgroup: the Rayleigh-Ritz step of
// LOBPCG (generalized symmetric eigenproblem of the projected pair
// (S^T A S, S^T B S), Section 4.3 asks for B-orthonormal generalized
// eigenvectors), the CholQR coefficients that B-orthonormalise the
// preconditioned residual block, and the dense solve used for graphs of at
// most 48 nodes.
//
// Method: the basis Gram S^T B S is scaled to unit diagonal and Cholesky
// factorised; a column whose pivot falls below a threshold is dropped from
// the basis (it is numerically dependent on the earlier ones) and the
// factorisation restarts.  The standard symmetric problem
// M = L^-1 (D S^T A S D) L^-T is solved by cyclic Jacobi with the parallel
// round-robin pairing (m/2 disjoint rotations per step), all in LDS.
#include <cmath>

#include "common.h"

namespace me {

constexpr int kLd = kMaxBasis + 1;  // padded LDS row stride
constexpr int kDenseThreads = 256;
constexpr int kMaxSweeps = 24;

struct SmallWS {
  double A[kMaxBasis][kLd];   // scaled G_A, then M
  double L[kMaxBasis][kLd];   // scaled G_B, then its Cholesky factor (lower)
  double Li[kMaxBasis][kLd];  // L^-1 (lower)
  double V[kMaxBasis][kLd];   // temporary, then eigenvectors
  double dsc[kMaxBasis];      // diag(G_B)^-1/2 of the active columns
  double ev[kMaxBasis];
  double red[kDenseThreads];
  double red2[kDenseThreads];
  double rc[kMaxBasis / 2], rs[kMaxBasis / 2], rt[kMaxBasis / 2];
  int rp[kMaxBasis / 2], rq[kMaxBasis / 2];
  int idx[kMaxBasis];    // original index of each active (compact) column
  int order[kMaxBasis];  // eigenvalues ascending
  int active[kMaxBasis];
  int ma;
  int fail;
  int flag;
};

// Compact the active columns, scale to unit B-diagonal, symmetrise.
__device__ void load_compact(SmallWS& w, int m, const double* ga, const double* gb) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    int c = 0;
    for (int i = 0; i < m; ++i)
      if (w.active[i]) w.idx[c++] = i;
    w.ma = c;
    w.fail = -1;
  }
  __syncthreads();
  const int ma = w.ma;
  for (int a = tid; a < ma; a += blockDim.x) w.dsc[a] = 1.0 / sqrt(gb[w.idx[a] * m + w.idx[a]]);
  __syncthreads();
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int a = u / ma, b = u % ma;
    const int ia = w.idx[a], ib = w.idx[b];
    const double s = w.dsc[a] * w.dsc[b];
    w.A[a][b] = 0.5 * (ga[ia * m + ib] + ga[ib * m + ia]) * s;
    w.L[a][b] = (a == b) ? 1.0 : 0.5 * (gb[ia * m + ib] + gb[ib * m + ia]) * s;
  }
  __syncthreads();
}

// Right-looking Cholesky of w.L (ma x ma) in place.  Returns the compact
// index of the first pivot below `tol` (or -1).
__device__ int cholesky_lds(SmallWS& w, int ma, double tol) {
  const int tid = threadIdx.x;
  for (int k = 0; k < ma; ++k) {
    if (tid == 0) {
      const double piv = w.L[k][k];
      if (!(piv > tol)) w.fail = k; else w.L[k][k] = sqrt(piv);
    }
    __syncthreads();
    if (w.fail >= 0) return w.fail;
    const double lkk = w.L[k][k];
    for (int i = k + 1 + tid; i < ma; i += blockDim.x) w.L[i][k] /= lkk;
    __syncthreads();
    const int r = ma - k - 1;  // trailing size
    for (int u = tid; u < r * r; u += blockDim.x) {
      const int i = k + 1 + u / r, j = k + 1 + u % r;
      if (j <= i) w.L[i][j] -= w.L[i][k] * w.L[j][k];
    }
    __syncthreads();
  }
  return -1;
}

// Li = L^-1, one column per thread (forward substitution).
__device__ void tri_inverse(SmallWS& w, int ma) {
  const int j = threadIdx.x;
  if (j < ma) {
    for (int i = 0; i < j; ++i) w.Li[i][j] = 0.0;
    for (int i = j; i < ma; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= w.L[i][k] * w.Li[k][j];
      w.Li[i][j] = s / w.L[i][i];
    }
  }
  __syncthreads();
}

// A <- Li A Li^T (symmetrised), using V as temporary.
__device__ void form_standard(SmallWS& w, int ma) {
  const int tid = threadIdx.x;
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int i = u / ma, j = u % ma;
    double s = 0.0;
    for (int k = 0; k <= j; ++k) s += w.A[i][k] * w.Li[j][k];
    w.V[i][j] = s;
  }
  __syncthreads();
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int i = u / ma, j = u % ma;
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += w.Li[i][k] * w.V[k][j];
    w.A[i][j] = s;
  }
  __syncthreads();
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int i = u / ma, j = u % ma;
    if (i < j) {
      const double s = 0.5 * (w.A[i][j] + w.A[j][i]);
      w.A[i][j] = s;
      w.A[j][i] = s;
    }
  }
  __syncthreads();
}

// Cyclic Jacobi with round-robin pairing on w.A (ma x ma, symmetric).
// Eigenvalues to w.ev, eigenvectors to the columns of w.V, ascending order
// of the ma eigenvalues to w.order.
__device__ void jacobi_eig(SmallWS& w, int ma) {
  const int tid = threadIdx.x;
  const int mm = ma + (ma & 1);  // even; index ma is an inert dummy when ma is odd
  const int P = mm / 2;
  for (int u = tid; u < mm * mm; u += blockDim.x) {
    const int i = u / mm, j = u % mm;
    w.V[i][j] = (i == j) ? 1.0 : 0.0;
    if (i >= ma || j >= ma) w.A[i][j] = 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int u = tid; u < ma * ma; u += blockDim.x) {
      const int i = u / ma, j = u % ma;
      const double v = w.A[i][j];
      if (i == j) dg += v * v; else off += v * v;
    }
    w.red[tid] = off;
    w.red2[tid] = dg;
    __syncthreads();
    if (tid == 0) {
      double so = 0.0, sd = 0.0;
      for (int q = 0; q < (int)blockDim.x; ++q) { so += w.red[q]; sd += w.red2[q]; }
      w.flag = (so <= 1e-30 * sd) || so == 0.0;
    }
    __syncthreads();
    if (w.flag) break;
    for (int r = 0; r < mm - 1; ++r) {
      if (tid < P) {
        int p, q;
        if (tid == 0) { p = r; q = mm - 1; }
        else { p = (r + tid) % (mm - 1); q = (r - tid + mm - 1) % (mm - 1); }
        const double apq = w.A[p][q];
        double c = 1.0, s = 0.0, t = 0.0;
        if (apq != 0.0) {
          const double app = w.A[p][p], aqq = w.A[q][q];
          const double theta = (aqq - app) / (2.0 * apq);
          if (fabs(theta) > 1e150) t = 0.5 / theta;
          else t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        w.rp[tid] = p; w.rq[tid] = q; w.rc[tid] = c; w.rs[tid] = s; w.rt[tid] = t;
      }
      __syncthreads();
      // A <- J^T A J on 2x2 blocks (a <= b, mirrored), V <- V J
      for (int u = tid; u < P * P; u += blockDim.x) {
        const int a = u / P, b = u % P;
        if (a > b) continue;
        const int p = w.rp[a], q = w.rq[a];
        if (a == b) {
          const double apq = w.A[p][q], t = w.rt[a];
          w.A[p][p] -= t * apq;
          w.A[q][q] += t * apq;
          if (w.rs[a] != 0.0) { w.A[p][q] = 0.0; w.A[q][p] = 0.0; }
          continue;
        }
        const int r2 = w.rp[b], s2 = w.rq[b];
        const double ca = w.rc[a], sa = w.rs[a], cb = w.rc[b], sb = w.rs[b];
        const double mpr = w.A[p][r2], mps = w.A[p][s2], mqr = w.A[q][r2], mqs = w.A[q][s2];
        const double ypr = cb * mpr - sb * mps, yps = sb * mpr + cb * mps;
        const double yqr = cb * mqr - sb * mqs, yqs = sb * mqr + cb * mqs;
        const double npr = ca * ypr - sa * yqr, nqr = sa * ypr + ca * yqr;
        const double nps = ca * yps - sa * yqs, nqs = sa * yps + ca * yqs;
        w.A[p][r2] = npr; w.A[r2][p] = npr;
        w.A[q][r2] = nqr; w.A[r2][q] = nqr;
        w.A[p][s2] = nps; w.A[s2][p] = nps;
        w.A[q][s2] = nqs; w.A[s2][q] = nqs;
      }
      for (int u = tid; u < mm * P; u += blockDim.x) {
        const int i = u / P, a = u % P;
        const int p = w.rp[a], q = w.rq[a];
        const double c = w.rc[a], s = w.rs[a];
        const double vp = w.V[i][p], vq = w.V[i][q];
        w.V[i][p] = c * vp - s * vq;
        w.V[i][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < ma; i += blockDim.x) w.ev[i] = w.A[i][i];
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < ma; ++i) w.order[i] = i;
    for (int i = 1; i < ma; ++i) {  // insertion sort, stable
      int v = w.order[i];
      int j = i - 1;
      while (j >= 0 && w.ev[w.order[j]] > w.ev[v]) { w.order[j + 1] = w.order[j]; --j; }
      w.order[j + 1] = v;
    }
  }
  __syncthreads();
}

// Generalized eigenpairs of (ga, gb) (m x m) with column dropping; on exit
// w.ma >= 0 active columns, w.Li, w.V, w.ev, w.order, w.dsc, w.idx valid.
__device__ void small_geneig(SmallWS& w, int m, const double* ga, const double* gb,
                             double piv_tol) {
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += blockDim.x) {
    const double bd = gb[i * m + i], ad = ga[i * m + i];
    w.active[i] = (bd > 0.0) && isfinite(bd) && isfinite(ad);
  }
  __syncthreads();
  for (int attempt = 0; attempt <= m; ++attempt) {
    load_compact(w, m, ga, gb);
    const int ma = w.ma;
    if (ma == 0) break;
    const int f = cholesky_lds(w, ma, piv_tol);
    if (f < 0) break;
    if (tid == 0) w.active[w.idx[f]] = 0;
    __syncthreads();
  }
  const int ma = w.ma;
  if (ma == 0 || w.fail >= 0) {
    if (tid == 0) w.ma = 0;
    __syncthreads();
    return;
  }
  tri_inverse(w, ma);
  form_standard(w, ma);
  jacobi_eig(w, ma);
}

// coef[:, t] (m rows) = D Li^T V[:, order[t]] scattered to the original rows.
__device__ void write_coef(SmallWS& w, int m, int kout, double* coef, double* lam) {
  const int tid = threadIdx.x;
  const int ma = w.ma;
  for (int u = tid; u < m * kout; u += blockDim.x) coef[u] = 0.0;
  __syncthreads();
  for (int u = tid; u < ma * kout; u += blockDim.x) {
    const int a = u / kout, t = u % kout;
    double s = 0.0;
    if (t < ma) {
      const int col = w.order[t];
      for (int j = a; j < ma; ++j) s += w.Li[j][a] * w.V[j][col];
      s *= w.dsc[a];
    }
    coef[w.idx[a] * kout + t] = s;
  }
  for (int t = tid; t < kout; t += blockDim.x) lam[t] = (t < ma) ? w.ev[w.order[t]] : 0.0;
  __syncthreads();
}

// coef holds two (m x kb) matrices: first the P update (rows of the X block
// zeroed), then the X update C = [C_X; C_W; C_P].
__global__ void __launch_bounds__(kDenseThreads) k_rayleigh_ritz(int kb, int nb, const double* ga,
                                                                 const double* gb, double piv_tol,
                                                                 double* coef, double* lam,
                                                                 Ctrl* ctrl, int final_pass) {
  __shared__ SmallWS w;
  if (!final_pass && ctrl->done) return;
  const int m = kb * nb;
  double* cp = coef;
  double* cx = coef + m * kb;
  small_geneig(w, m, ga, gb, piv_tol);
  if (w.ma < kb) {
    // the X block itself is degenerate or non-finite: keep X, flag it
    if (threadIdx.x == 0) {
      ctrl->nonfinite = 1;
      ctrl->done = 1;
    }
    for (int u = threadIdx.x; u < m * kb; u += blockDim.x) {
      const int i = u / kb, t = u % kb;
      cx[u] = (i == t) ? 1.0 : 0.0;
      cp[u] = 0.0;
    }
    return;
  }
  write_coef(w, m, kb, cx, lam);
  for (int u = threadIdx.x; u < m * kb; u += blockDim.x) cp[u] = (u / kb < kb) ? 0.0 : cx[u];
  if (threadIdx.x == 0) {
    ctrl->nbasis_last = w.ma;
    ctrl->dropped = m - w.ma;
  }
}

void launch_rayleigh_ritz(int kb, int nb, const double* ga, const double* gb, double piv_tol,
                          double* coef, double* lam, Ctrl* ctrl, int final_pass, hipStream_t s) {
  k_rayleigh_ritz<<<1, kDenseThreads, 0, s>>>(kb, nb, ga, gb, piv_tol, coef, lam, ctrl,
                                              final_pass);
}

// CholQR coefficients for W <- (W - X C) D R^-1, from g = [C; G] where
// C = X^T B W and G = W^T B W (both kb x kb, row-major, stacked).  The
// projected Gram is G - C^T C (X^T B X = I).  Columns whose projected norm
// or Cholesky pivot is below piv_tol (relative) become zero.
__global__ void __launch_bounds__(kDenseThreads) k_cholqr_coef(int kb, const double* g,
                                                               double piv_tol, double* coef,
                                                               const Ctrl* ctrl) {
  __shared__ SmallWS w;
  __shared__ double Gp[kMaxBlockCols][kMaxBlockCols + 1];
  if (ctrl && ctrl->done) return;
  const int tid = threadIdx.x;
  const double* C = g;
  const double* G = g + kb * kb;
  for (int u = tid; u < kb * kb; u += blockDim.x) {
    const int i = u / kb, j = u % kb;
    double s = 0.5 * (G[i * kb + j] + G[j * kb + i]);
    for (int l = 0; l < kb; ++l) s -= C[l * kb + i] * C[l * kb + j];
    Gp[i][j] = s;
  }
  __syncthreads();
  for (int i = tid; i < kb; i += blockDim.x) {
    const double gd = Gp[i][i], orig = G[i * kb + i];
    w.active[i] = (gd > piv_tol * orig) && isfinite(gd) && (orig > 0.0);
  }
  __syncthreads();
  int ma = 0;
  for (int attempt = 0; attempt <= kb; ++attempt) {
    if (tid == 0) {
      int c = 0;
      for (int i = 0; i < kb; ++i)
        if (w.active[i]) w.idx[c++] = i;
      w.ma = c;
      w.fail = -1;
    }
    __syncthreads();
    ma = w.ma;
    for (int a = tid; a < ma; a += blockDim.x) w.dsc[a] = 1.0 / sqrt(Gp[w.idx[a]][w.idx[a]]);
    __syncthreads();
    for (int u = tid; u < ma * ma; u += blockDim.x) {
      const int a = u / ma, b = u % ma;
      w.L[a][b] = (a == b) ? 1.0 : Gp[w.idx[a]][w.idx[b]] * w.dsc[a] * w.dsc[b];
    }
    __syncthreads();
    if (ma == 0) break;
    const int f = cholesky_lds(w, ma, piv_tol);
    if (f < 0) break;
    if (tid == 0) w.active[w.idx[f]] = 0;
    __syncthreads();
  }
  if (ma > 0 && w.fail < 0) tri_inverse(w, ma);
  // coef W-part: (D R^-1)[ia][it] = dsc[a] * Li[t][a]; X-part: -C * that
  double* cx = coef;
  double* cw = coef + kb * kb;
  for (int u = tid; u < kb * kb; u += blockDim.x) cw[u] = 0.0;
  __syncthreads();
  if (ma > 0 && w.fail < 0) {
    for (int u = tid; u < ma * ma; u += blockDim.x) {
      const int a = u / ma, t = u % ma;
      cw[w.idx[a] * kb + w.idx[t]] = (t >= a) ? w.dsc[a] * w.Li[t][a] : 0.0;
    }
  }
  __syncthreads();
  for (int u = tid; u < kb * kb; u += blockDim.x) {
    const int l = u / kb, t = u % kb;
    double s = 0.0;
    for (int a = 0; a < kb; ++a) s -= C[l * kb + a] * cw[a * kb + t];
    cx[u] = s;
  }
}

void launch_cholqr_coef(int kb, const double* g, double piv_tol, double* coef, const Ctrl* ctrl,
                        hipStream_t s) {
  k_cholqr_coef<<<1, kDenseThreads, 0, s>>>(kb, g, piv_tol, coef, ctrl);
}

// Dense generalized problem for graphs with n <= 48: all n pairs.
__global__ void __launch_bounds__(kDenseThreads) k_dense_geneig(int n, const double* a,
                                                                const double* bmat, double* vec,
                                                                double* lam) {
  __shared__ SmallWS w;
  small_geneig(w, n, a, bmat, 1e-300);
  write_coef(w, n, n, vec, lam);
}

void launch_dense_geneig(int n, const double* a_dense, const double* b_dense, double* vec,
                         double* lam, hipStream_t s) {
  k_dense_geneig<<<1, kDenseThreads, 0, s>>>(n, a_dense, b_dense, vec, lam);
}

}  // namespace me
