// Small dense FP64 solves on one workgroup: the Rayleigh-Ritz step of
// LOBPCG (generalized symmetric eigenproblem of the projected pair
// (S^T A S, S^T B S), Section 4.3 asks for B-orthonormal generalized
// eigenvectors), the CholQR coefficients that B-orthonormalise the
// preconditioned residual block, and the dense solve used for graphs of at
// most 48 nodes.
//
// Method: the basis Gram S^T B S is scaled to unit diagonal and Cholesky
// factorised; a column whose pivot falls below a threshold is dropped from
// the basis (it is numerically dependent on the earlier ones) and skipped by
// the rest of the factorisation.  The standard symmetric problem
// M = L^-1 (D S^T A S D) L^-T is solved by cyclic Jacobi with the parallel
// round-robin pairing (m/2 disjoint rotations per step), all in LDS.
#include <cmath>

#include "common.h"
#include "engine.h"

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
  double red[kDenseThreads / kWave];
  double red2[kDenseThreads / kWave];
  double rc[kMaxBasis / 2], rs[kMaxBasis / 2];
  int idx[kMaxBasis];    // original index of each active (compact) column
  int order[kMaxBasis];  // eigenvalues ascending
  int active[kMaxBasis];
  int keep[kMaxBasis];
  int ma;
  int flag;
};

// w.idx = indices i < m (m <= 64) with w.active[i], ascending; w.ma = count.
__device__ __forceinline__ void compact_active(SmallWS& w, int m) {
  const int tid = threadIdx.x;
  if (tid < kWave) {
    const bool a = tid < m && w.active[tid];
    const unsigned long long mask = __ballot(a);
    if (a) w.idx[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
    if (tid == 0) w.ma = __popcll(mask);
  }
  __syncthreads();
}

// Compact the active columns, scale to unit B-diagonal, symmetrise.
__device__ __forceinline__ void load_compact(SmallWS& w, int m, const double* ga, const double* gb) {
  const int tid = threadIdx.x;
  compact_active(w, m);
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

// Right-looking Cholesky of w.L (ma x ma) in place.  A column whose pivot
// falls below `tol` is skipped (keep[k] = 0): its entries are zeroed and it
// takes no part in later updates, so the factor restricted to the kept
// columns is the Cholesky factor of the kept principal submatrix.
__device__ __forceinline__ void cholesky_skip(SmallWS& w, int ma, double tol) {
  const int tid = threadIdx.x;
  for (int k = 0; k < ma; ++k) {
    if (tid == 0) {
      const double piv = w.L[k][k];
      const bool ok = piv > tol;
      w.keep[k] = ok;
      w.L[k][k] = ok ? sqrt(piv) : 1.0;
      w.ev[k] = ok ? 1.0 / sqrt(piv) : 0.0;
    }
    __syncthreads();
    const double rk = w.ev[k];
    for (int i = k + 1 + tid; i < ma; i += blockDim.x) w.L[i][k] *= rk;
    __syncthreads();
    if (rk != 0.0) {
      const int r = ma - k - 1;  // trailing size
      for (int u = tid; u < r * r; u += blockDim.x) {
        const int i = k + 1 + u / r, j = k + 1 + u % r;
        if (j <= i) w.L[i][j] -= w.L[i][k] * w.L[j][k];
      }
    }
    __syncthreads();
  }
}

// Keeps the columns with keep[] set: compacts idx, dsc, A (scaled G_A) and
// the Cholesky factor L to the kept positions (V is scratch).
__device__ __forceinline__ void compact_kept(SmallWS& w, int ma) {
  const int tid = threadIdx.x;
  if (tid < kWave) {
    const bool a = tid < ma && w.keep[tid];
    const unsigned long long mask = __ballot(a);
    if (a) w.order[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
    if (tid == 0) w.flag = __popcll(mask);
  }
  __syncthreads();
  const int mk = w.flag;
  for (int u = tid; u < mk * mk; u += blockDim.x) {
    const int a = u / mk, b = u % mk;
    w.V[a][b] = w.L[w.order[a]][w.order[b]];
  }
  double dsc = 0.0;
  int id = 0;
  if (tid < mk) {
    dsc = w.dsc[w.order[tid]];
    id = w.idx[w.order[tid]];
  }
  __syncthreads();
  for (int u = tid; u < mk * mk; u += blockDim.x) {
    const int a = u / mk, b = u % mk;
    w.L[a][b] = w.V[a][b];
  }
  for (int u = tid; u < mk * mk; u += blockDim.x) {
    const int a = u / mk, b = u % mk;
    w.V[a][b] = w.A[w.order[a]][w.order[b]];
  }
  if (tid < mk) {
    w.dsc[tid] = dsc;
    w.idx[tid] = id;
  }
  __syncthreads();
  for (int u = tid; u < mk * mk; u += blockDim.x) {
    const int a = u / mk, b = u % mk;
    w.A[a][b] = w.V[a][b];
  }
  if (tid == 0) w.ma = mk;
  __syncthreads();
}

// Li = L^-1 row by row: row i needs rows < i; entries of a row in parallel.
__device__ __forceinline__ void tri_inverse(SmallWS& w, int ma) {
  const int tid = threadIdx.x;
  for (int i = tid; i < ma; i += blockDim.x) w.ev[i] = 1.0 / w.L[i][i];
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int i = u / ma, j = u % ma;
    if (j > i) w.Li[i][j] = 0.0;
  }
  __syncthreads();
  for (int i = 0; i < ma; ++i) {
    for (int j = tid; j <= i; j += blockDim.x) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= w.L[i][k] * w.Li[k][j];
      w.Li[i][j] = s * w.ev[i];
    }
    __syncthreads();
  }
}

// A <- Li A Li^T (symmetrised), using V as temporary.
__device__ __forceinline__ void form_standard(SmallWS& w, int ma) {
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

// Rotation (c, s) that (nearly) annihilates a_pq of the 2x2 block
// [[a_pp, a_pq], [a_pq, a_qq]] (Rutishauser's formulas).  The angle is
// computed in FP32 with the native reciprocal and square root; (c, s) is
// then renormalised in FP64 so that c^2 + s^2 = 1 to FP64 rounding: the
// similarity stays exactly orthogonal, only the annihilation is inexact
// (relative 1e-7), which the next sweep removes.
__device__ __forceinline__ void rotation(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  const float h = (float)(2.0 * apq);
  if (h == 0.0f) return;
  const float th = (float)(aqq - app) * __builtin_amdgcn_rcpf(h);
  const float r = __builtin_amdgcn_sqrtf(fmaf(th, th, 1.0f));
  const float t = copysignf(1.0f, th) * __builtin_amdgcn_rcpf(fabsf(th) + r);
  if (!(t == t)) return;
  const float cf = __builtin_amdgcn_rsqf(fmaf(t, t, 1.0f));
  double cd = (double)cf, sd = (double)(t * cf);
  // two Newton steps of x^-1/2 about 1 for x = c^2 + s^2
  const double x = cd * cd + sd * sd;
  double g = 1.5 - 0.5 * x;
  g = g * (1.5 - 0.5 * x * g * g);
  c = cd * g;
  s = sd * g;
}

// Pair k of round r in the round-robin ordering of mm indices:
// (r, mm - 1) for k = 0, else ((r + k) mod (mm - 1), (r - k) mod (mm - 1)).
__device__ __forceinline__ void round_pair(int r, int k, int mm, int& p, int& q) {
  const int n1 = mm - 1;
  if (k == 0) {
    p = r;
    q = n1;
  } else {
    p = r + k;
    if (p >= n1) p -= n1;
    q = r - k + n1;
    if (q >= n1) q -= n1;
  }
}

// Cyclic Jacobi with round-robin pairing on w.A (ma x ma, symmetric): mm/2
// disjoint rotations per round, mm - 1 rounds per sweep.  Eigenvalues to
// w.ev, eigenvectors to the columns of w.V, ascending order to w.order.
__device__ __forceinline__ void jacobi_eig(SmallWS& w, int ma) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int mm = ma + (ma & 1);  // even; index ma is an inert dummy when ma is odd
  const int P = mm / 2;
  for (int u = tid; u < mm * mm; u += nt) {
    const int i = u / mm, j = u % mm;
    w.V[i][j] = (i == j) ? 1.0 : 0.0;
    if (i >= ma || j >= ma) w.A[i][j] = 0.0;
  }
  // work items of a round, fixed per thread: 2x2 blocks (a <= b), then
  // (row of V, pair) updates; decoded once into registers
  // 6 items per thread cover a 48-column basis on 256 threads and a
  // 16-column basis on 64 threads (the launch rule of dense_threads)
  constexpr int kMaxItems = 6;
  const int nblk = P * (P + 1) / 2;
  const int nitem = nblk + mm * P;
  int ia[kMaxItems], ib[kMaxItems];  // block: (a, b); V item: (a, -1 - row)
#pragma unroll
  for (int t = 0; t < kMaxItems; ++t) {
    const int u = tid + t * nt;
    ia[t] = -1;
    ib[t] = 0;
    if (u < nblk) {
      int a = 0, rem = u;
      while (rem >= P - a) { rem -= P - a; ++a; }
      ia[t] = a;
      ib[t] = a + rem;
    } else if (u < nitem) {
      const int v = u - nblk;
      ia[t] = v % P;
      ib[t] = -1 - v / P;
    }
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int u = tid; u < ma * ma; u += nt) {
      const int i = u / ma, j = u - i * ma;
      const double v = w.A[i][j];
      if (i == j) dg += v * v; else off += v * v;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dg += __shfl_xor(dg, o);
    }
    if ((tid & (kWave - 1)) == 0) {
      w.red[tid / kWave] = off;
      w.red2[tid / kWave] = dg;
    }
    __syncthreads();
    if (tid == 0) {
      double so = 0.0, sd = 0.0;
      for (int q = 0; q < nt / kWave; ++q) { so += w.red[q]; sd += w.red2[q]; }
      w.flag = (so <= 1e-26 * sd) || so == 0.0;
    }
    __syncthreads();
    if (w.flag) break;
    for (int r = 0; r < mm - 1; ++r) {
      if (tid < P) {
        int p, q;
        round_pair(r, tid, mm, p, q);
        double c, sn;
        rotation(w.A[p][p], w.A[q][q], w.A[p][q], c, sn);
        w.rc[tid] = c;
        w.rs[tid] = sn;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kMaxItems; ++t) {
        const int a = ia[t];
        if (a < 0 || t * nt >= nitem) continue;
        int p, q;
        round_pair(r, a, mm, p, q);
        const double ca = w.rc[a], sa = w.rs[a];
        if (ib[t] >= 0) {
          // A <- J^T A J on the 2x2 block (a, b), mirrored
          const int b = ib[t];
          int r2, s2;
          round_pair(r, b, mm, r2, s2);
          const double cb = w.rc[b], sb = w.rs[b];
          const double mpr = w.A[p][r2], mps = w.A[p][s2], mqr = w.A[q][r2], mqs = w.A[q][s2];
          const double ypr = cb * mpr - sb * mps, yps = sb * mpr + cb * mps;
          const double yqr = cb * mqr - sb * mqs, yqs = sb * mqr + cb * mqs;
          const double npr = ca * ypr - sa * yqr, nqr = sa * ypr + ca * yqr;
          const double nps = ca * yps - sa * yqs, nqs = sa * yps + ca * yqs;
          if (a == b) {
            w.A[p][p] = npr;
            w.A[q][q] = nqs;
            const double o2 = 0.5 * (nps + nqr);
            w.A[p][q] = o2;
            w.A[q][p] = o2;
          } else {
            w.A[p][r2] = npr; w.A[r2][p] = npr;
            w.A[q][r2] = nqr; w.A[r2][q] = nqr;
            w.A[p][s2] = nps; w.A[s2][p] = nps;
            w.A[q][s2] = nqs; w.A[s2][q] = nqs;
          }
        } else {
          // V <- V J on row i
          const int i = -1 - ib[t];
          const double vp = w.V[i][p], vq = w.V[i][q];
          w.V[i][p] = ca * vp - sa * vq;
          w.V[i][q] = sa * vp + ca * vq;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < ma; i += nt) w.ev[i] = w.A[i][i];
  __syncthreads();
  // stable rank sort, ascending
  for (int i = tid; i < ma; i += nt) {
    const double v = w.ev[i];
    int r = 0;
    for (int j = 0; j < ma; ++j) {
      const double u = w.ev[j];
      r += (u < v) || (u == v && j < i);
    }
    w.order[r] = i;
  }
  __syncthreads();
}

// Generalized eigenpairs of (ga, gb) (m x m) with column dropping; on exit
// w.ma >= 0 kept columns, w.Li, w.V, w.ev, w.order, w.dsc, w.idx valid.
__device__ __forceinline__ void small_geneig(SmallWS& w, int m, const double* ga, const double* gb,
                                             double piv_tol) {
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += blockDim.x) {
    const double bd = gb[i * m + i], ad = ga[i * m + i];
    w.active[i] = (bd > 0.0) && isfinite(bd) && isfinite(ad);
  }
  __syncthreads();
  load_compact(w, m, ga, gb);
  if (w.ma == 0) return;
  cholesky_skip(w, w.ma, piv_tol);
  compact_kept(w, w.ma);
  const int ma = w.ma;
  if (ma == 0) return;
  tri_inverse(w, ma);
  form_standard(w, ma);
  jacobi_eig(w, ma);
}

// coef[:, t] (m rows) = D Li^T V[:, order[t]] scattered to the original rows.
__device__ __forceinline__ void write_coef(SmallWS& w, int m, int kout, double* coef, double* lam) {
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
__device__ __forceinline__ void rr_body(SmallWS& w, int kb, int nb, const double* ga,
                                        const double* gb, double piv_tol, double* coef,
                                        double* lam, Ctrl* ctrl) {
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

// One workgroup per slot of the set; G_B = gram (m x m), G_A = gram + m^2.
__global__ void __launch_bounds__(kDenseThreads) k_sl_rayleigh_ritz(const SlotDev* sl,
                                                                    const int32_t* slots, int kb,
                                                                    int nb, double piv_tol,
                                                                    int final_pass) {
  __shared__ SmallWS w;
  const SlotDev& d = sl[slots[blockIdx.x]];
  if (!final_pass && d.ctrl->done) return;
  const int m = kb * nb;
  rr_body(w, kb, nb, d.gram + m * m, d.gram, piv_tol, d.coef, d.lam, d.ctrl);
}

// One wave suffices (and avoids cross-wave barriers) for bases up to 16.
static int dense_threads(int m) { return m <= 16 ? kWave : kDenseThreads; }

void sl_rayleigh_ritz(const SlotDev* sl, const TileSet& ts, int nb, double piv_tol,
                      int final_pass, hipStream_t s) {
  if (ts.nslots == 0) return;
  k_sl_rayleigh_ritz<<<ts.nslots, dense_threads(ts.kb * nb), 0, s>>>(sl, ts.slots, ts.kb, nb,
                                                                      piv_tol, final_pass);
}

// CholQR coefficients for W <- (W - X C) D R^-1, from g = [C; G] where
// C = X^T B W and G = W^T B W (both kb x kb, row-major, stacked).  The
// projected Gram is G - C^T C (X^T B X = I).  Columns whose projected norm
// or Cholesky pivot is below piv_tol (relative) become zero.
__global__ void __launch_bounds__(kWave) k_sl_cholqr_coef(const SlotDev* sl,
                                                          const int32_t* slots, int kb,
                                                          double piv_tol) {
  __shared__ SmallWS w;
  __shared__ double Gp[kMaxBlockCols][kMaxBlockCols + 1];
  const SlotDev& d = sl[slots[blockIdx.x]];
  if (d.ctrl->done) return;
  const double* g = d.gram;
  double* coef = d.coefw;
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
  compact_active(w, kb);
  int ma = w.ma;
  for (int a = tid; a < ma; a += blockDim.x) w.dsc[a] = 1.0 / sqrt(Gp[w.idx[a]][w.idx[a]]);
  __syncthreads();
  for (int u = tid; u < ma * ma; u += blockDim.x) {
    const int a = u / ma, b = u % ma;
    w.L[a][b] = (a == b) ? 1.0 : Gp[w.idx[a]][w.idx[b]] * w.dsc[a] * w.dsc[b];
  }
  __syncthreads();
  if (ma > 0) {
    cholesky_skip(w, ma, piv_tol);
    compact_kept(w, ma);
    ma = w.ma;
    if (ma > 0) tri_inverse(w, ma);
  }
  // coef W-part: (D R^-1)[ia][it] = dsc[a] * Li[t][a]; X-part: -C * that
  __shared__ double Cw[kMaxBlockCols][kMaxBlockCols + 1];
  for (int u = tid; u < kb * kb; u += blockDim.x) Cw[u / kb][u % kb] = 0.0;
  __syncthreads();
  if (ma > 0) {
    for (int u = tid; u < ma * ma; u += blockDim.x) {
      const int a = u / ma, t = u % ma;
      Cw[w.idx[a]][w.idx[t]] = (t >= a) ? w.dsc[a] * w.Li[t][a] : 0.0;
    }
  }
  __syncthreads();
  double* cx = coef;
  double* cw = coef + kb * kb;
  for (int u = tid; u < kb * kb; u += blockDim.x) {
    const int l = u / kb, t = u % kb;
    double s = 0.0;
    for (int a = 0; a < kb; ++a) s -= C[l * kb + a] * Cw[a][t];
    cx[u] = s;
    cw[u] = Cw[l][t];
  }
}

void sl_cholqr_coef(const SlotDev* sl, const TileSet& ts, double piv_tol, hipStream_t s) {
  if (ts.nslots == 0) return;
  k_sl_cholqr_coef<<<ts.nslots, kWave, 0, s>>>(sl, ts.slots, ts.kb, piv_tol);
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
  k_dense_geneig<<<1, dense_threads(n), 0, s>>>(n, a_dense, b_dense, vec, lam);
}

}  // namespace me
