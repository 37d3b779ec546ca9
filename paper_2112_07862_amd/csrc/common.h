// Internal declarations shared by the HIP translation units of libmembed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "membed.h"

#define ME_TRY(expr)                                  \
  do {                                                \
    hipError_t me_err_ = (expr);                      \
    if (me_err_ != hipSuccess) return ME_ERR_HIP;     \
  } while (0)

#define ME_TRY_STATUS(expr)                           \
  do {                                                \
    int me_st_ = (expr);                              \
    if (me_st_ < 0) return me_st_;                    \
  } while (0)

namespace me {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads of the streaming kernels
constexpr int kMaxBlockCols = 16;    // largest LOBPCG block width
constexpr int kMaxBasis = 48;        // 3 x kMaxBlockCols: Rayleigh-Ritz basis size
constexpr int kDenseMaxN = 48;       // graphs up to this size are solved densely
constexpr int kPartialBlocks = 256;  // grid of the reducing streaming kernels
constexpr int kMaxChebDegree = 64;   // largest Chebyshev preconditioner degree

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump allocator over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    if (off + bytes > cap) return nullptr;
    used = off + bytes;
    return reinterpret_cast<T*>(base + off);
  }
  static size_t round(size_t bytes) { return (bytes + 255) & ~size_t(255); }
};

// Device-side control block of one LOBPCG solve.  Written by the
// single-block finalize kernels, read by every iteration kernel (early exit
// once `done` is set) and copied to pinned host memory every few iterations.
struct Ctrl {
  int done;        // 1 = converged or out of iterations
  int iter;        // iterations completed
  int nconv;       // columns (of the required ones) with rho <= tol
  int max_iter;
  int need;        // number of leading columns that must converge
  int kb;          // block width
  int nbasis_last; // basis size used by the last Rayleigh-Ritz
  int dropped;     // basis columns dropped by the last Rayleigh-Ritz
  int nonfinite;   // a NaN / Inf was seen
  int pad;
  double tol;
  double lam_floor;          // |lambda| below this is treated as zero ...
  double lam_scale;          // ... and replaced by this operator scale in rho
  double rho[kMaxBlockCols]; // last residuals
  // Chebyshev preconditioner: spectrum of D^-1 Op taken as [cheb_a, cheb_b];
  // cheb_a follows the leading Ritz pair (cheb_afac times its D-Rayleigh
  // quotient).  Step k uses dd <- alpha_k dd + beta_k D^-1 (R - Op y).
  int cheb_deg;
  int pad2;
  double cheb_afac;
  double cheb_a, cheb_b, cheb_theta;
  double cheb_alpha[kMaxChebDegree];
  double cheb_beta[kMaxChebDegree];
};

// Packed graph operators (device pointers into one allocation).
struct GraphOps {
  int64_t n = 0, nnz_w = 0, nnz_t = 0;
  int components = 0;   // of the two-hop graph
  double eps = 0, mu = 0, maxden = 0, max_diag_a = 0;
  int eps_iters = 0;
  int status = 0;
  // W in CSR (copy of the input, int64 row pointers)
  int64_t* w_rp = nullptr;
  int32_t* w_col = nullptr;
  double* w_val = nullptr;
  // two-hop pattern
  int64_t* t_rp = nullptr;
  int32_t* t_col = nullptr;
  int32_t* t_cnt = nullptr;
  // per-node scalars
  double* d = nullptr;      // degree
  double* qdiag = nullptr;  // Q_ii
  double* r = nullptr;      // Gershgorin radius of row i of A
  double* b = nullptr;      // B = diag(b)
  double* dinv = nullptr;   // 1 / A_ii (Jacobi)
  double* invt = nullptr;   // 1 / T_i (0 if T_i = 0)
  double* qinv = nullptr;   // 1 / Q_ii (0 if Q_ii = 0)
  float* qinv32 = nullptr;
  double cheb_b_a = 2.0;    // Gershgorin bound of the spectrum of diag(A)^-1 A
  double cheb_b_q = 2.0;    // and of diag(Q)^-1 Q
  float* b32 = nullptr;
  float* dinv32 = nullptr;
  float* invt32 = nullptr;
  // Solver order (locality permutation): solver row i' is user row perm[i'].
  int32_t* perm = nullptr;     // solver index -> user index
  int32_t* iperm = nullptr;    // user index -> solver index
  double *invt_s = nullptr, *qinv_s = nullptr, *b_s = nullptr, *dinv_s = nullptr;
  float *invt32_s = nullptr, *qinv32_s = nullptr, *b32_s = nullptr, *dinv32_s = nullptr;
  // merged difference-form operator in solver order: row i = [W cols | T cols]
  int32_t* a_rp = nullptr;     // int32[n+1]
  int32_t* a_split = nullptr;  // int32[n]: first T position of row i
  int32_t* a_col = nullptr;    // int32[nnz_w + nnz_t]
  double* a_w = nullptr;       // W weights at the W positions (T positions unused)
  float* a_w32 = nullptr;
  void* mem = nullptr;   // per-node arrays, W copy
  void* mem2 = nullptr;  // T columns and the merged operator
  size_t mem_bytes = 0;
  int device = 0;
};

// ---- launchers: build.hip -------------------------------------------------
int build_graph_ops(const me_csr* W, const me_opts* o, hipStream_t s, GraphOps* g, me_info* info);

// ---- launchers: dense.hip -------------------------------------------------
// Rayleigh-Ritz on a basis of nb blocks of kb columns: ga, gb (m x m,
// m = nb*kb, row-major, device) -> coef (m x kb) and lam (kb); column-drop
// threshold `piv_tol` on the normalised Cholesky pivots.
void launch_rayleigh_ritz(int kb, int nb, const double* ga, const double* gb, double piv_tol,
                          double* coef, double* lam, Ctrl* ctrl, int final_pass, hipStream_t s);
// Projected CholQR coefficients for W <- (W - X C) R^-1 from
// g = [X W]^T B W ((2kb) x kb): writes coef ((2kb) x kb) = [-C R^-1; R^-1].
void launch_cholqr_coef(int kb, const double* g, double piv_tol, double* coef, const Ctrl* ctrl,
                        hipStream_t s);
// Dense generalized eigenproblem for graphs with n <= 48: all n pairs of
// (a_dense, b_dense), both n x n; vec n x n (column t = pair t), lam ascending.
void launch_dense_geneig(int n, const double* a_dense, const double* b_dense, double* vec,
                         double* lam, hipStream_t s);

// ---- launchers: stream_ops.hip ---------------------------------------------
enum OpKind { OP_A = 0, OP_Q = 1 };

template <typename T>
void launch_spmm(const GraphOps& g, int kb, OpKind op, const T* x, T* y, const int* done,
                 hipStream_t s);
// precond: 0 W = R, 1 W = dinv R (Jacobi); dinv (D^-1) is always read
template <typename T>
void launch_cheb_first(const GraphOps& g, int kb, const T* r, const T* dinv, const Ctrl* ctrl,
                       T* y, T* dd, hipStream_t s);
template <typename T>
void launch_cheb_step(const GraphOps& g, int kb, OpKind op, int k, const T* r, const T* dinv,
                      const Ctrl* ctrl, const T* yin, T* yout, T* dd, hipStream_t s);
template <typename T>
void launch_resid(int64_t n, int kb, const T* x, const T* ax, const T* bdiag, const T* dinv,
                  int precond, const double* lam, T* w, double* partials, int nparts,
                  const int* done, hipStream_t s);
void launch_resid_finalize(int kb, const double* partials, int nparts, const double* lam,
                           Ctrl* ctrl, int final_pass, hipStream_t s);
// G1 = U^T diag(wdiag) V, G2 = U^T V2 (partials per block, G1 then G2)
template <typename T>
void launch_gram(int64_t n, int kb, int nu, const T* const* u, int nv, const T* const* v,
                 const T* wdiag, int nv2, const T* const* v2, double* partials, int nparts,
                 const int* done, hipStream_t s);
void launch_reduce_partials(int nparts, int nent, const double* partials, double* out,
                            const int* done, hipStream_t s);
template <typename T>
void launch_combine(int64_t n, int kb, int nin, const T* const* in, int nout, T* const* out,
                    const double* coef, const int* done, hipStream_t s);
// Two groups sharing coefficients: group g maps in_g to out_g.
template <typename T>
void launch_combine2(int64_t n, int kb, int nin, int ngroup, const T* const* in0,
                     const T* const* in1, int nout, T* const* out0, T* const* out1,
                     const double* coef, const int* done, hipStream_t s);
template <typename T>
void launch_deflate_ones(int64_t n, int kb, T* x, double* partials, int nparts, double* sums,
                         const int* done, hipStream_t s);
// start block in solver order (perm: solver -> user row, may be null)
void launch_fill_random(int64_t n, int kb, int kcopy, const double* x0, uint64_t seed,
                        const int32_t* perm, double* x, hipStream_t s);
// scratch: 64 * kb * 16 bytes; x in solver order, out in user order
void launch_sign_fix_and_copy(int64_t n, int kb, int k, const double* x, double* out,
                              const double* lam, double* lam_out, double* scratch,
                              const int32_t* perm, const int32_t* iperm, hipStream_t s);
template <typename Tin, typename Tout>
void launch_convert(int64_t count, const Tin* in, Tout* out, hipStream_t s);
void launch_scale_rows(int64_t n, int k, const double* b, const double* x, double* y,
                       hipStream_t s);
// dense n x n operator (which 0: A, 1: Q) and matching B (diag(b) or I)
void launch_dense_ops(const GraphOps& g, int which, double* out, double* bmat, hipStream_t s);
// dst[i][j] = src[map ? map[i] : i][j]
void launch_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const int32_t* map,
                      const double* src, double* dst, hipStream_t s);

// ---- timing.hip -------------------------------------------------------------
enum KTimeKind { KT_OFF = 0, KT_SPMM_A = 1, KT_GRAM_RR = 2, KT_COMBINE = 3, KT_CHEB = 4 };
// Records HIP events around one launch when `kind` is the kind being timed.
struct KScope {
  KScope(int kind, hipStream_t s, double bytes, int tag);
  ~KScope();
  bool on;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  double bytes_ = 0.0;
  int tag_ = 0, phase_ = 0;
};
int ktimer_kind();
int ktimer_new_phase();
void ktimer_drop_after(int phase, int last_real);
void ktimer_collect();

// ---- lobpcg.hip -------------------------------------------------------------
int solve_eps(GraphOps& g, const me_opts* o, hipStream_t s, double* eps, int* iters);
int block_width(int K);
size_t embed_workspace_bytes(const GraphOps& g, int K, const me_opts* o);
int embed(const GraphOps& g, int K, double tol, const me_opts* o, const double* x0, void* ws,
          size_t ws_bytes, double* X, double* lambda, me_info* info, hipStream_t s);

}  // namespace me

struct me_graph_ops {
  me::GraphOps g;
};
