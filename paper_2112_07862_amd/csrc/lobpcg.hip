// LOBPCG driver (Section 4.3 computes the first K generalized eigenpairs of
// (A, B) with LOBPCG; the paper gives no algorithm text, so this follows the
// block method of Knyazev (2001) with Rayleigh-Ritz on the basis [X W P],
// CholQR B-orthonormalisation of the preconditioned residual block W, column
// dropping in place of an explicit restart, and an FP64 certificate pass).
//
// Per iteration, all on the caller's stream:
//   R = A X - B X Lambda, rho_j, convergence           k_resid + finalize
//   W = T R  (T = I or diag(A)^-1)                       (same kernel)
//   W <- (W - X X^T B W) R^-1   (CholQR)                Gram, 1-block Cholesky, combine
//   AW = A W                                            difference-form SpMM
//   G_B = S^T B S, G_A = S^T A S, S = [X W P]           MFMA Gram + partial sums
//   Rayleigh-Ritz in FP64                               1-block Jacobi
//   P <- W C_W + P C_P,  X <- X C_X + P                 combine (also AX, AP)
// Kernels check a device `done` flag and return at once after convergence,
// so the host enqueues `check_every` iterations between reads of the flag.
#include <chrono>
#include <cmath>
#include <cstring>

#include "common.h"

namespace me {

void launch_cholqr_coef(int kb, const double* g, double piv_tol, double* coef, const Ctrl* ctrl,
                        hipStream_t s);

int block_width(int K) {
  if (K <= 4) return 4;
  if (K <= 8) return 8;
  return 16;
}

// Drop threshold on the pivots of the unit-diagonal basis Gram (squared sine
// of the angle between a column and the span of the earlier ones).  Small
// thresholds let the inverse Cholesky factor grow without bound on nearly
// dependent bases; 1e-4 keeps it bounded and costs no iterations.
constexpr double kRrPivot = 1e-4;

static int partial_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kPartialBlocks, ceil_div(n, 64)));
}

// Workspace layout of one solve (bulk type T).
template <typename T>
struct SolveBufs {
  int64_t n = 0;
  int kb = 0;
  T *X = nullptr, *AX = nullptr, *W = nullptr, *AW = nullptr, *P = nullptr, *AP = nullptr;
  T *R = nullptr, *Y = nullptr, *DD = nullptr;  // Chebyshev preconditioner
  // FP32 copies for the mixed-precision preconditioner
  float *R32 = nullptr, *W32 = nullptr, *Y32 = nullptr, *DD32 = nullptr;
  double* partials = nullptr;  // kPartialBlocks x (2 (3kb)^2)
  double* gram = nullptr;      // 2 (3kb)^2
  double* coef = nullptr;      // 2 (3kb) kb
  double* coefw = nullptr;     // 2 kb kb
  double* lam = nullptr;       // kb
  double* sums = nullptr;      // kb
  double* scratch = nullptr;   // sign fix: 64 kb (double + int64)
  Ctrl* ctrl = nullptr;

  static size_t bytes(int64_t n, int kb) {
    const int m = 3 * kb;
    size_t b = 9 * Arena::round((size_t)n * kb * sizeof(T));
    b += 4 * Arena::round((size_t)n * kb * sizeof(float));
    b += Arena::round((size_t)kPartialBlocks * 2 * m * m * 8);
    b += Arena::round(2 * m * m * 8) + Arena::round(2 * m * kb * 8) + Arena::round(2 * kb * kb * 8);
    b += 2 * Arena::round(kb * 8) + Arena::round(64 * kb * 16) + Arena::round(sizeof(Ctrl));
    return b;
  }
  bool carve(void* base, size_t cap, int64_t n_, int kb_) {
    n = n_;
    kb = kb_;
    const int m = 3 * kb;
    Arena a{(char*)base, cap, 0};
    X = a.take<T>(n * kb);
    AX = a.take<T>(n * kb);
    W = a.take<T>(n * kb);
    AW = a.take<T>(n * kb);
    P = a.take<T>(n * kb);
    AP = a.take<T>(n * kb);
    R = a.take<T>(n * kb);
    Y = a.take<T>(n * kb);
    DD = a.take<T>(n * kb);
    R32 = a.take<float>(n * kb);
    W32 = a.take<float>(n * kb);
    Y32 = a.take<float>(n * kb);
    DD32 = a.take<float>(n * kb);
    partials = a.take<double>((size_t)kPartialBlocks * 2 * m * m);
    gram = a.take<double>(2 * m * m);
    coef = a.take<double>(2 * m * kb);
    coefw = a.take<double>(2 * kb * kb);
    lam = a.take<double>(kb);
    sums = a.take<double>(kb);
    scratch = a.take<double>(64 * kb * 2);
    ctrl = a.take<Ctrl>(1);
    return ctrl != nullptr;
  }
};

struct Problem {
  OpKind op;
  const double* bdiag;  // nullptr: B = I
  const double* dinv;   // D^-1, D = diag(Op)
  int precond;          // ME_PRECOND_NONE / _JACOBI / _CHEBYSHEV
  int cheb_deg;
  bool cheb_fp32;       // run the Chebyshev preconditioner in FP32
  const float* dinv32;  // D^-1 in FP32
  double cheb_afac;     // lower end of the Chebyshev interval: afac x Rayleigh quotient
  double cheb_b;        // upper end: Gershgorin bound of D^-1 Op
  bool deflate_ones;    // keep the iterates orthogonal to the constant vector
  int need;             // leading columns that must converge
  double tol;
  int max_iter;
  int check_every;
  double lam_floor;
  double lam_scale;
};

// Pinned host mirror of the control block.
struct HostCtrl {
  Ctrl* h = nullptr;
  int alloc() { return hipHostMalloc((void**)&h, sizeof(Ctrl), hipHostMallocDefault) == hipSuccess ? 0 : -1; }
  ~HostCtrl() { if (h) (void)hipHostFree(h); }
};

static int read_ctrl(const Ctrl* dev, Ctrl* host, hipStream_t s) {
  ME_TRY(hipMemcpyAsync(host, dev, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  return ME_OK;
}

template <typename T>
struct Lobpcg {
  const GraphOps& g;
  const Problem& pr;
  SolveBufs<T>& B;
  hipStream_t s;
  int nparts_gram, nparts_res;
  int phase = 0, tag = 0;  // kernel-timing bookkeeping

  int kt(int kind) const { return pr.op == OP_A ? kind : -1; }
  double spmm_bytes() const {
    const double sz = sizeof(T);
    return 4.0 * (double)(g.nnz_w + g.nnz_t) + sz * (double)g.nnz_w + (double)g.n * (8.0 + sz) +
           2.0 * (double)g.n * B.kb * sz;
  }

  Lobpcg(const GraphOps& g_, const Problem& p_, SolveBufs<T>& b_, hipStream_t s_)
      : g(g_), pr(p_), B(b_), s(s_) {
    nparts_gram = partial_blocks(B.n);
    nparts_res = partial_blocks(B.n);
  }

  const int* done() const { return &B.ctrl->done; }

  void gram(int nu, const T* const* u, int nv, const T* const* v, int nv2, const T* const* v2,
            const int* dn) {
    const int kb = B.kb;
    launch_gram<T>(B.n, kb, nu, u, nv, v, (const T*)pr.bdiag, nv2, v2, B.partials, nparts_gram,
                   dn, s);
    const int nent = nu * kb * (nv * kb + nv2 * kb);
    launch_reduce_partials(nparts_gram, nent, B.partials, B.gram, dn, s);
  }

  // Rayleigh-Ritz on [X] only (start and certificate): X, AX rotated to
  // B-orthonormal Ritz vectors, lam set.
  void rr_x(int final_pass) {
    const int kb = B.kb;
    const int* dn = final_pass ? nullptr : done();
    {
      KScope ks(kt(KT_SPMM_A), s, spmm_bytes(), 0);
      launch_spmm<T>(g, kb, pr.op, B.X, B.AX, dn, s);
    }
    const T* u[1] = {B.X};
    const T* v2[1] = {B.AX};
    gram(1, u, 1, u, 1, v2, dn);
    launch_rayleigh_ritz(kb, 1, B.gram + kb * kb, B.gram, 1e-14, B.coef, B.lam, B.ctrl,
                         final_pass, s);
    const double* cx = B.coef + kb * kb;
    T* outx[1] = {B.X};
    T* outa[1] = {B.AX};
    const T* inx[1] = {B.X};
    const T* ina[1] = {B.AX};
    launch_combine2<T>(B.n, kb, 1, 2, inx, ina, 1, outx, outa, cx, dn, s);
  }

  template <typename U>
  double cheb_bytes() const {
    const double sz = sizeof(U);
    return 4.0 * (double)(g.nnz_w + g.nnz_t) + sz * (double)g.nnz_w + (double)g.n * (8.0 + sz) +
           6.0 * (double)g.n * B.kb * sz;
  }

  // W = p(D^-1 Op) R by cheb_deg Chebyshev steps (type U); ping-pongs
  // between w and y so that the last step writes w.
  template <typename U>
  void cheb_block(const U* r, const U* dinv, U* w, U* y, U* dd) {
    const int deg = pr.cheb_deg;
    U* cur = ((deg - 1) % 2 == 0) ? w : y;
    U* nxt = (cur == w) ? y : w;
    launch_cheb_first<U>(g, B.kb, r, dinv, B.ctrl, cur, dd, s);
    for (int k = 1; k < deg; ++k) {
      KScope ks(kt(KT_CHEB), s, cheb_bytes<U>(), tag);
      launch_cheb_step<U>(g, B.kb, pr.op, k, r, dinv, B.ctrl, cur, nxt, dd, s);
      U* t = cur;
      cur = nxt;
      nxt = t;
    }
  }

  void iteration(bool first) {
    const int kb = B.kb;
    const int* dn = done();
    ++tag;
    // residual, preconditioned W, convergence test
    const bool cheb = pr.precond == ME_PRECOND_CHEBYSHEV;
    launch_resid<T>(B.n, kb, B.X, B.AX, (const T*)pr.bdiag, (const T*)pr.dinv,
                    pr.precond == ME_PRECOND_JACOBI ? 1 : 0, B.lam, cheb ? B.R : B.W, B.partials,
                    nparts_res, dn, s);
    launch_resid_finalize(kb, B.partials, nparts_res, B.lam, B.ctrl, 0, s);
    if (cheb && pr.cheb_fp32) {
      // mixed precision: the preconditioner only shapes the search direction
      launch_convert<T, float>(B.n * kb, B.R, B.R32, s);
      cheb_block<float>(B.R32, pr.dinv32, B.W32, B.Y32, B.DD32);
      launch_convert<float, T>(B.n * kb, B.W32, B.W, s);
    } else if (cheb) {
      cheb_block<T>(B.R, (const T*)pr.dinv, B.W, B.Y, B.DD);
    }
    if (pr.deflate_ones)
      launch_deflate_ones<T>(B.n, kb, B.W, B.partials, nparts_res, B.sums, dn, s);
    // W <- (W - X C) R^-1
    {
      const T* u[2] = {B.X, B.W};
      const T* v[1] = {B.W};
      gram(2, u, 1, v, 0, nullptr, dn);
      launch_cholqr_coef(kb, B.gram, 1e-10, B.coefw, B.ctrl, s);
      T* out[1] = {B.W};
      launch_combine<T>(B.n, kb, 2, u, 1, out, B.coefw, dn, s);
    }
    {
      KScope ks(kt(KT_SPMM_A), s, spmm_bytes(), tag);
      launch_spmm<T>(g, kb, pr.op, B.W, B.AW, dn, s);
    }
    const int nb = first ? 2 : 3;
    const int m = nb * kb;
    const double blk = (double)B.n * kb * sizeof(T);
    const T* S[3] = {B.X, B.W, B.P};
    const T* AS[3] = {B.AX, B.AW, B.AP};
    {
      KScope ks(kt(KT_GRAM_RR), s, 2.0 * nb * blk + (double)B.n * sizeof(T), tag);
      launch_gram<T>(B.n, kb, nb, S, nb, S, (const T*)pr.bdiag, nb, AS, B.partials, nparts_gram,
                     dn, s);
    }
    launch_reduce_partials(nparts_gram, 2 * m * m, B.partials, B.gram, dn, s);
    launch_rayleigh_ritz(kb, nb, B.gram + m * m, B.gram, kRrPivot, B.coef, B.lam, B.ctrl, 0, s);
    T* out_x[2] = {B.P, B.X};
    T* out_a[2] = {B.AP, B.AX};
    {
      KScope ks(kt(KT_COMBINE), s, 2.0 * (nb + 2) * blk, tag);
      launch_combine2<T>(B.n, kb, nb, 2, S, AS, 2, out_x, out_a, B.coef, dn, s);
    }
  }

  // Returns status; ctrl_out receives the final control block.
  int run(Ctrl* hc, double* orth_err) {
    const int kb = B.kb;
    Ctrl c0{};
    c0.max_iter = pr.max_iter;
    c0.need = pr.need;
    c0.kb = kb;
    c0.tol = pr.tol;
    c0.lam_floor = pr.lam_floor;
    c0.lam_scale = pr.lam_scale;
    c0.cheb_deg = pr.precond == ME_PRECOND_CHEBYSHEV ? pr.cheb_deg : 0;
    c0.cheb_afac = pr.cheb_afac;
    c0.cheb_b = pr.cheb_b;
    *hc = c0;
    ME_TRY(hipMemcpyAsync(B.ctrl, hc, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    if (pr.deflate_ones) launch_deflate_ones<T>(B.n, kb, B.X, B.partials, nparts_res, B.sums,
                                                nullptr, s);
    phase = ktimer_new_phase();
    rr_x(0);
    bool first = true;
    int reentries = 0;
    for (;;) {
      phase = ktimer_new_phase();
      tag = 0;
      const int iter0 = hc->iter;
      for (;;) {
        for (int q = 0; q < pr.check_every; ++q) {
          iteration(first);
          first = false;
        }
        ME_TRY_STATUS(read_ctrl(B.ctrl, hc, s));
        if (hc->done) break;
      }
      ktimer_drop_after(phase, hc->iter - iter0);
      if (hc->nonfinite) return ME_ERR_BREAKDOWN;
      // certificate: fresh A X, Rayleigh-Ritz on X, residuals in FP64
      phase = ktimer_new_phase();
      tag = 0;
      rr_x(1);
      launch_resid<T>(B.n, kb, B.X, B.AX, (const T*)pr.bdiag, (const T*)pr.dinv, 0, B.lam,
                      nullptr, B.partials, nparts_res, nullptr, s);
      launch_resid_finalize(kb, B.partials, nparts_res, B.lam, B.ctrl, 1, s);
      ME_TRY_STATUS(read_ctrl(B.ctrl, hc, s));
      if (hc->nonfinite) return ME_ERR_BREAKDOWN;
      double worst = 0.0;
      for (int j = 0; j < pr.need; ++j) worst = std::max(worst, hc->rho[j]);
      if (worst <= pr.tol || hc->iter >= pr.max_iter || reentries >= 3) break;
      // drift between the recurrences and a fresh product: keep iterating
      ++reentries;
      hc->done = 0;
      ME_TRY(hipMemcpyAsync(&B.ctrl->done, &hc->done, sizeof(int), hipMemcpyHostToDevice, s));
      first = true;
    }
    // B-orthonormality of the final X
    if (orth_err) {
      const T* u[1] = {B.X};
      gram(1, u, 1, u, 0, nullptr, nullptr);
      std::vector<double> gh(kb * kb);
      ME_TRY(hipMemcpyAsync(gh.data(), B.gram, kb * kb * 8, hipMemcpyDeviceToHost, s));
      ME_TRY(hipStreamSynchronize(s));
      double e = 0.0;
      for (int i = 0; i < pr.need; ++i)
        for (int j = 0; j < pr.need; ++j) e = std::max(e, std::fabs(gh[i * kb + j] - (i == j)));
      *orth_err = e;
    }
    double worst = 0.0;
    for (int j = 0; j < pr.need; ++j) worst = std::max(worst, hc->rho[j]);
    return worst <= pr.tol ? ME_OK : ME_WARN_NOT_CONVERGED;
  }
};

// ---------------------------------------------------------------------------
// eps = lambda_2(Q)
// ---------------------------------------------------------------------------

int solve_eps(GraphOps& g, const me_opts* o, hipStream_t s, double* eps, int* iters) {
  const int64_t n = g.n;
  if (n <= kDenseMaxN) {
    double* buf = nullptr;
    const size_t nn = (size_t)n * n;
    ME_TRY(hipMallocAsync((void**)&buf, (3 * nn + n) * 8, s));
    launch_dense_ops(g, 1, buf, buf + nn, s);
    launch_dense_geneig((int)n, buf, buf + nn, buf + 2 * nn, buf + 3 * nn, s);
    double lam2 = 0.0;
    ME_TRY(hipMemcpyAsync(&lam2, buf + 3 * nn + 1, 8, hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
    ME_TRY(hipFreeAsync(buf, s));
    *eps = lam2;
    *iters = 0;
    return ME_OK;
  }
  const int kb = 4;
  SolveBufs<double> B;
  const size_t wsb = SolveBufs<double>::bytes(n, kb);
  void* ws = nullptr;
  ME_TRY(hipMallocAsync(&ws, wsb, s));
  B.carve(ws, wsb, n, kb);
  Problem pr;
  pr.op = OP_Q;
  pr.bdiag = nullptr;
  pr.dinv = g.qinv_s;
  pr.dinv32 = g.qinv32_s;
  pr.cheb_fp32 = o->precision == ME_MIXED;
  pr.precond = o->precond;
  pr.cheb_deg = o->cheb_degree;
  pr.cheb_afac = 0.5;
  pr.cheb_b = g.cheb_b_q * 1.01;
  pr.deflate_ones = true;
  pr.need = 1;
  pr.tol = o->eps_tol;
  pr.max_iter = o->eps_max_iter;
  pr.check_every = o->check_every > 0 ? o->check_every : 16;
  pr.lam_scale = g.maxden > 0 ? g.maxden : 1.0;
  pr.lam_floor = 1e-8 * pr.lam_scale;
  launch_fill_random(n, kb, 0, nullptr, o->seed ^ 0x51ED2701D5ull, g.perm, B.X, s);
  HostCtrl hc;
  if (hc.alloc()) { (void)hipFreeAsync(ws, s); return ME_ERR_HIP; }
  Lobpcg<double> L(g, pr, B, s);
  int st = L.run(hc.h, nullptr);
  double lam0 = 0.0;
  if (st >= 0) {
    ME_TRY(hipMemcpyAsync(&lam0, B.lam, 8, hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
  }
  *iters = hc.h->iter;
  ME_TRY(hipFreeAsync(ws, s));
  if (st < 0) return st;
  *eps = lam0;
  return ME_OK;
}

// ---------------------------------------------------------------------------
// Embedding
// ---------------------------------------------------------------------------

size_t embed_workspace_bytes(const GraphOps& g, int K, const me_opts* o) {
  (void)o;
  if (g.n <= kDenseMaxN) return Arena::round((3 * (size_t)g.n * g.n + g.n + 64 * 16 * 2) * 8);
  return SolveBufs<double>::bytes(g.n, block_width(K));
}

int embed(const GraphOps& g, int K, double tol, const me_opts* o, const double* x0, void* ws,
          size_t ws_bytes, double* X, double* lambda, me_info* info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = g.n;
  if (K < 1 || K > kMaxBlockCols || K > n) return ME_ERR_K_RANGE;
  if (!X || !lambda || !(tol > 0.0)) return ME_ERR_INVALID_ARG;
  const size_t need_bytes = embed_workspace_bytes(g, K, o);
  bool own = false;
  if (!ws) {
    ME_TRY(hipMallocAsync(&ws, need_bytes, s));
    own = true;
  } else if (ws_bytes < need_bytes) {
    return ME_ERR_WORKSPACE;
  }
  int st = ME_OK;
  int iters = 0, kb = K;
  double worst = 0.0, orth = 0.0;
  if (n <= kDenseMaxN) {
    double* buf = (double*)ws;
    const size_t nn = (size_t)n * n;
    launch_dense_ops(g, 0, buf, buf + nn, s);
    launch_dense_geneig((int)n, buf, buf + nn, buf + 2 * nn, buf + 3 * nn, s);
    launch_sign_fix_and_copy(n, (int)n, K, buf + 2 * nn, X, buf + 3 * nn, lambda,
                             buf + 3 * nn + n, nullptr, nullptr, s);
    ME_TRY(hipStreamSynchronize(s));
    kb = (int)n;
  } else {
    kb = block_width(K);
    if (3 * kb > n) {
      if (own) (void)hipFreeAsync(ws, s);
      return ME_ERR_K_RANGE;
    }
    SolveBufs<double> B;
    B.carve(ws, need_bytes, n, kb);
    launch_fill_random(n, kb, x0 ? K : 0, x0, o->seed, g.perm, B.X, s);
    Problem pr;
    pr.op = OP_A;
    pr.bdiag = g.b_s;
    pr.dinv = g.dinv_s;
    pr.dinv32 = g.dinv32_s;
    pr.cheb_fp32 = o->precision == ME_MIXED;
    pr.precond = o->precond;
    pr.cheb_deg = o->cheb_degree;
    pr.cheb_afac = 0.5;
    pr.cheb_b = g.cheb_b_a * 1.01;
    pr.deflate_ones = false;
    pr.need = K;
    pr.tol = tol;
    pr.max_iter = o->max_iter;
    pr.check_every = o->check_every > 0 ? o->check_every : 16;
    pr.lam_scale = g.max_diag_a > 0 ? g.max_diag_a : 1.0;
    pr.lam_floor = 1e-8 * pr.lam_scale;
    HostCtrl hc;
    if (hc.alloc()) {
      if (own) (void)hipFreeAsync(ws, s);
      return ME_ERR_HIP;
    }
    Lobpcg<double> L(g, pr, B, s);
    st = L.run(hc.h, &orth);
    iters = hc.h->iter;
    for (int j = 0; j < K; ++j) worst = std::max(worst, hc.h->rho[j]);
    if (st >= 0) {
      launch_sign_fix_and_copy(n, kb, K, B.X, X, B.lam, lambda, B.scratch, g.perm, g.iperm, s);
      ME_TRY(hipStreamSynchronize(s));
    }
    ktimer_collect();
  }
  if (own) {
    ME_TRY(hipFreeAsync(ws, s));
    ME_TRY(hipStreamSynchronize(s));
  }
  if (st == ME_OK && g.status == ME_WARN_EPS_ZERO) st = ME_WARN_EPS_ZERO;
  if (info) {
    info->status = st;
    info->iterations = iters;
    info->eps_iterations = g.eps_iters;
    info->block = kb;
    info->eps = g.eps;
    info->mu = g.mu;
    info->max_residual = worst;
    info->orth_error = orth;
    info->ms_build = 0.0;
    info->ms_solve =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace me
