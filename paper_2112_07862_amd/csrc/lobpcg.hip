// The two LOBPCG solves of the method on top of the engine:
//   eps = lambda_2(Q) (Section 4.2): smallest eigenpair of Q on the
//     complement of the constant vector (Q is the Laplacian of the two-hop
//     graph, so lambda_1(Q) = 0 with the constant eigenvector);
//   the embedding (Section 4.3): the first K generalized eigenpairs of
//     (A, B), B-orthonormal.
// Graphs of at most kDenseMaxN nodes are solved densely instead.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "engine.h"

namespace me {

// Host threads of the per-graph build steps of a batch.
constexpr int kBuildThreads = 8;

// Runs fn(i, stream) for i in [0, G) on up to kBuildThreads host threads,
// each with a stream of its own: the per-graph build steps wait on the host
// several times, so graphs overlap across threads.  Every stream is idle on
// return.
template <typename F>
static void for_each_graph(int G, F fn) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::atomic<int> next{0};
  auto work = [&]() {
    (void)hipSetDevice(dev);
    hipStream_t ws = nullptr;
    if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) ws = nullptr;
    for (int i; (i = next.fetch_add(1)) < G;) {
      fn(i, ws);
      (void)hipStreamSynchronize(ws);
    }
    if (ws) (void)hipStreamDestroy(ws);
  };
  std::vector<std::thread> th;
  const int nt = std::max(1, std::min(G, kBuildThreads));
  try {
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
  } catch (...) {
    // no more threads: the calling thread takes the rest
  }
  work();
  for (auto& x : th) x.join();
}

SlotSpec eps_slot_spec(const GraphOps& g, const me_opts* o) {
  SlotSpec sp;
  sp.g = &g;
  sp.op = OP_Q;
  sp.kb = 4;
  sp.need = 1;
  sp.tol = o->eps_tol;
  sp.max_iter = o->eps_max_iter;
  sp.deflate = true;
  sp.cheb_b = g.cheb_b_q * 1.01;
  sp.lam_scale = g.maxden > 0 ? g.maxden : 1.0;
  sp.seed = o->seed ^ 0x51ED2701D5ull;
  // smooth start: lambda_2(Q)'s vector varies along the manifold, like the
  // level cosines of frequencies 1..4 (the constant is deflated)
  sp.nsmooth = 4;
  sp.jfreq = 1;
  return sp;
}

SlotSpec embed_slot_spec(const GraphOps& g, int K, double tol, const me_opts* o,
                         const double* x0, double* X, double* lambda) {
  SlotSpec sp;
  sp.g = &g;
  sp.op = OP_A;
  sp.kb = block_width(K);
  sp.need = K;
  sp.tol = tol;
  sp.max_iter = o->max_iter;
  sp.deflate = false;
  sp.cheb_b = (o->cheb_op == ME_CHEB_LAPLACIAN ? g.cheb_b_p : g.cheb_b_a) * 1.01;
  sp.lam_scale = g.max_diag_a > 0 ? g.max_diag_a : 1.0;
  sp.seed = o->seed;
  sp.x0 = x0;
  sp.kcopy = x0 ? K : 0;
  // a random start: level cosines fit only the modes along the search
  // direction, and a partly smooth block converged more slowly than a
  // random one on the manifold graphs measured
  sp.nsmooth = 0;
  sp.jfreq = 0;
  sp.out_x = X;
  sp.out_lam = lambda;
  sp.k_out = K;
  return sp;
}

int dense_eps_solve(const GraphOps& g, hipStream_t s, double* eps) {
  const int64_t n = g.n;
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
  return ME_OK;
}

int solve_eps(GraphOps& g, const me_opts* o, hipStream_t s, double* eps, int* iters) {
  *iters = 0;
  if (g.n <= kDenseMaxN) return dense_eps_solve(g, s, eps);
  Engine e(s, *o, 1, false);
  ME_TRY_STATUS(e.init());
  int id = -1;
  ME_TRY_STATUS(e.add(eps_slot_spec(g, o), nullptr, 0, &id));
  ME_TRY_STATUS(e.run());
  const SlotResult& r = e.result(id);
  *iters = r.iterations;
  if (r.status < 0) return r.status;
  *eps = r.lam[0];
  return ME_OK;
}

// ---------------------------------------------------------------------------
// Embedding
// ---------------------------------------------------------------------------

size_t embed_workspace_bytes(const GraphOps& g, int K, const me_opts* o) {
  (void)o;
  if (g.n <= kDenseMaxN) return Arena::round((3 * (size_t)g.n * g.n + g.n + 64 * 16 * 2) * 8);
  return Engine::slot_bytes(g.n, block_width(K));
}

int check_k_range(const GraphOps& g, int K) {
  if (K < 1 || K > kMaxBlockCols || K > g.n) return ME_ERR_K_RANGE;
  if (g.n > kDenseMaxN && 3 * block_width(K) > g.n) return ME_ERR_K_RANGE;
  return ME_OK;
}

// Dense solve of (A, B) for graphs with n <= kDenseMaxN (buf: 3 n^2 + n + 2048 doubles).
int dense_embed_solve(const GraphOps& g, int K, double* buf, double* X, double* lambda,
                      hipStream_t s) {
  const int64_t n = g.n;
  const size_t nn = (size_t)n * n;
  launch_dense_ops(g, 0, buf, buf + nn, s);
  launch_dense_geneig((int)n, buf, buf + nn, buf + 2 * nn, buf + 3 * nn, s);
  launch_sign_fix_and_copy(n, (int)n, K, buf + 2 * nn, X, buf + 3 * nn, lambda,
                           buf + 3 * nn + n, nullptr, nullptr, s);
  return ME_OK;
}

static void fill_info(me_info* info, const GraphOps& g, int st, int iters, int kb, double worst,
                      double orth, double ms) {
  if (!info) return;
  info->status = st;
  info->iterations = iters;
  info->eps_iterations = g.eps_iters;
  info->block = kb;
  info->eps = g.eps;
  info->mu = g.mu;
  info->max_residual = worst;
  info->orth_error = orth;
  info->ms_build = 0.0;
  info->ms_solve = ms;
}

int embed(const GraphOps& g, int K, double tol, const me_opts* o, const double* x0, void* ws,
          size_t ws_bytes, double* X, double* lambda, me_info* info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ME_TRY_STATUS(check_k_range(g, K));
  if (!X || !lambda || !(tol > 0.0)) return ME_ERR_INVALID_ARG;
  const size_t need_bytes = embed_workspace_bytes(g, K, o);
  if (ws && ws_bytes < need_bytes) return ME_ERR_WORKSPACE;
  int st = ME_OK, iters = 0, kb = K;
  double worst = 0.0, orth = 0.0;
  if (g.n <= kDenseMaxN) {
    bool own = false;
    if (!ws) {
      ME_TRY(hipMallocAsync(&ws, need_bytes, s));
      own = true;
    }
    dense_embed_solve(g, K, (double*)ws, X, lambda, s);
    if (own) ME_TRY(hipFreeAsync(ws, s));
    ME_TRY(hipStreamSynchronize(s));
    kb = (int)g.n;
  } else {
    kb = block_width(K);
    Engine e(s, *o, 1, true, /*solo=*/true);
    ME_TRY_STATUS(e.init());
    int id = -1;
    ME_TRY_STATUS(e.add(embed_slot_spec(g, K, tol, o, x0, X, lambda), ws, ws_bytes, &id));
    ME_TRY_STATUS(e.run());
    const SlotResult& r = e.result(id);
    st = r.status;
    iters = r.iterations;
    worst = r.worst;
    orth = r.orth;
    if (st < 0) return st;
  }
  if (st == ME_OK && g.status == ME_WARN_EPS_ZERO) st = ME_WARN_EPS_ZERO;
  fill_info(info, g, st, iters, kb, worst, orth,
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count());
  return st;
}

// ---------------------------------------------------------------------------
// Batch: every graph's build up to eps, all eps solves in one engine, the
// rest of each build, then all embedding solves in one engine.
// ---------------------------------------------------------------------------

int embed_batch(int G, const me_csr* Ws, const int* Ks, double tol, const me_opts* o,
                double* const* Xs, double* const* lams, me_info* infos, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<GraphOps> gs(G);
  struct Release {
    std::vector<GraphOps>& v;
    ~Release() {
      for (auto& g : v) free_graph_ops(g);
    }
  } release{gs};
  std::vector<int> st(G, ME_OK);
  std::vector<double> ms_build(G, 0.0);
  ME_TRY(hipStreamSynchronize(s));  // the caller's graphs are in place
  for_each_graph(G, [&](int i, hipStream_t ws) {
    if (!Xs[i] || !lams[i]) st[i] = ME_ERR_INVALID_ARG;
    else if (Ks[i] < 1 || Ks[i] > kMaxBlockCols) st[i] = ME_ERR_K_RANGE;
    if (st[i] < 0) return;
    st[i] = build_pre_a(&Ws[i], o, ws, &gs[i]);
    if (st[i] >= 0) st[i] = check_k_range(gs[i], Ks[i]);
  });
  // the breadth-first searches of every graph in one launch, then each
  // graph's operator in its order
  {
    std::vector<GraphOps*> ok;
    for (int i = 0; i < G; ++i)
      if (st[i] >= 0) ok.push_back(&gs[i]);
    void* args = nullptr;
    ME_TRY_STATUS(order_launch(ok.data(), (int)ok.size(), s, &args));
    ME_TRY_STATUS(order_finish(ok.data(), (int)ok.size(), s, args));
    for_each_graph(G, [&](int i, hipStream_t ws) {
      if (st[i] >= 0) st[i] = build_pre_b(&gs[i], ws);
    });
  }
  // eps
  std::vector<double> eps(G, 0.0);
  std::vector<int> eps_it(G, 0);
  {
    int cnt = 0;
    for (int i = 0; i < G; ++i) cnt += st[i] >= 0 && gs[i].needs_eps && gs[i].n > kDenseMaxN;
    Engine e(s, *o, std::max(cnt, 1), false);
    ME_TRY_STATUS(e.init());
    std::vector<int> id(G, -1);
    for (int i = 0; i < G; ++i) {
      if (st[i] < 0 || !gs[i].needs_eps) continue;
      if (gs[i].n <= kDenseMaxN) {
        st[i] = dense_eps_solve(gs[i], s, &eps[i]);
        continue;
      }
      const int a = e.add(eps_slot_spec(gs[i], o), nullptr, 0, &id[i]);
      if (a < 0) st[i] = a;
    }
    ME_TRY_STATUS(e.run());
    for (int i = 0; i < G; ++i) {
      if (id[i] < 0) continue;
      const SlotResult& r = e.result(id[i]);
      eps_it[i] = r.iterations;
      if (r.status < 0) st[i] = r.status;
      else eps[i] = r.lam[0];
    }
  }
  for_each_graph(G, [&](int i, hipStream_t ws) {
    if (st[i] < 0) return;
    st[i] = build_post(&gs[i], eps[i], eps_it[i], ws);
    (void)hipStreamSynchronize(ws);
    ms_build[i] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
  // embedding
  const auto t1 = std::chrono::steady_clock::now();
  {
    int cnt = 0;
    for (int i = 0; i < G; ++i) cnt += st[i] >= 0 && gs[i].n > kDenseMaxN;
    // FP16 iterates only for a batch of one input graph (decided by G, not by
    // how many graphs reach the engine)
    Engine e(s, *o, std::max(cnt, 1), false, /*solo=*/G == 1);
    ME_TRY_STATUS(e.init());
    std::vector<int> id(G, -1);
    for (int i = 0; i < G; ++i) {
      if (st[i] < 0) continue;
      if (gs[i].n <= kDenseMaxN) {
        double* buf = nullptr;
        const size_t bytes = embed_workspace_bytes(gs[i], Ks[i], o);
        ME_TRY(hipMallocAsync((void**)&buf, bytes, s));
        dense_embed_solve(gs[i], Ks[i], buf, Xs[i], lams[i], s);
        ME_TRY(hipFreeAsync(buf, s));
        continue;
      }
      const int a =
          e.add(embed_slot_spec(gs[i], Ks[i], tol, o, nullptr, Xs[i], lams[i]), nullptr, 0, &id[i]);
      if (a < 0) st[i] = a;
    }
    ME_TRY_STATUS(e.run());
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
    for (int i = 0; i < G; ++i) {
      if (st[i] < 0) {
        if (infos) infos[i].status = st[i];
        continue;
      }
      int s_i = ME_OK, iters = 0, kb = (int)gs[i].n;
      double worst = 0.0, orth = 0.0;
      if (id[i] >= 0) {
        const SlotResult& r = e.result(id[i]);
        s_i = r.status;
        iters = r.iterations;
        worst = r.worst;
        orth = r.orth;
        kb = block_width(Ks[i]);
      }
      if (s_i == ME_OK && gs[i].status == ME_WARN_EPS_ZERO) s_i = ME_WARN_EPS_ZERO;
      st[i] = s_i;
      fill_info(infos ? &infos[i] : nullptr, gs[i], s_i, iters, kb, worst, orth, ms);
      if (infos) infos[i].ms_build = ms_build[i];
    }
  }
  ME_TRY(hipStreamSynchronize(s));
  int worst_st = ME_OK;
  for (int i = 0; i < G; ++i) {
    if (st[i] < 0) return st[i];
    worst_st = std::max(worst_st, st[i]);
  }
  return worst_st;
}

}  // namespace me
