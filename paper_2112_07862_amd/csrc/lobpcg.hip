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

static size_t dense_eps_bytes(int64_t n) { return (3 * (size_t)n * n + n) * 8; }

int dense_eps_solve(const GraphOps& g, DevHeap& heap, hipStream_t s, double* eps) {
  const int64_t n = g.n;
  double* buf = nullptr;
  const size_t nn = (size_t)n * n;
  ME_TRY_STATUS(heap.alloc((void**)&buf, dense_eps_bytes(n), s));
  launch_dense_ops(g, 1, buf, buf + nn, s);
  launch_dense_geneig((int)n, buf, buf + nn, buf + 2 * nn, buf + 3 * nn, s);
  double lam2 = 0.0;
  const hipError_t e1 = hipMemcpyAsync(&lam2, buf + 3 * nn + 1, 8, hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  heap.release(buf, s);  // synchronised
  if (e1 != hipSuccess || e2 != hipSuccess) return ME_ERR_HIP;
  *eps = lam2;
  return ME_OK;
}

size_t eps_solve_bytes(int64_t n) {
  if (n <= kDenseMaxN) return DevHeap::round(dense_eps_bytes(n));
  return Engine::run_bytes({{n, 4}});
}

// Options of an eps solve: the embedding solve's, with the product in FP64
// (the FP32 product option concerns the embedding solve only).
static me_opts eps_opts(const me_opts& o) {
  me_opts e = o;
  e.product = ME_PRODUCT_FP64;
  return e;
}

int solve_eps(GraphOps& g, const me_opts* o, DevHeap& heap, hipStream_t s, double* eps,
              int* iters) {
  *iters = 0;
  if (g.n <= kDenseMaxN) return dense_eps_solve(g, heap, s, eps);
  const me_opts eo = eps_opts(*o);
  Engine e(s, eo, 1, false, false, &heap, Engine::tile_area_bytes(Engine::tile_bytes(g.n, 4)));
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

static size_t dense_embed_bytes(int64_t n) {
  return Arena::round((3 * (size_t)n * n + n + 64 * 16 * 2) * 8);
}

size_t dense_request_bytes(int64_t n) { return dense_embed_bytes(n); }

// Everything one embedding solve allocates: its slot, the engine's tables
// and work-list areas (or the dense solve's buffer).
size_t embed_workspace_bytes(int64_t n, int K, const me_opts* o) {
  (void)o;
  if (n <= kDenseMaxN) return DevHeap::round(dense_embed_bytes(n)) + kHeapAlign;
  return Engine::run_bytes({{n, block_width(K)}}) + kHeapAlign;
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
  if (ws && ws_bytes < embed_workspace_bytes(g.n, K, o)) return ME_ERR_WORKSPACE;
  // with a workspace every device allocation of the solve is carved from it
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
  int st = ME_OK, iters = 0, kb = K;
  double worst = 0.0, orth = 0.0;
  if (g.n <= kDenseMaxN) {
    double* buf = nullptr;
    ME_TRY_STATUS(heap.alloc((void**)&buf, dense_embed_bytes(g.n), s));
    dense_embed_solve(g, K, buf, X, lambda, s);
    heap.release_later(buf, s);
    ME_TRY(hipStreamSynchronize(s));
    heap.quiesce();
    kb = (int)g.n;
  } else {
    kb = block_width(K);
    Engine e(s, *o, 1, true, /*solo=*/true, &heap,
             Engine::tile_area_bytes(Engine::tile_bytes(g.n, kb)));
    ME_TRY_STATUS(e.init());
    int id = -1;
    ME_TRY_STATUS(e.add(embed_slot_spec(g, K, tol, o, x0, X, lambda), nullptr, 0, &id));
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

// Workspace of a batch: the sum of every allocation the batch makes (each
// graph's build with T at its degree bound, both engines with all slots,
// the dense solves and the searches' arguments), so that first fit over the
// region never fails whatever the order in which graphs finish.
int batch_workspace_bytes(int G, const me_csr* Ws, const int* Ks, const me_opts* o,
                          hipStream_t s, size_t* bytes) {
  (void)o;
  *bytes = 0;
  size_t total = kHeapAlign + DevHeap::round(order_args_bytes(G));
  std::vector<std::pair<int64_t, int>> eps_slots, emb_slots;
  for (int i = 0; i < G; ++i) {
    int64_t tb = 0;
    ME_TRY_STATUS(two_hop_bound(&Ws[i], s, &tb));
    const int64_t n = Ws[i].n;
    total += build_bytes_bound(n, Ws[i].nnz, tb);
    if (n <= kDenseMaxN) {
      total += DevHeap::round(dense_eps_bytes(n)) + DevHeap::round(dense_embed_bytes(n));
    } else {
      eps_slots.push_back({n, 4});
      emb_slots.push_back({n, block_width(std::max(1, std::min(Ks[i], kMaxBlockCols)))});
    }
  }
  total += Engine::run_bytes(eps_slots) + Engine::run_bytes(emb_slots);
  *bytes = total;
  return ME_OK;
}

static size_t sum_tiles(const std::vector<std::pair<int64_t, int>>& slots) {
  size_t t = 0;
  for (const auto& x : slots) t += Engine::tile_bytes(x.first, x.second);
  return Engine::tile_area_bytes(t);
}

int embed_batch(int G, const me_csr* Ws, const int* Ks, double tol, const me_opts* o, void* ws,
                size_t ws_bytes, double* const* Xs, double* const* lams, me_info* infos,
                hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (ws) {
    size_t need = 0;
    ME_TRY_STATUS(batch_workspace_bytes(G, Ws, Ks, o, s, &need));
    if (ws_bytes < need) return ME_ERR_WORKSPACE;
  }
  // with a workspace every device allocation of the batch is carved from it
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  DevHeap& heap = ws ? region : hip;
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
  for_each_graph(G, [&](int i, hipStream_t ws_i) {
    if (!Xs[i] || !lams[i]) st[i] = ME_ERR_INVALID_ARG;
    else if (Ks[i] < 1 || Ks[i] > kMaxBlockCols) st[i] = ME_ERR_K_RANGE;
    if (st[i] < 0) return;
    st[i] = build_pre_a(&Ws[i], o, heap, ws_i, &gs[i]);
    if (st[i] >= 0) st[i] = check_k_range(gs[i], Ks[i]);
  });
  heap.quiesce();  // every build stream is idle
  // the breadth-first searches of every graph in one launch, then each
  // graph's operator in its order
  {
    std::vector<GraphOps*> ok;
    for (int i = 0; i < G; ++i)
      if (st[i] >= 0) ok.push_back(&gs[i]);
    OrderJob job;
    ME_TRY_STATUS(order_launch(ok.data(), (int)ok.size(), heap, s, &job));
    ME_TRY_STATUS(order_finish(ok.data(), (int)ok.size(), heap, s, &job));
    for_each_graph(G, [&](int i, hipStream_t ws_i) {
      if (st[i] >= 0) st[i] = build_pre_b(&gs[i], ws_i);
    });
  }
  // eps
  std::vector<double> eps(G, 0.0);
  std::vector<int> eps_it(G, 0);
  {
    std::vector<std::pair<int64_t, int>> slots;
    for (int i = 0; i < G; ++i)
      if (st[i] >= 0 && gs[i].needs_eps && gs[i].n > kDenseMaxN) slots.push_back({gs[i].n, 4});
    const me_opts eo = eps_opts(*o);
    Engine e(s, eo, std::max((int)slots.size(), 1), false, false, &heap, sum_tiles(slots));
    ME_TRY_STATUS(e.init());
    std::vector<int> id(G, -1);
    for (int i = 0; i < G; ++i) {
      if (st[i] < 0 || !gs[i].needs_eps) continue;
      if (gs[i].n <= kDenseMaxN) {
        st[i] = dense_eps_solve(gs[i], heap, s, &eps[i]);
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
  for_each_graph(G, [&](int i, hipStream_t ws_i) {
    if (st[i] < 0) return;
    st[i] = build_post(&gs[i], eps[i], eps_it[i], ws_i);
    (void)hipStreamSynchronize(ws_i);
    ms_build[i] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
  // embedding
  const auto t1 = std::chrono::steady_clock::now();
  {
    std::vector<std::pair<int64_t, int>> slots;
    for (int i = 0; i < G; ++i)
      if (st[i] >= 0 && gs[i].n > kDenseMaxN) slots.push_back({gs[i].n, block_width(Ks[i])});
    // FP16 iterates only for a batch of one input graph (decided by G, not by
    // how many graphs reach the engine)
    Engine e(s, *o, std::max((int)slots.size(), 1), false, /*solo=*/G == 1, &heap,
             sum_tiles(slots));
    ME_TRY_STATUS(e.init());
    std::vector<int> id(G, -1);
    for (int i = 0; i < G; ++i) {
      if (st[i] < 0) continue;
      if (gs[i].n <= kDenseMaxN) {
        double* buf = nullptr;
        const int a = heap.alloc((void**)&buf, dense_embed_bytes(gs[i].n), s);
        if (a < 0) {
          st[i] = a;
          continue;
        }
        dense_embed_solve(gs[i], Ks[i], buf, Xs[i], lams[i], s);
        heap.release_later(buf, s);
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
  heap.quiesce();
  int worst_st = ME_OK;
  for (int i = 0; i < G; ++i) {
    if (st[i] < 0) return st[i];
    worst_st = std::max(worst_st, st[i]);
  }
  return worst_st;
}

}  // namespace me
