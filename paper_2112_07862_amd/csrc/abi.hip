// extern "C" entry points declared in include/membed.h.
#include <chrono>
#include <cstring>
#include <new>

#include "common.h"

using namespace me;

namespace me {
void free_graph_ops(GraphOps& g) {
  if (!g.in_region) {  // region memory belongs to the caller's workspace
    if (g.mem) (void)hipFree(g.mem);
    if (g.mem2) (void)hipFree(g.mem2);
    if (g.ord_mem) (void)hipFree(g.ord_mem);
  }
  g.mem = g.mem2 = g.ord_mem = nullptr;
}
}  // namespace me

static void free_ops(GraphOps& g) { free_graph_ops(g); }

bool me::opts_valid(const me_opts& o) {
  return o.max_iter >= 1 && o.eps_max_iter >= 1 && o.check_every >= 1 && o.precond >= 0 &&
         o.precond <= 2 && (o.precision == ME_FP64 || o.precision == ME_MIXED) &&
         o.eps_tol > 0 && (o.cheb_op == ME_CHEB_LAPLACIAN || o.cheb_op == ME_CHEB_FULL) &&
         (o.addressing == ME_ADDR_AUTO || o.addressing == ME_ADDR_GLOBAL) &&
         (o.cheb_iterates == ME_ITER_FP32 || o.cheb_iterates == ME_ITER_FP16) &&
         (o.launch == ME_LAUNCH_AUTO || o.launch == ME_LAUNCH_STREAM ||
          o.launch == ME_LAUNCH_GRAPH) &&
         (o.cholqr_passes == 1 || o.cholqr_passes == 2) &&
         (o.product == ME_PRODUCT_FP64 || (o.product == ME_PRODUCT_FP32 && o.precision == ME_MIXED)) &&
         (o.precond != ME_PRECOND_CHEBYSHEV ||
          (o.cheb_degree >= 2 && o.cheb_degree <= kMaxChebDegree));
}

extern "C" {

void me_opts_default(me_opts* o) {
  if (!o) return;
  o->precision = ME_FP64;
  o->precond = ME_PRECOND_CHEBYSHEV;
  o->max_iter = 20000;
  o->eps_max_iter = 20000;
  o->eps_tol = 1e-6;
  o->check_every = 16;
  o->seed = 0;
  o->cheb_degree = 128;
  o->cheb_op = ME_CHEB_LAPLACIAN;
  o->addressing = ME_ADDR_AUTO;
  o->cheb_iterates = ME_ITER_FP32;
  o->launch = ME_LAUNCH_AUTO;
  o->cholqr_passes = 1;
  o->product = ME_PRODUCT_FP64;
}

const char* me_status_string(int st) {
  switch (st) {
    case ME_OK: return "ok";
    case ME_WARN_NOT_CONVERGED: return "warning: not converged within max_iter";
    case ME_WARN_EPS_ZERO: return "warning: two-hop graph disconnected, eps = mu = 0";
    case ME_ERR_INVALID_ARG: return "error: invalid argument or malformed CSR";
    case ME_ERR_NOT_SYMMETRIC: return "error: W is not symmetric";
    case ME_ERR_SELF_LOOP: return "error: W has a self loop";
    case ME_ERR_BAD_WEIGHT: return "error: weight not finite or not positive";
    case ME_ERR_ISOLATED_NODE: return "error: isolated node";
    case ME_ERR_K_RANGE: return "error: K out of range for this graph";
    case ME_ERR_WORKSPACE: return "error: workspace too small";
    case ME_ERR_HIP: return "error: HIP runtime call failed";
    case ME_ERR_BREAKDOWN: return "error: non-finite values in the iteration";
    case ME_ERR_TOO_LARGE: return "error: graph too large (nnz(W) + nnz(T) >= 2^31)";
    default: return "unknown status";
  }
}


int me_build_workspace_bytes(const me_csr* W, const me_opts* opts, void* stream,
                             size_t* bytes) {
  if (!W || !bytes) return ME_ERR_INVALID_ARG;
  *bytes = 0;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  int64_t tb = 0;
  ME_TRY_STATUS(two_hop_bound(W, (hipStream_t)stream, &tb));
  *bytes = kHeapAlign + build_bytes_bound(W->n, W->nnz, tb) + eps_solve_bytes(W->n);
  return ME_OK;
}

int me_build_graph_ops(const me_csr* W, const me_opts* opts, void* ws, size_t ws_bytes,
                       void* stream, me_graph_ops** out, me_info* info) {
  if (!W || !out) return ME_ERR_INVALID_ARG;
  *out = nullptr;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (ws && ws_bytes < 2 * kHeapAlign) return ME_ERR_WORKSPACE;  // before any device call
  if (ws) {
    size_t need = 0;
    ME_TRY_STATUS(me_build_workspace_bytes(W, &o, stream, &need));
    if (ws_bytes < need) return ME_ERR_WORKSPACE;
  }
  const auto t0 = std::chrono::steady_clock::now();
  auto* h = new (std::nothrow) me_graph_ops();
  if (!h) return ME_ERR_HIP;
  // with a workspace the handle's arrays live in it and nothing is allocated
  DevHeap region(ws, ws_bytes);
  DevHeap hip;
  int st = build_graph_ops(W, &o, ws ? region : hip, s, &h->g, info);
  if (st < 0) {
    (void)hipStreamSynchronize(s);
    free_ops(h->g);
    delete h;
    if (info) info->status = st;
    return st;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    free_ops(h->g);
    delete h;
    return ME_ERR_HIP;
  }
  if (info) {
    info->ms_build =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  *out = h;
  return st;
}

int me_graph_ops_query(const me_graph_ops* ops, int64_t* n, int64_t* nnz_t, double* eps,
                       double* mu, int* components_gt1) {
  if (!ops) return ME_ERR_INVALID_ARG;
  if (n) *n = ops->g.n;
  if (nnz_t) *nnz_t = ops->g.nnz_t;
  if (eps) *eps = ops->g.eps;
  if (mu) *mu = ops->g.mu;
  if (components_gt1) *components_gt1 = ops->g.components > 1;
  return ME_OK;
}

size_t me_graph_ops_bytes(const me_graph_ops* ops) { return ops ? ops->g.mem_bytes : 0; }

int me_graph_ops_export(const me_graph_ops* ops, int64_t* t_rowptr, int32_t* t_col,
                        int32_t* t_count, double* d, double* qdiag, double* r, double* b,
                        void* stream) {
  if (!ops) return ME_ERR_INVALID_ARG;
  const GraphOps& g = ops->g;
  hipStream_t s = (hipStream_t)stream;
  const auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
  };
  ME_TRY(cp(t_rowptr, g.t_rp, (g.n + 1) * 8));
  ME_TRY(cp(t_col, g.t_col, g.nnz_t * 4));
  ME_TRY(cp(t_count, g.t_cnt, g.n * 4));
  ME_TRY(cp(d, g.d, g.n * 8));
  ME_TRY(cp(qdiag, g.qdiag, g.n * 8));
  ME_TRY(cp(r, g.r, g.n * 8));
  ME_TRY(cp(b, g.b, g.n * 8));
  ME_TRY(hipStreamSynchronize(s));
  return ME_OK;
}

int me_graph_ops_order(const me_graph_ops* ops, int32_t* perm, void* stream) {
  if (!ops || !perm) return ME_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  ME_TRY(hipMemcpyAsync(perm, ops->g.perm, ops->g.n * 4, hipMemcpyDeviceToDevice, s));
  ME_TRY(hipStreamSynchronize(s));
  return ME_OK;
}

int me_apply(const me_graph_ops* ops, int which, int k, const double* X, double* Y,
             void* stream) {
  if (!ops || !X || !Y || k < 1 || k > kMaxBlockCols || which < 0 || which > 2)
    return ME_ERR_INVALID_ARG;
  const GraphOps& g = ops->g;
  hipStream_t s = (hipStream_t)stream;
  if (which == 2) {
    launch_scale_rows(g.n, k, g.b, X, Y, s);
    ME_TRY(hipStreamSynchronize(s));
    return ME_OK;
  }
  const int kb = block_width(k);
  double* buf = nullptr;
  const size_t bytes = (size_t)g.n * kb * 8;
  ME_TRY(hipMallocAsync((void**)&buf, 2 * bytes, s));
  ME_TRY(hipMemsetAsync(buf, 0, bytes, s));
  // into the solver order, apply, back to the caller's order
  launch_copy_cols(g.n, k, kb, k, g.perm, X, buf, s);
  launch_spmm<double>(g, kb, which == 0 ? OP_A : OP_Q, buf, buf + (size_t)g.n * kb, nullptr, s);
  launch_copy_cols(g.n, kb, k, k, g.iperm, buf + (size_t)g.n * kb, Y, s);
  ME_TRY(hipFreeAsync(buf, s));
  ME_TRY(hipStreamSynchronize(s));
  return ME_OK;
}

size_t me_embed_workspace_bytes(const me_graph_ops* ops, int K, const me_opts* opts) {
  if (!ops || K < 1 || K > kMaxBlockCols) return 0;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  return embed_workspace_bytes(ops->g.n, K, &o);
}

int me_embed(const me_graph_ops* ops, int K, double tol, const me_opts* opts, const double* X0,
             void* ws, size_t ws_bytes, double* X, double* lambda, me_info* info, void* stream) {
  if (!ops) return ME_ERR_INVALID_ARG;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  return embed(ops->g, K, tol, &o, X0, ws, ws_bytes, X, lambda, info, (hipStream_t)stream);
}

int me_embed_batch_workspace_bytes(int G, const me_csr* Ws, const int* Ks, const me_opts* opts,
                                   void* stream, size_t* bytes) {
  if (!bytes || G < 0 || (G > 0 && (!Ws || !Ks))) return ME_ERR_INVALID_ARG;
  *bytes = 0;
  if (G == 0) return ME_OK;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  return batch_workspace_bytes(G, Ws, Ks, &o, (hipStream_t)stream, bytes);
}

int me_embed_batch(int G, const me_csr* Ws, const int* Ks, double tol, const me_opts* opts,
                   void* ws, size_t ws_bytes, double* const* Xs, double* const* lambdas,
                   me_info* infos, void* stream) {
  if (G < 0 || (G > 0 && (!Ws || !Ks || !Xs || !lambdas)) || !(tol > 0.0))
    return ME_ERR_INVALID_ARG;
  if (G == 0) return ME_OK;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  if (ws && ws_bytes < 2 * kHeapAlign) return ME_ERR_WORKSPACE;  // before any device call
  if (infos) std::memset(infos, 0, sizeof(me_info) * (size_t)G);
  return embed_batch(G, Ws, Ks, tol, &o, ws, ws_bytes, Xs, lambdas, infos, (hipStream_t)stream);
}

void me_graph_ops_destroy(me_graph_ops* ops) {
  if (!ops) return;
  (void)hipDeviceSynchronize();
  free_ops(ops->g);
  delete ops;
}

}  // extern "C"
