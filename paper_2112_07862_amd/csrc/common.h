// Internal declarations shared by the HIP translation units of libmembed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <thread>
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
#ifndef ME_HALO_ROWS
#define ME_HALO_ROWS 32
#endif
constexpr int kHaloRows = ME_HALO_ROWS;  // rows per tile of the halo-staged preconditioner step
constexpr int kHaloMaxE = 2048;      // entries of one tile and range the halo build sorts
constexpr int kMaxBlockCols = 16;    // largest LOBPCG block width
constexpr int kMaxBasis = 48;        // 3 x kMaxBlockCols: Rayleigh-Ritz basis size
constexpr int kDenseMaxN = 48;       // graphs up to this size are solved densely
constexpr int kPartialBlocks = 256;  // grid of the reducing streaming kernels
constexpr int kMaxChebDegree = 256;  // largest Chebyshev preconditioner degree
constexpr int kRhoHist = 32;         // residual history kept per solve
constexpr int kXcd = 8;              // accelerator complex dies (one L2 each)
// largest array (bytes) the buffer-resource kernels address with 32-bit offsets
constexpr int64_t kBufMaxBytes = (int64_t)1 << 31;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroup i of a launch runs on XCD i mod kXcd.  Gathering kernels remap
// their workgroups so that each XCD runs one contiguous range of logical
// blocks: rows that are close in the locality order then meet in the same
// L2.  Launch xcd_grid(nblocks) workgroups; logical blocks >= nblocks exit.
__host__ __device__ inline int64_t xcd_grid(int64_t nblocks) {
  return kXcd * ((nblocks + kXcd - 1) / kXcd);
}
__device__ __forceinline__ int64_t xcd_block(int64_t nblocks) {
  const int64_t per = (nblocks + kXcd - 1) / kXcd;
  return (int64_t)(blockIdx.x % kXcd) * per + blockIdx.x / kXcd;
}

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

constexpr size_t kHeapAlign = 256;

// Device memory of one call (or of one server).  Without a region every
// request is a stream-ordered hipMallocAsync / hipFreeAsync.  Over a
// caller-owned region (the workspace arguments of the C ABI) requests are
// carved first-fit in kHeapAlign units and no HIP allocation is made; a
// released range is reused at once, so `release` is only for memory whose
// work is complete (its stream synchronised), and `release_later` defers the
// range to the next `quiesce`, which the owner calls once every stream that
// used the heap is idle.  If the region holds at least the sum of every
// request of a call (each rounded to kHeapAlign), first fit never fails,
// whatever the order of releases: each request lands either in a hole below
// the highest byte in use or right above it.  Thread-safe.
class DevHeap {
 public:
  DevHeap() = default;
  DevHeap(void* base, size_t bytes);
  DevHeap(const DevHeap&) = delete;
  DevHeap& operator=(const DevHeap&) = delete;
  // ME_ERR_WORKSPACE when the region has no free range of `bytes`.
  int alloc(void** p, size_t bytes, hipStream_t s);
  template <typename T>
  int alloc_n(T** p, size_t count, hipStream_t s) {
    return alloc(reinterpret_cast<void**>(p), count * sizeof(T), s);
  }
  void release(void* p, hipStream_t s);
  void release_later(void* p, hipStream_t s);
  void quiesce();
  bool region() const { return region_; }
  bool owns(const void* p) const;
  size_t high_water() const { return hw_; }
  size_t capacity() const { return cap_; }
  size_t largest_free();
  static size_t round(size_t bytes) { return (bytes + kHeapAlign - 1) & ~(kHeapAlign - 1); }

 private:
  void put_back(size_t off, size_t len);
  std::mutex mu_;
  char* base_ = nullptr;
  size_t cap_ = 0;
  bool region_ = false;
  std::map<size_t, size_t> free_;  // offset -> bytes
  std::map<size_t, size_t> live_;  // offset -> bytes
  std::vector<void*> later_;
  size_t hw_ = 0;
};

// Device-side control block of one LOBPCG solve.  Written by the per-slot
// finalize kernels, read by every iteration kernel (early exit once `done`)
// and copied to the host at each convergence check.
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
  int cheb_deg;    // Chebyshev preconditioner degree (0: none)
  double tol;
  double lam_floor;          // |lambda| below this is treated as zero ...
  double lam_scale;          // ... and replaced by this operator scale in rho
  // Chebyshev preconditioner: spectrum of D^-1 Op taken as [a, cheb_b];
  // a follows the leading nonzero Ritz pair (cheb_afac times its
  // D-Rayleigh quotient).
  double cheb_afac;
  double cheb_b;
  double orth;               // max |X^T B X - I| at exit
  double rho[kMaxBlockCols]; // last residuals
  double lam[kMaxBlockCols]; // Ritz values of the certificate pass
  // largest residual of the required columns at iteration i, at
  // rho_hist[i % kRhoHist] (the host's convergence-rate estimate)
  double rho_hist[kRhoHist];
  // 1 / |r_j| of the last residual block: the FP16 preconditioner path
  // scales its input columns to unit norm (FP16's range)
  double rinv[kMaxBlockCols];
};

// Arguments of the breadth-first searches of one graph (device scratch; one
// workgroup per graph).
struct OrderArgs {
  int64_t n;
  const int64_t* rp;
  const int32_t* col;
  int32_t *level, *fa, *fb, *ev, *ei, *ef, *start, *perm;
  int32_t* maxlev;  // receives the deepest level
  // > 0: the first component is already placed in perm[0, resume_off),
  // its last level resume_last; the one-workgroup ordering continues with
  // the further components
  int64_t resume_off;
  int32_t resume_last;
};

// Searches in flight between order_launch and order_finish.
struct OrderJob {
  void* args = nullptr;  // device argument array
  std::thread th;        // drives the per-level launches of large graphs
  int status = 0;
  ~OrderJob() {
    if (th.joinable()) th.join();
  }
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
  double cheb_b_p = 2.0;    // and of diag(L + eps I)^-1 (L + eps I)
  double* pdinv = nullptr;  // 1 / (d_i + eps): Jacobi scaling of L + eps I
  float* pdinv32 = nullptr;
  float* b32 = nullptr;
  float* dinv32 = nullptr;
  float* invt32 = nullptr;
  // Solver order (locality permutation): solver row i' is user row perm[i'].
  int32_t* perm = nullptr;     // solver index -> user index
  int32_t* lev_s = nullptr;    // breadth-first level of each solver row
  int32_t max_level = 0;       // deepest level
  int32_t* iperm = nullptr;    // user index -> solver index
  double *qinv_s = nullptr, *b_s = nullptr, *dinv_s = nullptr, *pdinv_s = nullptr;
  double* invt_s = nullptr;    // 1 / T_i in solver order (two-hop weights of the FP64 products)
  float *qinv32_s = nullptr, *b32_s = nullptr, *dinv32_s = nullptr, *pdinv32_s = nullptr;
  // difference-form operator in solver order: W entries of row i at [a_rp[i], a_rp[i+1]),
  // T entries at [a_tp[i], a_tp[i+1]) (all W entries precede all T entries)
  int32_t* a_rp = nullptr;     // int32[n+1]
  int32_t* a_tp = nullptr;     // int32[n+1]
  int32_t* a_col = nullptr;    // int32[nnz_w + nnz_t]
  double* a_w = nullptr;       // w_ij at the W positions, 1/T_i + 1/T_j at the T positions
  float* a_w32 = nullptr;
  // the same entries packed for the FP32 preconditioner: bits 0-15 the
  // column minus the row (int16), bits 16-31 the weight (FP16); usable when
  // every |column - row| fits (pk_ok)
  uint32_t* a_pk = nullptr;
  bool pk_ok = false;
  bool w32_ok = true;  // every W weight finite in FP32 (the FP32 copies a_w32, a_pk)
  // the two-hop entries packed for the FP64 products: bits 0-15 the column
  // minus the row (int16), bits 16-31 T_j of the column (the weight is
  // 1/T_i + 1/T_j, formed on the fly); usable when offsets and counts fit
  // (tq_ok).  Entry k of the T block (position nnz_w + k) is a_tq[k].
  uint32_t* a_tq = nullptr;
  bool tq_ok = false;
  // Neighbour halos of the FP32 preconditioner (tiles of kHaloRows rows in
  // the solver order, per entry range W and T): h_list holds each tile's
  // distinct columns, sorted, at the position of the tile's first entry of
  // the range (a tile has no more distinct columns than entries); h_pk holds
  // per entry its column's slot in that list (bits 0-15) and the FP16 weight
  // of a_pk (bits 16-31); h_cnt_w / h_cnt_t the list lengths, h_max_w /
  // h_max_t their maxima; halo_w / halo_t whether every tile fitted.
  uint32_t* h_pk = nullptr;
  int32_t* h_list = nullptr;
  int32_t* h_cnt_w = nullptr;
  int32_t* h_cnt_t = nullptr;
  int32_t h_max_w = 0, h_max_t = 0;
  bool halo_w = false, halo_t = false;
  double* scratch_d = nullptr;  // n doubles of build scratch
  int64_t *woff = nullptr, *toff = nullptr;  // row offsets of the packed blocks
  OrderArgs ord{};              // search arguments while the order is pending
  void* ord_mem = nullptr;      // their scratch
  int* dflags = nullptr;        // 64 ints of build flags and reductions
  bool needs_eps = false;       // two-hop graph connected: eps = lambda_2(Q) > 0
  void* mem = nullptr;   // per-node arrays, W copy
  void* mem2 = nullptr;  // T columns and the merged operator
  size_t mem_bytes = 0;
  bool in_region = false;  // memory carved from a caller's workspace (not freed here)
  int device = 0;
};

// ---- launchers: build.hip -------------------------------------------------
int build_graph_ops(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g,
                    me_info* info);
// Device bytes of the build's allocations (see build_bytes_bound).
size_t build_mem1_bytes(int64_t n, int64_t nnz);
size_t build_mem2_bytes(int64_t nnz, int64_t nnz_t);
size_t order_scratch_bytes(int64_t n, int64_t nnz);
size_t order_args_bytes(int G);
size_t twohop_bitmap_bytes(int64_t n);
// Every allocation of build_pre for a graph of n nodes, nnz entries and at
// most nnz_t_max two-hop entries (each rounded to the heap's unit).
size_t build_bytes_bound(int64_t n, int64_t nnz, int64_t nnz_t_max);
// Exclusive scan of int32 counts into int64 offsets out[0..n] (out[n] = the
// total); tile_tmp holds scan_tmp_count(n) int64.
int64_t scan_tmp_count(int64_t n);
void scan_counts(int64_t n, const int32_t* cnt, int64_t* out, int64_t* tile_tmp, hipStream_t s);
// Upper bound of nnz(T) from W's degrees (reads W's row pointers).
int two_hop_bound(const me_csr* W, hipStream_t s, int64_t* bound);
// option ranges of me_opts (shared by every entry point that takes them)
bool opts_valid(const me_opts& o);
// build_pre = build_pre_a (validation, T, Q_ii, connectivity; the order's
// scratch) + the locality order + build_pre_b (operator packed in that
// order).  Batches run the searches of all graphs in one launch.
int build_pre(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g);
int build_pre_a(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g);
int order_launch(GraphOps* const* gs, int G, DevHeap& heap, hipStream_t s, OrderJob* job);
int order_finish(GraphOps* const* gs, int G, DevHeap& heap, hipStream_t s, OrderJob* job);
int build_pre_b(GraphOps* g, hipStream_t s);
int build_post(GraphOps* g, double eps, int eps_iters, hipStream_t s);

// ---- launchers: dense.hip -------------------------------------------------
// Dense generalized eigenproblem for graphs with n <= 48: all n pairs of
// (a_dense, b_dense), both n x n; vec n x n (column t = pair t), lam ascending.
void launch_dense_geneig(int n, const double* a_dense, const double* b_dense, double* vec,
                         double* lam, hipStream_t s);

// ---- launchers: stream_ops.hip ---------------------------------------------
enum OpKind { OP_A = 0, OP_Q = 1 };

template <typename T>
void launch_spmm(const GraphOps& g, int kb, OpKind op, const T* x, T* y, const int* done,
                 hipStream_t s);
// scratch: 64 * kb * 16 bytes; x in solver order, out in user order
void launch_sign_fix_and_copy(int64_t n, int kb, int k, const double* x, double* out,
                              const double* lam, double* lam_out, double* scratch,
                              const int32_t* perm, const int32_t* iperm, hipStream_t s);
void launch_scale_rows(int64_t n, int k, const double* b, const double* x, double* y,
                       hipStream_t s);
// dense n x n operator (which 0: A, 1: Q) and matching B (diag(b) or I)
void launch_dense_ops(const GraphOps& g, int which, double* out, double* bmat, hipStream_t s);
// dst[i][j] = src[map ? map[i] : i][j]
void launch_copy_cols(int64_t n, int ksrc, int kdst, int kcopy, const int32_t* map,
                      const double* src, double* dst, hipStream_t s);

// ---- timing.hip -------------------------------------------------------------
enum KTimeKind { KT_OFF = 0, KT_SPMM_A = 1, KT_GRAM_RR = 2, KT_COMBINE = 3, KT_CHEB = 4 };
// Records HIP events around `launches` back-to-back launches of one kernel
// (bytes: their algorithmic total) when `kind` is the kind being timed.
struct KScope {
  KScope(int kind, hipStream_t s, double bytes, int tag, int launches = 1);
  ~KScope();
  bool on;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  double bytes_ = 0.0;
  int tag_ = 0, phase_ = 0, launches_ = 1;
};
int ktimer_kind();
int ktimer_new_phase();
void ktimer_drop_after(int phase, int last_real);
void ktimer_collect();

// ---- knn.hip ----------------------------------------------------------------
size_t knn_workspace_bytes(int64_t n, int k);
int knn_graph(const double* x, int64_t n, int dim, int k, void* ws, size_t ws_bytes,
              int64_t* rowptr, int32_t* col, double* val, int64_t* nnz, double* sigma,
              hipStream_t s);

// ---- cluster.hip ------------------------------------------------------------
size_t cluster_workspace_bytes(int64_t n, int K, int C);

// ---- vbc.hip ----------------------------------------------------------------
size_t betweenness_workspace_bytes(int64_t n);
int betweenness(const me_csr* W, void* ws, size_t ws_bytes, double* cb, double* vbc,
                hipStream_t s);

// ---- lobpcg.hip -------------------------------------------------------------
int solve_eps(GraphOps& g, const me_opts* o, DevHeap& heap, hipStream_t s, double* eps,
              int* iters);
// Device bytes the eps solve of a graph with n nodes allocates.
size_t eps_solve_bytes(int64_t n);
int block_width(int K);
size_t embed_workspace_bytes(int64_t n, int K, const me_opts* o);
int embed(const GraphOps& g, int K, double tol, const me_opts* o, const double* x0, void* ws,
          size_t ws_bytes, double* X, double* lambda, me_info* info, hipStream_t s);
// Footprint of one server request (build bound and both solver slots).
size_t request_bytes(int64_t n, int64_t nnz, int64_t nnz_t_max, int K);
size_t dense_request_bytes(int64_t n);
// Workspace bound of embed_batch (reads every graph's row pointers).
int batch_workspace_bytes(int G, const me_csr* Ws, const int* Ks, const me_opts* o,
                          hipStream_t s, size_t* bytes);
int embed_batch(int G, const me_csr* Ws, const int* Ks, double tol, const me_opts* o, void* ws,
                size_t ws_bytes, double* const* Xs, double* const* lams, me_info* infos,
                hipStream_t s);
// Releases the device memory of a GraphOps (partially built ones too).
void free_graph_ops(GraphOps& g);

}  // namespace me

struct me_graph_ops {
  me::GraphOps g;
};
