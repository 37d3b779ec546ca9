// Row-streaming kernels of the LOBPCG engine.  Every launch covers one set
// of slots with a common block width KB through a work list of tiles; a
// tile belongs to one slot, so all lanes of a workgroup share the slot's
// pointers (scalar loads) and its early-exit flag.
//
// Blocks are row-major n x KB.  Elementwise kernels give each row
// LPR = KB / VEC lanes with one 16-byte vector each; the gathering kernels
// (operator products) give each row G lanes (RowCfg: two entries per round
// per 16-byte chunk by default) that split the row's entries, 32 rows per
// workgroup.
//
// Difference-form operator (eq. (obj2) with the Laplacian identity of
// Section 3.1): with a row's W entries (weight w_ij) and T entries (weight
// 1/T_i + 1/T_j),
//   (A x)_i = sum_{j in N(i)} w_ij (x_i - x_j)
//             - mu sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j) + eps x_i
//   (Q x)_i = sum_{j in T_i} (1/T_i + 1/T_j) (x_i - x_j)
#include <cmath>
#include <cstddef>
#include <cstdlib>

#include "common.h"
#include "engine.h"
#include "rowops.h"

namespace me {

// FP64 rows of at most two 16-byte chunks (block width 4: the eps solve)
// read the packed two-hop entries (measured faster there: 78 against 87 us
// for the 1M sphere's Q product); wider rows repeat the entry decode, a
// correctly rounded 1 / T_j, in every chunk lane and read the stored weight
// instead (692 against 536-600 us at width 16).
template <typename T, int KB>
constexpr bool kTqRows = sizeof(T) == 8 && RowCfg<T, KB>::NCH <= 2;

template <typename T>
struct SB;
template <>
struct SB<double> {
  static __device__ __forceinline__ double* blk(const SlotDev& d, int id) { return d.b64[id]; }
  static __device__ __forceinline__ const double* w(const SlotDev& d) { return d.a_w; }
  static __device__ __forceinline__ const double* dinv(const SlotDev& d) { return d.dinv; }
  static __device__ __forceinline__ const double* cdinv(const SlotDev& d) { return d.cheb_dinv; }
};
template <>
struct SB<float> {
  static __device__ __forceinline__ float* blk(const SlotDev& d, int id) { return d.b32[id]; }
  static __device__ __forceinline__ const float* w(const SlotDev& d) { return d.a_w32; }
  static __device__ __forceinline__ const float* dinv(const SlotDev& d) { return d.dinv32; }
  static __device__ __forceinline__ const float* cdinv(const SlotDev& d) { return d.cheb_dinv32; }
};

// rows per tile of the elementwise kernels
template <typename T, int KB>
struct ElemCfg {
  using L = Lay<T, KB>;
  static constexpr int VEC = L::VEC, LPR = L::LPR, RB = kBlock / LPR;
};

__device__ __forceinline__ bool slot_done(const SlotDev& d) { return *glob(&d.ctrl->done) != 0; }
__device__ __forceinline__ bool skip_slot(const SlotDev& d, int cert) {
  return !cert && slot_done(d);
}

// ---------------------------------------------------------------------------
// Operator product Y = Op X (gathering; XCD-aware tile order)
// ---------------------------------------------------------------------------

template <typename T, int KB, bool BUF>
__global__ void __launch_bounds__((RowCfg<T, KB>::THREADS)) k_sl_spmm(const SlotDev* __restrict__ sl,
                                                    const Tile* __restrict__ tiles,
                                                    int64_t ntiles, int in, int out, int cert) {
  using C = RowCfg<T, KB>;
  const int64_t b = xcd_block(ntiles);
  if (b >= ntiles) return;
  const Tile t = tiles[b];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert)) return;
  const int64_t row = (int64_t)t.blk * kGatherRows + threadIdx.x / C::G;
  const int q = threadIdx.x % C::G;
  const bool live = row < d.n;
  const T* x = SB<T>::blk(d, in);
  const int ch = q % C::NCH;
  T xi[C::V16], acc[C::V16];
  // own row (row 0 stands in for rows past the end; their lanes add nothing)
  if constexpr (BUF) {
    const BufRsrc rx = buf_rsrc(x, d.n * KB * (int64_t)sizeof(T));
    const auto own = buf_vec16<T, C::V16>(
        rx, (uint32_t)(live ? row : 0) * (uint32_t)(KB * sizeof(T)) + (uint32_t)(ch * 16));
#pragma unroll
    for (int v = 0; v < C::V16; ++v) xi[v] = own.v[v];
    const RowSpan sp = row_span(live, row, d.a_rp, d.a_tp, d.range);
    const int64_t rs = live ? row : 0;
    BufRsrc rq{};
    T ti = 0;
    const bool tq = kTqRows<T, KB> && d.tq_ok;
    if (tq) {
      rq = buf_rsrc(d.a_tq, (d.nnz_ops - d.tq_base) * 4);
      ti = (T)glob(d.invt)[rs];
    }
    spmm_span_buf<T, KB>(sp.ws, sp.nw, sp.ts, sp.len, q, rs, buf_rsrc(d.a_col, d.nnz_ops * 4),
                         buf_rsrc(SB<T>::w(d), d.nnz_ops * (int64_t)sizeof(T)), rq,
                         (uint32_t)d.tq_base, tq, ti, rx, (T)d.c_t, xi, acc);
  } else {
    load_chunk<T, C::V16>(x + (live ? row : 0) * KB + ch * C::V16, xi);
    spmm_row<T, KB>(live, row, q, d.a_rp, d.a_tp, d.a_col, SB<T>::w(d), (T)d.c_t, d.range, x,
                    xi, acc);
  }
  if (!live || q >= C::NCH) return;
  // lane q < NCH holds chunk q of the row
  const T sd = (T)d.s_diag;
  VecT<T, C::V16> o;
#pragma unroll
  for (int v = 0; v < C::V16; ++v) o.v[v] = fmaT(sd, xi[v], acc[v]);
  stv<T, C::V16>(SB<T>::blk(d, out) + row * KB + q * C::V16, o);
}

template <typename T>
void sl_spmm(const SlotDev* sl, const TileSet& ts, int in, int out, int cert, hipStream_t s) {
  if (ts.n_gather == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    static_assert(RowCfg<T, KB>::ROWS == kGatherRows, "gather tile rows");
    if (ts.buf)
      k_sl_spmm<T, KB, true><<<xcd_grid(ts.n_gather), RowCfg<T, KB>::THREADS, 0, s>>>(
          sl, ts.gather, ts.n_gather, in, out, cert);
    else
      k_sl_spmm<T, KB, false><<<xcd_grid(ts.n_gather), RowCfg<T, KB>::THREADS, 0, s>>>(
          sl, ts.gather, ts.n_gather, in, out, cert);
  });
}
template void sl_spmm<double>(const SlotDev*, const TileSet&, int, int, int, hipStream_t);
template void sl_spmm<float>(const SlotDev*, const TileSet&, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Chebyshev preconditioner: approximate solve of Op y = R with Jacobi
// scaling D, spectrum of D^-1 Op taken as [a, b], theta = (a + b) / 2, in
// three-term form (y_0 = 0):
//   y_1 = D^-1 R / theta,
//   y_{k+1} = y_k + alpha_k (y_k - y_{k-1}) + beta_k D^-1 (R - Op y_k).
// Step k gathers y_k and overwrites y_{k-1} with y_{k+1} (each row reads its
// own y_{k-1} before writing it; neighbours only read y_k).
// ---------------------------------------------------------------------------

template <typename T, int KB, bool R16>
__global__ void __launch_bounds__(kBlock) k_sl_cheb_first(const SlotDev* __restrict__ sl,
                                                          const Tile* __restrict__ tiles, int r,
                                                          int y, int yprev) {
  using E = ElemCfg<T, KB>;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (slot_done(d)) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / E::LPR;
  const int sub = threadIdx.x % E::LPR;
  if (row >= d.n) return;
  const T sc = (T)(1.0 / *glob(&d.cheb->theta)) * glob(SB<T>::cdinv(d))[row];
  const int64_t o = row * KB + sub * E::VEC;
  VecT<T, E::VEC> v;
  if constexpr (R16) {  // right-hand side in FP16
    static_assert(sizeof(T) == 4 && E::VEC % 4 == 0, "FP16 right-hand side of FP32 steps");
    const _Float16* rh = reinterpret_cast<const _Float16*>(SB<T>::blk(d, r)) + o;
#pragma unroll
    for (int h = 0; h < E::VEC / 4; ++h) {
      const auto f = ld_half4(rh + 4 * h);
#pragma unroll
      for (int q = 0; q < 4; ++q) v.v[4 * h + q] = f.v[q];
    }
  } else {
    v = ldv<T, E::VEC>(SB<T>::blk(d, r) + o);
  }
#pragma unroll
  for (int q = 0; q < E::VEC; ++q) v.v[q] *= sc;
  stv<T, E::VEC>(SB<T>::blk(d, y) + o, v);
#pragma unroll
  for (int q = 0; q < E::VEC; ++q) v.v[q] = 0;
  stv<T, E::VEC>(SB<T>::blk(d, yprev) + o, v);
}

// What one step needs of a slot, gathered in one place: read from the slot
// table by the work-list kernel, passed by value (kernel arguments, one
// scalar load) by the one-slot kernel.
template <typename T>
struct ChebView {
  int64_t n, nnz_ops;
  const int32_t *a_rp, *a_tp, *a_col;
  const uint32_t* a_pk;
  const T *a_w, *cdinv, *yin, *r;
  T* yout;
  const double* invt;      // 1 / T_i in solver order (FP64 two-hop weights)
  const uint32_t* a_tq;    // packed two-hop entries of the FP64 form (tq_ok)
  int64_t tq_base;
  int tq_ok;
  const uint32_t* h_pk;    // halos of the range (h_cnt null: none)
  const int32_t* h_list;
  const int32_t* h_cnt;
  int h_max;
  const double *alpha, *beta;
  const int* done;
  double c_t, s_diag;
  int range;
};

template <typename T>
__device__ __forceinline__ ChebView<T> cheb_view(const SlotDev& d, int r, int yin, int yout) {
  ChebView<T> v;
  v.n = d.n;
  v.nnz_ops = d.nnz_ops;
  v.a_rp = d.a_rp;
  v.a_tp = d.a_tp;
  v.a_col = d.a_col;
  v.a_pk = d.a_pk;
  v.a_w = SB<T>::w(d);
  v.cdinv = SB<T>::cdinv(d);
  v.yin = SB<T>::blk(d, yin);
  v.r = SB<T>::blk(d, r);
  v.yout = SB<T>::blk(d, yout);
  v.invt = d.invt;
  v.a_tq = d.a_tq;
  v.tq_base = d.tq_base;
  v.tq_ok = d.tq_ok;
  v.h_pk = d.h_pk;
  v.h_list = d.h_list;
  v.h_cnt = d.h_cnt;
  v.h_max = d.h_max;
  v.alpha = d.cheb->alpha;
  v.beta = d.cheb->beta;
  v.done = &d.ctrl->done;
  v.c_t = d.c_t;
  v.s_diag = d.cheb_s_diag;
  v.range = d.cheb_range;
  return v;
}

// Rows row0, row0 + 1, ... (blockDim.x / G of them) through buffer resources.  Everything a row needs
// besides its neighbours is requested before the slot's done flag is tested
// (all of it in bounds either way), so the flag, the row bounds and the
// row's own data share one memory latency.
template <typename T, int KB, int RANGE, bool PK>
__device__ __forceinline__ void cheb_step_rows(const ChebView<T>& d, int64_t row0, int k) {
  using C = RowCfg<T, KB>;
  const int64_t row = row0 + threadIdx.x / C::G;
  const int q = threadIdx.x % C::G;
  const bool live = row < d.n;
  const int ch = q % C::NCH;
  const T sd = (T)d.s_diag;
  T yi[C::V16], acc[C::V16];
  const int64_t rs = live ? row : 0;
  const uint32_t oo = (uint32_t)rs * (uint32_t)(KB * sizeof(T)) + (uint32_t)(ch * 16);
  const int64_t xb = d.n * KB * (int64_t)sizeof(T);
  const BufRsrc rx = buf_rsrc(d.yin, xb);
  const auto own = buf_vec16<T, C::V16>(rx, oo);
  VecT<T, C::V16> ri;
  if constexpr (PK) {  // packed sets: right-hand side in FP16
    static_assert(sizeof(T) == 4, "packed entries serve the FP32 preconditioner");
    ri = buf_half4(buf_rsrc(d.r, d.n * KB * 2), (uint32_t)rs * (uint32_t)(KB * 2) + (uint32_t)(ch * 8));
  } else {
    ri = buf_vec16<T, C::V16>(buf_rsrc(d.r, xb), oo);
  }
  auto yo = buf_vec16<T, C::V16>(buf_rsrc(d.yout, xb), oo);  // y_{k-1}
  const T cd = glob(d.cdinv)[rs];
  const T alpha = (T)*glob(&d.alpha[k]);
  const T bk = (T)*glob(&d.beta[k]);
  const RowSpan sp = row_span(live, row, d.a_rp, d.a_tp, d.range);
  asm volatile("" ::: "memory");  // keeps the requests above ahead of the test
  if (*glob(d.done)) return;
#pragma unroll
  for (int v = 0; v < C::V16; ++v) yi[v] = own.v[v];
  if constexpr (PK) {
    static_assert(sizeof(T) == 4, "packed entries serve the FP32 preconditioner");
    spmm_span_pk<KB, RANGE, true>(sp.ws, sp.nw, sp.ts, sp.len, q, rs, d.a_pk, d.nnz_ops, d.yin,
                                  d.n, (float)d.c_t, yi, acc);
  } else {
    BufRsrc rq{};
    T ti = 0;
    const bool tq = kTqRows<T, KB> && d.tq_ok;
    if (tq) {
      rq = buf_rsrc(d.a_tq, (d.nnz_ops - d.tq_base) * 4);
      ti = (T)glob(d.invt)[rs];
    }
    spmm_span_buf<T, KB, RANGE>(sp.ws, sp.nw, sp.ts, sp.len, q, rs,
                                buf_rsrc(d.a_col, d.nnz_ops * 4),
                                buf_rsrc(d.a_w, d.nnz_ops * (int64_t)sizeof(T)), rq,
                                (uint32_t)d.tq_base, tq, ti, rx, (T)d.c_t, yi, acc);
  }
  if (!live || q >= C::NCH) return;
  // lane q < NCH updates chunk q of the row
  const T beta = bk * cd;
#pragma unroll
  for (int v = 0; v < C::V16; ++v) {
    const T res = ri.v[v] - fmaT(sd, yi[v], acc[v]);
    yo.v[v] = yi[v] + fmaT(alpha, yi[v] - yo.v[v], beta * res);
  }
  stv<T, C::V16>(d.yout + row * KB + q * C::V16, yo);
}

// Work-list form (any number of slots).
template <typename T, int KB, bool BUF, bool PK>
__global__ void __launch_bounds__((RowCfg<T, KB>::THREADS)) k_sl_cheb_step(const SlotDev* __restrict__ sl,
                                                         const Tile* __restrict__ tiles,
                                                         int64_t ntiles, int k, int r, int yin,
                                                         int yout) {
  using C = RowCfg<T, KB>;
  const int64_t b = xcd_block(ntiles);
  if (b >= ntiles) return;
  const Tile t = tiles[b];
  const SlotDev& d = sl[t.slot];
  if constexpr (BUF) {
    cheb_step_rows<T, KB, -1, PK>(cheb_view<T>(d, r, yin, yout), (int64_t)t.blk * kGatherRows, k);
  } else {
    const int64_t row = (int64_t)t.blk * kGatherRows + threadIdx.x / C::G;
    const int q = threadIdx.x % C::G;
    const bool live = row < d.n;
    const int ch = q % C::NCH;
    const T sd = (T)d.cheb_s_diag;
    T yi[C::V16], acc[C::V16];
    if (slot_done(d)) return;
    const T* yi_p = SB<T>::blk(d, yin);
    load_chunk<T, C::V16>(yi_p + (live ? row : 0) * KB + ch * C::V16, yi);
    if constexpr (PK) {
      static_assert(sizeof(T) == 4, "packed entries serve the FP32 preconditioner");
      const RowSpan sp = row_span(live, row, d.a_rp, d.a_tp, d.cheb_range);
      spmm_span_pk<KB, -1, false>(sp.ws, sp.nw, sp.ts, sp.len, q, live ? row : 0, d.a_pk,
                                  d.nnz_ops, yi_p, d.n, (float)d.c_t, yi, acc);
    } else {
      spmm_row<T, KB>(live, row, q, d.a_rp, d.a_tp, d.a_col, SB<T>::w(d), (T)d.c_t,
                      d.cheb_range, yi_p, yi, acc);
    }
    if (!live || q >= C::NCH) return;
    const T alpha = (T)*glob(&d.cheb->alpha[k]);
    const T beta = (T)*glob(&d.cheb->beta[k]) * glob(SB<T>::cdinv(d))[row];
    const int64_t o = row * KB + q * C::V16;
    VecT<T, C::V16> ri;
    if constexpr (PK)  // packed sets: right-hand side in FP16
      ri = ld_half4(reinterpret_cast<const _Float16*>(SB<T>::blk(d, r)) + o);
    else
      ri = ldv<T, C::V16>(SB<T>::blk(d, r) + o);
    T* yo_p = SB<T>::blk(d, yout);
    auto yo = ldv<T, C::V16>(yo_p + o);  // y_{k-1} of this row
#pragma unroll
    for (int v = 0; v < C::V16; ++v) {
      const T res = ri.v[v] - fmaT(sd, yi[v], acc[v]);
      yo.v[v] = yi[v] + fmaT(alpha, yi[v] - yo.v[v], beta * res);
    }
    stv<T, C::V16>(yo_p + o, yo);
  }
}

// One-slot form: the slot's view arrives in the kernel arguments, so no
// table is read before the rows; the entry range is a template argument.
// Workgroups of kStep1Rows rows (one wave for the default row mapping):
// measured faster than 32-, 64- and 128-row workgroups.
constexpr int kStep1Rows = kGatherRows / 2;
template <typename T, int KB>
constexpr int step1_threads() {
  return kStep1Rows * RowCfg<T, KB>::G;
}
template <typename T, int KB, int RANGE, bool PK>
__global__ void __launch_bounds__((step1_threads<T, KB>())) k_sl_cheb_step1(ChebView<T> v,
                                                                          int64_t nblocks, int k) {
  const int64_t b = xcd_block(nblocks);
  if (b >= nblocks) return;
  cheb_step_rows<T, KB, RANGE, PK>(v, b * kStep1Rows, k);
}

// One-slot FP32 step over packed entries with the tile's neighbour rows of
// y_k staged in LDS: the tile's distinct columns (its halo list) are loaded
// once, coalesced, and each entry reads its neighbour's chunk from LDS at
// the entry's halo slot.  Entries, weights and their order are those of the
// packed product (an entry past the span reads the row itself with weight
// 0), so the step equals k_sl_cheb_step1's bit for bit.  The tile's first
// round of entries and its list are requested with the row's own data,
// before the rows of the halo.
static_assert(kGatherRows % kHaloRows == 0, "a gather tile is a whole number of halo tiles");
template <int KB>
constexpr int halo_threads() {
  return kHaloRows * RowCfg<float, KB>::G;
}
// halo chunks a thread stages per pass (4 measured faster than 8: fewer
// registers)
constexpr int kHaloStage = 4;
// One halo tile (kHaloRows rows from row0 = tile kHaloRows) by NT =
// kHaloRows G threads (tid in [0, NT)), its halo staged at hl.  RANGE is the
// entry range (kRangeW, kRangeT) or -1: taken from the slot (tr: T range).
// Every thread of the workgroup reaches the one barrier (the done test and
// the tile's existence are the same for all of them).
template <int KB, int RANGE>
__device__ __forceinline__ void cheb_tile_halo(const ChebView<float>& d, int64_t tile, int tid,
                                               int k, float* hl) {
  using C = RowCfg<float, KB>;
  constexpr int V = C::V16, EPL = C::EPL, UNR = C::UNR, NCH = C::NCH, G = C::G;
  constexpr int NT = kHaloRows * G;
  const bool tr = RANGE == -1 ? d.range == kRangeT : RANGE == kRangeT;
  const int64_t row0 = tile * kHaloRows;
  const int64_t row = row0 + tid / G;
  const int q = tid % G;
  const bool tile_live = row0 < d.n;
  const bool live = row < d.n;
  const int ch = q % NCH, e0 = q / NCH;
  const int64_t rs = live ? row : 0;
  const uint32_t oo = (uint32_t)rs * (uint32_t)(KB * 4) + (uint32_t)(ch * 16);
  const int64_t xb = d.n * KB * 4;
  const BufRsrc rx = buf_rsrc(d.yin, xb);
  const auto own = buf_vec16<float, V>(rx, oo);
  // right-hand side in FP16 (packed sets)
  const auto ri = buf_half4(buf_rsrc(d.r, d.n * KB * 2),
                            (uint32_t)rs * (uint32_t)(KB * 2) + (uint32_t)(ch * 8));
  auto yo = buf_vec16<float, V>(buf_rsrc(d.yout, xb), oo);  // y_{k-1}
  const float cd = glob(d.cdinv)[rs];
  const float alpha = (float)*glob(&d.alpha[k]);
  const float bk = (float)*glob(&d.beta[k]);
  const RowSpan sp = row_span(live, row, d.a_rp, d.a_tp, tr ? kRangeT : kRangeW);
  const int32_t hs = tile_live ? glob(tr ? d.a_tp : d.a_rp)[row0] : 0;  // the tile's list
  const int H = tile_live ? glob(d.h_cnt)[tile] : 0;
  asm volatile("" ::: "memory");  // keeps the requests above ahead of the test
  if (*glob(d.done)) return;      // the same slot for the whole workgroup
  const BufRsrc rh = buf_rsrc(d.h_pk, d.nnz_ops * 4);
  const int32_t base = tr ? sp.ts : sp.ws;
  const int32_t mine = sp.len > e0 ? (sp.len - e0 + EPL - 1) / EPL : 0;  // this lane's entries
  uint32_t pv[UNR];
#pragma unroll
  for (int u = 0; u < UNR; ++u)
    pv[u] = (uint32_t)buf_i32(rh, u < mine ? (uint32_t)(base + u * EPL + e0) * 4u : kBufOut);
  // stage the halo: chunk c of halo row h at hl[(h NCH + c) V]
  const BufRsrc rl = buf_rsrc(d.h_list, d.nnz_ops * 4);
  for (int i0 = tid; i0 < H * NCH; i0 += NT * kHaloStage) {
    uint32_t col[kHaloStage];
#pragma unroll
    for (int j = 0; j < kHaloStage; ++j) {
      const int i = i0 + j * NT;
      col[j] = (uint32_t)buf_i32(rl, i < H * NCH ? (uint32_t)(hs + i / NCH) * 4u : kBufOut);
    }
    VecT<float, V> hv[kHaloStage];
#pragma unroll
    for (int j = 0; j < kHaloStage; ++j) {
      const int i = i0 + j * NT;
      hv[j] = buf_vec16<float, V>(
          rx, i < H * NCH ? col[j] * (uint32_t)(KB * 4) + (uint32_t)((i % NCH) * 16) : kBufOut);
    }
#pragma unroll
    for (int j = 0; j < kHaloStage; ++j) {
      const int i = i0 + j * NT;
      if (i < H * NCH) {
#pragma unroll
        for (int v = 0; v < V; ++v) hl[i * V + v] = hv[j].v[v];
      }
    }
  }
  __syncthreads();
  float yi[V], acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    yi[v] = own.v[v];
    acc[v] = 0.0f;
  }
  const float ct = (float)d.c_t;
  for (int32_t r = 0; r < mine; r += UNR) {
    if (r > 0) {
#pragma unroll
      for (int u = 0; u < UNR; ++u)
        pv[u] = (uint32_t)buf_i32(
            rh, r + u < mine ? (uint32_t)(base + (r + u) * EPL + e0) * 4u : kBufOut);
    }
    float cf[UNR];
    VecT<float, V> xj[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const float w = (float)__builtin_bit_cast(_Float16, (uint16_t)(pv[u] >> 16));
      cf[u] = tr ? ct * w : w;
      if (r + u < mine) {
        const float* src = hl + ((pv[u] & 0xffffu) * NCH + ch) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) xj[u].v[v] = src[v];
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) xj[u].v[v] = yi[v];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fmaT(cf[u], yi[v] - xj[u].v[v], acc[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    for (int o = NCH; o < G; o <<= 1) acc[v] += __shfl_xor(acc[v], o);
  if (!live || q >= NCH) return;
  const float sd = (float)d.s_diag;
  const float beta = bk * cd;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const float res = ri.v[v] - fmaT(sd, yi[v], acc[v]);
    yo.v[v] = yi[v] + fmaT(alpha, yi[v] - yo.v[v], beta * res);
  }
  stv<float, V>(d.yout + row * KB + q * V, yo);
}

template <int KB, int RANGE>
__global__ void __launch_bounds__((halo_threads<KB>())) k_sl_cheb_step1_halo(
    ChebView<float> d, int64_t nblocks, int k) {
  static_assert(RANGE == kRangeW || RANGE == kRangeT, "halos exist per entry range");
  extern __shared__ float4 halo_lds[];
  const int64_t b = xcd_block(nblocks);
  if (b >= nblocks) return;
  cheb_tile_halo<KB, RANGE>(d, b, threadIdx.x, k, reinterpret_cast<float*>(halo_lds));
}

// Work-list form over slots with halos (every slot of the set has them):
// a tile of kGatherRows rows is kGatherRows / kHaloRows halo tiles, each
// staged in its own part of the LDS (hstride floats each).  Equal bit for
// bit to k_sl_cheb_step.
template <int KB>
__global__ void __launch_bounds__((RowCfg<float, KB>::THREADS)) k_sl_cheb_step_halo(
    const SlotDev* __restrict__ sl, const Tile* __restrict__ tiles, int64_t ntiles, int k, int r,
    int yin, int yout, int hstride) {
  constexpr int NT = halo_threads<KB>();
  constexpr int PARTS = kGatherRows / kHaloRows;
  extern __shared__ float4 halo_lds[];
  const int64_t b = xcd_block(ntiles);
  if (b >= ntiles) return;
  const Tile t = tiles[b];
  const ChebView<float> d = cheb_view<float>(sl[t.slot], r, yin, yout);
  const int part = threadIdx.x / NT;
  cheb_tile_halo<KB, -1>(d, PARTS * (int64_t)t.blk + part, threadIdx.x % NT, k,
                         reinterpret_cast<float*>(halo_lds) + part * hstride);
}

// Dynamic LDS of the halo step (its largest list), or 0 when the slot has
// no halos or they would not fit.
constexpr int kHaloMaxLds = 32768;
template <int KB>
static int halo_lds_bytes(const ChebView<float>& v) {
  if (!v.h_cnt || (v.range != kRangeW && v.range != kRangeT)) return 0;
  const int64_t b = (int64_t)v.h_max * KB * 4;
  return b <= kHaloMaxLds ? (int)(b > 16 ? b : 16) : 0;
}

template <typename T>
void sl_cheb_first(const SlotDev* sl, const TileSet& ts, int r, int y, int yprev, hipStream_t s) {
  const Tile* tl = sizeof(T) == 8 ? ts.elem64 : ts.elem32;
  const int64_t nt = sizeof(T) == 8 ? ts.n_elem64 : ts.n_elem32;
  if (nt == 0) return;
  // packed FP32 sets read the right-hand side in FP16 (sl_to16_scaled)
  ME_DISPATCH_KB(ts.kb, {
    if (sizeof(T) == 4 && ts.pk)
      k_sl_cheb_first<T, KB, sizeof(T) == 4><<<nt, kBlock, 0, s>>>(sl, tl, r, y, yprev);
    else
      k_sl_cheb_first<T, KB, false><<<nt, kBlock, 0, s>>>(sl, tl, r, y, yprev);
  });
}
// The view of a slot from the host copy of its descriptor (device
// addresses of the same fields the device-side view reads).
template <typename T>
static ChebView<T> cheb_view_host(const SlotDev& d, int r, int yin, int yout) {
  ChebView<T> v;
  v.n = d.n;
  v.nnz_ops = d.nnz_ops;
  v.a_rp = d.a_rp;
  v.a_tp = d.a_tp;
  v.a_col = d.a_col;
  v.a_pk = d.a_pk;
  if constexpr (sizeof(T) == 8) {
    v.a_w = d.a_w;
    v.cdinv = d.cheb_dinv;
    v.yin = d.b64[yin];
    v.r = d.b64[r];
    v.yout = d.b64[yout];
  } else {
    v.a_w = d.a_w32;
    v.cdinv = d.cheb_dinv32;
    v.yin = d.b32[yin];
    v.r = d.b32[r];
    v.yout = d.b32[yout];
  }
  v.invt = d.invt;
  v.a_tq = d.a_tq;
  v.tq_base = d.tq_base;
  v.tq_ok = d.tq_ok;
  v.h_pk = d.h_pk;
  v.h_list = d.h_list;
  v.h_cnt = d.h_cnt;
  v.h_max = d.h_max;
  v.alpha = (const double*)((const char*)d.cheb + offsetof(ChebCoef, alpha));
  v.beta = (const double*)((const char*)d.cheb + offsetof(ChebCoef, beta));
  v.done = (const int*)((const char*)d.ctrl + offsetof(Ctrl, done));
  v.c_t = d.c_t;
  v.s_diag = d.cheb_s_diag;
  v.range = d.cheb_range;
  return v;
}

template <typename T, int KB, bool PK>
static void launch_cheb_step(const SlotDev* sl, const SlotDev* host_sl, const TileSet& ts, int k,
                             int r, int yin, int yout, int form, hipStream_t s) {
  const dim3 grid(xcd_grid(ts.n_gather)), blk(RowCfg<T, KB>::THREADS);
  if (ts.buf && ts.nslots == 1) {
    const ChebView<T> v = cheb_view_host<T>(host_sl[ts.ids[0]], r, yin, yout);
    const int64_t nb = (v.n + kStep1Rows - 1) / kStep1Rows;
    const dim3 g1(xcd_grid(nb)), b1(step1_threads<T, KB>());
    if constexpr (PK && sizeof(T) == 4) {
      const int lds = form == kFormGather ? 0 : halo_lds_bytes<KB>(v);
      if (lds > 0) {
        const int64_t nh = (v.n + kHaloRows - 1) / kHaloRows;
        const dim3 gh(xcd_grid(nh)), bh(halo_threads<KB>());
        if (v.range == kRangeW)
          k_sl_cheb_step1_halo<KB, kRangeW><<<gh, bh, lds, s>>>(v, nh, k);
        else
          k_sl_cheb_step1_halo<KB, kRangeT><<<gh, bh, lds, s>>>(v, nh, k);
        return;
      }
    }
    if (v.range == kRangeW)
      k_sl_cheb_step1<T, KB, kRangeW, PK><<<g1, b1, 0, s>>>(v, nb, k);
    else if (v.range == kRangeT)
      k_sl_cheb_step1<T, KB, kRangeT, PK><<<g1, b1, 0, s>>>(v, nb, k);
    else
      k_sl_cheb_step1<T, KB, kRangeAll, PK><<<g1, b1, 0, s>>>(v, nb, k);
  } else if (ts.buf) {
    if constexpr (PK && sizeof(T) == 4) {
      // halos when every slot of the set has them and two fit the LDS
      int64_t hmax = 0;
      bool all = true;
      for (int id : ts.ids) {
        const SlotDev& h = host_sl[id];
        all = all && h.h_cnt && (h.cheb_range == kRangeW || h.cheb_range == kRangeT);
        hmax = std::max<int64_t>(hmax, h.h_max);
      }
      const int64_t hstride = std::max<int64_t>(hmax, 1) * KB;  // floats per halo tile
      constexpr int parts = kGatherRows / kHaloRows;
      if (all && parts * hstride * 4 <= kHaloMaxLds) {
        k_sl_cheb_step_halo<KB><<<grid, blk, parts * hstride * 4, s>>>(
            sl, ts.gather, ts.n_gather, k, r, yin, yout, (int)hstride);
        return;
      }
    }
    k_sl_cheb_step<T, KB, true, PK><<<grid, blk, 0, s>>>(sl, ts.gather, ts.n_gather, k, r, yin,
                                                          yout);
  } else {
    k_sl_cheb_step<T, KB, false, PK><<<grid, blk, 0, s>>>(sl, ts.gather, ts.n_gather, k, r, yin,
                                                           yout);
  }
}

template <typename T>
void sl_cheb_step(const SlotDev* sl, const SlotDev* host_sl, const TileSet& ts, int k, int r,
                  int yin, int yout, hipStream_t s, int form) {
  if (ts.n_gather == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    static_assert(RowCfg<T, KB>::ROWS == kGatherRows, "gather tile rows");
    if constexpr (sizeof(T) == 4) {
      if (ts.pk) launch_cheb_step<T, KB, true>(sl, host_sl, ts, k, r, yin, yout, form, s);
      else launch_cheb_step<T, KB, false>(sl, host_sl, ts, k, r, yin, yout, form, s);
    } else {
      launch_cheb_step<T, KB, false>(sl, host_sl, ts, k, r, yin, yout, form, s);
    }
  });
}
// FP16 storage of the iterates (arithmetic in FP32), one slot, W entries
// only, packed entries: the input block is the FP32 residual scaled per
// column to unit norm, so the iterates sit well inside FP16's range; the
// column scale leaves the span of the preconditioned block unchanged.
struct ChebViewH {
  int64_t n, nnz_ops;
  const int32_t *a_rp, *a_tp;
  const uint32_t* a_pk;
  const float *cdinv, *r;
  const _Float16* yin;
  _Float16* yout;
  const double *alpha, *beta;
  const int* done;
  double s_diag;
};

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_cheb_first_h(const SlotDev* __restrict__ sl,
                                                            const Tile* __restrict__ tiles, int r,
                                                            int y, int yprev) {
  using E = ElemCfg<float, KB>;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (slot_done(d)) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / E::LPR;
  const int sub = threadIdx.x % E::LPR;
  if (row >= d.n) return;
  const float sc = (float)(1.0 / *glob(&d.cheb->theta)) * glob(d.cheb_dinv32)[row];
  const int64_t o = row * KB + sub * E::VEC;
  const auto v = ldv<float, E::VEC>(d.b32[r] + o);
  VecT<_Float16, E::VEC> h, z;
#pragma unroll
  for (int q = 0; q < E::VEC; ++q) {
    h.v[q] = (_Float16)(v.v[q] * sc);
    z.v[q] = (_Float16)0;
  }
  stv<_Float16, E::VEC>((_Float16*)d.b32[y] + o, h);
  stv<_Float16, E::VEC>((_Float16*)d.b32[yprev] + o, z);
}

template <int KB>
__global__ void __launch_bounds__((RowCfg<_Float16, KB>::THREADS)) k_sl_cheb_step_h(ChebViewH d,
                                                                                 int64_t ntiles,
                                                                                 int k) {
  using C = RowCfg<_Float16, KB>;
  constexpr int V = C::V16;
  const int64_t blk = xcd_block(ntiles);
  if (blk >= ntiles) return;
  const int64_t row = blk * kGatherRows + threadIdx.x / C::G;
  const int q = threadIdx.x % C::G;
  const bool live = row < d.n;
  const int ch = q % C::NCH;
  const int64_t rs = live ? row : 0;
  const uint32_t oh = (uint32_t)rs * (uint32_t)(KB * 2) + (uint32_t)(ch * 16);
  const uint32_t of = (uint32_t)rs * (uint32_t)(KB * 4) + (uint32_t)(ch * 32);
  const BufRsrc rx = buf_rsrc(d.yin, d.n * KB * 2);
  const BufRsrc rr = buf_rsrc(d.r, d.n * KB * 4);
  const auto own = buf_vec16<_Float16, V>(rx, oh);
  const auto r0 = buf_vec16<float, 4>(rr, of);
  const auto r1 = buf_vec16<float, 4>(rr, of + 16);
  const auto yo = buf_vec16<_Float16, V>(buf_rsrc(d.yout, d.n * KB * 2), oh);  // y_{k-1}
  const float cd = glob(d.cdinv)[rs];
  const float alpha = (float)*glob(&d.alpha[k]);
  const float bk = (float)*glob(&d.beta[k]);
  const RowSpan sp = row_span(live, row, d.a_rp, d.a_tp, kRangeW);
  asm volatile("" ::: "memory");  // keeps the requests above ahead of the test
  if (*glob(d.done)) return;
  float yi[V], acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) yi[v] = (float)own.v[v];
  spmm_span_pk_h<KB, kRangeW>(sp.ws, sp.nw, sp.ts, sp.len, q, rs, d.a_pk, d.nnz_ops, d.yin, d.n,
                              0.0f, yi, acc);
  if (!live || q >= C::NCH) return;
  const float beta = bk * cd, sd = (float)d.s_diag;
  VecT<_Float16, V> out;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const float ri = v < 4 ? r0.v[v] : r1.v[v - 4];
    const float res = ri - fmaT(sd, yi[v], acc[v]);
    out.v[v] = (_Float16)(yi[v] + fmaT(alpha, yi[v] - (float)yo.v[v], beta * res));
  }
  stv<_Float16, V>(d.yout + row * KB + q * V, out);
}

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_to64_h(const SlotDev* __restrict__ sl,
                                                      const Tile* __restrict__ tiles, int from,
                                                      int to) {
  using E = ElemCfg<float, KB>;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (slot_done(d)) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / E::LPR;
  const int sub = threadIdx.x % E::LPR;
  if (row >= d.n) return;
  const int64_t o = row * KB + sub * E::VEC;
  const auto h = ldv<_Float16, E::VEC>((const _Float16*)d.b32[from] + o);
#pragma unroll
  for (int p = 0; p < E::VEC / 2; ++p) {
    VecT<double, 2> v;
    v.v[0] = (double)h.v[2 * p];
    v.v[1] = (double)h.v[2 * p + 1];
    stv<double, 2>(d.b64[to] + o + 2 * p, v);
  }
}

bool sl_cheb_h_ok(const SlotDev* host_sl, const TileSet& ts) {
  return ts.buf && ts.pk && ts.nslots == 1 && (ts.kb == 8 || ts.kb == 16) &&
         host_sl[ts.ids[0]].cheb_range == kRangeW;
}

void sl_cheb_first_h(const SlotDev* sl, const TileSet& ts, int r, int y, int yprev,
                     hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, { k_sl_cheb_first_h<KB><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, r, y, yprev); });
}

void sl_cheb_step_h(const SlotDev* host_sl, const TileSet& ts, int k, int r, int yin, int yout,
                    hipStream_t s) {
  if (ts.n_gather == 0) return;
  const SlotDev& h = host_sl[ts.ids[0]];
  ChebViewH v;
  v.n = h.n;
  v.nnz_ops = h.nnz_ops;
  v.a_rp = h.a_rp;
  v.a_tp = h.a_tp;
  v.a_pk = h.a_pk;
  v.cdinv = h.cheb_dinv32;
  v.r = h.b32[r];
  v.yin = (const _Float16*)h.b32[yin];
  v.yout = (_Float16*)h.b32[yout];
  v.alpha = (const double*)((const char*)h.cheb + offsetof(ChebCoef, alpha));
  v.beta = (const double*)((const char*)h.cheb + offsetof(ChebCoef, beta));
  v.done = (const int*)((const char*)h.ctrl + offsetof(Ctrl, done));
  v.s_diag = h.cheb_s_diag;
  const dim3 grid(xcd_grid(ts.n_gather));
  if (ts.kb == 8) {
    static_assert(RowCfg<_Float16, 8>::ROWS == kGatherRows, "gather tile rows");
    k_sl_cheb_step_h<8><<<grid, RowCfg<_Float16, 8>::THREADS, 0, s>>>(v, ts.n_gather, k);
  } else if (ts.kb == 16) {
    k_sl_cheb_step_h<16><<<grid, RowCfg<_Float16, 16>::THREADS, 0, s>>>(v, ts.n_gather, k);
  } else {
    abort();
  }
}

void sl_to64_h(const SlotDev* sl, const TileSet& ts, int from, int to, hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, { k_sl_to64_h<KB><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, from, to); });
}

template void sl_cheb_first<double>(const SlotDev*, const TileSet&, int, int, int, hipStream_t);
template void sl_cheb_first<float>(const SlotDev*, const TileSet&, int, int, int, hipStream_t);
template void sl_cheb_step<double>(const SlotDev*, const SlotDev*, const TileSet&, int, int,
                                   int, int, hipStream_t, int);
template void sl_cheb_step<float>(const SlotDev*, const SlotDev*, const TileSet&, int, int, int,
                                  int, hipStream_t, int);

// ---------------------------------------------------------------------------
// Residual R = AX - B X Lambda; W = R or D^-1 R (Jacobi); per tile: column
// sums of |r|^2, |B x|^2 and x^T D x with D the diagonal of the operator the
// Chebyshev preconditioner inverts (3 KB partials).
// ---------------------------------------------------------------------------

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_resid(const SlotDev* __restrict__ sl,
                                                     const Tile* __restrict__ tiles, int wblk,
                                                     int jacobi, int cert) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR, NE = 3 * KB;
  __shared__ double sh[kBlock / kWave][NE];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert)) return;
  const int tid = threadIdx.x, sub = tid % LPR;
  const int64_t r0 = (int64_t)t.blk * d.per;
  const int64_t r1 = r0 + d.per < d.n ? r0 + d.per : d.n;
  const double* x = d.b64[BX];
  const double* ax = d.b64[BAX];
  double* w = wblk >= 0 ? d.b64[wblk] : nullptr;
  double r2[VEC], b2[VEC], xd[VEC], lm[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    r2[v] = b2[v] = xd[v] = 0.0;
    lm[v] = d.lam[sub * VEC + v];
  }
  for (int64_t row = r0 + tid / LPR; row < r1; row += E::RB) {
    const int64_t o = row * KB + sub * VEC;
    const auto xi = ldv<double, VEC>(x + o);
    const auto ai = ldv<double, VEC>(ax + o);
    const double bi = d.bdiag ? d.bdiag[row] : 1.0;
    const double di = jacobi ? d.dinv[row] : 1.0;
    const double rdv = 1.0 / d.cheb_dinv[row];
    VecT<double, VEC> wv;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const double bx = bi * xi.v[v];
      const double r = ai.v[v] - lm[v] * bx;
      r2[v] += r * r;
      b2[v] += bx * bx;
      xd[v] += xi.v[v] * xi.v[v] * rdv;
      wv.v[v] = di * r;
    }
    if (w) stv<double, VEC>(w + o, wv);
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    for (int off = kWave / 2; off >= LPR; off >>= 1) {
      r2[v] += __shfl_xor(r2[v], off);
      b2[v] += __shfl_xor(b2[v], off);
      xd[v] += __shfl_xor(xd[v], off);
    }
  }
  const int lane = tid % kWave, wv_ = tid / kWave;
  if (lane < LPR) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      sh[wv_][lane * VEC + v] = r2[v];
      sh[wv_][KB + lane * VEC + v] = b2[v];
      sh[wv_][2 * KB + lane * VEC + v] = xd[v];
    }
  }
  __syncthreads();
  if (tid < NE) {
    double acc = 0;
    for (int q = 0; q < kBlock / kWave; ++q) acc += sh[q][tid];
    d.partials[(int64_t)t.blk * NE + tid] = acc;
  }
}

void sl_resid(const SlotDev* sl, const TileSet& ts, int w, int jacobi, int cert, hipStream_t s) {
  if (ts.n_red == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_resid<KB><<<ts.n_red, kBlock, 0, s>>>(sl, ts.red, w, jacobi, cert);
  });
}

// rho_j = |r_j| / (|lambda_j| |B x_j|), with |lambda_j| replaced by the
// operator scale when it is below the zero threshold; convergence
// bookkeeping; Chebyshev interval and coefficients for this iteration.
// One wave per slot: lane l sums tiles l, l + 64, ...; then a fixed xor tree.
template <int KB>
__global__ void __launch_bounds__(kWave) k_sl_resid_finalize(const SlotDev* __restrict__ sl,
                                                             const int32_t* __restrict__ slots,
                                                             int final_pass) {
  constexpr int NE = 3 * KB;
  __shared__ double tot[NE];
  const SlotDev& d = sl[slots[blockIdx.x]];
  Ctrl* ctrl = d.ctrl;
  if (!final_pass && ctrl->done) return;
  const int lane = threadIdx.x;
  double acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) acc[e] = 0.0;
  for (int p = lane; p < d.nparts; p += kWave) {
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] += d.partials[(int64_t)p * NE + e];
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    double v = acc[e];
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) tot[e] = v;
  }
  __syncthreads();
  const double* lam = d.lam;
  int conv = 0, bad = 0;
  double worst = 0.0;  // largest residual of the required columns
  if (lane < KB) {
    const double al = fabs(lam[lane]);
    const double den = (al >= ctrl->lam_floor ? al : ctrl->lam_scale) * sqrt(tot[KB + lane]);
    const double rho = sqrt(tot[lane]) / den;
    ctrl->rho[lane] = rho;
    ctrl->rinv[lane] = tot[lane] > 0.0 ? 1.0 / sqrt(tot[lane]) : 0.0;
    if (final_pass) ctrl->lam[lane] = lam[lane];
    conv = (lane < ctrl->need) && (rho <= ctrl->tol);
    if (lane < ctrl->need) worst = rho;
    bad = !isfinite(rho);
  }
  const int nc = __popcll(__ballot(conv));
  const int nb = __popcll(__ballot(bad));
  for (int o = kWave / 2; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o));
  if (lane == 0) {
    ctrl->nconv = nc;
    if (nb) ctrl->nonfinite = 1;
    if (!final_pass) {
      ctrl->rho_hist[ctrl->iter % kRhoHist] = worst;
      if (nc >= ctrl->need || nb || ctrl->iter >= ctrl->max_iter) ctrl->done = 1;
      else ctrl->iter += 1;
    }
  }
  const int deg = ctrl->cheb_deg;
  if (final_pass || deg < 2) return;
  // [a, b]: a = afac * (x_j^T A x_j) / (x_j^T D x_j) with x_j^T B x_j = 1,
  // j the leading Ritz pair with a nonzero value (the eps = 0 case has
  // lambda_1 = 0)
  const double b = ctrl->cheb_b;
  double a = -1.0;
  for (int j = 0; j < KB; ++j) {
    if (fabs(lam[j]) >= ctrl->lam_floor) {
      a = ctrl->cheb_afac * fabs(lam[j]) / tot[2 * KB + j];
      break;
    }
  }
  if (!(a > 0.0) || !isfinite(a)) a = 1e-3 * b;
  a = fmin(fmax(a, 1e-9 * b), 0.5 * b);
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
  const double phi = acosh(theta / delta);
  // rho_k = T_k(sigma) / T_{k+1}(sigma) = cosh(k phi) / cosh((k+1) phi),
  // written with decaying exponentials so that no cosh overflows
  const double e1 = exp(-phi);
  ChebCoef* cc = d.cheb;
  for (int k = lane + 1; k < deg; k += kWave) {
    const double rk = e1 * (1.0 + exp(-2.0 * k * phi)) / (1.0 + exp(-2.0 * (k + 1) * phi));
    const double rkm = e1 * (1.0 + exp(-2.0 * (k - 1) * phi)) / (1.0 + exp(-2.0 * k * phi));
    cc->alpha[k] = rk * rkm;
    cc->beta[k] = 2.0 * rk / delta;
  }
  if (lane == 0) {
    cc->a = a;
    cc->theta = theta;
  }
}

void sl_resid_finalize(const SlotDev* sl, const TileSet& ts, int final_pass, hipStream_t s) {
  if (ts.nslots == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_resid_finalize<KB><<<ts.nslots, kWave, 0, s>>>(sl, ts.slots, final_pass);
  });
}

// ---------------------------------------------------------------------------
// Tall-skinny Gram products on MFMA (FP64):
//   G1 = U^T diag(b) V ((nu KB) x (nv KB)),  G2 = U^T V2 ((nu KB) x (nv2 KB))
// per reduction tile of a slot.  Each 16x16x4 step consumes 4 rows; lane l
// supplies U[row + l/16][16a + l%16] (A operand) and V[row + l/16][16b + l%16]
// (B operand).  Tiles write partial Grams; sl_reduce sums them in tile order.
// ---------------------------------------------------------------------------

struct Ids {
  int v[3];
};

// Grams of one reduction tile, G1 = U^T diag(b) V and G2 = U^T V2, where V's
// blocks are blocks of U (vsel[i] = position in U of V's block i).  Each wave
// takes 16-row chunks (rows r0 + 16 wave, + 16 NW, ...): it stages the chunk
// of every U and V2 block in its own LDS area (a 16-row chunk of a row-major
// n x KB block is 16 KB contiguous doubles: one contiguous load per block),
// requests the next chunk into registers, and feeds the FP64 MFMA 16x16x4
// from LDS while those loads are in flight.  SYM (V = U, V2 = A U: both Grams
// symmetric) computes only the 16x16 tiles on and above the diagonal and
// mirrors them, so both triangles of an off-diagonal tile hold the same sums.
// The waves' sums are added in wave order in LDS and written as the tile's
// partial.
template <int KB, int NU, int NV, int NV2, int NTH>
struct GramCfg {
  static constexpr int MU = NU * KB, MV = NV * KB, MV2 = NV2 * KB;
  static constexpr int TU = (MU + 15) / 16, TV = (MV + 15) / 16, TV2 = (MV2 + 15) / 16;
  static constexpr int E1 = MU * MV, E2 = MU * MV2;
  static constexpr int NB = NU + NV2;         // staged blocks
  static constexpr int LD = NB * KB + 1;      // LDS row stride (doubles)
  static constexpr int NW = NTH / kWave;
  static constexpr int WAVE_LDS = 16 * LD + 16;  // chunk + row weights
  static constexpr int LDS = NW * WAVE_LDS > E1 + E2 ? NW * WAVE_LDS : E1 + E2;
  static constexpr int EPL = KB / 4;          // doubles per lane when staging
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KB, int NU, int NV, int NV2, bool SYM, int NTH>
__global__ void __launch_bounds__(NTH) k_sl_gram(const SlotDev* __restrict__ sl,
                                                 const Tile* __restrict__ tiles, Ids u, Ids vsel,
                                                 Ids v2, int use_b, int cert) {
  using C = GramCfg<KB, NU, NV, NV2, NTH>;
  constexpr int MU = C::MU, MV = C::MV, MV2 = C::MV2, TU = C::TU, TV = C::TV, TV2 = C::TV2;
  constexpr int E1 = C::E1, E2 = C::E2, LD = C::LD, NW = C::NW, EPL = C::EPL, NB = C::NB;
  static_assert(!SYM || (NU == NV && (NV2 == 0 || NV2 == NU)), "symmetric Grams are square");
  using Acc = typename Mfma<double>::Acc;
  __shared__ double lds[C::LDS];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert)) return;
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
  const int64_t r0 = (int64_t)t.blk * d.per;
  const int64_t r1 = r0 + d.per < d.n ? r0 + d.per : d.n;
  const double* wd = use_b ? d.bdiag : nullptr;
  const double* bp[NB];
#pragma unroll
  for (int i = 0; i < NU; ++i) bp[i] = d.b64[u.v[i]];
#pragma unroll
  for (int i = 0; i < NV2; ++i) bp[NU + i] = d.b64[v2.v[i]];
  // LDS column of V's column j (V's block j / KB is U's block vsel)
  int vcol[TV > 0 ? TV : 1];
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int b = 0; b < TV; ++b) {
    const int j = 16 * b + li;
    vcol[b] = j < MV ? vsel.v[j / KB] * KB + j % KB : -1;
  }
  double* st = lds + wave * C::WAVE_LDS;
  const int se = lane * EPL, sr = se / KB, sc = se % KB;  // staging: row, column
  // one chunk's share of this lane: EPL doubles of each block, a row weight
  VecT<double, EPL> nx[NB];
  double nwt = 0.0;
  auto fetch = [&](int64_t base) {
    const bool ok = base + sr < r1;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      if (ok) {
        nx[bi] = ldv<double, EPL>(bp[bi] + (base + sr) * KB + sc);
      } else {
#pragma unroll
        for (int q = 0; q < EPL; ++q) nx[bi].v[q] = 0.0;
      }
    }
    if (lane < 16) nwt = (base + lane < r1) ? (wd ? glob(wd)[base + lane] : 1.0) : 0.0;
  };
  int64_t base = r0 + 16 * wave;
  if (base < r1) fetch(base);
  for (; base < r1; base += 16 * NW) {
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int q = 0; q < EPL; ++q) st[sr * LD + bi * KB + sc + q] = nx[bi].v[q];
    }
    if (lane < 16) st[16 * LD + lane] = nwt;
    if (base + 16 * NW < r1) fetch(base + 16 * NW);  // in flight during the MFMAs
    wave_lds_sync();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int row = 4 * ks + lk;
      const double* sr_p = st + row * LD;
      double ua[TU], vb[TV > 0 ? TV : 1], v2b[TV2 > 0 ? TV2 : 1];
#pragma unroll
      for (int a = 0; a < TU; ++a) ua[a] = 16 * a + li < MU ? sr_p[16 * a + li] : 0.0;
      const double wr = TV > 0 ? st[16 * LD + row] : 0.0;
#pragma unroll
      for (int b = 0; b < TV; ++b) vb[b] = vcol[b] >= 0 ? wr * sr_p[vcol[b]] : 0.0;
#pragma unroll
      for (int b = 0; b < TV2; ++b)
        v2b[b] = 16 * b + li < MV2 ? sr_p[NU * KB + 16 * b + li] : 0.0;
#pragma unroll
      for (int a = 0; a < TU; ++a) {
#pragma unroll
        for (int b = 0; b < TV; ++b)
          if (!SYM || b >= a) acc1[a][b] = Mfma<double>::step(ua[a], vb[b], acc1[a][b]);
#pragma unroll
        for (int b = 0; b < TV2; ++b)
          if (!SYM || b >= a) acc2[a][b] = Mfma<double>::step(ua[a], v2b[b], acc2[a][b]);
      }
    }
    wave_lds_sync();  // the chunk is read before the next one overwrites it
  }
  __syncthreads();  // staging areas are reused for the sums
  double* sh = lds;
  for (int wv = 0; wv < NW; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int a = 0; a < TU; ++a) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * a + Mfma<double>::row(lk, q);
          if (i >= MU) continue;
#pragma unroll
          for (int b = 0; b < TV; ++b) {
            if (SYM && b < a) continue;
            const int j = 16 * b + li;
            if (j < MV) {
              const double val = acc1[a][b][q];
              if (wv == 0) sh[i * MV + j] = val; else sh[i * MV + j] += val;
              if (SYM && b > a) {
                if (wv == 0) sh[j * MV + i] = val; else sh[j * MV + i] += val;
              }
            }
          }
#pragma unroll
          for (int b = 0; b < TV2; ++b) {
            if (SYM && b < a) continue;
            const int j = 16 * b + li;
            if (j < MV2) {
              const double val = acc2[a][b][q];
              if (wv == 0) sh[E1 + i * MV2 + j] = val; else sh[E1 + i * MV2 + j] += val;
              if (SYM && b > a) {
                if (wv == 0) sh[E1 + j * MV2 + i] = val; else sh[E1 + j * MV2 + i] += val;
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
  double* out = d.partials + (int64_t)t.blk * (E1 + E2);
  for (int e = tid; e < E1 + E2; e += NTH) out[e] = sh[e];
}

void sl_gram(const SlotDev* sl, const TileSet& ts, int nu, const int* u, int nv, const int* v,
             int nv2, const int* v2, int use_b, int cert, hipStream_t s) {
  if (ts.n_red == 0) return;
  Ids iu{{0, 0, 0}}, iv{{0, 0, 0}}, iv2{{0, 0, 0}};
  for (int i = 0; i < nu; ++i) iu.v[i] = u[i];
  // V's blocks are blocks of U: pass their positions in U
  bool same = nv == nu;
  for (int i = 0; i < nv; ++i) {
    iv.v[i] = -1;
    for (int j = 0; j < nu; ++j)
      if (u[j] == v[i]) iv.v[i] = j;
    if (iv.v[i] < 0) std::abort();  // no caller asks for a V outside U
    same = same && iv.v[i] == i;
  }
  for (int i = 0; i < nv2; ++i) iv2.v[i] = v2[i];
  // tiles of tall slots in 8 waves (one wave per 16-row chunk column of
  // the tile), the others in 4; a slot's tiles always run in the same form
  const int64_t nb = ts.n_red_big, ns = ts.n_red - ts.n_red_big;
#define ME_SL_GRAM(NU_, NV_, NV2_, SYM_)                                                    \
  if (nu == NU_ && nv == NV_ && nv2 == NV2_ && (!(SYM_) || same)) {                          \
    ME_DISPATCH_KB(ts.kb, {                                                                  \
      if (nb > 0)                                                                            \
        k_sl_gram<KB, NU_, NV_, NV2_, SYM_, 512><<<nb, 512, 0, s>>>(sl, ts.red, iu, iv, iv2, \
                                                                    use_b, cert);           \
      if (ns > 0)                                                                            \
        k_sl_gram<KB, NU_, NV_, NV2_, SYM_, 256><<<ns, 256, 0, s>>>(sl, ts.red + nb, iu, iv, \
                                                                    iv2, use_b, cert);      \
    });                                                                                      \
    return;                                                                                  \
  }
  // symmetric pairs: U^T B U with U^T (A U) (each call passes V2 = A U)
  ME_SL_GRAM(3, 3, 3, true)   // [X W P] pair
  ME_SL_GRAM(1, 1, 1, true)   // X^T B X, X^T AX
  ME_SL_GRAM(1, 1, 0, true)   // X^T B X
  ME_SL_GRAM(2, 1, 0, false)  // [X W]^T B W
#undef ME_SL_GRAM
  std::abort();  // no other shape is requested
}

// out[e] = sum_p partials[p][e], p ascending, per slot (target 0: gram,
// 1: sums, only for slots that deflate).
__global__ void __launch_bounds__(kBlock) k_sl_reduce(const SlotDev* __restrict__ sl,
                                                      const int32_t* __restrict__ slots, int nent,
                                                      int target, int cert) {
  __shared__ double sh[8][33];
  const SlotDev& d = sl[slots[blockIdx.y]];
  if (skip_slot(d, cert)) return;
  if (target == 1 && !d.deflate) return;
  const int el = threadIdx.x % 32, pl = threadIdx.x / 32;
  const int e = blockIdx.x * 32 + el;
  double s = 0;
  if (e < nent) {
    for (int p = pl; p < d.nparts; p += 8) s += d.partials[(int64_t)p * nent + e];
  }
  sh[pl][el] = s;
  __syncthreads();
  if (pl == 0 && e < nent) {
    double t = 0;
    for (int q = 0; q < 8; ++q) t += sh[q][el];
    (target == 0 ? d.gram : d.sums)[e] = t;
  }
}

void sl_reduce(const SlotDev* sl, const TileSet& ts, int nent, int cert, hipStream_t s) {
  if (ts.nslots == 0) return;
  k_sl_reduce<<<dim3(ceil_div(nent, 32), ts.nslots), kBlock, 0, s>>>(sl, ts.slots, nent, 0, cert);
}

// ---------------------------------------------------------------------------
// Block combination: out_o = sum_s in_s C_o.  Each tile stages its rows in
// LDS (coalesced), then every lane forms VEC output columns.  Outputs may
// alias inputs: a tile reads all of its rows before writing any.
// ---------------------------------------------------------------------------

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_combine(const SlotDev* __restrict__ sl,
                                                       const Tile* __restrict__ tiles, int nin,
                                                       int ngroup, Ids in0, Ids in1, int nout,
                                                       Ids out0, Ids out1, int which, int off,
                                                       int cert) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR, RB = E::RB;
  __shared__ double rows[2][RB][3 * KB + 1];
  __shared__ double cf[2][3 * KB][KB];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert)) return;
  const int tid = threadIdx.x;
  const int m = nin * KB;
  const double* coef = (which == 0 ? d.coef : d.coefw) + off;
  for (int u = tid; u < nout * m * KB; u += kBlock) {
    const int o = u / (m * KB), rem = u % (m * KB);
    cf[o][rem / KB][rem % KB] = coef[u];
  }
  const int rloc = tid / LPR, sub = tid % LPR;
  const int64_t row = (int64_t)t.blk * RB + rloc;
  if (row < d.n) {
    for (int g = 0; g < ngroup; ++g) {
      const Ids& in = g == 0 ? in0 : in1;
      for (int sidx = 0; sidx < nin; ++sidx) {
        const auto v = ldv<double, VEC>(d.b64[in.v[sidx]] + row * KB + sub * VEC);
#pragma unroll
        for (int q = 0; q < VEC; ++q) rows[g][rloc][sidx * KB + sub * VEC + q] = v.v[q];
      }
    }
  }
  __syncthreads();
  if (row >= d.n) return;
  for (int g = 0; g < ngroup; ++g) {
    const Ids& out = g == 0 ? out0 : out1;
    for (int o = 0; o < nout; ++o) {
      double acc[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] = 0;
      for (int k = 0; k < m; ++k) {
        const double a = rows[g][rloc][k];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] += a * cf[o][k][sub * VEC + q];
      }
      VecT<double, VEC> ov;
#pragma unroll
      for (int q = 0; q < VEC; ++q) ov.v[q] = acc[q];
      stv<double, VEC>(d.b64[out.v[o]] + row * KB + sub * VEC, ov);
    }
  }
}

void sl_combine(const SlotDev* sl, const TileSet& ts, int nin, int ngroup, const int* in0,
                const int* in1, int nout, const int* out0, const int* out1, int which, int off,
                int cert, hipStream_t s) {
  if (ts.n_elem64 == 0) return;
  Ids a{{0, 0, 0}}, b{{0, 0, 0}}, c{{0, 0, 0}}, e{{0, 0, 0}};
  for (int i = 0; i < nin; ++i) {
    a.v[i] = in0[i];
    if (ngroup > 1) b.v[i] = in1[i];
  }
  for (int i = 0; i < nout; ++i) {
    c.v[i] = out0[i];
    if (ngroup > 1) e.v[i] = out1[i];
  }
  ME_DISPATCH_KB(ts.kb, {
    k_sl_combine<KB><<<ts.n_elem64, kBlock, 0, s>>>(sl, ts.elem64, nin, ngroup, a, b, nout, c, e,
                                                    which, off, cert);
  });
}

// ---------------------------------------------------------------------------
// Deflation of the constant vector (slots with `deflate`): x <- x - mean(x)
// per column.
// ---------------------------------------------------------------------------

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_colsum(const SlotDev* __restrict__ sl,
                                                      const Tile* __restrict__ tiles, int blk,
                                                      int cert) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  __shared__ double sh[kBlock / kWave][KB];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert) || !d.deflate) return;
  const int tid = threadIdx.x, sub = tid % LPR;
  const int64_t r0 = (int64_t)t.blk * d.per;
  const int64_t r1 = r0 + d.per < d.n ? r0 + d.per : d.n;
  const double* x = d.b64[blk];
  double acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  for (int64_t row = r0 + tid / LPR; row < r1; row += E::RB) {
    const auto xv = ldv<double, VEC>(x + row * KB + sub * VEC);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += xv.v[v];
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
    d.partials[(int64_t)t.blk * KB + tid] = s;
  }
}

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_sub_mean(const SlotDev* __restrict__ sl,
                                                        const Tile* __restrict__ tiles, int blk,
                                                        int cert) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (skip_slot(d, cert) || !d.deflate) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (row >= d.n) return;
  double* p = d.b64[blk] + row * KB + sub * VEC;
  auto xv = ldv<double, VEC>(p);
#pragma unroll
  for (int v = 0; v < VEC; ++v) xv.v[v] -= d.sums[sub * VEC + v] / (double)d.n;
  stv<double, VEC>(p, xv);
}

void sl_deflate(const SlotDev* sl, const TileSet& ts, int blk, int cert, hipStream_t s) {
  if (ts.n_red == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_colsum<KB><<<ts.n_red, kBlock, 0, s>>>(sl, ts.red, blk, cert);
    k_sl_reduce<<<dim3(1, ts.nslots), kBlock, 0, s>>>(sl, ts.slots, KB, 1, cert);
    k_sl_sub_mean<KB><<<ts.n_elem64, kBlock, 0, s>>>(sl, ts.elem64, blk, cert);
  });
}

// ---------------------------------------------------------------------------
// FP64 <-> FP32 copies of a block (mixed-precision preconditioner)
// ---------------------------------------------------------------------------

template <int KB, bool TO32, bool SC = false>
__global__ void __launch_bounds__(kBlock) k_sl_convert(const SlotDev* __restrict__ sl,
                                                       const Tile* __restrict__ tiles, int b64,
                                                       int b32) {
  using E = ElemCfg<float, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (slot_done(d)) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (row >= d.n) return;
  const int64_t o = row * KB + sub * VEC;
  double* p64 = d.b64[b64] + o;
  float* p32 = d.b32[b32] + o;
  if (TO32) {
    VecT<float, VEC> f;
#pragma unroll
    for (int h = 0; h < VEC / 2; ++h) {
      const auto v = ldv<double, 2>(p64 + 2 * h);
      if constexpr (SC) {  // columns scaled by 1 / |r_j|
        const double* ri = d.ctrl->rinv + sub * VEC + 2 * h;
        f.v[2 * h] = (float)(v.v[0] * glob(ri)[0]);
        f.v[2 * h + 1] = (float)(v.v[1] * glob(ri)[1]);
      } else {
        f.v[2 * h] = (float)v.v[0];
        f.v[2 * h + 1] = (float)v.v[1];
      }
    }
    stv<float, VEC>(p32, f);
  } else {
    const auto f = ldv<float, VEC>(p32);
#pragma unroll
    for (int h = 0; h < VEC / 2; ++h) {
      VecT<double, 2> v;
      v.v[0] = (double)f.v[2 * h];
      v.v[1] = (double)f.v[2 * h + 1];
      stv<double, 2>(p64 + 2 * h, v);
    }
  }
}

void sl_to32(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_convert<KB, true><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, from64, to32);
  });
}
void sl_to32_scaled(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_convert<KB, true, true><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, from64, to32);
  });
}
// R (FP64) to FP16 in the FP32 block's memory, each column scaled by
// 1 / |r_j| from the residual pass (unit columns: FP16's range; the scale
// leaves the span of the preconditioned block unchanged).
template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_to16_scaled(const SlotDev* __restrict__ sl,
                                                           const Tile* __restrict__ tiles, int b64,
                                                           int b32) {
  using E = ElemCfg<float, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  if (slot_done(d)) return;
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (row >= d.n) return;
  const int64_t o = row * KB + sub * VEC;
  const double* p64 = d.b64[b64] + o;
  const double* ri = d.ctrl->rinv + sub * VEC;
  VecT<_Float16, VEC> h;
#pragma unroll
  for (int q = 0; q < VEC; q += 2) {
    const auto v = ldv<double, 2>(p64 + q);
    h.v[q] = (_Float16)(float)(v.v[0] * glob(ri)[q]);
    h.v[q + 1] = (_Float16)(float)(v.v[1] * glob(ri)[q + 1]);
  }
  stv<_Float16, VEC>(reinterpret_cast<_Float16*>(d.b32[b32]) + o, h);
}
void sl_to16_scaled(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_to16_scaled<KB><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, from64, to32);
  });
}

void sl_to64(const SlotDev* sl, const TileSet& ts, int from32, int to64, hipStream_t s) {
  if (ts.n_elem32 == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_convert<KB, false><<<ts.n_elem32, kBlock, 0, s>>>(sl, ts.elem32, to64, from32);
  });
}

// ---------------------------------------------------------------------------
// Starting block: copies x0 (user order, n x kcopy) and fills the remaining
// columns with a counter-based generator (SplitMix64 of seed and element
// index, Steele, Lea & Flood 2014), uniform in [-1, 1), or -- smooth start
// -- with cos(pi f t) of the row's breadth-first depth t in (0, 1) plus a
// tenth of that random value: on a manifold graph the depth from a
// peripheral node is a coordinate along the manifold, and these cosines
// approximate its lowest eigenvectors along that direction.
// ---------------------------------------------------------------------------

__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_fill_start(const SlotDev* __restrict__ sl,
                                                          const Tile* __restrict__ tiles) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (row >= d.n) return;
  const int64_t u = d.perm ? d.perm[row] : row;
  VecT<double, VEC> v;
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const int j = sub * VEC + q;
    if (d.x0 && j < d.kcopy) {
      v.v[q] = d.x0[u * d.kcopy + j];
    } else {
      const uint64_t h = splitmix64(d.seed * 0x2545F4914F6CDD1Dull + (uint64_t)(u * KB + j));
      const double rnd = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
      if (d.lev && j < d.nsmooth) {
        const double t = ((double)d.lev[row] + 0.5) / ((double)d.max_lev + 1.0);
        v.v[q] = cos(3.141592653589793 * (double)(j + d.jfreq) * t) + 0.1 * rnd;
      } else {
        v.v[q] = rnd;
      }
    }
  }
  stv<double, VEC>(d.b64[BX] + row * KB + sub * VEC, v);
}

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_zero(const SlotDev* __restrict__ sl,
                                                    const Tile* __restrict__ tiles, int blk) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  const int64_t row = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (row >= d.n) return;
  VecT<double, VEC> v;
#pragma unroll
  for (int q = 0; q < VEC; ++q) v.v[q] = 0.0;
  stv<double, VEC>(d.b64[blk] + row * KB + sub * VEC, v);
}

void sl_fill_start(const SlotDev* sl, const TileSet& ts, hipStream_t s) {
  if (ts.n_elem64 == 0) return;
  ME_DISPATCH_KB(ts.kb, { k_sl_fill_start<KB><<<ts.n_elem64, kBlock, 0, s>>>(sl, ts.elem64); });
}
void sl_zero(const SlotDev* sl, const TileSet& ts, int blk, hipStream_t s) {
  if (ts.n_elem64 == 0) return;
  ME_DISPATCH_KB(ts.kb, { k_sl_zero<KB><<<ts.n_elem64, kBlock, 0, s>>>(sl, ts.elem64, blk); });
}

// ---------------------------------------------------------------------------
// Per-slot bookkeeping
// ---------------------------------------------------------------------------

// ctrl->orth = max |G_ij - delta_ij| over i, j < need, G = X^T B X (gram)
__global__ void __launch_bounds__(kWave) k_sl_orth(const SlotDev* __restrict__ sl,
                                                   const int32_t* __restrict__ slots, int kb) {
  const SlotDev& d = sl[slots[blockIdx.x]];
  const int need = d.need;
  double e = 0.0;
  for (int u = threadIdx.x; u < need * need; u += kWave) {
    const int i = u / need, j = u % need;
    e = fmax(e, fabs(d.gram[i * kb + j] - (i == j ? 1.0 : 0.0)));
  }
  for (int o = kWave / 2; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o));
  if (threadIdx.x == 0) d.ctrl->orth = e;
}

void sl_orth(const SlotDev* sl, const TileSet& ts, hipStream_t s) {
  if (ts.nslots == 0) return;
  k_sl_orth<<<ts.nslots, kWave, 0, s>>>(sl, ts.slots, ts.kb);
}

__global__ void k_sl_reenter(const SlotDev* __restrict__ sl, const int32_t* __restrict__ slots) {
  if (threadIdx.x == 0) sl[slots[blockIdx.x]].ctrl->done = 0;
}

void sl_reenter(const SlotDev* sl, const TileSet& ts, hipStream_t s) {
  if (ts.nslots == 0) return;
  k_sl_reenter<<<ts.nslots, kWave, 0, s>>>(sl, ts.slots);
}

// Output: sign convention (largest |x| of each column positive, lowest user
// row on ties) and the copy of the first k_out columns in user order.
template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_col_argmax(const SlotDev* __restrict__ sl,
                                                          const Tile* __restrict__ tiles) {
  __shared__ double sv[kBlock];
  __shared__ int64_t si[kBlock];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  const int64_t r0 = (int64_t)t.blk * d.per;
  const int64_t r1 = r0 + d.per < d.n ? r0 + d.per : d.n;
  const double* x = d.b64[BX];
  double* pval = d.scratch;
  int64_t* pidx = reinterpret_cast<int64_t*>(d.scratch + (int64_t)d.nparts * KB);
  for (int j = 0; j < KB; ++j) {
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
      const double a = fabs(x[i * KB + j]);
      const int64_t u = d.perm ? d.perm[i] : i;
      if (a > best || (a == best && u < bi)) {
        best = a;
        bi = u;
      }
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
      pval[(int64_t)t.blk * KB + j] = sv[0];
      pidx[(int64_t)t.blk * KB + j] = si[0];
    }
    __syncthreads();
  }
}

template <int KB>
__global__ void __launch_bounds__(kBlock) k_sl_signed_copy(const SlotDev* __restrict__ sl,
                                                           const Tile* __restrict__ tiles) {
  using E = ElemCfg<double, KB>;
  constexpr int VEC = E::VEC, LPR = E::LPR;
  __shared__ double sgn[KB];
  const Tile t = tiles[blockIdx.x];
  const SlotDev& d = sl[t.slot];
  const double* x = d.b64[BX];
  if (threadIdx.x < KB) {
    const int j = threadIdx.x;
    const double* pval = d.scratch;
    const int64_t* pidx = reinterpret_cast<const int64_t*>(d.scratch + (int64_t)d.nparts * KB);
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int p = 0; p < d.nparts; ++p) {
      const double v = pval[p * KB + j];
      const int64_t ii = pidx[p * KB + j];
      if (v > best || (v == best && ii < bi)) {
        best = v;
        bi = ii;
      }
    }
    double val = 1.0;
    if (bi < d.n) val = x[(d.iperm ? (int64_t)d.iperm[bi] : bi) * KB + j];
    sgn[j] = val < 0.0 ? -1.0 : 1.0;
    if (t.blk == 0 && j < d.k_out && d.out_lam) d.out_lam[j] = d.lam[j];
  }
  __syncthreads();
  if (!d.out_x) return;
  const int64_t u = (int64_t)t.blk * E::RB + threadIdx.x / LPR;
  const int sub = threadIdx.x % LPR;
  if (u >= d.n) return;
  const int64_t i = d.iperm ? d.iperm[u] : u;
  const auto v = ldv<double, VEC>(x + i * KB + sub * VEC);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const int j = sub * VEC + q;
    if (j < d.k_out) d.out_x[u * d.k_out + j] = sgn[j] * v.v[q];
  }
}

void sl_output(const SlotDev* sl, const TileSet& ts, hipStream_t s) {
  if (ts.n_red == 0) return;
  ME_DISPATCH_KB(ts.kb, {
    k_sl_col_argmax<KB><<<ts.n_red, kBlock, 0, s>>>(sl, ts.red);
    k_sl_signed_copy<KB><<<ts.n_elem64, kBlock, 0, s>>>(sl, ts.elem64);
  });
}

}  // namespace me
