// Device helpers shared by the row-streaming kernels: 16-byte vector
// access to row-major n x kb blocks, the difference-form row product of the
// operator, and the 16x16x4 MFMA accumulator layouts.
#pragma once

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

// Every pointer these helpers take refers to global (device) memory.  The
// engine's kernels fetch their pointers from the slot table, so the compiler
// cannot infer the address space and would emit flat accesses; casting to
// the global address space gives global loads and stores.
#define ME_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const ME_GLOBAL T* glob(const T* p) {
  return (const ME_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ ME_GLOBAL T* globw(T* p) {
  return (ME_GLOBAL T*)p;
}
template <typename T, int V>
__device__ __forceinline__ VecT<T, V> ldv(const T* p) {
  typedef T vt __attribute__((ext_vector_type(V)));
  const vt x = *(const ME_GLOBAL vt*)glob(p);
  VecT<T, V> r;
#pragma unroll
  for (int q = 0; q < V; ++q) r.v[q] = x[q];
  return r;
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const VecT<T, V>& v) {
  typedef T vt __attribute__((ext_vector_type(V)));
  vt x;
#pragma unroll
  for (int q = 0; q < V; ++q) x[q] = v.v[q];
  *(ME_GLOBAL vt*)globw(p) = x;
}

// Raw buffer access: a 128-bit resource (base, byte size) in scalar
// registers and a 32-bit byte offset per lane.  Loads past the size return
// zero, which the row product uses for its padding entries.  Used where
// every array of a launch is below kBufMaxBytes.
typedef int32_t BufRsrc __attribute__((ext_vector_type(4)));
typedef int32_t BufI4 __attribute__((ext_vector_type(4)));
typedef int32_t BufI2 __attribute__((ext_vector_type(2)));
__device__ int32_t me_buf_load_i32(BufRsrc r, uint32_t voff, int32_t soff, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.i32");
__device__ BufI2 me_buf_load_v2i32(BufRsrc r, uint32_t voff, int32_t soff, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ BufI4 me_buf_load_v4i32(BufRsrc r, uint32_t voff, int32_t soff, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v4i32");
constexpr uint32_t kBufOut = 0x80000000u;  // an offset past every buffer
__device__ __forceinline__ BufRsrc buf_rsrc(const void* p, int64_t bytes) {
  const uint64_t a = (uint64_t)p;
  BufRsrc r;
  r.x = (int32_t)(uint32_t)a;
  r.y = (int32_t)(uint32_t)(a >> 32);  // stride 0
  r.z = (int32_t)(uint32_t)bytes;
  r.w = 0x00020000;  // 32-bit data format (gfx9 family)
  return r;
}
__device__ __forceinline__ int32_t buf_i32(BufRsrc r, uint32_t off) {
  return me_buf_load_i32(r, off, 0, 0);
}
template <typename T>
__device__ __forceinline__ T buf_scalar(BufRsrc r, uint32_t off) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, me_buf_load_i32(r, off, 0, 0));
  } else {
    return __builtin_bit_cast(T, me_buf_load_v2i32(r, off, 0, 0));
  }
}
template <typename T, int V>
__device__ __forceinline__ VecT<T, V> buf_vec16(BufRsrc r, uint32_t off) {
  static_assert(sizeof(T) * V == 16, "16-byte chunk");
  return __builtin_bit_cast(VecT<T, V>, me_buf_load_v4i32(r, off, 0, 0));
}
// Four FP16 values (8 bytes) widened to FP32: the preconditioner's
// right-hand side beside a 16-byte chunk of FP32 iterates.
__device__ __forceinline__ VecT<float, 4> buf_half4(BufRsrc r, uint32_t off) {
  const auto h = __builtin_bit_cast(VecT<_Float16, 4>, me_buf_load_v2i32(r, off, 0, 0));
  VecT<float, 4> f;
#pragma unroll
  for (int q = 0; q < 4; ++q) f.v[q] = (float)h.v[q];
  return f;
}
__device__ __forceinline__ VecT<float, 4> ld_half4(const _Float16* p) {
  const auto h = ldv<_Float16, 4>(p);
  VecT<float, 4> f;
#pragma unroll
  for (int q = 0; q < 4; ++q) f.v[q] = (float)h.v[q];
  return f;
}

// Multiply-adds of the products and recurrences are written out, so that
// every kernel form of the same arithmetic rounds identically, whatever the
// compiler would contract on its own.
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

#define ME_DISPATCH_KB(kb, ...)                       \
  switch (kb) {                                       \
    case 4: { constexpr int KB = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int KB = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int KB = 16; __VA_ARGS__; } break; \
    default: break;                                   \
  }

// Row i of the product, without the diagonal term.  A group of G
// consecutive lanes owns one row.  A row of KB values is NCH 16-byte chunks;
// lane q takes chunk c = q % NCH of the entries e = q / NCH, e + EPL,
// e + 2 EPL, ... (EPL = G / NCH entries per round), so the lanes of one
// instruction that load the same neighbour row share its cache lines.
// Row i has W entries [a_rp[i], a_rp[i+1]) (weight w_ij) and T entries
// [a_tp[i], a_tp[i+1]) (stored weight 1/T_i + 1/T_j, scaled by c_t) in
// separate blocks of a_col / a_w; `range` selects both (the W entries come
// first in the row's sequence), the W entries only or the T entries only.  Each lane accumulates its
// chunk; a butterfly over the lanes of equal chunk leaves the row's chunk c
// in every lane.  All lanes of the wave must call it (shuffles).
// entry ranges of a row of the merged operator
enum { kRangeAll = 0, kRangeW = 1, kRangeT = 2 };

// Row mapping of the gathering kernels (build-time parameters; the defaults
// are the fastest measured by paper_2112_07862_amd.tune on the manifold
// workloads): lanes per row for one-chunk rows, entries per round for wider
// rows, rounds in flight for each.
#ifndef ME_ROW_LANES_1
#define ME_ROW_LANES_1 4
#endif
#ifndef ME_ROW_EPL
#define ME_ROW_EPL 2
#endif
#ifndef ME_ROW_UNR_1
#define ME_ROW_UNR_1 6
#endif
#ifndef ME_ROW_UNR
#define ME_ROW_UNR 8
#endif

template <typename T, int KB>
struct RowCfg {
  static constexpr int V16 = 16 / (int)sizeof(T);      // values per 16-byte chunk
  static constexpr int NCH = KB * (int)sizeof(T) / 16; // chunks per row
  // lanes per row (a power of two up to 32): by default two entries per
  // round (four lanes for one-chunk rows), eight rounds in flight (six for
  // one-chunk rows); fewer lanes per row and more loads in flight per lane
  // measured faster than wider lane groups on the gather-bound products
  static constexpr int G = NCH == 1 ? ME_ROW_LANES_1 : ME_ROW_EPL * NCH;
  static constexpr int EPL = G / NCH;                  // entries per round
  static constexpr int UNR = NCH == 1 ? ME_ROW_UNR_1 : ME_ROW_UNR;  // rounds in flight
  static_assert(G >= NCH && G <= 32 && (G & (G - 1)) == 0, "lanes per row");
  static_assert(UNR >= 1, "rounds in flight");
  static constexpr int ROWS = 32;                      // rows per workgroup
  static constexpr int THREADS = ROWS * G;
};

// Entry span of a row: W entries [ws, ws + nw), then T entries at ts + k for
// positions k in [nw, len) (the range selects which kinds are present).
struct RowSpan {
  int32_t ws, nw, ts, len;
};
__device__ __forceinline__ RowSpan row_span(bool live, int64_t row,
                                            const int32_t* __restrict__ a_rp,
                                            const int32_t* __restrict__ a_tp, int range) {
  const ME_GLOBAL int32_t* rp = glob(a_rp);
  const ME_GLOBAL int32_t* tp = glob(a_tp);
  const int64_t r = live ? row : 0;
  const int32_t w0 = rp[r], w1 = rp[r + 1], t0 = tp[r], t1 = tp[r + 1];
  RowSpan s;
  s.ws = w0;
  s.nw = (live && range != kRangeT) ? w1 - w0 : 0;
  s.ts = t0 - s.nw;
  s.len = s.nw + ((live && range != kRangeW) ? t1 - t0 : 0);
  return s;
}

// The row product over buffer resources: rc / rw hold the column indices and
// weights, rx the block.  Lane q takes the entries e0, e0 + EPL, ... of the
// span; an entry past the span loads column 0 and weight 0 (out-of-range
// loads) and adds 0 * (x_i - x_0).  Loop counts are per lane.  RANGE fixes
// the entry kinds at compile time (kRangeW: W only, kRangeT: T only) or
// leaves them to the span (-1).  In FP64 with tq (two-hop entries packed as
// column offset and T_j in rq, entry position minus tq_base), a T entry is
// one 4-byte load and its weight is formed as ti + 1 / T_j: the same two
// doubles the stored weight was summed from (1 / T_j correctly rounded), so
// the products equal those over the stored weights bit for bit.  An entry
// past the span loads 0: offset 0 (the row itself), weight 0.
template <typename T, int KB, int RANGE = -1>
__device__ __forceinline__ void spmm_span_buf(int32_t ws, int32_t nw, int32_t ts, int32_t len,
                                              int q, int64_t rs, BufRsrc rc, BufRsrc rw,
                                              BufRsrc rq, uint32_t tq_base, bool tq, T ti,
                                              BufRsrc rx, T c_t,
                                              const T (&xi)[RowCfg<T, KB>::V16],
                                              T (&acc)[RowCfg<T, KB>::V16]) {
  constexpr bool TQ = sizeof(T) == 8;
  using C = RowCfg<T, KB>;
  constexpr int V = C::V16, EPL = C::EPL, UNR = C::UNR;
  const int ch = q % C::NCH, e0 = q / C::NCH;
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  const int32_t mine = len > e0 ? (len - e0 + EPL - 1) / EPL : 0;  // this lane's entries
  for (int32_t r = 0; r < mine; r += UNR) {
    int32_t c[UNR];
    T cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = (r + u) * EPL + e0;
      const bool ok = r + u < mine;
      const bool isw = RANGE == kRangeW ? true : (RANGE == kRangeT ? false : k < nw);
      const uint32_t at = (uint32_t)((isw ? ws : ts) + k);
      if (TQ && tq && !isw) {
        const uint32_t pv = (uint32_t)buf_i32(rq, ok ? (at - tq_base) * 4u : kBufOut);
        c[u] = (int32_t)rs + (int32_t)(int16_t)(pv & 0xffffu);
        const T tj = (T)(pv >> 16);
        cf[u] = ok ? c_t * (ti + (T)1 / tj) : (T)0;
      } else {
        c[u] = buf_i32(rc, ok ? at * 4u : kBufOut);
        const T w = buf_scalar<T>(rw, ok ? at * (uint32_t)sizeof(T) : kBufOut);
        cf[u] = isw ? w : c_t * w;
      }
    }
    VecT<T, V> xj[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      xj[u] = buf_vec16<T, V>(rx, (uint32_t)c[u] * (uint32_t)(KB * sizeof(T)) +
                                      (uint32_t)(ch * 16));
    // every gather of the round is in flight before the first is used (the
    // scheduler would otherwise trade them for registers)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fmaT(cf[u], xi[v] - xj[u].v[v], acc[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    for (int o = C::NCH; o < C::G; o <<= 1) acc[v] += __shfl_xor(acc[v], o);
}

// The FP32 row product over packed entries (column - row in 16 bits, FP16
// weight): one 32-bit load per entry.  rs is the row, clamped to 0 past the
// end; an entry past the span (its load gives 0, by the buffer's range check
// or by the explicit test of the 64-bit form) points at row rs with weight 0
// and adds exactly 0.  BUFA selects buffer or 64-bit global addressing; both
// visit the entries in the same order.
template <int KB, int RANGE, bool BUFA>
__device__ __forceinline__ void spmm_span_pk(int32_t ws, int32_t nw, int32_t ts, int32_t len,
                                             int q, int64_t rs, const uint32_t* __restrict__ a_pk,
                                             int64_t nnz_ops, const float* __restrict__ x,
                                             int64_t n, float c_t,
                                             const float (&xi)[RowCfg<float, KB>::V16],
                                             float (&acc)[RowCfg<float, KB>::V16]) {
  using C = RowCfg<float, KB>;
  constexpr int V = C::V16, EPL = C::EPL, UNR = C::UNR;
  const int ch = q % C::NCH, e0 = q / C::NCH;
  BufRsrc rp{}, rx{};
  if constexpr (BUFA) {
    rp = buf_rsrc(a_pk, nnz_ops * 4);
    rx = buf_rsrc(x, n * KB * 4);
  }
  const ME_GLOBAL uint32_t* gp = glob(a_pk);
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  const int32_t mine = len > e0 ? (len - e0 + EPL - 1) / EPL : 0;  // this lane's entries
  for (int32_t r = 0; r < mine; r += UNR) {
    int32_t c[UNR];
    float cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = (r + u) * EPL + e0;
      const bool ok = r + u < mine;
      bool isw;
      uint32_t at;
      if constexpr (RANGE == kRangeW) {
        isw = true;
        at = (uint32_t)(ws + k);
      } else if constexpr (RANGE == kRangeT) {
        isw = false;
        at = (uint32_t)(ts + k);
      } else {
        isw = k < nw;
        at = (uint32_t)((isw ? ws : ts) + k);
      }
      uint32_t pv;
      if constexpr (BUFA) pv = (uint32_t)buf_i32(rp, ok ? at * 4u : kBufOut);
      else pv = ok ? gp[at] : 0u;
      c[u] = (int32_t)rs + (int32_t)(int16_t)(pv & 0xffffu);
      const float w = (float)__builtin_bit_cast(_Float16, (uint16_t)(pv >> 16));
      cf[u] = isw ? w : c_t * w;
    }
    VecT<float, V> xj[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      if constexpr (BUFA)
        xj[u] = buf_vec16<float, V>(rx, (uint32_t)c[u] * (uint32_t)(KB * 4) + (uint32_t)(ch * 16));
      else
        xj[u] = ldv<float, V>(x + (int64_t)c[u] * KB + ch * V);
    }
    asm volatile("" ::: "memory");  // every gather of the round in flight first
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fmaT(cf[u], xi[v] - xj[u].v[v], acc[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    for (int o = C::NCH; o < C::G; o <<= 1) acc[v] += __shfl_xor(acc[v], o);
}

// The same product over a block stored in FP16 (arithmetic in FP32): one
// 16-byte chunk is 8 values.
template <int KB, int RANGE>
__device__ __forceinline__ void spmm_span_pk_h(int32_t ws, int32_t nw, int32_t ts, int32_t len,
                                               int q, int64_t rs, const uint32_t* __restrict__ a_pk,
                                               int64_t nnz_ops, const _Float16* __restrict__ x,
                                               int64_t n, float c_t, const float (&xi)[8],
                                               float (&acc)[8]) {
  using C = RowCfg<_Float16, KB>;
  constexpr int V = C::V16, EPL = C::EPL, UNR = C::UNR;
  static_assert(V == 8, "8 FP16 values per chunk");
  const int ch = q % C::NCH, e0 = q / C::NCH;
  const BufRsrc rp = buf_rsrc(a_pk, nnz_ops * 4);
  const BufRsrc rx = buf_rsrc(x, n * KB * 2);
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  const int32_t mine = len > e0 ? (len - e0 + EPL - 1) / EPL : 0;  // this lane's entries
  for (int32_t r = 0; r < mine; r += UNR) {
    int32_t c[UNR];
    float cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = (r + u) * EPL + e0;
      const bool ok = r + u < mine;
      bool isw;
      uint32_t at;
      if constexpr (RANGE == kRangeW) {
        isw = true;
        at = (uint32_t)(ws + k);
      } else if constexpr (RANGE == kRangeT) {
        isw = false;
        at = (uint32_t)(ts + k);
      } else {
        isw = k < nw;
        at = (uint32_t)((isw ? ws : ts) + k);
      }
      const uint32_t pv = (uint32_t)buf_i32(rp, ok ? at * 4u : kBufOut);
      c[u] = (int32_t)rs + (int32_t)(int16_t)(pv & 0xffffu);
      const float w = (float)__builtin_bit_cast(_Float16, (uint16_t)(pv >> 16));
      cf[u] = isw ? w : c_t * w;
    }
    VecT<_Float16, V> xj[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      xj[u] = buf_vec16<_Float16, V>(rx, (uint32_t)c[u] * (uint32_t)(KB * 2) + (uint32_t)(ch * 16));
    asm volatile("" ::: "memory");  // every gather of the round in flight first
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fmaT(cf[u], xi[v] - (float)xj[u].v[v], acc[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    for (int o = C::NCH; o < C::G; o <<= 1) acc[v] += __shfl_xor(acc[v], o);
}

template <typename T, int KB>
__device__ __forceinline__ void spmm_row(bool live, int64_t row, int q,
                                         const int32_t* __restrict__ a_rp,
                                         const int32_t* __restrict__ a_tp,
                                         const int32_t* __restrict__ a_col,
                                         const T* __restrict__ a_w, T c_t, int range,
                                         const T* __restrict__ x,
                                         const T (&xi)[RowCfg<T, KB>::V16],
                                         T (&acc)[RowCfg<T, KB>::V16]) {
  using C = RowCfg<T, KB>;
  constexpr int V = C::V16, EPL = C::EPL, UNR = C::UNR;
  const int ch = q % C::NCH, e0 = q / C::NCH;
  const ME_GLOBAL int32_t* rp = glob(a_rp);
  const ME_GLOBAL int32_t* tp = glob(a_tp);
  const ME_GLOBAL int32_t* cl = glob(a_col);
  const ME_GLOBAL T* wt = glob(a_w);
  // the row's entries as one sequence: positions [0, nw) are W entries at
  // ws + k, positions [nw, len) T entries at ts + (k - nw)
  int32_t ws = 0, nw = 0, ts = 0, len = 0;
  if (live) {
    if (range != kRangeT) {
      ws = rp[row];
      nw = rp[row + 1] - ws;
    }
    len = nw;
    if (range != kRangeW) {
      ts = tp[row] - nw;
      len += tp[row + 1] - tp[row];
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  // rounds of EPL entries; loop to the wave's longest row
  int32_t rounds = (len + EPL - 1) / EPL;
  for (int o = kWave / 2; o > 0; o >>= 1) rounds = max(rounds, __shfl_xor(rounds, o));
  for (int32_t r = 0; r < rounds; r += UNR) {
    int32_t c[UNR];
    T cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = (r + u) * EPL + e0;
      const bool ok = k < len, isw = k < nw;
      const int32_t at = (isw ? ws : ts) + k;
      c[u] = ok ? cl[at] : -1;
      const T w = ok ? wt[at] : (T)0;
      cf[u] = isw ? w : c_t * w;
    }
    T xj[UNR][V];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      if (c[u] >= 0) {
        const auto t = ldv<T, V>(x + (int64_t)c[u] * KB + ch * V);
#pragma unroll
        for (int v = 0; v < V; ++v) xj[u][v] = t.v[v];
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) xj[u][v] = xi[v];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fmaT(cf[u], xi[v] - xj[u][v], acc[v]);
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    for (int o = C::NCH; o < C::G; o <<= 1) acc[v] += __shfl_xor(acc[v], o);
}

// One 16-byte chunk of a row into registers.
template <typename T, int V>
__device__ __forceinline__ void load_chunk(const T* __restrict__ p, T (&v)[V]) {
  const auto t = ldv<T, V>(p);
#pragma unroll
  for (int q = 0; q < V; ++q) v[q] = t.v[q];
}

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

}  // namespace me
