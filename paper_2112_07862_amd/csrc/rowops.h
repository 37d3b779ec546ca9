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

template <typename T, int V>
__device__ inline VecT<T, V> ldv(const T* p) {
  return *reinterpret_cast<const VecT<T, V>*>(p);
}
template <typename T, int V>
__device__ inline void stv(T* p, const VecT<T, V>& v) {
  *reinterpret_cast<VecT<T, V>*>(p) = v;
}

#define ME_DISPATCH_KB(kb, ...)                       \
  switch (kb) {                                       \
    case 4: { constexpr int KB = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int KB = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int KB = 16; __VA_ARGS__; } break; \
    default: break;                                   \
  }

// Row i of the product, without the diagonal term.  A group of G
// consecutive lanes owns one row and splits the row's entries: lane q takes
// entries q, q + G, q + 2G, ..., loads their columns and weights (coalesced
// over the group), gathers the neighbour rows x_j whole (KB values, 16-byte
// loads) UNR at a time, and accumulates the full row; a butterfly over the
// group leaves the sum in every lane.  Entries before a_split are W entries
// (weight w_ij), the rest T entries (weight c_t (1/T_i + 1/T_j)).  All
// lanes of the wave must call it (shuffles).
template <typename T, int KB>
struct RowCfg {
  static constexpr int G = 8;                                  // lanes per row
  static constexpr int UNR = (KB * sizeof(T) >= 128) ? 2 : 4;  // entries in flight per lane
  static constexpr int V16 = 16 / sizeof(T);                   // values per 16-byte load
  static constexpr int NLD = KB * sizeof(T) / 16;              // 16-byte loads per row
};

template <typename T, int KB>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[KB]) {
  using C = RowCfg<T, KB>;
#pragma unroll
  for (int l = 0; l < C::NLD; ++l) {
    const auto t = ldv<T, C::V16>(p + l * C::V16);
#pragma unroll
    for (int q = 0; q < C::V16; ++q) v[l * C::V16 + q] = t.v[q];
  }
}

template <typename T, int KB>
__device__ __forceinline__ void spmm_row(bool live, int64_t row, int q,
                                         const int32_t* __restrict__ a_rp,
                                         const int32_t* __restrict__ a_split,
                                         const int32_t* __restrict__ a_col,
                                         const T* __restrict__ a_w, const T* __restrict__ invt,
                                         T c_t, int skip_w, const T* __restrict__ x,
                                         const T (&xi)[KB], T (&acc)[KB]) {
  using C = RowCfg<T, KB>;
  constexpr int G = C::G, UNR = C::UNR;
  int32_t s = 0, sp = 0, e = 0;
  T ti = 0;
  if (live) {
    s = skip_w ? a_split[row] : a_rp[row];
    sp = a_split[row];
    e = a_rp[row + 1];
    ti = invt[row];
  }
#pragma unroll
  for (int v = 0; v < KB; ++v) acc[v] = 0;
  // steps of G entries; loop to the wave's longest row
  int32_t steps = (e - s + G - 1) / G;
  for (int o = kWave / 2; o > 0; o >>= 1) steps = max(steps, __shfl_xor(steps, o));
  for (int32_t st = 0; st < steps; st += UNR) {
    int32_t c[UNR];
    T cf[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = s + (st + u) * G + q;
      const bool ok = k < e;
      c[u] = ok ? a_col[k] : -1;
      cf[u] = (ok && k < sp) ? a_w[k] : (T)0;
    }
    T xj[UNR][KB];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int32_t k = s + (st + u) * G + q;
      if (c[u] >= 0) {
        load_row<T, KB>(x + (int64_t)c[u] * KB, xj[u]);
        if (k >= sp) cf[u] = c_t * (ti + invt[c[u]]);
      } else {
#pragma unroll
        for (int v = 0; v < KB; ++v) xj[u][v] = xi[v];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int v = 0; v < KB; ++v) acc[v] += cf[u] * (xi[v] - xj[u][v]);
  }
#pragma unroll
  for (int v = 0; v < KB; ++v)
    for (int o = G / 2; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
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
