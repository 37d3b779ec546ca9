// Graph-operator build: validation of W (Section 3.1), degrees, the
// disconnected two-hop pattern T (Section 4.1.1), Q's diagonal and the mu
// denominators (eq. (Q), eq. (mu)), connectivity of the two-hop graph
// (lambda_2(Q) = 0 iff it is disconnected), eps (Section 4.2), r and b
// (Section 4.3), and the packed difference-form operator A = L - mu Q + eps I
// (eq. (obj2)).
#include <cmath>
#include <cstring>

#include "common.h"

namespace me {

enum : int {
  F_INVALID = 1,
  F_SELF_LOOP = 2,
  F_BAD_WEIGHT = 4,
  F_NOT_SYMMETRIC = 8,
  F_ISOLATED = 16,
};

static int flags_to_status(int f) {
  if (f & F_INVALID) return ME_ERR_INVALID_ARG;
  if (f & F_SELF_LOOP) return ME_ERR_SELF_LOOP;
  if (f & F_BAD_WEIGHT) return ME_ERR_BAD_WEIGHT;
  if (f & F_NOT_SYMMETRIC) return ME_ERR_NOT_SYMMETRIC;
  if (f & F_ISOLATED) return ME_ERR_ISOLATED_NODE;
  return ME_OK;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------

__global__ void k_check_rowptr(int64_t n, int64_t nnz, const int64_t* rp, int* flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  int64_t v = rp[i];
  bool bad = (i == 0 && v != 0) || (i == n && v != nnz) || (v < 0) || (v > nnz);
  if (i < n && rp[i + 1] < v) bad = true;
  if (bad) atomicOr(flags, F_INVALID);
}

// One thread per row: column range and order, self loops, weights,
// exact symmetry (binary search of i in row j), isolated nodes, degree.
__global__ void k_validate_rows(int64_t n, const int64_t* rp, const int32_t* col,
                                const double* val, double* deg, int* flags) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t s = rp[i], e = rp[i + 1];
  int f = 0;
  if (s == e) f |= F_ISOLATED;
  double d = 0.0;
  int32_t prev = -1;
  for (int64_t t = s; t < e; ++t) {
    int32_t c = col[t];
    double v = val[t];
    if (c < 0 || c >= n) { f |= F_INVALID; continue; }
    if (c <= prev) f |= F_INVALID;
    prev = c;
    if (c == i) f |= F_SELF_LOOP;
    if (!(v > 0.0) || !isfinite(v)) f |= F_BAD_WEIGHT;
    d += v;
    int64_t lo = rp[c], hi = rp[c + 1];
    bool found = false;
    while (lo < hi) {
      int64_t mid = lo + ((hi - lo) >> 1);
      int32_t cm = col[mid];
      if (cm == (int32_t)i) { found = (val[mid] == v); break; }
      if (cm < (int32_t)i) lo = mid + 1; else hi = mid;
    }
    if (!found) f |= F_NOT_SYMMETRIC;
  }
  deg[i] = d;
  if (f) atomicOr(flags, f);
}

// ---------------------------------------------------------------------------
// Two-hop pattern.  Row i's candidates are the members of N(k) for k in N(i);
// T_i is that union minus N(i) and i.  Rows whose candidate count fits an
// LDS table use an open-addressing hash in LDS (one wave per row): a small
// table first (the rows of kNN graphs; little LDS, many waves per CU), the
// rows it cannot take a large one, the rest a bitmap kernel.  Output columns
// are sorted ascending.
// ---------------------------------------------------------------------------

constexpr int kHashSmall = 512;   // slots per row table (powers of two) ...
constexpr int kHashLarge = 2048;  // ... admitting half as many keys (load factor <= 1/2)

template <int CAP>
__device__ inline unsigned hash_slot(int32_t j) {
  constexpr int bits = __builtin_ctz(CAP);
  return ((uint32_t)j * 2654435761u) >> (32 - bits);
}

template <int CAP>
__device__ inline void hash_insert(int* table, int32_t j, bool excluded) {
  int key = excluded ? -(j + 1) : (j + 1);
  unsigned h = hash_slot<CAP>(j);
  for (;;) {
    int prev = atomicCAS(&table[h], 0, key);
    if (prev == 0 || prev == j + 1 || prev == -(j + 1)) return;
    h = (h + 1) & (CAP - 1);
  }
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Rows `rows[0..nrows)` (rows null: every row, nrows = n) with a table of
// CAP slots.  mode 0: count (tcnt[i] = T_i; a row with more candidates than
// the table admits is appended to over_list with tcnt = 0); mode 1: fill
// (writes sorted columns at t_rp[i]; such rows skipped, over_list unused).
template <int CAP>
__global__ void __launch_bounds__(64) k_twohop_lds(int64_t n, const int64_t* rp, const int32_t* col,
                                                   int mode, int32_t* tcnt, const int64_t* t_rp,
                                                   int32_t* t_col, const int32_t* rows,
                                                   int64_t nrows, int32_t* over_list,
                                                   int32_t* over_count) {
  constexpr int kMaxKeys = CAP / 2;
  __shared__ int table[CAP];
  __shared__ int32_t list[kMaxKeys];
  __shared__ int lane_off[kWave];
  const int lane = threadIdx.x;
  constexpr int per = CAP / kWave;  // slots per lane
  for (int q = 0; q < per; ++q) table[lane * per + q] = 0;
  __syncthreads();
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int64_t row = rows ? (int64_t)rows[r] : r;
    const int64_t s = rp[row], e = rp[row + 1];
    int64_t cand = 0;
    for (int64_t t = s + lane; t < e; t += kWave) {
      int32_t k = col[t];
      cand += rp[k + 1] - rp[k];
    }
    cand = wave_sum_i64(cand);
    if (cand + (e - s) + 1 > kMaxKeys) {
      if (mode == 0 && lane == 0) {
        int slot = atomicAdd(over_count, 1);
        over_list[slot] = (int32_t)row;
        tcnt[row] = 0;
      }
      continue;
    }
    if (lane == 0) hash_insert<CAP>(table, (int32_t)row, true);
    for (int64_t t = s + lane; t < e; t += kWave) hash_insert<CAP>(table, col[t], true);
    __syncthreads();
    for (int64_t t = s; t < e; ++t) {
      int32_t k = col[t];
      const int64_t ks = rp[k], ke = rp[k + 1];
      for (int64_t u = ks + lane; u < ke; u += kWave) hash_insert<CAP>(table, col[u], false);
    }
    __syncthreads();
    int mine = 0;
    for (int q = 0; q < per; ++q) mine += table[lane * per + q] > 0;
    if (mode == 0) {
      int64_t total = wave_sum_i64(mine);
      if (lane == 0) tcnt[row] = (int32_t)total;
    } else {
      // exclusive prefix of `mine` over lanes
      lane_off[lane] = mine;
      __syncthreads();
      int off = 0;
      for (int q = 0; q < lane; ++q) off += lane_off[q];
      int total = off;
      for (int q = lane; q < kWave; ++q) total += lane_off[q];
      for (int q = 0; q < per; ++q) {
        int v = table[lane * per + q];
        if (v > 0) list[off++] = v - 1;
      }
      __syncthreads();
      const int64_t base = t_rp[row];
      for (int a = lane; a < total; a += kWave) {
        int32_t v = list[a];
        int rank = 0;
        for (int c = 0; c < total; ++c) rank += list[c] < v;
        t_col[base + rank] = v;
      }
      __syncthreads();
    }
    for (int q = 0; q < per; ++q) table[lane * per + q] = 0;
    __syncthreads();
  }
}

// Rows too large for the LDS table: one block per row, a bitmap over all
// nodes in global scratch (one bitmap per block).  Scanning the bitmap in
// order yields sorted columns.
__global__ void __launch_bounds__(256) k_twohop_big(int64_t n, const int64_t* rp, const int32_t* col,
                                                    int mode, const int32_t* big_list, int nbig,
                                                    uint32_t* bitmaps, int32_t* tcnt,
                                                    const int64_t* t_rp, int32_t* t_col) {
  __shared__ int64_t part[256];
  const int64_t nwords = (n + 31) / 32;
  uint32_t* bm = bitmaps + (int64_t)blockIdx.x * nwords;
  for (int qi = blockIdx.x; qi < nbig; qi += gridDim.x) {
    const int64_t row = big_list[qi];
    const int64_t s = rp[row], e = rp[row + 1];
    for (int64_t t = s; t < e; ++t) {
      int32_t k = col[t];
      for (int64_t u = rp[k] + threadIdx.x; u < rp[k + 1]; u += blockDim.x) {
        uint32_t j = (uint32_t)col[u];
        atomicOr(&bm[j >> 5], 1u << (j & 31));
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicAnd(&bm[row >> 5], ~(1u << (row & 31)));
    for (int64_t t = s + threadIdx.x; t < e; t += blockDim.x) {
      uint32_t j = (uint32_t)col[t];
      atomicAnd(&bm[j >> 5], ~(1u << (j & 31)));
    }
    __syncthreads();
    // contiguous word chunk per thread
    const int64_t chunk = (nwords + blockDim.x - 1) / blockDim.x;
    const int64_t w0 = threadIdx.x * chunk;
    const int64_t w1 = (w0 + chunk < nwords) ? w0 + chunk : nwords;
    int64_t cnt = 0;
    for (int64_t w = w0; w < w1; ++w) cnt += __popc(bm[w]);
    part[threadIdx.x] = cnt;
    __syncthreads();
    if (mode == 0) {
      if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int q = 0; q < (int)blockDim.x; ++q) tot += part[q];
        tcnt[row] = (int32_t)tot;
      }
    } else {
      int64_t off = t_rp[row];
      for (int q = 0; q < (int)threadIdx.x; ++q) off += part[q];
      for (int64_t w = w0; w < w1; ++w) {
        uint32_t bits = bm[w];
        while (bits) {
          int b = __ffs(bits) - 1;
          bits &= bits - 1;
          t_col[off++] = (int32_t)(w * 32 + b);
        }
      }
    }
    __syncthreads();
    // clear what this row set
    for (int64_t t = s; t < e; ++t) {
      int32_t k = col[t];
      for (int64_t u = rp[k] + threadIdx.x; u < rp[k + 1]; u += blockDim.x) {
        uint32_t j = (uint32_t)col[u];
        bm[j >> 5] = 0u;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts into int64 offsets (out[n] = total).
// ---------------------------------------------------------------------------

constexpr int kScanPer = 4;
constexpr int kScanTile = kBlock * kScanPer;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_tiles(int64_t n, const int32_t* in, int64_t* out,
                                                       int64_t* tile_sums) {
  __shared__ int64_t sh[kBlock];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t sum = 0;
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    sum += v[q];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(sum, sh, &tot);
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) out[base + q] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_sums(int64_t ntiles, int64_t* tile_sums,
                                                      int64_t* out_total) {
  __shared__ int64_t sh[kBlock];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += kBlock) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < ntiles ? tile_sums[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < ntiles) tile_sums[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ void k_scan_add(int64_t n, int64_t* out, const int64_t* tile_sums) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_sums[i / kScanTile];
}

int64_t scan_tmp_count(int64_t n) { return std::max<int64_t>(1, ceil_div(n, kScanTile)); }

void scan_counts(int64_t n, const int32_t* cnt, int64_t* out, int64_t* tile_tmp, hipStream_t s) {
  int64_t ntiles = ceil_div(n, kScanTile);
  if (ntiles == 0) ntiles = 1;
  k_scan_tiles<<<ntiles, kBlock, 0, s>>>(n, cnt, out, tile_tmp);
  k_scan_sums<<<1, kBlock, 0, s>>>(ntiles, tile_tmp, out + n);
  k_scan_add<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, out, tile_tmp);
}

// ---------------------------------------------------------------------------
// Connected components of the two-hop graph (union-find: hook the larger
// root under the smaller one, path halving; parents only decrease, so every
// loop ends).
// ---------------------------------------------------------------------------

__device__ inline int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    int32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    if (p == x) return x;
    int32_t gp = __atomic_load_n(&parent[p], __ATOMIC_RELAXED);
    if (gp != p) __atomic_store_n(&parent[x], gp, __ATOMIC_RELAXED);
    x = gp;
  }
}

__global__ void k_uf_init(int64_t n, int32_t* parent) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) parent[i] = (int32_t)i;
}

__global__ void k_uf_hook(int64_t n, const int64_t* t_rp, const int32_t* t_col, int32_t* parent) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t t = t_rp[i]; t < t_rp[i + 1]; ++t) {
    int32_t j = t_col[t];
    if (j >= i) break;  // sorted: each undirected pair once
    int32_t a = uf_find(parent, (int32_t)i), b = uf_find(parent, j);
    while (a != b) {
      if (a < b) { int32_t tmp = a; a = b; b = tmp; }  // a > b: hook a under b
      int32_t old = atomicCAS(&parent[a], a, b);
      if (old == a) break;
      a = uf_find(parent, old);
      b = uf_find(parent, b);
    }
  }
}

__global__ void k_uf_count_roots(int64_t n, int32_t* parent, int* roots) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int is_root = 0;
  if (i < n) is_root = uf_find(parent, (int32_t)i) == (int32_t)i;
  // wave-level count then one atomic per wave
  unsigned long long m = __ballot(is_root);
  if ((threadIdx.x & (kWave - 1)) == 0 && m) atomicAdd(roots, __popcll(m));
}

// ---------------------------------------------------------------------------
// Locality order of the solver.  The LOBPCG kernels gather the rows of the
// neighbours (one- and two-hop) of every row; with the caller's node order
// (random for sampled point clouds) each gather touches its own cache line.
// Nodes are put in Cuthill-McKee order from a pseudo-peripheral node (the
// lowest-numbered node on the last level of a search from node 0),
// components one after the other: neighbours then lie within a few level
// widths of each other.  Both searches are level-synchronous, one workgroup
// per graph (a batch runs the searches of all its graphs in one launch), and
// deterministic: the order equals that of the sequential algorithm.
// ---------------------------------------------------------------------------


// Breadth-first levels in one workgroup, with frontier counters in LDS.
//
// bfs_levels: plain levels from one node (used to find the pseudo-peripheral
// start: the lowest-numbered node on the last level of a search from 0).
//
// cm_order: the Cuthill-McKee order, written straight into perm.  Level 0 is
// the start; level l+1 holds the unvisited neighbours of level l, ordered by
// the position of their first (lowest-positioned) neighbour in level l and
// then by node id -- exactly the order of a sequential search that scans
// level l in order and each row's neighbours in increasing id.  Further
// components follow, each started at its lowest unvisited node.
// level[] and key[] change through device-scope atomics, which are performed
// in L2; every read of them is an agent-scope atomic load so that no stale
// L1 copy is used.
__device__ __forceinline__ int32_t ld_coherent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kBfsThreads = 1024;
// Neighbours of one node whose loads and atomics are issued together in the
// node-parallel levels of the plain search.
constexpr int kNbrGrp = 8;

// A frontier of at most kBfsThreads nodes staged in LDS: node ids, first
// edges and the exclusive scan of their degrees, so that one thread per edge
// finds its node by a binary search in LDS.
struct FrontierLds {
  int32_t off[kBfsThreads + 1];
  int32_t u[kBfsThreads];
  int64_t rs[kBfsThreads];
};

// The edges of a narrow level in LDS (neighbour, frontier position, "my
// child" flag) when there are at most kEdgeLds of them.
constexpr int kEdgeLds = 8192;
struct EdgeLds {
  int32_t ev[kEdgeLds];
  int32_t ei[kEdgeLds];
  int32_t ef[kEdgeLds];
};

__device__ __forceinline__ int32_t find_owner(const int32_t* off, int32_t n, int32_t e);

// Stages fin[0..nin) (nin <= kBfsThreads); returns the number of edges.
__device__ __forceinline__ int32_t stage_frontier(const int64_t* __restrict__ rp,
                                                  const int32_t* fin, int32_t nin,
                                                  FrontierLds* f, int32_t* s_wave);

__device__ __forceinline__ int32_t bfs_levels(const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col, int32_t* level,
                                              int32_t* fa, int32_t* fb, int32_t start,
                                              int32_t* s_cnt, FrontierLds* f, int32_t* s_wave) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    level[start] = 0;
    fa[0] = start;
    s_cnt[0] = 1;
  }
  __syncthreads();
  int32_t lev = 0;
  int32_t* fin = fa;
  int32_t* fout = fb;
  for (;;) {
    const int32_t nin = s_cnt[0];
    if (tid == 0) s_cnt[1] = 0;
    __syncthreads();
    if (nin <= kBfsThreads) {
      // narrow level: one thread per frontier edge
      const int32_t m = stage_frontier(rp, fin, nin, f, s_wave);
      for (int32_t e = tid; e < m; e += kBfsThreads) {
        const int32_t i = find_owner(f->off, nin, e);
        const int32_t v = col[f->rs[i] + (e - f->off[i])];
        if (ld_coherent(&level[v]) < 0 && atomicCAS(&level[v], -1, lev + 1) == -1)
          fout[atomicAdd(&s_cnt[1], 1)] = v;
      }
    } else {
      for (int32_t i = tid; i < nin; i += kBfsThreads) {
        const int32_t u = fin[i];
        const int64_t t0 = rp[u], t1 = rp[u + 1];
        for (int64_t t = t0; t < t1; t += kNbrGrp) {
          int32_t v[kNbrGrp], lv[kNbrGrp];
#pragma unroll
          for (int j = 0; j < kNbrGrp; ++j)
            if (t + j < t1) v[j] = col[t + j];
#pragma unroll
          for (int j = 0; j < kNbrGrp; ++j)
            if (t + j < t1) lv[j] = ld_coherent(&level[v[j]]);
#pragma unroll
          for (int j = 0; j < kNbrGrp; ++j)
            if (t + j < t1 && lv[j] < 0 && atomicCAS(&level[v[j]], -1, lev + 1) == -1)
              fout[atomicAdd(&s_cnt[1], 1)] = v[j];
        }
      }
    }
    __syncthreads();
    const int32_t nout = s_cnt[1];
    if (nout == 0) break;
    if (tid == 0) s_cnt[0] = nout;
    int32_t* t = fin;
    fin = fout;
    fout = t;
    ++lev;
    __syncthreads();
  }
  return lev;
}

// Exclusive scan of a[0..n) in place by one workgroup of NT threads
// (s_wave: NT / kWave ints); returns the total.  COH: a[] was written by
// other workgroups of the same launch, so it is read past the L1.
template <int NT = kBfsThreads, bool COH = false>
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t* a, int32_t n, int32_t* s_wave) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  constexpr int NW = NT / kWave;
  int32_t carry = 0;
  for (int32_t base = 0; base < n; base += NT) {
    const int32_t i = base + tid;
    const int32_t v = i < n ? (COH ? ld_coherent(&a[i]) : a[i]) : 0;
    int32_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[wave] = x;
    __syncthreads();
    if (wave == 0) {
      int32_t w = lane < NW ? s_wave[lane] : 0;
      for (int o = 1; o < NW; o <<= 1) {
        const int32_t y = __shfl_up(w, o);
        if (lane >= o) w += y;
      }
      if (lane < NW) s_wave[lane] = w;
    }
    __syncthreads();
    const int32_t before = wave > 0 ? s_wave[wave - 1] : 0;
    if (i < n) a[i] = carry + before + x - v;
    const int32_t chunk = s_wave[NW - 1];
    __syncthreads();
    carry += chunk;
  }
  return carry;
}

// Largest i < n with off[i] <= e (off strictly increasing, off[0] = 0).
__device__ __forceinline__ int32_t find_owner(const int32_t* off, int32_t n, int32_t e) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int32_t stage_frontier(const int64_t* __restrict__ rp,
                                                  const int32_t* fin, int32_t nin,
                                                  FrontierLds* f, int32_t* s_wave) {
  const int tid = threadIdx.x;
  if (tid < nin) {
    const int32_t u = fin[tid];
    const int64_t rs = rp[u];
    f->u[tid] = u;
    f->rs[tid] = rs;
    f->off[tid] = (int32_t)(rp[u + 1] - rs);
  }
  __syncthreads();
  const int32_t m = block_exclusive_scan(f->off, nin, s_wave);
  __syncthreads();
  return m;
}

// One component of the Cuthill-McKee order: perm[off] = start, levels from
// lev0.  Scratch: key (n ints, INT32_MAX for unvisited nodes), eoff (n ints)
// and ev, ei, ef (one int per edge).  Every level-l node claims its
// unvisited neighbours and lowers their key to its own position (atomic
// min); a child belongs to the node whose position is its key.  A narrow
// level (fewer than kBfsThreads nodes, staged in LDS) works on its
// frontier's edges in (frontier position, neighbour id) order, one thread
// per edge, and an exclusive scan of the "my child" flags over the edges
// places every child (edges and flags in LDS up to kEdgeLds of them); a wide
// level (one thread per frontier node) scans per-node child counts and each
// node writes its children in row order.  Both give the sequential
// Cuthill-McKee order.
// Returns the number of nodes placed; *last_lev receives the last level.
__device__ __forceinline__ int64_t cm_component(const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col, int32_t* level,
                                                int32_t* key, int32_t* eoff, int32_t* ev,
                                                int32_t* ei, int32_t* ef, int32_t* perm,
                                                int64_t off, int32_t start, int32_t lev0,
                                                int32_t* s_wave, FrontierLds* f, EdgeLds* el,
                                                int32_t* last_lev) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    level[start] = lev0;
    perm[off] = start;
  }
  __syncthreads();
  int64_t placed = 1;
  int32_t nin = 1, lev = lev0;
  for (;;) {
    const int32_t* fin = perm + off + placed - nin;
    int32_t* fout = perm + off + placed;
    int32_t nout = 0;
    if (nin >= kBfsThreads) {
      // wide level: one thread per frontier node
      for (int32_t i = tid; i < nin; i += kBfsThreads) {
        const int32_t u = fin[i];
        for (int64_t t = rp[u]; t < rp[u + 1]; ++t) {
          const int32_t v = col[t];
          int32_t lv = ld_coherent(&level[v]);
          if (lv < 0) {
            const int32_t old = atomicCAS(&level[v], -1, lev + 1);
            lv = old < 0 ? lev + 1 : old;
          }
          if (lv == lev + 1) atomicMin(&key[v], i);
        }
      }
      __syncthreads();
      for (int32_t i = tid; i < nin; i += kBfsThreads) {
        const int32_t u = fin[i];
        int32_t c = 0;
        for (int64_t t = rp[u]; t < rp[u + 1]; ++t) {
          const int32_t v = col[t];
          c += (ld_coherent(&level[v]) == lev + 1 && ld_coherent(&key[v]) == i) ? 1 : 0;
        }
        eoff[i] = c;
      }
      __syncthreads();
      nout = block_exclusive_scan(eoff, nin, s_wave);
      for (int32_t i = tid; i < nin; i += kBfsThreads) {
        const int32_t u = fin[i];
        int32_t j = eoff[i];
        for (int64_t t = rp[u]; t < rp[u + 1]; ++t) {
          const int32_t v = col[t];
          if (ld_coherent(&level[v]) == lev + 1 && ld_coherent(&key[v]) == i) fout[j++] = v;
        }
      }
    } else {
      // narrow level: one thread per frontier edge
      const int32_t m = stage_frontier(rp, fin, nin, f, s_wave);
      if (m <= kEdgeLds) {
        // edges, flags and their scan in LDS
        for (int32_t e = tid; e < m; e += kBfsThreads) {
          const int32_t i = find_owner(f->off, nin, e);
          const int32_t v = col[f->rs[i] + (e - f->off[i])];
          el->ev[e] = v;
          el->ei[e] = i;
          int32_t lv = ld_coherent(&level[v]);
          if (lv < 0) {
            const int32_t old = atomicCAS(&level[v], -1, lev + 1);
            lv = old < 0 ? lev + 1 : old;
          }
          if (lv == lev + 1) atomicMin(&key[v], i);
        }
        __syncthreads();
        for (int32_t e = tid; e < m; e += kBfsThreads) {
          const int32_t v = el->ev[e];
          el->ef[e] = (ld_coherent(&level[v]) == lev + 1 && ld_coherent(&key[v]) == el->ei[e]);
        }
        __syncthreads();
        nout = block_exclusive_scan(el->ef, m, s_wave);
        for (int32_t e = tid; e < m; e += kBfsThreads) {
          const int32_t nxt = e + 1 < m ? el->ef[e + 1] : nout;
          if (nxt != el->ef[e]) fout[el->ef[e]] = el->ev[e];
        }
        __syncthreads();
        if (nout == 0) break;
        placed += nout;
        nin = nout;
        ++lev;
        continue;
      }
      for (int32_t e = tid; e < m; e += kBfsThreads) {
        const int32_t i = find_owner(f->off, nin, e);
        const int32_t v = col[f->rs[i] + (e - f->off[i])];
        ev[e] = v;
        ei[e] = i;
        int32_t lv = ld_coherent(&level[v]);
        if (lv < 0) {
          const int32_t old = atomicCAS(&level[v], -1, lev + 1);
          lv = old < 0 ? lev + 1 : old;
        }
        if (lv == lev + 1) atomicMin(&key[v], i);
      }
      __syncthreads();
      for (int32_t e = tid; e < m; e += kBfsThreads) {
        const int32_t v = ev[e];
        ef[e] = (ld_coherent(&level[v]) == lev + 1 && ld_coherent(&key[v]) == ei[e]) ? 1 : 0;
      }
      __syncthreads();
      // after the scan, edge e was flagged iff the next prefix differs
      nout = block_exclusive_scan(ef, m, s_wave);
      for (int32_t e = tid; e < m; e += kBfsThreads) {
        const int32_t nxt = e + 1 < m ? ef[e + 1] : nout;
        if (nxt != ef[e]) fout[ef[e]] = ev[e];
      }
    }
    __syncthreads();
    if (nout == 0) break;
    placed += nout;
    nin = nout;
    ++lev;
  }
  *last_lev = lev;
  return placed;
}

__global__ void __launch_bounds__(kBfsThreads) k_pseudo_peripheral(const OrderArgs* args) {
  const OrderArgs& ga = args[blockIdx.x];
  const int64_t n = ga.n;
  const int64_t* rp = ga.rp;
  const int32_t* col = ga.col;
  int32_t* level = ga.level;
  int32_t* fa = ga.fa;
  int32_t* fb = ga.fb;
  int32_t* out = ga.start;
  __shared__ int32_t s_cnt[2];
  __shared__ int32_t s_min;
  __shared__ int32_t s_wave[kBfsThreads / kWave];
  __shared__ FrontierLds f;
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < n; i += kBfsThreads) level[i] = -1;
  __syncthreads();
  const int32_t last = bfs_levels(rp, col, level, fa, fb, 0, s_cnt, &f, s_wave);
  if (tid == 0) s_min = INT32_MAX;
  __syncthreads();
  for (int64_t i = tid; i < n; i += kBfsThreads)
    if (ld_coherent(&level[i]) == last) atomicMin(&s_min, (int32_t)i);
  __syncthreads();
  if (tid == 0) *out = s_min;
}

__global__ void __launch_bounds__(kBfsThreads) k_cm_order(const OrderArgs* args) {
  const OrderArgs& ga = args[blockIdx.x];
  const int64_t n = ga.n;
  const int64_t* rp = ga.rp;
  const int32_t* col = ga.col;
  int32_t* level = ga.level;
  int32_t* key = ga.fa;   // the first search's frontiers serve as key ...
  int32_t* eoff = ga.fb;  // ... and frontier edge offsets
  int32_t *ev = ga.ev, *ei = ga.ei, *ef = ga.ef, *start = ga.start, *perm = ga.perm;
  __shared__ int32_t s_wave[kBfsThreads / kWave];
  __shared__ int32_t s_min;
  __shared__ FrontierLds f;
  __shared__ EdgeLds el;
  const int tid = threadIdx.x;
  int32_t last = 0;
  int64_t off = 0;
  if (ga.resume_off > 0) {
    // the first component is placed (by the per-level kernels)
    off = ga.resume_off;
    last = ga.resume_last;
  } else {
    for (int64_t i = tid; i < n; i += kBfsThreads) {
      level[i] = -1;
      key[i] = INT32_MAX;
    }
    __syncthreads();
    off = cm_component(rp, col, level, key, eoff, ev, ei, ef, perm, 0, *start, 0, s_wave, &f, &el,
                       &last);
  }
  // further components: the lowest unvisited node only grows
  int64_t ptr = 0;
  for (;;) {
    if (tid == 0) s_min = INT32_MAX;
    __syncthreads();
    for (; ptr < n; ptr += kBfsThreads) {
      const int64_t i = ptr + tid;
      if (i < n && ld_coherent(&level[i]) < 0) atomicMin(&s_min, (int32_t)i);
      __syncthreads();
      if (s_min != INT32_MAX) break;
      __syncthreads();
    }
    const int32_t nxt = s_min;
    __syncthreads();
    if (nxt == INT32_MAX) break;
    off += cm_component(rp, col, level, key, eoff, ev, ei, ef, perm, off, nxt, last + 1, s_wave,
                        &f, &el, &last);
  }
  if (tid == 0) {
    start[1] = last;
    *ga.maxlev = last;
  }
}


// ---------------------------------------------------------------------------
// The same two searches for large graphs, one launch per level over many
// workgroups (a single workgroup is bound by one CU's memory throughput on
// the wide levels of a large graph).  The host enqueues rounds of levels
// from a thread of its own and reads the frontier size between rounds;
// levels past the end of a search exit at once.  The results are those of
// the one-workgroup kernels (and of the sequential algorithm): levels are
// claimed with the same compare-and-swap, a child's parent is the lowest
// frontier position that reaches it, and children are placed by a scan over
// the frontier in position order, each parent's in row order.
// ---------------------------------------------------------------------------
constexpr int64_t kWideOrderMin = 32768;  // graphs of at least this many nodes
constexpr int kLvlGrid = 256;             // workgroups of a per-level launch
constexpr int kLvlThreads = 256;
constexpr int kNodeLanes = 16;            // lanes per frontier node
constexpr int kLvlChunk = kLvlThreads / kNodeLanes;  // frontier nodes per workgroup pass
constexpr int kLevelsPerRound = 32;       // levels enqueued between host reads

// Frontier state of one level (device).  The plain search keeps three (level
// t reads [t % 3], appends to [(t + 1) % 3] and clears [(t + 2) % 3]); the
// ordering keeps two (level t reads [t % 2], its last chunk writes
// [(t + 1) % 2]).
struct LevelCtl {
  int32_t nin;     // frontier size
  int32_t lev;     // level of the frontier
  int64_t placed;  // ordering: nodes placed so far (the frontier is the last nin)
};

__device__ __forceinline__ int32_t ld_ctl(const int32_t* p) { return ld_coherent(p); }

// Level t of the plain search: the frontier fin (level t) claims level t + 1
// into fout.  res[0] = last level with a non-empty frontier.
__global__ void __launch_bounds__(kLvlThreads) k_bfs_level(const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           int32_t* level, const int32_t* fin,
                                                           int32_t* fout, LevelCtl* ctl, int t,
                                                           int32_t* res) {
  // res[1] = 1 once a level came out empty: every later level exits (a
  // buffer that cycles back still holds an old frontier)
  if (ld_coherent(&res[1])) return;
  LevelCtl* cur = ctl + t % 3;
  LevelCtl* nxt = ctl + (t + 1) % 3;
  const int32_t nin = ld_ctl(&cur->nin);
  if (nin == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) res[1] = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    LevelCtl* clr = ctl + (t + 2) % 3;
    clr->nin = 0;
    res[0] = t;
  }
  const int sub = threadIdx.x % kNodeLanes;
  const int64_t stride = (int64_t)gridDim.x * (kLvlThreads / kNodeLanes);
  for (int64_t i = ((int64_t)blockIdx.x * kLvlThreads + threadIdx.x) / kNodeLanes; i < nin;
       i += stride) {
    const int32_t u = fin[i];
    const int64_t e1 = rp[u + 1];
    for (int64_t e = rp[u] + sub; e < e1; e += kNodeLanes) {
      const int32_t v = col[e];
      if (ld_coherent(&level[v]) < 0 && atomicCAS(&level[v], -1, t + 1) == -1)
        fout[atomicAdd(&nxt->nin, 1)] = v;
    }
  }
}

// Lowest node id on the last level (one workgroup): the pseudo-peripheral
// start.  Level t's frontier is in fa for even t, fb for odd t.
__global__ void __launch_bounds__(kLvlThreads) k_frontier_min(const int32_t* fa, const int32_t* fb,
                                                              const LevelCtl* ctl,
                                                              const int32_t* res, int32_t* out) {
  __shared__ int32_t s_min;
  if (threadIdx.x == 0) s_min = INT32_MAX;
  __syncthreads();
  const int32_t t = res[0];
  const int32_t nin = ctl[t % 3].nin;
  const int32_t* f = (t & 1) ? fb : fa;
  int32_t m = INT32_MAX;
  for (int32_t i = threadIdx.x; i < nin; i += kLvlThreads) m = min(m, f[i]);
  atomicMin(&s_min, m);
  __syncthreads();
  if (threadIdx.x == 0) *out = s_min;
}

__global__ void k_fill_i32(int64_t n, int32_t* a, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Search starts: plain search from node 0, ordering from the
// pseudo-peripheral node.
__global__ void k_bfs_start(int32_t* level, int32_t* fa, LevelCtl* ctl, int32_t* res) {
  level[0] = 0;
  fa[0] = 0;
  ctl[0] = LevelCtl{1, 0, 1};
  ctl[1] = LevelCtl{0, 0, 0};
  ctl[2] = LevelCtl{0, 0, 0};
  res[0] = 0;
  res[1] = 0;
  res[2] = 0;  // the ordering's ticket (k_cm_count)
}

__global__ void k_store_i32(int32_t* p, int32_t v) { *p = v; }

__global__ void k_cm_start(int32_t* level, int32_t* perm, const int32_t* start, LevelCtl* ctl) {
  const int32_t v = *start;
  level[v] = 0;
  perm[0] = v;
  ctl[0] = LevelCtl{1, 0, 1};
  ctl[1] = LevelCtl{0, 0, 0};
}

// Ordering, level t, step 1: every frontier node claims its unvisited
// neighbours for the next level and lowers their key to its position.
__global__ void __launch_bounds__(kLvlThreads) k_cm_claim(const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          int32_t* level, int32_t* key,
                                                          const int32_t* perm, const LevelCtl* ctl,
                                                          int t) {
  const LevelCtl* cur = ctl + (t & 1);
  const int32_t nin = ld_ctl(&cur->nin);
  if (nin == 0) return;
  const int32_t lev = cur->lev;
  const int32_t* fin = perm + (cur->placed - nin);
  const int sub = threadIdx.x % kNodeLanes;
  const int64_t stride = (int64_t)gridDim.x * (kLvlThreads / kNodeLanes);
  for (int64_t i = ((int64_t)blockIdx.x * kLvlThreads + threadIdx.x) / kNodeLanes; i < nin;
       i += stride) {
    const int32_t u = fin[i];
    const int64_t e1 = rp[u + 1];
    for (int64_t e = rp[u] + sub; e < e1; e += kNodeLanes) {
      const int32_t v = col[e];
      int32_t lv = ld_coherent(&level[v]);
      if (lv < 0) {
        const int32_t old = atomicCAS(&level[v], -1, lev + 1);
        lv = old < 0 ? lev + 1 : old;
      }
      if (lv == lev + 1) atomicMin(&key[v], (int32_t)i);
    }
  }
}

// Children of frontier position i among its row's edges, e in row order:
// flag = the neighbour is on the next level and i is its parent.
__device__ __forceinline__ bool cm_child(const int32_t* level, const int32_t* key, int32_t v,
                                         int32_t lev, int32_t i) {
  return ld_coherent(&level[v]) == lev + 1 && ld_coherent(&key[v]) == i;
}

// Step 2: children per frontier node, and per chunk of kLvlChunk positions
// (one chunk per workgroup pass, kNodeLanes lanes per node); then, in the
// workgroup that finishes last (a ticket taken after its counts are
// published), the exclusive scan of the chunk counts in place and the next
// level's state (its frontier is the children just counted).  The ticket
// returns to 0 for the next level.
__global__ void __launch_bounds__(kLvlThreads) k_cm_count(const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const int32_t* level, const int32_t* key,
                                                          const int32_t* perm, int32_t* cnt,
                                                          int32_t* partial, LevelCtl* ctl,
                                                          int32_t* ticket, int t) {
  const LevelCtl* cur = ctl + (t & 1);
  LevelCtl* nxt = ctl + ((t + 1) & 1);
  const int32_t nin = ld_ctl(&cur->nin);
  if (nin == 0) {  // past the end: the empty state carries forward
    if (blockIdx.x == 0 && threadIdx.x == 0) *nxt = *cur;
    return;
  }
  const int32_t lev = cur->lev;
  const int32_t* fin = perm + (cur->placed - nin);
  __shared__ int32_t s_k[kLvlChunk];
  const int sub = threadIdx.x % kNodeLanes, slot = threadIdx.x / kNodeLanes;
  const int32_t nchunks = (nin + kLvlChunk - 1) / kLvlChunk;
  for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int32_t i = c * kLvlChunk + slot;
    int32_t k = 0;
    if (i < nin) {
      const int32_t u = fin[i];
      const int64_t e1 = rp[u + 1];
      for (int64_t e = rp[u] + sub; e < e1; e += kNodeLanes) k += cm_child(level, key, col[e], lev, i);
    }
    for (int o = kNodeLanes / 2; o > 0; o >>= 1) k += __shfl_xor(k, o, kNodeLanes);
    if (sub == 0) {
      if (i < nin) cnt[i] = k;
      s_k[slot] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t x = 0;
      for (int q = 0; q < kLvlChunk; ++q) x += s_k[q];
      partial[c] = x;
    }
    __syncthreads();
  }
  __shared__ int32_t s_last;
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's counts before its ticket
    s_last = atomicAdd(ticket, 1) == (int32_t)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  __shared__ int32_t s_wave[kLvlThreads / kWave];
  const int32_t total = block_exclusive_scan<kLvlThreads, true>(partial, nchunks, s_wave);
  if (threadIdx.x == 0) {
    *nxt = LevelCtl{total, cur->lev + 1, cur->placed + total};
    *ticket = 0;
  }
}

// Step 3: place every child: a chunk starts at its scanned offset, a node at
// the counts of the chunk's nodes before it, and a node's children keep row
// order.
__global__ void __launch_bounds__(kLvlThreads) k_cm_place(const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const int32_t* level, const int32_t* key,
                                                          int32_t* perm, const int32_t* cnt,
                                                          const int32_t* partial,
                                                          const LevelCtl* ctl, int t) {
  const LevelCtl* cur = ctl + (t & 1);
  const int32_t nin = ld_ctl(&cur->nin);
  if (nin == 0) return;
  const int32_t lev = cur->lev;
  const int64_t placed = cur->placed;
  const int32_t* fin = perm + (placed - nin);
  int32_t* fout = perm + placed;
  __shared__ int32_t s_k[kLvlChunk];
  const int tid = threadIdx.x, lane = tid % kWave;
  const int sub = tid % kNodeLanes, slot = tid / kNodeLanes, grp = lane / kNodeLanes;
  const int32_t nchunks = (nin + kLvlChunk - 1) / kLvlChunk;
  for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int32_t i = c * kLvlChunk + slot;
    const bool live = i < nin;
    if (sub == 0) s_k[slot] = live ? cnt[i] : 0;
    __syncthreads();
    int32_t pos = partial[c];
    for (int q = 0; q < slot; ++q) pos += s_k[q];
    int64_t e0 = 0, e1 = 0;
    if (live) {
      const int32_t u = fin[i];
      e0 = rp[u];
      e1 = rp[u + 1];
    }
    for (int64_t e = e0; e < e1; e += kNodeLanes) {
      const int64_t my = e + sub;
      int32_t v = 0;
      bool f = false;
      if (my < e1) {
        v = col[my];
        f = cm_child(level, key, v, lev, i);
      }
      const uint64_t m = (__ballot(f) >> (grp * kNodeLanes)) & ((1ull << kNodeLanes) - 1);
      if (f) fout[pos + __popcll(m & ((1ull << sub) - 1))] = v;
      pos += __popcll(m);
    }
    __syncthreads();
  }
}

// lev_s[i'] = breadth-first level of solver row i'
__global__ void k_gather_level(int64_t n, const int32_t* perm, const int32_t* level,
                               int32_t* lev_s) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) lev_s[i] = level[perm[i]];
}

__global__ void k_iota(int64_t n, int32_t* a) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_invert_perm(int64_t n, const int32_t* perm, int32_t* iperm) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) iperm[perm[i]] = (int32_t)i;
}

// perm (solver index -> user index), iperm (user -> solver).
// Scratch and arguments of a graph's searches (graphs of at most kDenseMaxN
// nodes take the identity order and need none).
size_t order_scratch_bytes(int64_t n, int64_t nnz) {
  if (n <= kDenseMaxN) return 0;
  return Arena::round((n + 2) * 4) * 3 + Arena::round((nnz + 2) * 4) * 3 + Arena::round(64);
}

size_t order_args_bytes(int G) {
  return Arena::round(sizeof(OrderArgs) * (G > 0 ? G : 1)) + Arena::round(4 * (size_t)G + 4);
}

static int order_alloc(GraphOps* g, DevHeap& heap, hipStream_t s) {
  const int64_t n = g->n;
  g->ord = OrderArgs{};
  g->ord.n = n;
  g->ord.perm = g->perm;
  if (n <= kDenseMaxN) return ME_OK;
  const int64_t nnz = g->nnz_w;
  const size_t bytes = order_scratch_bytes(n, nnz);
  ME_TRY_STATUS(heap.alloc(&g->ord_mem, bytes, s));
  Arena a{(char*)g->ord_mem, bytes, 0};
  g->ord.rp = g->w_rp;
  g->ord.col = g->w_col;
  g->ord.level = a.take<int32_t>(n + 2);
  g->ord.fa = a.take<int32_t>(n + 2);
  g->ord.fb = a.take<int32_t>(n + 2);
  g->ord.ev = a.take<int32_t>(nnz + 2);
  g->ord.ei = a.take<int32_t>(nnz + 2);
  g->ord.ef = a.take<int32_t>(nnz + 2);
  g->ord.start = a.take<int32_t>(16);
  return ME_OK;
}

static bool wide_graph(const GraphOps* g) { return g->ord_mem && g->n >= kWideOrderMin; }

// Both searches of one large graph by per-level launches on s (see the
// per-level kernels); dargs: the graph's arguments on the device.
static int wide_order(GraphOps* g, OrderArgs* dargs, hipStream_t s) {
  const int64_t n = g->n;
  const OrderArgs& a = g->ord;
  LevelCtl* ctl = reinterpret_cast<LevelCtl*>(a.ei);  // 3 plain-search + 2 ordering states
  int32_t* res = reinterpret_cast<int32_t*>(ctl + 5);
  int32_t* partial = a.ev;  // one count per frontier chunk
  int32_t* key = a.fa;
  int32_t* cnt = a.fb;
  const int64_t nb = ceil_div(n, kBlock);
  // plain search from node 0: its last level gives the start
  k_fill_i32<<<nb, kBlock, 0, s>>>(n, a.level, -1);
  k_bfs_start<<<1, 1, 0, s>>>(a.level, a.fa, ctl, res);
  int64_t t = 0;
  for (;;) {
    for (int q = 0; q < kLevelsPerRound; ++q, ++t) {
      const bool odd = t & 1;
      k_bfs_level<<<kLvlGrid, kLvlThreads, 0, s>>>(a.rp, a.col, a.level, odd ? a.fb : a.fa,
                                                  odd ? a.fa : a.fb, ctl, (int)t, res);
    }
    int32_t h[2] = {0, 0};
    ME_TRY(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
    if (h[1]) break;
    if (t > n + kLevelsPerRound) return ME_ERR_HIP;  // a search has at most n levels
  }
  k_frontier_min<<<1, kLvlThreads, 0, s>>>(a.fa, a.fb, ctl, res, a.start);
  // Cuthill-McKee order of the start's component
  LevelCtl* cc = ctl + 3;
  k_fill_i32<<<nb, kBlock, 0, s>>>(n, a.level, -1);
  k_fill_i32<<<nb, kBlock, 0, s>>>(n, key, INT32_MAX);
  k_cm_start<<<1, 1, 0, s>>>(a.level, a.perm, a.start, cc);
  LevelCtl h{};
  t = 0;
  for (;;) {
    for (int q = 0; q < kLevelsPerRound; ++q, ++t) {
      k_cm_claim<<<kLvlGrid, kLvlThreads, 0, s>>>(a.rp, a.col, a.level, key, a.perm, cc, (int)t);
      k_cm_count<<<kLvlGrid, kLvlThreads, 0, s>>>(a.rp, a.col, a.level, key, a.perm, cnt, partial,
                                                 cc, res + 2, (int)t);
      k_cm_place<<<kLvlGrid, kLvlThreads, 0, s>>>(a.rp, a.col, a.level, key, a.perm, cnt, partial,
                                                 cc, (int)t);
    }
    ME_TRY(hipMemcpyAsync(&h, cc + (t & 1), sizeof(h), hipMemcpyDeviceToHost, s));
    ME_TRY(hipStreamSynchronize(s));
    if (h.nin == 0) break;
    if (t > n + kLevelsPerRound) return ME_ERR_HIP;
  }
  if (h.placed < n) {
    // further components: the one-workgroup kernel continues from here
    OrderArgs r = a;
    r.resume_off = h.placed;
    r.resume_last = h.lev - 1;
    ME_TRY(hipMemcpyAsync(dargs, &r, sizeof(OrderArgs), hipMemcpyHostToDevice, s));
    k_cm_order<<<1, kBfsThreads, 0, s>>>(dargs);
    ME_TRY(hipStreamSynchronize(s));  // r is read by the copy
  } else {
    k_store_i32<<<1, 1, 0, s>>>(a.maxlev, h.lev - 1);
  }
  return ME_OK;
}

// The pseudo-peripheral starts and the Cuthill-McKee orders of G graphs
// (one workgroup per graph in each launch; graphs of kWideOrderMin nodes or
// more by per-level launches driven from a host thread of the job), then
// iperm and the solver-order levels of each.  job->args receives the
// argument array (device) that order_finish releases.
int order_launch(GraphOps* const* gs, int G, DevHeap& heap, hipStream_t s, OrderJob* job) {
  job->args = nullptr;
  job->status = ME_OK;
  std::vector<OrderArgs> host;
  std::vector<GraphOps*> wide;
  for (int i = 0; i < G; ++i)
    if (gs[i]->ord_mem && !wide_graph(gs[i])) host.push_back(gs[i]->ord);
  const int m = (int)host.size();
  for (int i = 0; i < G; ++i)
    if (wide_graph(gs[i])) {
      host.push_back(gs[i]->ord);
      wide.push_back(gs[i]);
    }
  const int mt = (int)host.size();
  ME_TRY_STATUS(heap.alloc(&job->args, order_args_bytes(G), s));
  OrderArgs* dargs = (OrderArgs*)job->args;
  int32_t* maxlev =
      (int32_t*)((char*)job->args + Arena::round(sizeof(OrderArgs) * (G > 0 ? G : 1)));
  for (int q = 0; q < mt; ++q) host[q].maxlev = maxlev + q;
  for (size_t w = 0; w < wide.size(); ++w) wide[w]->ord.maxlev = maxlev + m + w;
  if (mt > 0)
    ME_TRY(hipMemcpyAsync(dargs, host.data(), sizeof(OrderArgs) * mt, hipMemcpyHostToDevice, s));
  if (m > 0) {
    k_pseudo_peripheral<<<m, kBfsThreads, 0, s>>>(dargs);
    k_cm_order<<<m, kBfsThreads, 0, s>>>(dargs);
  }
  for (int i = 0; i < G; ++i) {
    GraphOps* g = gs[i];
    const int64_t n = g->n;
    if (!g->ord_mem) {
      k_iota<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm);
      k_iota<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->iperm);
      continue;
    }
    if (wide_graph(g)) continue;
    k_invert_perm<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->iperm);
    k_gather_level<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->ord.level, g->lev_s);
  }
  if (!wide.empty()) {
    // the wide searches wait on the host between rounds of levels: a thread
    // of their own keeps the caller free to enqueue other work meanwhile
    int dev = 0;
    ME_TRY(hipGetDevice(&dev));
    const hipError_t ready = hipStreamSynchronize(s);  // the argument copy has landed
    if (ready != hipSuccess) return ME_ERR_HIP;
    job->th = std::thread([job, wide, dargs, m, s, dev]() {
      if (hipSetDevice(dev) != hipSuccess) {
        job->status = ME_ERR_HIP;
        return;
      }
      for (size_t w = 0; w < wide.size(); ++w) {
        GraphOps* g = wide[w];
        const int st = wide_order(g, dargs + m + w, s);
        if (st < 0) {
          job->status = st;
          return;
        }
        const int64_t n = g->n;
        k_invert_perm<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->iperm);
        k_gather_level<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->ord.level,
                                                              g->lev_s);
      }
    });
  }
  return ME_OK;
}

// Waits for the searches, reads the deepest levels, frees their scratch.
int order_finish(GraphOps* const* gs, int G, DevHeap& heap, hipStream_t s, OrderJob* job) {
  if (job->th.joinable()) job->th.join();
  std::vector<int32_t> lev(G > 0 ? G : 1, 0);
  int narrow = 0, nwide = 0;
  for (int i = 0; i < G; ++i) {
    if (!gs[i]->ord_mem) continue;
    if (wide_graph(gs[i])) ++nwide; else ++narrow;
  }
  const size_t off = Arena::round(sizeof(OrderArgs) * (G > 0 ? G : 1));
  if (narrow + nwide > 0 && job->args)
    ME_TRY(hipMemcpyAsync(lev.data(), (char*)job->args + off, 4 * (narrow + nwide),
                          hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (job->status < 0) return job->status;
  int qn = 0, qw = narrow;
  for (int i = 0; i < G; ++i) {
    GraphOps* g = gs[i];
    if (g->ord_mem) g->max_level = wide_graph(g) ? lev[qw++] : lev[qn++];
    else g->max_level = 0;
  }
  for (int i = 0; i < G; ++i) {
    heap.release(gs[i]->ord_mem, s);  // the searches are complete (synchronised above)
    gs[i]->ord_mem = nullptr;
  }
  heap.release(job->args, s);
  job->args = nullptr;
  return ME_OK;
}

// A side stream for one graph's searches: they occupy one workgroup, so the
// two-hop construction and the connectivity pass of the main stream run
// beside them.  The destructor waits for it after an early return.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ready = nullptr;
  ~SideStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    if (ready) (void)hipEventDestroy(ready);
  }
  int fork(hipStream_t main) {
    ME_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ME_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    ME_TRY(hipEventRecord(ready, main));
    ME_TRY(hipStreamWaitEvent(s, ready, 0));
    return ME_OK;
  }
};

// ---------------------------------------------------------------------------
// Per-node scalars
// ---------------------------------------------------------------------------

__global__ void k_invt(int64_t n, const int32_t* tcnt, double* invt, float* invt32) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t t = tcnt[i];
  double v = t > 0 ? 1.0 / (double)t : 0.0;
  invt[i] = v;
  invt32[i] = (float)v;
}

__device__ inline void atomic_max_pos_double(unsigned long long* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// Q_ii = sum_{j in T_i} (1/T_i + 1/T_j) and the eq. (mu) denominator
// den_i = Q_ii - sum_{j != i} Q_ij with Q_ij = -(1/T_i + 1/T_j).
__global__ void k_qdiag(int64_t n, const int64_t* t_rp, const int32_t* t_col, const double* invt,
                        double* qdiag, double* qinv, float* qinv32,
                        unsigned long long* maxden_bits) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double den = 0.0;
  if (i < n) {
    const double ti = invt[i];
    double qii = 0.0, off = 0.0;
    for (int64_t t = t_rp[i]; t < t_rp[i + 1]; ++t) {
      double q = ti + invt[t_col[t]];
      qii += q;
      off -= q;
    }
    qdiag[i] = qii;
    qinv[i] = qii > 0.0 ? 1.0 / qii : 0.0;
    qinv32[i] = (float)qinv[i];
    den = qii - off;
  }
  for (int o = 32; o > 0; o >>= 1) den = fmax(den, __shfl_xor(den, o));
  if ((threadIdx.x & (kWave - 1)) == 0) atomic_max_pos_double(maxden_bits, den);
}

// Merged difference-form operator rows in the solver order: solver row i'
// is user row o = perm[i'], entries [W columns | T columns] in the user
// row's order, columns renumbered by iperm.
// W and T row lengths of the rows in solver order
__global__ void k_row_len_perm(int64_t n, const int32_t* perm, const int64_t* w_rp,
                               const int64_t* t_rp, int32_t* wlen, int32_t* tlen) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t o = perm[i];
  wlen[i] = (int32_t)(w_rp[o + 1] - w_rp[o]);
  tlen[i] = (int32_t)(t_rp[o + 1] - t_rp[o]);
}

// The operator in solver order as two CSR blocks in one array: the W entries
// of all rows ([a_rp[i], a_rp[i+1]), weight w_ij), then the T entries of all
// rows ([a_tp[i], a_tp[i+1]), stored weight 1/T_i + 1/T_j).  A solve that
// reads one kind of entry reads whole cache lines of it.
// Packed preconditioner entry: column - row in the low 16 bits (two's
// complement, clamped: only used when every offset fits), FP16 weight above.
__device__ __forceinline__ uint32_t pack_entry(int64_t row, int32_t col, double w) {
  int64_t d = (int64_t)col - row;
  d = d > 32767 ? 32767 : (d < -32768 ? -32768 : d);
  const _Float16 h = (_Float16)(float)w;
  return (uint32_t)(uint16_t)(int16_t)d | ((uint32_t)__builtin_bit_cast(uint16_t, h) << 16);
}

__global__ void __launch_bounds__(kBlock) k_pack_perm(
    int64_t n, int64_t nnz_w, const int32_t* perm, const int32_t* iperm, const int64_t* woff,
    const int64_t* toff, const int64_t* w_rp, const int32_t* w_col, const double* w_val,
    const int64_t* t_rp, const int32_t* t_col, const int32_t* t_cnt, const double* invt,
    int32_t* a_rp, int32_t* a_tp, int32_t* a_col, double* a_w, float* a_w32, uint32_t* a_pk,
    uint32_t* a_tq, int* max_offset, int* max_tcnt, int* wide_w) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t far = 0;  // largest |column - row| of this row
  int32_t tmax = 0;  // largest T_j over the row's two-hop columns
  int wide = 0;      // W weights beyond FP16's finite range (bit 0), beyond FP32's (bit 1)
  if (i <= n) {
    const int64_t ws = woff[i], ts = nnz_w + toff[i];
    a_rp[i] = (int32_t)ws;
    a_tp[i] = (int32_t)ts;
  }
  if (i < n) {
    const int64_t ws = woff[i], ts = nnz_w + toff[i];
    const int32_t o = perm[i];
    const int64_t nw = w_rp[o + 1] - w_rp[o];
    for (int64_t t = 0; t < nw; ++t) {
      const int32_t c = iperm[w_col[w_rp[o] + t]];
      const double v = w_val[w_rp[o] + t];
      a_col[ws + t] = c;
      a_w[ws + t] = v;
      a_w32[ws + t] = (float)v;
      a_pk[ws + t] = pack_entry(i, c, v);
      wide |= (!(fabsf((float)(_Float16)(float)v) <= 65504.0f) ? 1 : 0) |
              (!(fabsf((float)v) <= 3.4028234663852886e38f) ? 2 : 0);
      far = max(far, (int64_t)llabs((int64_t)c - i));
    }
    // T entries: weight 1/T_i + 1/T_j of the two-hop term (eq. (Q), reading R1)
    const int64_t tb = t_rp[o], te = t_rp[o + 1];
    for (int64_t t = tb; t < te; ++t) {
      const int64_t k = ts + (t - tb);
      const int32_t c = iperm[t_col[t]];
      const double q = invt[o] + invt[t_col[t]];
      const int32_t tj = t_cnt[t_col[t]];
      a_col[k] = c;
      a_w[k] = q;
      a_w32[k] = (float)q;
      a_pk[k] = pack_entry(i, c, q);
      int64_t dd = (int64_t)c - i;
      dd = dd > 32767 ? 32767 : (dd < -32768 ? -32768 : dd);
      a_tq[k - nnz_w] = (uint32_t)(uint16_t)(int16_t)dd | ((uint32_t)(tj & 0xffff) << 16);
      far = max(far, (int64_t)llabs((int64_t)c - i));
      tmax = max(tmax, tj);
    }
  }
  int32_t f = far > INT32_MAX ? INT32_MAX : (int32_t)far;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    f = max(f, __shfl_xor(f, o));
    tmax = max(tmax, __shfl_xor(tmax, o));
    wide |= __shfl_xor(wide, o);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(max_offset, f);
    atomicMax(max_tcnt, tmax);
    if (wide) atomicOr(wide_w, wide);
  }
}

// Halo of one tile of kHaloRows consecutive solver rows over one entry range
// (row pointers rp: a_rp for W, a_tp for T; the tile's entries are
// contiguous): its distinct columns, sorted (bitonic sort in LDS, then a
// block scan of first occurrences), written at the tile's first entry
// position; each entry's slot in that list (binary search) with the FP16
// weight of the packed entry.  Entries keep their order, so a product over
// the halo visits them exactly as the packed product does.  A tile with more
// than kHaloMaxE entries sets *fail (the range then runs without halos).
constexpr int kHaloBuildThreads = 256;
__global__ void __launch_bounds__(kHaloBuildThreads) k_halo_build(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ a_col,
    const uint32_t* __restrict__ a_pk, uint32_t* __restrict__ h_pk, int32_t* __restrict__ h_list,
    int32_t* __restrict__ h_cnt, int* hmax, int* fail) {
  __shared__ int32_t key[kHaloMaxE];
  __shared__ int32_t wsum[kHaloBuildThreads / kWave];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kHaloRows;
  const int64_t r1 = r0 + kHaloRows < n ? r0 + kHaloRows : n;
  const int32_t e0 = rp[r0], e1 = rp[r1];
  const int E = e1 - e0;
  if (E > kHaloMaxE) {
    if (tid == 0) {
      h_cnt[blockIdx.x] = 0;
      atomicOr(fail, 1);
    }
    return;
  }
  int P = 1;
  while (P < E) P <<= 1;
  for (int i = tid; i < P; i += kHaloBuildThreads) key[i] = i < E ? a_col[e0 + i] : INT32_MAX;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P / 2; i += kHaloBuildThreads) {
        const int lo = 2 * i - (i & (stride - 1));  // pair (lo, lo + stride)
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int32_t a = key[lo], b = key[hi];
        if ((a > b) == up) {
          key[lo] = b;
          key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  // first occurrences, compacted in order (chunks of kHaloBuildThreads)
  int32_t base = 0;
  for (int c0 = 0; c0 < E; c0 += kHaloBuildThreads) {
    const int i = c0 + tid;
    const bool first = i < E && (i == 0 || key[i] != key[i - 1]);
    const int32_t v = i < E ? key[i] : 0;
    const unsigned long long m = __ballot(first);
    const int lane = tid % kWave, wv = tid / kWave;
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int q = 0; q < wv; ++q) off += wsum[q];
    int all = 0;
    for (int q = 0; q < kHaloBuildThreads / kWave; ++q) all += wsum[q];
    __syncthreads();  // every read of key[i - 1] and wsum is done
    if (first) key[base + off + before] = v;  // base + off + before <= i
    __syncthreads();
    base += all;
  }
  const int H = base;
  for (int j = tid; j < H; j += kHaloBuildThreads) h_list[e0 + j] = key[j];
  for (int i = tid; i < E; i += kHaloBuildThreads) {
    const int32_t c = a_col[e0 + i];
    int lo = 0, hi = H - 1;  // key[0..H) sorted, distinct; c is among them
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (key[mid] < c) lo = mid + 1; else hi = mid;
    }
    h_pk[e0 + i] = (uint32_t)lo | (a_pk[e0 + i] & 0xffff0000u);
  }
  if (tid == 0) {
    h_cnt[blockIdx.x] = H;
    atomicMax(hmax, H);
  }
}

// dst[i'] = src[perm[i']] for a double array and its FP32 copy
__global__ void k_gather_node(int64_t n, const int32_t* perm, const double* src, double* dst,
                              float* dst32) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src[perm[i]];
  dst[i] = v;
  if (dst32) dst32[i] = (float)v;
}

// r_i = sum_{j != i} |A_ij| = d_i + mu Q_ii; log r partial sums (fixed order).
__global__ void __launch_bounds__(kBlock) k_radius(int64_t n, const double* d, const double* qdiag,
                                                   double mu, double* r, double* partial) {
  __shared__ double sh[kBlock];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double ri = d[i] + mu * qdiag[i];
    r[i] = ri;
    acc += log(ri);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// b_i = r_i / (prod r)^(1/N) through logs; Jacobi 1 / A_ii, A_ii = d_i - mu Q_ii + eps.
__global__ void k_bvec(int64_t n, const double* r, const double* d, const double* qdiag,
                       const double* partial, int nparts, double mu, double eps, double* b,
                       float* b32, double* dinv, float* dinv32, double* pdinv, float* pdinv32,
                       unsigned long long* maxdiag_bits, unsigned long long* maxratio_bits,
                       unsigned long long* maxpratio_bits) {
  double sum = 0.0;
  for (int q = 0; q < nparts; ++q) sum += partial[q];
  const double mean = sum / (double)n;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double diag = 0.0, ratio = 0.0, pratio = 0.0;
  if (i < n) {
    double bi = exp(log(r[i]) - mean);
    b[i] = bi;
    b32[i] = (float)bi;
    diag = d[i] - mu * qdiag[i] + eps;
    dinv[i] = 1.0 / diag;
    dinv32[i] = (float)(1.0 / diag);
    ratio = (diag + r[i]) / diag;  // Gershgorin right end of row i of diag(A)^-1 A
    const double pd = d[i] + eps;  // L + eps I: diagonal d_i + eps, radius d_i
    pdinv[i] = 1.0 / pd;
    pdinv32[i] = (float)(1.0 / pd);
    pratio = (pd + d[i]) / pd;
  }
  for (int o = 32; o > 0; o >>= 1) {
    diag = fmax(diag, __shfl_xor(diag, o));
    ratio = fmax(ratio, __shfl_xor(ratio, o));
    pratio = fmax(pratio, __shfl_xor(pratio, o));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomic_max_pos_double(maxdiag_bits, diag);
    atomic_max_pos_double(maxratio_bits, ratio);
    atomic_max_pos_double(maxpratio_bits, pratio);
  }
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------

template <typename T>
static int read_scalar(const T* dev, T* host, hipStream_t s) {
  ME_TRY(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  return ME_OK;
}

// Everything up to eps: validation, degrees, T, Q, the locality order and
// the packed operator.  g->needs_eps tells whether eps = lambda_2(Q) must be
// computed (connected two-hop graph); otherwise eps = 0 (ME_WARN_EPS_ZERO).
static int build_pre_a_impl(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s,
                            GraphOps* g, SideStream* side, OrderJob* job);

int build_pre(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g) {
  SideStream side;
  OrderJob job;
  struct Pending {  // waits for the searches and releases their arguments if a step fails
    OrderJob& job;
    DevHeap& heap;
    ~Pending() {
      if (job.th.joinable()) job.th.join();
      if (job.args) {
        (void)hipDeviceSynchronize();
        heap.release(job.args, nullptr);
      }
    }
  } pending{job, heap};
  ME_TRY_STATUS(build_pre_a_impl(W, o, heap, s, g, &side, &job));
  const int st = order_finish(&g, 1, heap, side.s, &job);
  if (st < 0) return st;
  return build_pre_b(g, s);
}

int build_pre_a(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g) {
  return build_pre_a_impl(W, o, heap, s, g, nullptr, nullptr);
}

size_t build_mem1_bytes(int64_t n, int64_t nnz) {
  const int64_t ne = nnz > 0 ? nnz : 1;  // W's arrays hold one entry at least
  size_t b1 = 0;
  b1 += Arena::round((n + 1) * 8) + Arena::round(ne * 4) + Arena::round(ne * 8);  // W
  b1 += Arena::round((n + 1) * 8) + Arena::round(n * 4);                            // t_rp, t_cnt
  b1 += 9 * Arena::round(n * 8) + 5 * Arena::round(n * 4);                          // per node
  b1 += 2 * Arena::round((n + 1) * 4);                                              // a_rp, a_tp
  b1 += 3 * Arena::round(n * 4) + 5 * Arena::round(n * 8) + 4 * Arena::round(n * 4);  // solver order
  b1 += 2 * Arena::round((n + 1) * 8);                                              // offsets
  b1 += 2 * Arena::round((n / kHaloRows + 1) * 4);                                  // halo sizes
  b1 += Arena::round(sizeof(int) * 64);
  return b1;
}

size_t build_mem2_bytes(int64_t nnz, int64_t nnz_t) {
  return 2 * Arena::round(nnz_t * 4 + 4) + Arena::round((nnz + nnz_t) * 4 + 4) +
         Arena::round((nnz + nnz_t) * 8 + 8) + 4 * Arena::round((nnz + nnz_t) * 4 + 4);
}

// Bitmaps of the two-hop rows with more than the LDS hash's candidates.
static int64_t twohop_big_grid(int64_t nbig) { return std::min<int64_t>(nbig, 128); }
size_t twohop_bitmap_bytes(int64_t n) {
  return (size_t)twohop_big_grid(n) * ((n + 31) / 32) * 4;
}

size_t build_bytes_bound(int64_t n, int64_t nnz, int64_t nnz_t_max) {
  return DevHeap::round(build_mem1_bytes(n, nnz)) + DevHeap::round(build_mem2_bytes(nnz, nnz_t_max)) +
         DevHeap::round(order_scratch_bytes(n, nnz)) + DevHeap::round(order_args_bytes(1)) +
         DevHeap::round(twohop_bitmap_bytes(n));
}

// Largest two-hop pattern W's degrees allow: T_i lies in the union over
// k in N(i) of N(k) minus i, so nnz(T) <= sum_k d_k (d_k - 1), and
// nnz(T) <= n (n - 1) - nnz(W).  Reads the row pointers (device) to the host.
int two_hop_bound(const me_csr* W, hipStream_t s, int64_t* bound) {
  *bound = 0;
  const int64_t n = W->n, nnz = W->nnz;
  if (n < 1 || nnz < 0 || !W->rowptr) return ME_ERR_INVALID_ARG;
  std::vector<int64_t> rp((size_t)n + 1);
  ME_TRY(hipMemcpyAsync(rp.data(), W->rowptr, (n + 1) * 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  if (rp[0] != 0 || rp[n] != nnz) return ME_ERR_INVALID_ARG;
  __int128 sum = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = rp[i + 1] - rp[i];
    if (d < 0) return ME_ERR_INVALID_ARG;
    if (d > 0) sum += (__int128)d * (d - 1);
  }
  const __int128 full = (__int128)n * (n - 1) - nnz;
  __int128 b = sum < full ? sum : full;
  if (b < 0) b = 0;
  *bound = b > (__int128)INT64_MAX ? INT64_MAX : (int64_t)b;
  return ME_OK;
}

// side != null: the graph's searches start on a side stream right after
// validation and run beside the two-hop construction.
static int build_pre_a_impl(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s,
                            GraphOps* g, SideStream* side, OrderJob* job) {
  const int64_t n = W->n, nnz = W->nnz;
  if (n < 1 || nnz < 0 || !W->rowptr || (nnz > 0 && (!W->col || !W->val)))
    return ME_ERR_INVALID_ARG;
  if (n >= (int64_t)INT32_MAX) return ME_ERR_TOO_LARGE;
  ME_TRY(hipGetDevice(&g->device));
  g->n = n;
  g->nnz_w = nnz;

  g->in_region = heap.region();
  // ---- allocation 1: W copy, per-node arrays, scratch of the count phase
  const size_t b1 = build_mem1_bytes(n, nnz);
  void* mem1 = nullptr;
  ME_TRY_STATUS(heap.alloc(&mem1, b1, s));
  g->mem = mem1;
  g->mem_bytes = b1;
  Arena ar{(char*)mem1, b1, 0};
  g->w_rp = ar.take<int64_t>(n + 1);
  g->w_col = ar.take<int32_t>(nnz > 0 ? nnz : 1);
  g->w_val = ar.take<double>(nnz > 0 ? nnz : 1);
  g->t_rp = ar.take<int64_t>(n + 1);
  g->t_cnt = ar.take<int32_t>(n);
  g->d = ar.take<double>(n);
  g->qdiag = ar.take<double>(n);
  g->r = ar.take<double>(n);
  g->b = ar.take<double>(n);
  g->dinv = ar.take<double>(n);
  g->invt = ar.take<double>(n);
  g->qinv = ar.take<double>(n);
  g->pdinv = ar.take<double>(n);
  g->pdinv32 = ar.take<float>(n);
  double* scratch_d = ar.take<double>(n);  // tile sums / partials / parents
  g->b32 = ar.take<float>(n);
  g->dinv32 = ar.take<float>(n);
  g->invt32 = ar.take<float>(n);
  g->qinv32 = ar.take<float>(n);
  g->a_rp = ar.take<int32_t>(n + 1);
  g->a_tp = ar.take<int32_t>(n + 1);
  g->perm = ar.take<int32_t>(n);
  g->lev_s = ar.take<int32_t>(n);
  g->iperm = ar.take<int32_t>(n);
  g->qinv_s = ar.take<double>(n);
  g->b_s = ar.take<double>(n);
  g->dinv_s = ar.take<double>(n);
  g->pdinv_s = ar.take<double>(n);
  g->invt_s = ar.take<double>(n);
  g->qinv32_s = ar.take<float>(n);
  g->b32_s = ar.take<float>(n);
  g->dinv32_s = ar.take<float>(n);
  g->pdinv32_s = ar.take<float>(n);
  g->woff = ar.take<int64_t>(n + 1);
  g->toff = ar.take<int64_t>(n + 1);
  g->h_cnt_w = ar.take<int32_t>(n / kHaloRows + 1);
  g->h_cnt_t = ar.take<int32_t>(n / kHaloRows + 1);

  int* dflags = ar.take<int>(64);
  if (!dflags) return ME_ERR_HIP;
  g->scratch_d = scratch_d;
  g->dflags = dflags;

  ME_TRY(hipMemcpyAsync(g->w_rp, W->rowptr, (n + 1) * 8, hipMemcpyDeviceToDevice, s));
  if (nnz > 0) {
    ME_TRY(hipMemcpyAsync(g->w_col, W->col, nnz * 4, hipMemcpyDeviceToDevice, s));
    ME_TRY(hipMemcpyAsync(g->w_val, W->val, nnz * 8, hipMemcpyDeviceToDevice, s));
  }
  ME_TRY(hipMemsetAsync(dflags, 0, sizeof(int) * 64, s));

  // ---- validation (row pointers first: the row kernel indexes with them)
  k_check_rowptr<<<ceil_div(n + 1, kBlock), kBlock, 0, s>>>(n, nnz, g->w_rp, dflags);
  int hflags = 0;
  ME_TRY_STATUS(read_scalar(dflags, &hflags, s));
  if (hflags) return flags_to_status(hflags);
  k_validate_rows<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->w_rp, g->w_col, g->w_val, g->d,
                                                         dflags);
  ME_TRY_STATUS(read_scalar(dflags, &hflags, s));
  if (hflags) return flags_to_status(hflags);

  ME_TRY_STATUS(order_alloc(g, heap, s));
  if (side) {
    ME_TRY_STATUS(side->fork(s));
    ME_TRY_STATUS(order_launch(&g, 1, heap, side->s, job));
  }

  // ---- two-hop pattern: count
  // rows the small table cannot take (mid) and rows the large one cannot
  // (big): 2n int32 fit in g->r's n doubles
  int32_t* big_list = reinterpret_cast<int32_t*>(g->r);
  int32_t* mid_list = big_list + n;
  int32_t* big_count = dflags + 1;
  int32_t* mid_count = dflags + 19;
  const int grid_small = (int)std::min<int64_t>(n, 256 * 32);
  k_twohop_lds<kHashSmall><<<grid_small, kWave, 0, s>>>(
      n, g->w_rp, g->w_col, 0, g->t_cnt, nullptr, nullptr, nullptr, n, mid_list, mid_count);
  int nmid = 0;
  ME_TRY_STATUS(read_scalar(mid_count, &nmid, s));
  const int grid_mid = (int)std::min<int64_t>(nmid, 256 * 20);
  if (nmid > 0)
    k_twohop_lds<kHashLarge><<<grid_mid, kWave, 0, s>>>(n, g->w_rp, g->w_col, 0, g->t_cnt,
                                                        nullptr, nullptr, mid_list, nmid,
                                                        big_list, big_count);
  int nbig = 0;
  ME_TRY_STATUS(read_scalar(big_count, &nbig, s));
  uint32_t* bitmaps = nullptr;
  const int64_t nwords = (n + 31) / 32;
  const int grid_big = nbig > 0 ? (int)twohop_big_grid(nbig) : 0;
  if (nbig > 0) {
    ME_TRY_STATUS(heap.alloc((void**)&bitmaps, (size_t)grid_big * nwords * 4, s));
    ME_TRY(hipMemsetAsync(bitmaps, 0, (size_t)grid_big * nwords * 4, s));
    k_twohop_big<<<grid_big, 256, 0, s>>>(n, g->w_rp, g->w_col, 0, big_list, nbig, bitmaps,
                                          g->t_cnt, nullptr, nullptr);
  }
  int64_t* tile_tmp = reinterpret_cast<int64_t*>(scratch_d);
  scan_counts(n, g->t_cnt, g->t_rp, tile_tmp, s);
  int64_t nnz_t = 0;
  ME_TRY_STATUS(read_scalar(g->t_rp + n, &nnz_t, s));
  g->nnz_t = nnz_t;
  if (nnz + nnz_t >= (int64_t)INT32_MAX) {
    heap.release_later(bitmaps, s);
    return ME_ERR_TOO_LARGE;
  }

  // ---- allocation 2: T columns and the merged operator
  const size_t b2 = build_mem2_bytes(nnz, nnz_t);
  void* mem2 = nullptr;
  {
    const int st2 = heap.alloc(&mem2, b2, s);
    if (st2 < 0) {
      heap.release_later(bitmaps, s);
      return st2;
    }
  }
  g->mem2 = mem2;
  Arena ar2{(char*)mem2, b2, 0};
  g->t_col = ar2.take<int32_t>(nnz_t + 1);
  g->a_col = ar2.take<int32_t>(nnz + nnz_t + 1);
  g->a_w = ar2.take<double>(nnz + nnz_t + 1);
  g->a_w32 = ar2.take<float>(nnz + nnz_t + 1);
  g->a_pk = ar2.take<uint32_t>(nnz + nnz_t + 1);
  g->a_tq = ar2.take<uint32_t>(nnz_t + 1);
  g->h_pk = ar2.take<uint32_t>(nnz + nnz_t + 1);
  g->h_list = ar2.take<int32_t>(nnz + nnz_t + 1);
  g->mem_bytes += b2;

  k_twohop_lds<kHashSmall><<<grid_small, kWave, 0, s>>>(
      n, g->w_rp, g->w_col, 1, g->t_cnt, g->t_rp, g->t_col, nullptr, n, nullptr, nullptr);
  if (nmid > 0)
    k_twohop_lds<kHashLarge><<<grid_mid, kWave, 0, s>>>(n, g->w_rp, g->w_col, 1, g->t_cnt,
                                                        g->t_rp, g->t_col, mid_list, nmid,
                                                        nullptr, nullptr);
  if (nbig > 0) {
    k_twohop_big<<<grid_big, 256, 0, s>>>(n, g->w_rp, g->w_col, 1, big_list, nbig, bitmaps,
                                          g->t_cnt, g->t_rp, g->t_col);
    heap.release_later(bitmaps, s);  // free at the call's next quiesce
  }

  // ---- connectivity of the two-hop graph
  int32_t* parent = reinterpret_cast<int32_t*>(scratch_d);
  int* roots = dflags + 2;
  k_uf_init<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, parent);
  k_uf_hook<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->t_rp, g->t_col, parent);
  k_uf_count_roots<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, parent, roots);

  // ---- Q diagonal, mu denominators, packed operator
  k_invt<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->t_cnt, g->invt, g->invt32);
  unsigned long long* maxden_bits = reinterpret_cast<unsigned long long*>(dflags + 4);
  k_qdiag<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->t_rp, g->t_col, g->invt, g->qdiag,
                                                 g->qinv, g->qinv32, maxden_bits);
  return ME_OK;
}

// The operator packed in the solver order (perm, iperm set), the solver-order
// copies of the per-node arrays, the connectivity and mu denominator reads.
int build_pre_b(GraphOps* g, hipStream_t s) {
  const int64_t n = g->n, nnz = g->nnz_w;
  int64_t* tile_tmp = reinterpret_cast<int64_t*>(g->scratch_d);
  int64_t *woff = g->woff, *toff = g->toff;
  int* roots = g->dflags + 2;
  unsigned long long* maxden_bits = reinterpret_cast<unsigned long long*>(g->dflags + 4);
  int32_t* wlen = reinterpret_cast<int32_t*>(g->r);  // 2n int32 fit in n doubles
  int32_t* tlen = wlen + n;
  k_row_len_perm<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->w_rp, g->t_rp, wlen, tlen);
  scan_counts(n, wlen, woff, tile_tmp, s);
  scan_counts(n, tlen, toff, tile_tmp, s);
  int* max_offset = g->dflags + 12;
  int* max_tcnt = g->dflags + 13;
  int* wide_w = g->dflags + 18;
  k_pack_perm<<<ceil_div(n + 1, kBlock), kBlock, 0, s>>>(
      n, nnz, g->perm, g->iperm, woff, toff, g->w_rp, g->w_col, g->w_val, g->t_rp, g->t_col,
      g->t_cnt, g->invt, g->a_rp, g->a_tp, g->a_col, g->a_w, g->a_w32, g->a_pk, g->a_tq,
      max_offset, max_tcnt, wide_w);
  k_gather_node<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->qinv, g->qinv_s,
                                                       g->qinv32_s);
  k_gather_node<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->invt, g->invt_s, nullptr);
  // halos of the W and T ranges (largest list: 14, 15; overflow: 16, 17)
  const int64_t ntile = ceil_div(n, kHaloRows);
  k_halo_build<<<ntile, kHaloBuildThreads, 0, s>>>(n, g->a_rp, g->a_col, g->a_pk, g->h_pk,
                                                   g->h_list, g->h_cnt_w, g->dflags + 14,
                                                   g->dflags + 16);
  k_halo_build<<<ntile, kHaloBuildThreads, 0, s>>>(n, g->a_tp, g->a_col, g->a_pk, g->h_pk,
                                                   g->h_list, g->h_cnt_t, g->dflags + 15,
                                                   g->dflags + 17);
  // roots (2), the mu denominator's bits (4, 5), the largest offset (12),
  // the largest two-hop count of a column (13), the halo sizes (14-17) and
  // whether a W weight lies beyond FP16's (18, bit 0) or FP32's (bit 1)
  // range in one read
  int hf[20];
  ME_TRY(hipMemcpyAsync(hf, g->dflags, sizeof(hf), hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  const int hroots = hf[roots - g->dflags];
  unsigned long long hmaxden = 0;
  std::memcpy(&hmaxden, &hf[(int*)maxden_bits - g->dflags], 8);
  g->components = hroots;
  double maxden;
  std::memcpy(&maxden, &hmaxden, 8);
  g->maxden = maxden;
  // packed entries: every offset fits 16 bits (both packings) and every W
  // weight FP16 (the FP32 preconditioner's; otherwise it reads the FP32
  // weights, and its halos go with the packed form)
  const bool off_ok = hf[12] <= 32767;
  g->pk_ok = off_ok && (hf[18] & 1) == 0;
  g->w32_ok = (hf[18] & 2) == 0;
  g->tq_ok = off_ok && hf[13] <= 65535;
  g->h_max_w = hf[14];
  g->h_max_t = hf[15];
  g->halo_w = g->pk_ok && hf[16] == 0;
  g->halo_t = g->pk_ok && hf[17] == 0;

  g->needs_eps = !(hroots > 1 || n < 2);
  return ME_OK;
}

// eps, mu and everything that depends on them: r, b, the Jacobi diagonal.
int build_post(GraphOps* g, double eps, int eps_iters, hipStream_t s) {
  const int64_t n = g->n;
  int st = ME_OK;
  if (!g->needs_eps || !(eps > 0.0)) st = ME_WARN_EPS_ZERO, eps = 0.0;
  const double maxden = g->maxden;
  g->eps = eps;
  g->eps_iters = eps_iters;
  // mu = min_i eps / den_i over den_i > 0 = eps / max_i den_i
  g->mu = (eps > 0.0 && maxden > 0.0) ? eps / maxden : 0.0;
  double* scratch_d = g->scratch_d;
  int* dflags = g->dflags;
  unsigned long long* maxdiag_bits = reinterpret_cast<unsigned long long*>(dflags + 6);
  unsigned long long* maxratio_bits = reinterpret_cast<unsigned long long*>(dflags + 8);

  // ---- r, b, Jacobi diagonal
  const int nparts = (int)std::min<int64_t>(ceil_div(n, kBlock), kPartialBlocks);
  double* partial = reinterpret_cast<double*>(scratch_d);
  k_radius<<<nparts, kBlock, 0, s>>>(n, g->d, g->qdiag, g->mu, g->r, partial);
  unsigned long long* maxpratio_bits = reinterpret_cast<unsigned long long*>(dflags + 10);
  k_bvec<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->r, g->d, g->qdiag, partial, nparts, g->mu,
                                                g->eps, g->b, g->b32, g->dinv, g->dinv32,
                                                g->pdinv, g->pdinv32, maxdiag_bits, maxratio_bits,
                                                maxpratio_bits);
  unsigned long long hmax[3] = {0, 0, 0};
  ME_TRY(hipMemcpyAsync(hmax, maxdiag_bits, 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipMemcpyAsync(hmax + 1, maxratio_bits, 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipMemcpyAsync(hmax + 2, maxpratio_bits, 8, hipMemcpyDeviceToHost, s));
  ME_TRY(hipStreamSynchronize(s));
  std::memcpy(&g->max_diag_a, &hmax[0], 8);
  std::memcpy(&g->cheb_b_a, &hmax[1], 8);
  std::memcpy(&g->cheb_b_p, &hmax[2], 8);
  k_gather_node<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->pdinv, g->pdinv_s,
                                                       g->pdinv32_s);
  k_gather_node<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->b, g->b_s, g->b32_s);
  k_gather_node<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, g->perm, g->dinv, g->dinv_s,
                                                       g->dinv32_s);
  g->status = st;
  return st;
}

int build_graph_ops(const me_csr* W, const me_opts* o, DevHeap& heap, hipStream_t s, GraphOps* g,
                    me_info* info) {
  ME_TRY_STATUS(build_pre(W, o, heap, s, g));
  double eps = 0.0;
  int eps_iters = 0;
  if (g->needs_eps) ME_TRY_STATUS(solve_eps(*g, o, heap, s, &eps, &eps_iters));
  const int st = build_post(g, eps, eps_iters, s);
  if (info && st >= 0) {
    info->eps = g->eps;
    info->mu = g->mu;
    info->eps_iterations = eps_iters;
    info->status = st;
  }
  return st;
}

}  // namespace me
