// Host side of the multi-problem LOBPCG engine (Section 4.3 asks for the
// first K generalized eigenpairs by LOBPCG and gives no algorithm text; the
// iteration is the block method of Knyazev (2001): Rayleigh-Ritz on the
// basis [X W P], CholQR B-orthonormalisation of the preconditioned residual
// block W, column dropping instead of an explicit restart, and an FP64
// certificate pass before a solve is accepted).
//
// Per iteration, for every active slot, all on the caller's stream:
//   R = A X - B X Lambda, rho_j, convergence           sl_resid + finalize
//   W = T R  (T = I, Jacobi, or Chebyshev)             (+ sl_cheb_*)
//   W <- (W - X X^T B W) R^-1   (CholQR)                Gram, Cholesky, combine
//   AW = A W                                            difference-form product
//   G_B = S^T B S, G_A = S^T A S, S = [X W P]           MFMA Gram + tile sums
//   Rayleigh-Ritz in FP64                               one workgroup per slot
//   P <- W C_W + P C_P,  X <- X C_X + P                 combine (also AX, AP)
// Kernels skip slots whose device `done` flag is set, so the host enqueues
// a round of iterations between reads of the flags: at most `check_every`,
// fewer when the device's residual history says the first slot to finish
// needs fewer.  A slot that stops
// is certified (fresh A X, Rayleigh-Ritz on X, FP64 residuals); if the
// certificate misses the tolerance the slot iterates again (at most three
// times).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "engine.h"
#include "rowops.h"

namespace me {

int block_width(int K) {
  if (K <= 4) return 4;
  if (K <= 8) return 8;
  return 16;
}

int partial_tiles(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kPartialBlocks, ceil_div(n, 64)));
}

// Drop threshold on the pivots of the unit-diagonal basis Gram (squared sine
// of the angle between a column and the span of the earlier ones).  Small
// thresholds let the inverse Cholesky factor grow without bound on nearly
// dependent bases; 1e-4 keeps it bounded and costs no iterations.
constexpr double kRrPivot = 1e-4;

static int lpr64(int kb) { return kb / std::min(2, kb); }
static int lpr32(int kb) { return kb / std::min(4, kb); }

size_t Engine::slot_bytes(int64_t n, int kb) {
  const int m = 3 * kb;
  const int np = partial_tiles(n);
  size_t b = kNumBlk64 * Arena::round((size_t)n * kb * 8);
  b += kNumBlk32 * Arena::round((size_t)n * kb * 4);
  b += Arena::round((size_t)np * 2 * m * m * 8);
  b += Arena::round((size_t)2 * m * m * 8) + Arena::round((size_t)2 * m * kb * 8);
  b += Arena::round((size_t)2 * kb * kb * 8) + 2 * Arena::round((size_t)kb * 8);
  b += Arena::round((size_t)np * kb * 16);
  return b;
}

size_t Engine::table_bytes(int capacity) {
  const size_t c = (size_t)std::max(capacity, 1);
  return Arena::round(sizeof(SlotDev) * c) + Arena::round(sizeof(Ctrl) * c) +
         Arena::round(sizeof(ChebCoef) * c);
}

size_t Engine::tile_bytes(int64_t n, int kb) {
  const int64_t rb64 = kBlock / lpr64(kb), rb32 = kBlock / lpr32(kb);
  return 4 + sizeof(Tile) * (size_t)(ceil_div(n, kGatherRows) + ceil_div(n, rb64) +
                                     ceil_div(n, rb32) + partial_tiles(n));
}

size_t Engine::tile_area_bytes(size_t sum) {
  // each of at most six lists (per block width, packed entries or not)
  // rounds five sections and its start to the heap's unit
  return DevHeap::round(sum + 6 * 6 * kHeapAlign);
}

size_t Engine::run_bytes(const std::vector<std::pair<int64_t, int>>& slots) {
  size_t tiles = 0, b = DevHeap::round(table_bytes((int)slots.size()));
  for (const auto& s : slots) {
    b += DevHeap::round(slot_bytes(s.first, s.second));
    tiles += tile_bytes(s.first, s.second);
  }
  return b + DevHeap::round(2 * tile_area_bytes(tiles));
}

Engine::Engine(hipStream_t s, const me_opts& o, int capacity, bool timed, bool solo,
               DevHeap* heap, size_t tile_area)
    : s_(s), o_(o), cap_(capacity), timed_(timed), solo_(solo),
      heap_(heap ? heap : &own_heap_), tile_area_(tile_area) {
  cheb_ = o.precond == ME_PRECOND_CHEBYSHEV;
  cheb32_ = cheb_ && o.precision == ME_MIXED;
}

int Engine::init() {
  sh_.assign(cap_, SlotHost());
  res_.assign(cap_, SlotResult());
  hdev_.assign(cap_, SlotDev());
  const size_t tb = table_bytes(cap_);
  ME_TRY_STATUS(heap_->alloc(&tables_, tb, s_));
  Arena a{(char*)tables_, tb, 0};
  d_slots_ = a.take<SlotDev>(cap_);
  d_ctrl_ = a.take<Ctrl>(cap_);
  d_cheb_ = a.take<ChebCoef>(cap_);
  if (heap_->region()) {
    // no allocation of any kind over a caller region: a pageable mirror and
    // both work-list areas carved from the region
    h_ctrl_pageable_.assign(cap_, Ctrl{});
    h_ctrl_ = h_ctrl_pageable_.data();
    if (tile_area_ == 0) return ME_ERR_WORKSPACE;
    ME_TRY_STATUS(heap_->alloc(&tile_mem_, 2 * tile_area_, s_));
    for (int q = 0; q < 2; ++q) {
      areas_[q].base = (char*)tile_mem_ + q * tile_area_;
      areas_[q].cap = tile_area_;
      areas_[q].used = 0;
    }
  } else {
    ME_TRY(hipHostMalloc((void**)&h_ctrl_, sizeof(Ctrl) * cap_, hipHostMallocDefault));
  }
  std::memset(h_ctrl_, 0, sizeof(Ctrl) * cap_);
  return ME_OK;
}

// The form of the one-slot FP32 preconditioner step per kind of slot
// (block width, entry range, log2 of the rows): kFormHalo or kFormGather
// once timed, -1 while its first iteration times both.  Process-wide: every
// engine of the process shares what was measured.
static std::mutex g_form_mu;
static std::map<std::array<int, 3>, int> g_form;

Engine::~Engine() {
  (void)hipStreamSynchronize(s_);
  if (tune_.live) {  // timed but never read: time that kind again later
    std::lock_guard<std::mutex> l(g_form_mu);
    g_form.erase({tune_.key[0], tune_.key[1], tune_.key[2]});
  }
  for (auto& e : tune_.ev) (void)hipEventDestroy(e);
  drop_graph();
  if (cap_s_) (void)hipStreamDestroy(cap_s_);
  free_sets(&sets_);
  for (auto& h : sh_)
    if (h.used && h.own_ws && h.ws) heap_->release(h.ws, s_);
  heap_->release(tables_, s_);
  heap_->release(tile_mem_, s_);
  (void)hipStreamSynchronize(s_);
  if (h_ctrl_ && !heap_->region()) (void)hipHostFree(h_ctrl_);
}

bool Engine::idle() const {
  for (const auto& h : sh_)
    if (h.used && !h.finished) return false;
  return true;
}

int Engine::active() const {
  int c = 0;
  for (const auto& h : sh_) c += h.used && !h.finished;
  return c;
}

int Engine::add(const SlotSpec& sp, void* ws, size_t ws_bytes, int* id_out) {
  int id = -1;
  for (int i = 0; i < cap_; ++i)
    if (!sh_[i].used) {
      id = i;
      break;
    }
  if (id < 0) return ME_ERR_INVALID_ARG;
  const GraphOps& g = *sp.g;
  // the FP32 preconditioner and the FP32 product read W's weights in FP32
  if (sp.op != OP_Q && (cheb32_ || o_.product == ME_PRODUCT_FP32) && !g.w32_ok)
    return ME_ERR_BAD_WEIGHT;
  const int64_t n = g.n;
  const int kb = sp.kb;
  const size_t need = slot_bytes(n, kb);
  bool own = false;
  if (!ws) {
    ME_TRY_STATUS(heap_->alloc(&ws, need, s_));
    own = true;
  } else if (ws_bytes < need) {
    return ME_ERR_WORKSPACE;
  }
  SlotHost& h = sh_[id];
  h = SlotHost();
  h.used = true;
  h.own_ws = own;
  h.ws = ws;
  h.ws_bytes = need;
  h.sp = sp;
  bytes_in_use_ += need;
  res_[id] = SlotResult();

  SlotDev d{};
  Arena a{(char*)ws, need, 0};
  for (int b = 0; b < kNumBlk64; ++b) d.b64[b] = a.take<double>((size_t)n * kb);
  for (int b = 0; b < kNumBlk32; ++b) d.b32[b] = a.take<float>((size_t)n * kb);
  const int m = 3 * kb;
  const int np = partial_tiles(n);
  d.partials = a.take<double>((size_t)np * 2 * m * m);
  d.gram = a.take<double>((size_t)2 * m * m);
  d.coef = a.take<double>((size_t)2 * m * kb);
  d.coefw = a.take<double>((size_t)2 * kb * kb);
  d.lam = a.take<double>(kb);
  d.sums = a.take<double>(kb);
  d.scratch = a.take<double>((size_t)np * kb * 2);
  if (!d.scratch) return ME_ERR_WORKSPACE;
  d.n = n;
  d.nparts = np;
  d.per = ((ceil_div(n, np) + 15) / 16) * 16;
  d.need = sp.need;
  d.deflate = sp.deflate;
  d.range = sp.op == OP_Q ? kRangeT : kRangeAll;
  d.kcopy = sp.x0 ? sp.kcopy : 0;
  d.k_out = sp.k_out;
  d.a_rp = g.a_rp;
  d.a_tp = g.a_tp;
  d.a_col = g.a_col;
  d.a_w = g.a_w;
  d.a_w32 = g.a_w32;
  d.nnz_ops = g.nnz_w + g.nnz_t + 1;
  d.a_pk = g.a_pk;
  d.pk_ok = g.pk_ok ? 1 : 0;
  d.invt = g.invt_s;
  d.a_tq = g.a_tq;
  d.tq_base = g.nnz_w;
  d.tq_ok = g.tq_ok ? 1 : 0;
  d.h_pk = g.h_pk;
  d.h_list = g.h_list;
  d.h_cnt = nullptr;
  d.h_max = 0;
  if (sp.op == OP_A) {
    d.c_t = -g.mu;
    d.s_diag = g.eps;
    d.bdiag = g.b_s;
    d.dinv = g.dinv_s;
    d.dinv32 = g.dinv32_s;
    const bool lap = o_.cheb_op == ME_CHEB_LAPLACIAN;
    d.cheb_range = lap ? kRangeW : kRangeAll;
    d.cheb_s_diag = g.eps;
    d.cheb_dinv = lap ? g.pdinv_s : g.dinv_s;
    d.cheb_dinv32 = lap ? g.pdinv32_s : g.dinv32_s;
  } else {
    d.c_t = 1.0;
    d.s_diag = 0.0;
    d.bdiag = nullptr;
    d.dinv = g.qinv_s;
    d.dinv32 = g.qinv32_s;
    // eps solve: the preconditioner inverts Q itself (the one-hop
    // Laplacian is a poor stand-in: ten times the iterations)
    d.cheb_range = kRangeT;
    d.cheb_s_diag = 0.0;
    d.cheb_dinv = g.qinv_s;
    d.cheb_dinv32 = g.qinv32_s;
  }
  if (d.cheb_range == kRangeW && g.halo_w) {
    d.h_cnt = g.h_cnt_w;
    d.h_max = g.h_max_w;
  } else if (d.cheb_range == kRangeT && g.halo_t) {
    d.h_cnt = g.h_cnt_t;
    d.h_max = g.h_max_t;
  }
  d.perm = g.perm;
  d.iperm = g.iperm;
  d.x0 = sp.x0;
  d.seed = sp.seed;
  d.lev = (sp.nsmooth > 0 && g.max_level > 0) ? g.lev_s : nullptr;
  d.max_lev = g.max_level;
  d.jfreq = sp.jfreq;
  d.nsmooth = sp.nsmooth;
  d.out_x = sp.out_x;
  d.out_lam = sp.out_lam;
  d.ctrl = d_ctrl_ + id;
  d.cheb = d_cheb_ + id;
  hdev_[id] = d;

  Ctrl& c = h_ctrl_[id];
  std::memset(&c, 0, sizeof(Ctrl));
  c.max_iter = sp.max_iter;
  c.need = sp.need;
  c.kb = kb;
  c.tol = sp.tol;
  c.lam_scale = sp.lam_scale > 0 ? sp.lam_scale : 1.0;
  c.lam_floor = 1e-8 * c.lam_scale;
  c.cheb_deg = cheb_ ? o_.cheb_degree : 0;
  c.cheb_afac = 0.5;
  c.cheb_b = sp.cheb_b;
  ME_TRY(hipMemcpyAsync(d_slots_ + id, &hdev_[id], sizeof(SlotDev), hipMemcpyHostToDevice, s_));
  ME_TRY(hipMemcpyAsync(d_ctrl_ + id, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s_));
  // the pageable SlotDev copy and the pinned Ctrl must not change before the
  // copies complete: callers add between synchronised rounds
  ME_TRY(hipStreamSynchronize(s_));
  *id_out = id;
  return ME_OK;
}

void Engine::release(int id) {
  if (id < 0 || id >= cap_ || !sh_[id].used) return;
  SlotHost& h = sh_[id];
  if (h.own_ws && h.ws) heap_->release(h.ws, s_);  // the slot's work is complete
  bytes_in_use_ -= h.ws_bytes;
  h = SlotHost();
}

// Work lists of the slots `ids` (all of block width kb).
int Engine::build_set(const std::vector<int>& ids, int kb, TileSet* ts, int area) {
  ts->kb = kb;
  ts->nslots = (int)ids.size();
  ts->ids = ids;
  const int rb64 = kBlock / lpr64(kb), rb32 = kBlock / lpr32(kb);
  std::vector<Tile> gat, e64, e32, red;
  ts->buf = o_.addressing == ME_ADDR_AUTO;
  ts->pk = true;
  ts->n_red_big = 0;
  for (int id : ids) {
    const SlotDev& d = hdev_[id];
    ts->buf = ts->buf && d.n * kb * 8 < kBufMaxBytes && d.nnz_ops * 8 < kBufMaxBytes;
    ts->pk = ts->pk && d.pk_ok;
    for (int64_t b = 0; b < ceil_div(d.n, kGatherRows); ++b) gat.push_back({id, (int32_t)b});
    for (int64_t b = 0; b < ceil_div(d.n, rb64); ++b) e64.push_back({id, (int32_t)b});
    for (int64_t b = 0; b < ceil_div(d.n, rb32); ++b) e32.push_back({id, (int32_t)b});
  }
  // reduction tiles: slots with tall tiles first (their Grams run in wider
  // workgroups; the split depends on the slot alone)
  for (int big = 1; big >= 0; --big)
    for (int id : ids) {
      const SlotDev& d = hdev_[id];
      if ((d.per >= kGramBigRows) != (big == 1)) continue;
      for (int b = 0; b < d.nparts; ++b) red.push_back({id, b});
      if (big) ts->n_red_big += d.nparts;
    }
  ts->n_gather = (int64_t)gat.size();
  ts->n_elem64 = (int64_t)e64.size();
  ts->n_elem32 = (int64_t)e32.size();
  ts->n_red = (int64_t)red.size();
  const size_t nt = gat.size() + e64.size() + e32.size() + red.size();
  const size_t bytes = Arena::round(ids.size() * 4) + nt * sizeof(Tile) + 4 * 256;
  ts->host.assign(bytes, 0);
  size_t off = 0;
  auto put = [&](const void* src, size_t sz) {
    std::memcpy(ts->host.data() + off, src, sz);
    const size_t at = off;
    off = Arena::round(off + sz);
    return at;
  };
  const size_t o_sl = put(ids.data(), ids.size() * 4);
  const size_t o_g = put(gat.data(), gat.size() * sizeof(Tile));
  const size_t o_e64 = put(e64.data(), e64.size() * sizeof(Tile));
  const size_t o_e32 = put(e32.data(), e32.size() * sizeof(Tile));
  const size_t o_r = put(red.data(), red.size() * sizeof(Tile));
  const size_t dev_bytes = DevHeap::round(off > 0 ? off : 1);
  if (heap_->region()) {
    Area& ar = areas_[area];
    if (ar.used + dev_bytes > ar.cap) return ME_ERR_WORKSPACE;
    ts->mem = ar.base + ar.used;
    ar.used += dev_bytes;
  } else {
    ME_TRY_STATUS(heap_->alloc(&ts->mem, dev_bytes, s_));
  }
  ME_TRY(hipMemcpyAsync(ts->mem, ts->host.data(), off, hipMemcpyHostToDevice, s_));
  char* base = (char*)ts->mem;
  ts->slots = (const int32_t*)(base + o_sl);
  ts->gather = (const Tile*)(base + o_g);
  ts->elem64 = (const Tile*)(base + o_e64);
  ts->elem32 = (const Tile*)(base + o_e32);
  ts->red = (const Tile*)(base + o_r);
  return ME_OK;
}

// Callers free a set only once the stream has finished the work that used it.
void Engine::free_set(TileSet* ts) {
  if (ts->mem && !heap_->region()) heap_->release(ts->mem, s_);
  *ts = TileSet();
}

int Engine::sets_for(const std::vector<int>& ids, std::vector<TileSet>* sets, int area) {
  areas_[area].used = 0;  // the area's previous lists are freed
  // one set per block width and kind of preconditioner entries (packed or
  // not), so that the kernels a slot runs depend on the slot alone
  for (int kb : {4, 8, 16})
    for (int pk : {1, 0}) {
      std::vector<int> sub;
      for (int id : ids)
        if (sh_[id].sp.kb == kb && (hdev_[id].pk_ok != 0) == (pk == 1)) sub.push_back(id);
      if (sub.empty()) continue;
      sets->emplace_back();
      ME_TRY_STATUS(build_set(sub, kb, &sets->back(), area));
    }
  return ME_OK;
}

void Engine::free_sets(std::vector<TileSet>* sets) {
  for (auto& t : *sets) free_set(&t);
  sets->clear();
}

int Engine::read_ctrl() {
  ME_TRY(hipGetLastError());
  ME_TRY(hipMemcpyAsync(h_ctrl_, d_ctrl_, sizeof(Ctrl) * cap_, hipMemcpyDeviceToHost, s_));
  ME_TRY(hipStreamSynchronize(s_));
  return ME_OK;
}

// Rayleigh-Ritz on [X] alone (start and certificate): X, AX rotated to
// B-orthonormal Ritz vectors, lam set.
void Engine::rr_x(const TileSet& ts, int final_pass) {
  const int kb = ts.kb;
  sl_spmm<double>(d_slots_, ts, BX, BAX, 1, s_);
  const int u[1] = {BX}, v2[1] = {BAX};
  sl_gram(d_slots_, ts, 1, u, 1, u, 1, v2, 1, 1, s_);
  sl_reduce(d_slots_, ts, 2 * kb * kb, 1, s_);
  sl_rayleigh_ritz(d_slots_, ts, 1, 1e-14, final_pass, s_);
  const int ix[1] = {BX}, ia[1] = {BAX};
  sl_combine(d_slots_, ts, 1, 2, ix, ia, 1, ix, ia, 0, kb * kb, 1, s_);
}

void Engine::start_pass(const TileSet& ts) {
  sl_fill_start(d_slots_, ts, s_);
  sl_zero(d_slots_, ts, BP, s_);
  sl_zero(d_slots_, ts, BAP, s_);
  sl_deflate(d_slots_, ts, BX, 1, s_);
  rr_x(ts, 0);
}


int Engine::step_form(const TileSet& ts, bool* tune) {
  *tune = false;
  if (!cheb32_ || !ts.pk || ts.nslots != 1 || capturing_ || tune_.live) return kFormHalo;
  const SlotDev& h = hdev_[ts.ids[0]];
  if (!h.h_cnt) return kFormHalo;  // no halos: the gathering step in either case
  int lg = 0;
  while ((int64_t)1 << (lg + 1) <= h.n) ++lg;
  const std::array<int, 3> key{ts.kb, h.cheb_range, lg};
  std::lock_guard<std::mutex> l(g_form_mu);
  const auto it = g_form.find(key);
  if (it != g_form.end()) return it->second < 0 ? kFormHalo : it->second;
  g_form[key] = -1;
  for (int q = 0; q < 3; ++q) tune_.key[q] = key[q];
  *tune = true;
  return kFormHalo;
}

// After the round of a timed iteration: keep the faster form per step.
void Engine::finish_tune() {
  if (!tune_.live) return;
  tune_.live = false;
  double t[2] = {0.0, 0.0};
  int n[2] = {0, 0};
  bool ok = tune_.used >= 3;
  for (int b = 0; ok && b + 1 < tune_.used; ++b) {
    float ms = 0.f;
    ok = hipEventElapsedTime(&ms, tune_.ev[b], tune_.ev[b + 1]) == hipSuccess;
    t[b % 2] += ms;
    n[b % 2] += tune_.steps[b];
  }
  ok = ok && n[0] > 0 && n[1] > 0;
  const double t0 = ok ? t[0] : 0.0, t1 = ok ? t[1] : 0.0;
  const int n0 = n[0], n1 = n[1];
  const std::array<int, 3> key{tune_.key[0], tune_.key[1], tune_.key[2]};
  std::lock_guard<std::mutex> l(g_form_mu);
  if (!ok) {
    (void)hipGetLastError();
    g_form.erase(key);  // time it again later
    return;
  }
  // the halo form unless the gathering one is clearly faster (timing noise)
  g_form[key] = t1 / n1 < 0.97 * (t0 / n0) ? kFormGather : kFormHalo;
}

void Engine::iteration(const TileSet& ts) {
  const int kb = ts.kb;
  ++tag_;
  const bool tm = timed_;
  // residual, preconditioned W, convergence test
  sl_resid(d_slots_, ts, cheb_ ? BR : BW, o_.precond == ME_PRECOND_JACOBI ? 1 : 0, 0, s_);
  sl_resid_finalize(d_slots_, ts, 0, s_);
  if (cheb_) {
    const int deg = o_.cheb_degree;
    double cb = 0.0;
    // only when the caller solves one input graph, so that a graph's result
    // never depends on which other graphs share its batch
    const bool h16 = cheb32_ && solo_ && o_.cheb_iterates == ME_ITER_FP16 &&
                     sl_cheb_h_ok(hdev_.data(), ts);
    if (tm) {
      for (int id : ts.ids) {
        const GraphOps& g = *sh_[id].sp.g;
        // algorithmic bytes of one step: every entry of the preconditioner's
        // operator (packed: 4 B; else column index and weight; FP64 two-hop
        // entries: the column, with 1/T_i per row), row bounds (8 B), D^-1_i,
        // and the blocks y_k (neighbour rows counted once), y_{k-1}, R
        // (packed FP32 sets: FP16) read and y_{k+1} written
        const double sz = cheb32_ ? 4.0 : 8.0;
        const double ent = (cheb32_ && ts.pk) ? 4.0 : 4.0 + sz;
        const bool tq = !cheb32_ && g.tq_ok && kb <= 4;  // packed two-hop entries
        const double ent_t = ((cheb32_ && ts.pk) || tq) ? 4.0 : 4.0 + sz;
        const int rg = hdev_[id].cheb_range;
        const double nw = rg == kRangeT ? 0.0 : (double)g.nnz_w;
        const double nt = rg == kRangeW ? 0.0 : (double)g.nnz_t;
        const double tin = (tq && nt > 0.0) ? 8.0 * (double)g.n : 0.0;
        if (h16)  // y_k, y_{k-1} read and y_{k+1} written in FP16, R in FP32
          cb += 4.0 * (nw + nt) + (double)g.n * 12.0 + 10.0 * (double)g.n * kb;
        else
          cb += ent * nw + ent_t * nt + tin + (double)g.n * (8.0 + sz) +
                (3.0 * sz + ((cheb32_ && ts.pk) ? 2.0 : sz)) * (double)g.n * kb;
      }
    }
    const int w = cheb32_ ? BW32 : BW, y = cheb32_ ? BY32 : BY;
    const int r = cheb32_ ? BR32 : BR;
    int cur = ((deg - 1) % 2 == 0) ? w : y;
    int nxt = cur == w ? y : w;
    if (h16) {
      sl_to32_scaled(d_slots_, ts, BR, BR32, s_);
      sl_cheb_first_h(d_slots_, ts, r, cur, nxt, s_);
    } else if (cheb32_) {
      if (ts.pk) sl_to16_scaled(d_slots_, ts, BR, BR32, s_);  // packed: FP16 right-hand side
      else sl_to32(d_slots_, ts, BR, BR32, s_);
      sl_cheb_first<float>(d_slots_, ts, r, cur, nxt, s_);
    } else {
      sl_cheb_first<double>(d_slots_, ts, r, cur, nxt, s_);
    }
    {
      KScope ks(tm ? KT_CHEB : -1, s_, (deg - 1) * cb, tag_, deg - 1);
      bool tune = false;
      int form = h16 ? kFormHalo : step_form(ts, &tune);
      if (tune) {  // blocks of kTuneBlock steps, alternating halo and gathering
        const int nb = (deg - 1 + kTuneBlock - 1) / kTuneBlock;
        while ((int)tune_.ev.size() < nb + 1) {
          hipEvent_t e = nullptr;
          if (hipEventCreate(&e) != hipSuccess) break;
          tune_.ev.push_back(e);
        }
        tune = (int)tune_.ev.size() >= nb + 1;
        if (tune) {
          tune_.live = true;
          tune_.used = 0;
          tune_.steps.assign(nb, 0);
        }
      }
      for (int k = 1; k < deg; ++k) {
        if (tune && (k - 1) % kTuneBlock == 0) {
          const int b = (k - 1) / kTuneBlock;
          (void)hipEventRecord(tune_.ev[b], s_);
          tune_.used = b + 1;
          form = b % 2 == 0 ? kFormHalo : kFormGather;
        }
        if (tune) ++tune_.steps[(k - 1) / kTuneBlock];
        if (h16) sl_cheb_step_h(hdev_.data(), ts, k, r, cur, nxt, s_);
        else if (cheb32_) sl_cheb_step<float>(d_slots_, hdev_.data(), ts, k, r, cur, nxt, s_, form);
        else sl_cheb_step<double>(d_slots_, hdev_.data(), ts, k, r, cur, nxt, s_);
        std::swap(cur, nxt);
      }
      if (tune) {
        (void)hipEventRecord(tune_.ev[tune_.used], s_);
        ++tune_.used;
      }
    }
    if (h16) sl_to64_h(d_slots_, ts, BW32, BW, s_);
    else if (cheb32_) sl_to64(d_slots_, ts, BW32, BW, s_);
  }
  sl_deflate(d_slots_, ts, BW, 0, s_);
  // W <- (W - X C) R^-1, once, or twice (CholQR2)
  for (int pass = 0; pass < o_.cholqr_passes; ++pass) {
    const int u[2] = {BX, BW}, v[1] = {BW}, o[1] = {BW};
    sl_gram(d_slots_, ts, 2, u, 1, v, 0, nullptr, 1, 0, s_);
    sl_reduce(d_slots_, ts, 2 * kb * kb, 0, s_);
    sl_cholqr_coef(d_slots_, ts, 1e-10, s_);
    sl_combine(d_slots_, ts, 2, 1, u, nullptr, 1, o, nullptr, 1, 0, 0, s_);
  }
  double sb = 0.0, blk = 0.0;
  if (tm) {
    for (int id : ts.ids) {
      const GraphOps& g = *sh_[id].sp.g;
      // column index and weight of every one-hop entry, the packed word of
      // every two-hop entry (its weight is 1/T_i + 1/T_j) with 1/T_i per row
      // (else column index and weight), row bounds, x in, y out
      const bool tq = g.tq_ok && kb <= 4;
      sb += 12.0 * (double)g.nnz_w + (tq ? 4.0 : 12.0) * (double)g.nnz_t +
            (double)g.n * (tq ? 16.0 : 8.0) + 2.0 * (double)g.n * kb * 8.0;
      blk += (double)g.n * kb * 8.0;
    }
  }
  {
    KScope ks(tm ? KT_SPMM_A : -1, s_, sb, tag_);
    if (o_.product == ME_PRODUCT_FP32) {  // W rounded to FP32, product in FP32
      sl_to32(d_slots_, ts, BW, BY32, s_);
      sl_spmm<float>(d_slots_, ts, BY32, BR32, 0, s_);
      sl_to64(d_slots_, ts, BR32, BAW, s_);
    } else {
      sl_spmm<double>(d_slots_, ts, BW, BAW, 0, s_);
    }
  }
  const int m = 3 * kb;
  const int S[3] = {BX, BW, BP}, AS[3] = {BAX, BAW, BAP};
  {
    KScope ks(tm ? KT_GRAM_RR : -1, s_, 6.0 * blk + blk / kb, tag_);
    sl_gram(d_slots_, ts, 3, S, 3, S, 3, AS, 1, 0, s_);
  }
  sl_reduce(d_slots_, ts, 2 * m * m, 0, s_);
  sl_rayleigh_ritz(d_slots_, ts, 3, kRrPivot, 0, s_);
  const int ox[2] = {BP, BX}, oa[2] = {BAP, BAX};
  {
    KScope ks(tm ? KT_COMBINE : -1, s_, 2.0 * 5.0 * blk, tag_);
    sl_combine(d_slots_, ts, 3, 2, S, AS, 2, ox, oa, 0, 0, 0, s_);
  }
}

int Engine::certify(const std::vector<int>& ids, std::vector<int>* finished) {
  std::vector<TileSet> cs;
  ME_TRY_STATUS(sets_for(ids, &cs, 1));
  for (auto& ts : cs) {
    rr_x(ts, 1);
    sl_resid(d_slots_, ts, -1, 0, 1, s_);
    sl_resid_finalize(d_slots_, ts, 1, s_);
  }
  int st = read_ctrl();
  free_sets(&cs);
  if (st < 0) return st;
  std::vector<int> fin, again;
  for (int id : ids) {
    const Ctrl& c = h_ctrl_[id];
    SlotHost& h = sh_[id];
    SlotResult& r = res_[id];
    double worst = 0.0;
    for (int j = 0; j < h.sp.need; ++j) worst = std::max(worst, c.rho[j]);
    r.iterations = c.iter;
    r.worst = worst;
    for (int j = 0; j < h.sp.kb && j < kMaxBlockCols; ++j) r.lam[j] = c.lam[j];
    if (c.nonfinite || !std::isfinite(worst)) {
      r.status = ME_ERR_BREAKDOWN;
      h.finished = true;
      continue;
    }
    if (worst <= h.sp.tol || c.iter >= h.sp.max_iter || h.reentries >= 3) {
      r.status = worst <= h.sp.tol ? ME_OK : ME_WARN_NOT_CONVERGED;
      fin.push_back(id);
    } else {
      // drift between the recurrences and a fresh product: iterate again
      ++h.reentries;
      again.push_back(id);
    }
  }
  if (!fin.empty()) {
    ME_TRY_STATUS(sets_for(fin, &cs, 1));
    for (auto& ts : cs) {
      const int u[1] = {BX};
      sl_gram(d_slots_, ts, 1, u, 1, u, 0, nullptr, 1, 1, s_);
      sl_reduce(d_slots_, ts, ts.kb * ts.kb, 1, s_);
      sl_orth(d_slots_, ts, s_);
      sl_output(d_slots_, ts, s_);
    }
    st = read_ctrl();
    free_sets(&cs);
    if (st < 0) return st;
    for (int id : fin) {
      res_[id].orth = h_ctrl_[id].orth;
      sh_[id].finished = true;
    }
  }
  if (!again.empty()) {
    ME_TRY_STATUS(sets_for(again, &cs, 1));
    for (auto& ts : cs) {
      sl_reenter(d_slots_, ts, s_);
      sl_zero(d_slots_, ts, BP, s_);
      sl_zero(d_slots_, ts, BAP, s_);
    }
    ME_TRY(hipStreamSynchronize(s_));
    free_sets(&cs);
    for (int id : again) h_ctrl_[id].done = 0;
  }
  for (int id : ids)
    if (sh_[id].finished && finished) finished->push_back(id);
  return ME_OK;
}

// Iterations to enqueue before the next check: check_every, shortened to
// the fewest iterations any active slot still needs by the linear
// convergence rate of its largest required rho over the last round (so that
// few iterations are enqueued after the first slot has stopped).
int Engine::round_length() {
  const int ce = o_.check_every > 0 ? o_.check_every : 16;
  double best = 1e300;
  for (int id : active_) {
    // convergence rate from the device's residual history (iterations
    // 0 .. iter - 1 have entries), the faster of the last 4 and the last 8
    // iterations: a round that ends early costs one host read, an iteration
    // past convergence costs a round of launches that do nothing
    const Ctrl& c = h_ctrl_[id];
    const int last = c.iter - 1;
    const double rho = last >= 0 ? c.rho_hist[last % kRhoHist] : 0.0;
    double rate = 0.0;
    for (int m : {4, 8}) {
      if (m > last || m >= kRhoHist) continue;
      const double old = c.rho_hist[(last - m) % kRhoHist];
      if (rho > 0.0 && rho < old) rate = std::max(rate, std::log(old / rho) / (double)m);
    }
    if (rate > 0.0) {
      const double rem = rho > sh_[id].sp.tol ? std::log(rho / sh_[id].sp.tol) / rate : 0.0;
      best = std::min(best, rem);
    }
  }
  if (best >= 1e300) return ce;
  return (int)std::max(1.0, std::min((double)ce, std::ceil(best)));
}

// Starts the slots added since the last round, then enqueues one round of
// iterations of every active slot (returns without waiting for them).
int Engine::begin_round() {
  round_open_ = false;
  std::vector<int> fresh;
  for (int id = 0; id < cap_; ++id)
    if (sh_[id].used && !sh_[id].started) fresh.push_back(id);
  if (!fresh.empty()) {
    std::vector<TileSet> cs;
    ME_TRY_STATUS(sets_for(fresh, &cs, 1));
    for (auto& ts : cs) start_pass(ts);
    ME_TRY(hipStreamSynchronize(s_));
    free_sets(&cs);
    for (int id : fresh) {
      sh_[id].started = true;
      active_.push_back(id);
    }
    sets_dirty_ = true;
  }
  if (active_.empty()) return ME_OK;
  if (sets_dirty_) {
    ME_TRY(hipStreamSynchronize(s_));
    free_sets(&sets_);
    std::sort(active_.begin(), active_.end());
    ME_TRY_STATUS(sets_for(active_, &sets_, 0));
    sets_dirty_ = false;
    ++sets_ver_;
  }
  iter0_.resize(active_.size());
  for (size_t q = 0; q < active_.size(); ++q) iter0_[q] = h_ctrl_[active_[q]].iter;
  if (timed_) phase_ = ktimer_new_phase();
  tag_ = 0;
  const int ce = round_length();
  ME_TRY_STATUS(enqueue_round(ce));
  round_open_ = true;
  return ME_OK;
}

void Engine::drop_graph() {
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  gexec_ = nullptr;
  gexec_ver_ = -1;
}

// ce iterations of every active set: kernel by kernel, or one captured
// iteration replayed ce times (captured again whenever the active sets
// change).  Captures run on a private stream (the caller's may be the
// legacy default stream, which cannot be captured); the replays go to the
// engine's stream.
// Largest one-graph solve that ME_LAUNCH_AUTO replays as a graph.
constexpr int64_t kGraphMaxRows = 16384;

int Engine::enqueue_round(int ce) {
  bool graph = o_.launch == ME_LAUNCH_GRAPH;
  if (o_.launch == ME_LAUNCH_AUTO) {
    int64_t rows = 0;
    for (int id : active_) rows += hdev_[id].n;
    graph = cap_ == 1 && rows <= kGraphMaxRows;
  }
  graph = graph && !heap_->region() && !(timed_ && ktimer_kind() != 0);
  if (!graph) {
    for (int q = 0; q < ce; ++q)
      for (auto& ts : sets_) iteration(ts);
    return ME_OK;
  }
  if (!gexec_ || gexec_ver_ != sets_ver_) {
    drop_graph();
    if (!cap_s_) ME_TRY(hipStreamCreateWithFlags(&cap_s_, hipStreamNonBlocking));
    hipStream_t keep = s_;
    s_ = cap_s_;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap_s_, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      capturing_ = true;
      for (auto& ts : sets_) iteration(ts);
      capturing_ = false;
      e = hipStreamEndCapture(cap_s_, &g);
    }
    s_ = keep;
    if (e == hipSuccess) e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      gexec_ = nullptr;
      return ME_ERR_HIP;
    }
    gexec_ver_ = sets_ver_;
  }
  for (int q = 0; q < ce; ++q) ME_TRY(hipGraphLaunch(gexec_, s_));
  return ME_OK;
}

// Waits for the round, then certifies the slots that stopped; appends the
// ids that finished.
int Engine::end_round(std::vector<int>* finished) {
  if (!round_open_) return ME_OK;
  round_open_ = false;
  ME_TRY_STATUS(read_ctrl());
  finish_tune();  // the round's events are complete
  int adv = 0;
  std::vector<int> stopped;
  for (size_t q = 0; q < active_.size(); ++q) {
    const int id = active_[q];
    adv = std::max(adv, h_ctrl_[id].iter - iter0_[q]);
    if (h_ctrl_[id].done) stopped.push_back(id);
  }
  // launches of the round after every slot had stopped did no work
  if (timed_) ktimer_drop_after(phase_, adv * (int)sets_.size());
  if (!stopped.empty()) {
    ME_TRY_STATUS(certify(stopped, finished));
    std::vector<int> keep;
    for (int id : active_)
      if (!sh_[id].finished) keep.push_back(id);
    if (keep.size() != active_.size()) {
      active_.swap(keep);
      sets_dirty_ = true;
    }
  }
  return ME_OK;
}

int Engine::step(std::vector<int>* finished) {
  ME_TRY_STATUS(begin_round());
  return end_round(finished);
}

int Engine::run() {
  while (!idle()) ME_TRY_STATUS(step(nullptr));
  if (timed_) ktimer_collect();
  return ME_OK;
}

}  // namespace me

extern "C" {

int me_step_form(int block_width, int range, int64_t rows) {
  int lg = 0;
  while (rows > 0 && ((int64_t)1 << (lg + 1)) <= rows) ++lg;
  std::lock_guard<std::mutex> l(me::g_form_mu);
  const auto it = me::g_form.find({block_width, range, lg});
  return it == me::g_form.end() ? -1 : it->second;
}

void me_step_form_reset(void) {
  std::lock_guard<std::mutex> l(me::g_form_mu);
  me::g_form.clear();
}

}  // extern "C"
