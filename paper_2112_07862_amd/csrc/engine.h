// Multi-problem LOBPCG engine: every LOBPCG solve (the eps = lambda_2(Q)
// solve of Section 4.2 and the embedding solve of Section 4.3) is a "slot"
// with its own device state.  One launch per stage covers every active slot
// of one block width through a work list of (slot, row tile) entries; the
// small per-slot solves run one workgroup per slot.  A slot's tiles and
// reduction orders depend only on its own size, so its arithmetic is the
// same whether it runs alone or beside other slots.
#pragma once

#include "common.h"

namespace me {

// Chebyshev preconditioner coefficients of one slot (written on the device
// by the residual finalize kernel each iteration).
struct ChebCoef {
  double a, theta;
  double alpha[kMaxChebDegree];
  double beta[kMaxChebDegree];
};

// Dense blocks of a slot (row-major n x kb).
enum Blk64 { BX = 0, BAX, BW, BAW, BP, BAP, BR, BY, kNumBlk64 };
enum Blk32 { BR32 = 0, BW32, BY32, kNumBlk32 };

// Device view of one slot.
struct SlotDev {
  int64_t n;
  int64_t per;      // rows per reduction tile (multiple of 16)
  int nparts;       // reduction tiles
  int need;         // leading columns that must converge
  int deflate;      // keep the iterates orthogonal to the constant vector
  int range;        // entries of the operator: all (A) or T only (Q)
  int kcopy;        // columns of x0 copied into the start block
  int k_out;        // columns written to out_x
  // operator Op in difference form: W entries w_ij, T entries
  // c_t (1/T_i + 1/T_j) (a_w holds both weights), diagonal shift s_diag
  const int32_t* a_rp;
  const int32_t* a_tp;
  const int32_t* a_col;
  const double* a_w;
  const float* a_w32;
  int64_t nnz_ops;  // entries of a_col / a_w (W and T)
  const uint32_t* a_pk;  // packed entries of the FP32 preconditioner (pk_ok)
  int pk_ok;
  // FP64 products with tq_ok read a two-hop entry as one packed word (column
  // offset, T_j) at a_tq[position - tq_base] and form its weight 1/T_i + 1/T_j
  // from invt (1 / T_i, solver order) and 1 / T_j
  const double* invt;
  const uint32_t* a_tq;
  int64_t tq_base;
  int tq_ok;
  // halos of the preconditioner's entry range (tiles of kHaloRows rows;
  // null h_cnt: none): per entry its slot in the tile's list and its FP16
  // weight, the lists, their lengths and the largest
  const uint32_t* h_pk;
  const int32_t* h_list;
  const int32_t* h_cnt;
  int h_max;
  double c_t, s_diag;
  const double* bdiag;  // null: B = I
  const double* dinv;   // diag(Op)^-1 (Jacobi preconditioner)
  const float* dinv32;
  // operator the Chebyshev preconditioner inverts: the same rows restricted
  // to an entry range (all, W only or T only; T entries scaled by c_t), with
  // its own diagonal shift and Jacobi scaling
  int cheb_range;
  double cheb_s_diag;
  const double* cheb_dinv;
  const float* cheb_dinv32;
  const int32_t* perm;   // solver row -> user row (null: identity)
  const int32_t* iperm;  // user row -> solver row
  const double* x0;      // user-order n x kcopy start columns (may be null)
  uint64_t seed;
  // smooth start: column j < nsmooth is cos(pi (j + jfreq) (level + 1/2) /
  // (max_level + 1)) plus a tenth of the seeded random column (null lev:
  // random start)
  const int32_t* lev;
  int32_t max_lev;
  int32_t jfreq;
  int32_t nsmooth;
  double* out_x;         // user-order n x k_out output (may be null)
  double* out_lam;       // k_out
  double* b64[kNumBlk64];
  float* b32[kNumBlk32];
  double* partials;  // nparts x 2 (3kb)^2
  double* gram;      // 2 (3kb)^2
  double* coef;      // 2 (3kb) kb
  double* coefw;     // 2 kb kb
  double* lam;       // kb
  double* sums;      // kb
  double* scratch;   // nparts x kb x (double, int64): sign convention
  Ctrl* ctrl;
  ChebCoef* cheb;
};

// One entry of a work list: block `blk` of slot `slot`.
struct Tile {
  int32_t slot;
  int32_t blk;
};

constexpr int kGatherRows = 32;  // rows per workgroup of the gathering kernels
constexpr int kGramBigRows = 512;  // reduction tiles this tall run the Grams in 8 waves

// Work lists of one set of slots with a common block width kb (device).
struct TileSet {
  int kb = 0;
  int nslots = 0;
  const int32_t* slots = nullptr;  // slot ids
  const Tile* gather = nullptr;    // kGatherRows rows per tile
  const Tile* elem64 = nullptr;    // kBlock / LPR(double, kb) rows per tile
  const Tile* elem32 = nullptr;    // kBlock / LPR(float, kb) rows per tile
  const Tile* red = nullptr;       // reduction tiles (slot.per rows)
  int64_t n_gather = 0, n_elem64 = 0, n_elem32 = 0, n_red = 0;
  int64_t n_red_big = 0;           // leading reduction tiles of slots with kGramBigRows rows and more
  bool buf = false;                // every array below kBufMaxBytes (buffer loads)
  bool pk = false;                 // every slot has packed preconditioner entries
  void* mem = nullptr;             // device allocation behind the lists
  std::vector<char> host;          // staging copy (kept until the next sync)
  std::vector<int> ids;            // slot ids (host)
};

// ---- slot_ops.hip: one launch per stage over a TileSet ---------------------
// `cert` = 1 runs the stage for slots whose done flag is set (start and
// certificate passes); otherwise such slots are skipped.
template <typename T>
void sl_spmm(const SlotDev* sl, const TileSet& ts, int in, int out, int cert, hipStream_t s);
// y <- D^-1 R / theta, yprev <- 0; then y_{k+1} into yout (which holds y_{k-1})
template <typename T>
void sl_cheb_first(const SlotDev* sl, const TileSet& ts, int r, int y, int yprev, hipStream_t s);
// host_sl: the host copy of the slot table (a one-slot set passes its
// slot's pointers in the kernel arguments).  form: kFormHalo (the
// halo-staged step where the slots have halos that fit) or kFormGather (the
// gathering step); both give the same results bit for bit.
enum { kFormHalo = 0, kFormGather = 1 };
template <typename T>
void sl_cheb_step(const SlotDev* sl, const SlotDev* host_sl, const TileSet& ts, int k, int r,
                  int yin, int yout, hipStream_t s, int form = kFormHalo);
// R = AX - B X Lambda (-> block w unless w < 0; Jacobi-scaled if jacobi),
// per-tile sums of |r|^2, |Bx|^2, x^T D x.
void sl_resid(const SlotDev* sl, const TileSet& ts, int w, int jacobi, int cert, hipStream_t s);
void sl_resid_finalize(const SlotDev* sl, const TileSet& ts, int final_pass, hipStream_t s);
// Gram products per slot: G1 = U^T diag(b) V (or U^T V), G2 = U^T V2.
void sl_gram(const SlotDev* sl, const TileSet& ts, int nu, const int* u, int nv, const int* v,
             int nv2, const int* v2, int use_b, int cert, hipStream_t s);
void sl_reduce(const SlotDev* sl, const TileSet& ts, int nent, int cert, hipStream_t s);
// out_o = sum_s in_s C_o (C_o: (nin kb) x kb, stacked per output) for
// ngroup groups sharing the coefficients; coefficients at coef (which 0) or
// coefw (which 1) plus `off`.
void sl_combine(const SlotDev* sl, const TileSet& ts, int nin, int ngroup, const int* in0,
                const int* in1, int nout, const int* out0, const int* out1, int which, int off,
                int cert, hipStream_t s);
void sl_deflate(const SlotDev* sl, const TileSet& ts, int blk, int cert, hipStream_t s);
void sl_to32(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s);
void sl_to64(const SlotDev* sl, const TileSet& ts, int from32, int to64, hipStream_t s);
void sl_to32_scaled(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s);
void sl_to16_scaled(const SlotDev* sl, const TileSet& ts, int from64, int to32, hipStream_t s);
bool sl_cheb_h_ok(const SlotDev* host_sl, const TileSet& ts);
void sl_cheb_first_h(const SlotDev* sl, const TileSet& ts, int r, int y, int yprev, hipStream_t s);
void sl_cheb_step_h(const SlotDev* host_sl, const TileSet& ts, int k, int r, int yin, int yout,
                    hipStream_t s);
void sl_to64_h(const SlotDev* sl, const TileSet& ts, int from, int to, hipStream_t s);
void sl_fill_start(const SlotDev* sl, const TileSet& ts, hipStream_t s);
void sl_zero(const SlotDev* sl, const TileSet& ts, int blk, hipStream_t s);
// max |X^T B X - I| over the first `need` columns -> ctrl->orth (uses gram)
void sl_orth(const SlotDev* sl, const TileSet& ts, hipStream_t s);
void sl_reenter(const SlotDev* sl, const TileSet& ts, hipStream_t s);
void sl_output(const SlotDev* sl, const TileSet& ts, hipStream_t s);

// ---- dense.hip ---------------------------------------------------------------
void sl_rayleigh_ritz(const SlotDev* sl, const TileSet& ts, int nb, double piv_tol,
                      int final_pass, hipStream_t s);
void sl_cholqr_coef(const SlotDev* sl, const TileSet& ts, double piv_tol, hipStream_t s);

// ---- engine.hip ----------------------------------------------------------------
// Host description of one problem.
struct SlotSpec {
  const GraphOps* g = nullptr;
  OpKind op = OP_A;
  int kb = 4;
  int need = 1;
  double tol = 1e-6;
  int max_iter = 1000;
  bool deflate = false;
  double cheb_b = 2.0;     // upper end of the Chebyshev interval
  double lam_scale = 1.0;  // operator scale (replaces |lambda| near zero)
  uint64_t seed = 0;
  const double* x0 = nullptr;  // user-order n x kcopy (device)
  int nsmooth = 0;             // leading columns of the start from the breadth-first levels
  int jfreq = 0;               // frequency of column 0 of the smooth start
  int kcopy = 0;
  double* out_x = nullptr;  // user-order n x k_out (device)
  double* out_lam = nullptr;
  int k_out = 0;
};

// Result of a finished slot.
struct SlotResult {
  int status = 0;  // ME_OK, ME_WARN_NOT_CONVERGED, ME_ERR_BREAKDOWN
  int iterations = 0;
  double worst = 0.0;  // largest rho over the required columns
  double orth = 0.0;
  double lam[kMaxBlockCols] = {};
};

class Engine {
 public:
  // solo: the caller solves one input graph (me_embed, a batch of one
  // graph), which alone may take FP16 Chebyshev iterates; the engine's
  // capacity is not used for that, so that a graph's arithmetic never
  // depends on which other graphs share a batch or a server
  // heap: device memory of the engine (null: stream-ordered HIP
  // allocations).  Over a caller region the engine also needs tile_area
  // bytes twice (work lists of the active slots and of the slots being
  // started or certified): at least tile_area_bytes of the summed
  // tile_bytes of the slots that can be active at once.
  Engine(hipStream_t s, const me_opts& o, int capacity, bool timed, bool solo = false,
         DevHeap* heap = nullptr, size_t tile_area = 0);
  ~Engine();
  int init();
  // Workspace of one slot (device bytes).
  static size_t slot_bytes(int64_t n, int kb);
  // Slot table, control blocks and Chebyshev coefficients of `capacity` slots.
  static size_t table_bytes(int capacity);
  // Work-list entries of one slot (device bytes, before rounding).
  static size_t tile_bytes(int64_t n, int kb);
  // One work-list area for slots whose tile_bytes sum to `sum`.
  static size_t tile_area_bytes(size_t sum);
  // Every allocation of an engine of these slots that runs to completion
  // (tables, slots, both work-list areas), each rounded to the heap's unit.
  static size_t run_bytes(const std::vector<std::pair<int64_t, int>>& slots);
  // Registers a problem (ws: caller memory of slot_bytes, or null to let the
  // engine allocate); it starts at the next run()/step().  id >= 0 on success.
  int add(const SlotSpec& sp, void* ws, size_t ws_bytes, int* id);
  // Iterates until every registered problem has finished.
  int run();
  // One round: starts new problems, check_every iterations of the active
  // ones, certification and output of those that stopped; appends the ids
  // that finished in this round.
  int step(std::vector<int>* finished);
  // step() in two halves, so that host work can overlap the round on the GPU
  int begin_round();
  int end_round(std::vector<int>* finished);
  bool idle() const;
  int active() const;
  const SlotResult& result(int id) const { return res_[id]; }
  // Frees a finished slot's id (and its workspace if the engine owned it).
  void release(int id);
  size_t bytes_in_use() const { return bytes_in_use_; }

 private:
  struct SlotHost {
    bool used = false;
    bool started = false;
    bool finished = false;
    bool own_ws = false;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    SlotSpec sp;
    int reentries = 0;
  };
  // area: 0 for the active slots' lists, 1 for start and certificate passes
  int build_set(const std::vector<int>& ids, int kb, TileSet* ts, int area);
  void free_set(TileSet* ts);
  int upload_slot(int id);
  void start_pass(const TileSet& ts);
  void rr_x(const TileSet& ts, int final_pass);
  void iteration(const TileSet& ts);
  int read_ctrl();
  int sets_for(const std::vector<int>& ids, std::vector<TileSet>* sets, int area);
  void free_sets(std::vector<TileSet>* sets);
  int certify(const std::vector<int>& ids, std::vector<int>* finished);

  hipStream_t s_;
  me_opts o_;
  int cap_;
  bool timed_;
  bool solo_;
  bool cheb_, cheb32_;
  std::vector<SlotHost> sh_;
  std::vector<SlotResult> res_;
  std::vector<SlotDev> hdev_;
  DevHeap own_heap_;   // stream-ordered HIP allocations when no heap is given
  DevHeap* heap_;
  size_t tile_area_ = 0;
  void* tables_ = nullptr;
  void* tile_mem_ = nullptr;
  struct Area {
    char* base = nullptr;
    size_t cap = 0, used = 0;
  } areas_[2];
  SlotDev* d_slots_ = nullptr;
  Ctrl* d_ctrl_ = nullptr;
  ChebCoef* d_cheb_ = nullptr;
  Ctrl* h_ctrl_ = nullptr;  // host mirror (pinned in HIP mode, pageable over a region)
  std::vector<Ctrl> h_ctrl_pageable_;
  std::vector<int> active_;
  std::vector<TileSet> sets_;  // work lists of active_, one per block width
  // convergence history per slot (largest required rho at the last check)
  std::vector<int> iter0_;
  bool round_open_ = false;
  int round_length();
  bool sets_dirty_ = true;
  // one iteration of every active set as a replayable graph (ME_LAUNCH_GRAPH)
  int enqueue_round(int ce);
  void drop_graph();
  hipStream_t cap_s_ = nullptr;  // private capture stream
  bool capturing_ = false;        // iterations are being recorded into a graph
  // run-time choice of the one-slot preconditioner step's form: the first
  // iteration of a kind of slot not seen before in this process runs its
  // steps in blocks of kTuneBlock, alternating the two forms, and times each
  // block; the form with the shorter time per step is kept for that kind
  static constexpr int kTuneBlock = 8;
  struct FormTune {
    bool live = false;
    int key[3] = {0, 0, 0};      // block width, entry range, log2 of the rows
    std::vector<hipEvent_t> ev;  // block boundaries
    std::vector<int> steps;      // steps of each block (even blocks: halo form)
    int used = 0;                // boundaries recorded
  } tune_;
  int step_form(const TileSet& ts, bool* tune);
  void finish_tune();
  hipGraphExec_t gexec_ = nullptr;
  int sets_ver_ = 0, gexec_ver_ = -1;
  size_t bytes_in_use_ = 0;
  int phase_ = 0, tag_ = 0;
};

int block_width(int K);
int partial_tiles(int64_t n);

}  // namespace me
