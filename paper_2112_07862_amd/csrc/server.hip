// Serving loop over the LOBPCG engine (continuous batching).  Requests wait
// in a queue until their device footprint fits the memory budget; an
// admitted request is built (operators up to eps) on a side stream while the
// engine's current round runs on the main stream, solves eps = lambda_2(Q)
// as one engine slot, finishes its build (mu, r, b), solves the embedding as
// another slot, and is retired as soon as that slot is certified; the freed
// memory and slot admit the next request.  Every slot's arithmetic depends
// only on its own graph, so a result is the same whether its request ran
// alone or beside others.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "engine.h"

namespace me {

SlotSpec eps_slot_spec(const GraphOps& g, const me_opts* o);
SlotSpec embed_slot_spec(const GraphOps& g, int K, double tol, const me_opts* o, const double* x0,
                         double* X, double* lambda);
int check_k_range(const GraphOps& g, int K);
int dense_eps_solve(const GraphOps& g, DevHeap& heap, hipStream_t s, double* eps);
int dense_embed_solve(const GraphOps& g, int K, double* buf, double* X, double* lambda,
                      hipStream_t s);
size_t dense_request_bytes(int64_t n);

void free_graph_ops_async(GraphOps& g, hipStream_t s) {
  if (!g.in_region) {
    if (g.mem) (void)hipFreeAsync(g.mem, s);
    if (g.mem2) (void)hipFreeAsync(g.mem2, s);
  }
  g.mem = g.mem2 = nullptr;
}

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket = 0;
  me_csr W{};
  int K = 0;
  double tol = 0.0;
  double* X = nullptr;
  double* lambda = nullptr;
  GraphOps g;
  size_t est = 0;   // footprint charged against the budget (an upper bound)
  size_t tiles = 0; // work-list bytes charged against the engine's area
  // over a caller region: the request's block (est bytes) and the heap that
  // carves its operators, scratch and solver slots
  void* block = nullptr;
  DevHeap* sub = nullptr;
  void* slot_ws = nullptr;
  int slot = -1;
  int phase = 0;  // 0 queued / building, 1 eps slot, 2 embedding slot
  int status = ME_OK;
  int eps_iters = 0;
  me_info info{};
  Clock::time_point t_admit, t_ops;
};

// Work-list area of a server over a caller region: a 128th of the region
// (at least 256 KiB); each admitted request is charged its own entries.
static size_t server_tile_sum(const me_server_opts& so) {
  if (!so.workspace) return 0;
  return std::max<size_t>(so.mem_budget / 128, (size_t)256 << 10);
}

class Server {
 public:
  Server(const me_server_opts& so, hipStream_t s)
      : so_(so), main_(s), region_(so.workspace, so.workspace ? so.mem_budget : 0),
        heap_(so.workspace ? &region_ : &hip_), tile_cap_(server_tile_sum(so)),
        eng_(s, so.opts, std::max(1, so.max_active), false, false, heap_,
             so.workspace ? Engine::tile_area_bytes(server_tile_sum(so)) : 0) {}
  ~Server();
  int init();
  int submit(const me_csr* W, int K, double tol, double* X, double* lambda, int64_t* ticket);
  int step(int* in_flight);
  int poll(int64_t* tickets, me_info* infos, int max, int* count);

 private:
  int estimate(Request* r);
  void finish(Request* r, int st);
  void drop(Request* r);
  int admit();
  int add_slots();

  me_server_opts so_;
  hipStream_t main_;
  hipStream_t side_ = nullptr;
  DevHeap hip_;      // no region: stream-ordered HIP allocations
  DevHeap region_;   // the caller's region, when one is given
  DevHeap* heap_;
  size_t tile_cap_ = 0, tiles_held_ = 0;
  Engine eng_;
  size_t budget_ = 0, held_ = 0;
  int64_t next_ticket_ = 0;
  int admitted_ = 0;  // requests past the queue and not yet finished
  std::deque<Request*> queue_;
  std::vector<Request*> want_eps_;    // built up to eps, slot not yet added
  std::vector<Request*> want_post_;   // eps known, build_post pending
  std::vector<Request*> want_embed_;  // built, embedding slot not yet added
  std::map<int, Request*> in_slot_;   // engine slot -> request
  std::vector<Request*> done_;
};

// Releases a request's device memory (its work is complete).
void Server::drop(Request* r) {
  if (r->block) {
    delete r->sub;
    r->sub = nullptr;
    heap_->release(r->block, main_);
    r->block = nullptr;
    r->g.mem = r->g.mem2 = nullptr;
  } else {
    free_graph_ops_async(r->g, main_);
  }
}

Server::~Server() {
  (void)hipStreamSynchronize(main_);
  if (side_) (void)hipStreamSynchronize(side_);
  auto drop = [&](Request* r) {
    this->drop(r);
    delete r;
  };
  for (auto* r : queue_) drop(r);
  for (auto* r : want_eps_) drop(r);
  for (auto* r : want_post_) drop(r);
  for (auto* r : want_embed_) drop(r);
  for (auto& kv : in_slot_) drop(kv.second);
  for (auto* r : done_) drop(r);
  (void)hipStreamSynchronize(main_);
  if (side_) (void)hipStreamDestroy(side_);
}

int Server::init() {
  ME_TRY(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
  ME_TRY_STATUS(eng_.init());
  budget_ = so_.mem_budget;
  if (budget_ == 0) {
    size_t fr = 0, tot = 0;
    ME_TRY(hipMemGetInfo(&fr, &tot));
    budget_ = fr / 10 * 6;
  }
  return ME_OK;
}

// Device bytes of one request, an upper bound: its build (T sized by the
// degree bound of the two-hop set, search scratch), both solver slots (eps
// and the embedding, each allocated once) or the dense solves.  Reads the
// row pointers of W.
size_t request_bytes(int64_t n, int64_t nnz, int64_t nnz_t_max, int K) {
  size_t b = build_bytes_bound(n, nnz, nnz_t_max);
  if (n <= kDenseMaxN)
    b += eps_solve_bytes(n) + DevHeap::round(dense_request_bytes(n));
  else
    b += DevHeap::round(Engine::slot_bytes(n, 4)) +
         DevHeap::round(Engine::slot_bytes(n, block_width(K)));
  return b + kHeapAlign;
}

int Server::estimate(Request* r) {
  int64_t tb = 0;
  ME_TRY_STATUS(two_hop_bound(&r->W, side_, &tb));
  const int64_t n = r->W.n;
  r->est = request_bytes(n, r->W.nnz, tb, r->K);
  r->tiles = n <= kDenseMaxN ? 0 : Engine::tile_bytes(n, std::max(4, block_width(r->K)));
  return ME_OK;
}

int Server::submit(const me_csr* W, int K, double tol, double* X, double* lambda,
                   int64_t* ticket) {
  if (!W || !X || !lambda || !ticket || !(tol > 0.0)) return ME_ERR_INVALID_ARG;
  if (K < 1 || K > kMaxBlockCols) return ME_ERR_K_RANGE;
  auto* r = new (std::nothrow) Request();
  if (!r) return ME_ERR_HIP;
  r->ticket = next_ticket_++;
  r->W = *W;
  r->K = K;
  r->tol = tol;
  r->X = X;
  r->lambda = lambda;
  queue_.push_back(r);
  *ticket = r->ticket;
  return ME_OK;
}

void Server::finish(Request* r, int st) {
  // build work of this request may still be queued on the side stream
  (void)hipStreamSynchronize(side_);
  r->status = st;
  r->info.status = st;
  if (r->slot >= 0) {
    eng_.release(r->slot);
    in_slot_.erase(r->slot);
    r->slot = -1;
  }
  drop(r);
  held_ -= std::min(held_, r->est);
  tiles_held_ -= std::min(tiles_held_, r->tiles);
  --admitted_;
  done_.push_back(r);
}

// Admission (host side, overlapping the round): builds up to eps on the side
// stream for queued requests that fit, and finishes the builds whose eps is
// known.  Graphs of at most kDenseMaxN nodes are solved here completely.
int Server::admit() {
  for (auto* r : want_post_) {
    const int st = build_post(&r->g, r->g.eps, r->eps_iters, side_);
    if (st < 0) {
      r->slot = -1;
      finish(r, st);
      continue;
    }
    r->t_ops = Clock::now();
    want_embed_.push_back(r);
  }
  want_post_.clear();
  while (!queue_.empty() && admitted_ < so_.max_active) {
    Request* r = queue_.front();
    if (r->est == 0) {
      const int se = estimate(r);
      if (se < 0) {  // malformed row pointers: the request's own error
        queue_.pop_front();
        ++admitted_;
        finish(r, se);
        continue;
      }
    }
    if (heap_->region()) {
      // reserve the request's whole footprint in the region; a request that
      // cannot fit even in an idle server fails, others wait for retirements
      const bool tiles_fit = tiles_held_ + r->tiles <= tile_cap_;
      void* blk = nullptr;
      if (tiles_fit && heap_->alloc(&blk, r->est, side_) == ME_OK) {
        r->block = blk;
        r->sub = new (std::nothrow) DevHeap(blk, r->est);
      }
      if (!r->sub) {
        if (blk) heap_->release(blk, side_);
        r->block = nullptr;
        if (admitted_ > 0) break;
        queue_.pop_front();
        ++admitted_;
        finish(r, ME_ERR_WORKSPACE);
        continue;
      }
    } else if (held_ + r->est > budget_ && admitted_ > 0) {
      // a request larger than the budget runs when nothing else is admitted
      break;
    }
    queue_.pop_front();
    ++admitted_;
    held_ += r->est;
    tiles_held_ += r->tiles;
    r->t_admit = Clock::now();
    DevHeap& rh = r->sub ? *r->sub : hip_;
    int st = build_pre(&r->W, &so_.opts, rh, side_, &r->g);
    if (st >= 0) st = check_k_range(r->g, r->K);
    if (st < 0) {
      finish(r, st);
      continue;
    }
    if (r->g.n <= kDenseMaxN) {
      double eps = 0.0;
      if (r->g.needs_eps) st = dense_eps_solve(r->g, rh, side_, &eps);
      if (st >= 0) st = build_post(&r->g, eps, 0, side_);
      if (st >= 0) {
        // a failure here is this request's error: finish() releases its
        // budget and reports it through me_server_poll
        double* buf = nullptr;
        st = rh.alloc((void**)&buf, dense_request_bytes(r->g.n), side_);
        if (st >= 0) {
          dense_embed_solve(r->g, r->K, buf, r->X, r->lambda, side_);
          if (hipStreamSynchronize(side_) != hipSuccess) st = ME_ERR_HIP;
          rh.release(buf, side_);
        }
      }
      if (st >= 0) {
        r->info.block = (int)r->g.n;
        r->info.eps = r->g.eps;
        r->info.mu = r->g.mu;
        if (st == ME_OK && r->g.status == ME_WARN_EPS_ZERO) st = ME_WARN_EPS_ZERO;
      }
      finish(r, st);
      continue;
    }
    if (r->g.needs_eps) {
      want_eps_.push_back(r);
    } else {
      st = build_post(&r->g, 0.0, 0, side_);
      if (st < 0) {
        finish(r, st);
        continue;
      }
      r->t_ops = Clock::now();
      want_embed_.push_back(r);
    }
  }
  ME_TRY(hipStreamSynchronize(side_));
  return ME_OK;
}

// Over a region a slot's memory comes from its request's block (the engine
// does not own it); otherwise the engine allocates it.
static int slot_memory(Request* r, int kb, void** ws, size_t* bytes) {
  *ws = nullptr;
  *bytes = 0;
  if (!r->sub) return ME_OK;
  *bytes = Engine::slot_bytes(r->g.n, kb);
  ME_TRY_STATUS(r->sub->alloc(ws, *bytes, nullptr));
  r->slot_ws = *ws;
  return ME_OK;
}

int Server::add_slots() {
  for (auto* r : want_eps_) {
    int id = -1;
    void* ws = nullptr;
    size_t wb = 0;
    int st = slot_memory(r, 4, &ws, &wb);
    if (st >= 0) st = eng_.add(eps_slot_spec(r->g, &so_.opts), ws, wb, &id);
    if (st < 0) {
      finish(r, st);
      continue;
    }
    r->slot = id;
    r->phase = 1;
    in_slot_[id] = r;
  }
  want_eps_.clear();
  for (auto* r : want_embed_) {
    int id = -1;
    void* ws = nullptr;
    size_t wb = 0;
    int st = slot_memory(r, block_width(r->K), &ws, &wb);
    if (st >= 0)
      st = eng_.add(embed_slot_spec(r->g, r->K, r->tol, &so_.opts, nullptr, r->X, r->lambda),
                    ws, wb, &id);
    if (st < 0) {
      finish(r, st);
      continue;
    }
    r->slot = id;
    r->phase = 2;
    in_slot_[id] = r;
  }
  want_embed_.clear();
  return ME_OK;
}

int Server::step(int* in_flight) {
  ME_TRY_STATUS(eng_.begin_round());
  ME_TRY_STATUS(admit());
  std::vector<int> fin;
  ME_TRY_STATUS(eng_.end_round(&fin));
  for (int id : fin) {
    auto it = in_slot_.find(id);
    if (it == in_slot_.end()) continue;
    Request* r = it->second;
    const SlotResult res = eng_.result(id);
    if (res.status < 0) {
      finish(r, res.status);
      continue;
    }
    const bool eps_phase = r->phase == 1;
    eng_.release(id);
    in_slot_.erase(it);
    r->slot = -1;
    if (r->sub && r->slot_ws) {  // the round is complete: the slot's memory is free
      r->sub->release(r->slot_ws, main_);
      r->slot_ws = nullptr;
    }
    if (eps_phase) {
      r->g.eps = res.lam[0];
      r->eps_iters = res.iterations;
      want_post_.push_back(r);
    } else {
      int st = res.status;
      if (st == ME_OK && r->g.status == ME_WARN_EPS_ZERO) st = ME_WARN_EPS_ZERO;
      const double ms_b =
          std::chrono::duration<double, std::milli>(r->t_ops - r->t_admit).count();
      const double ms_s = std::chrono::duration<double, std::milli>(Clock::now() - r->t_ops).count();
      r->info.iterations = res.iterations;
      r->info.eps_iterations = r->g.eps_iters;
      r->info.block = block_width(r->K);
      r->info.eps = r->g.eps;
      r->info.mu = r->g.mu;
      r->info.max_residual = res.worst;
      r->info.orth_error = res.orth;
      r->info.ms_build = ms_b;
      r->info.ms_solve = ms_s;
      finish(r, st);
    }
  }
  ME_TRY_STATUS(add_slots());
  if (in_flight) *in_flight = admitted_ + (int)queue_.size();
  return ME_OK;
}

int Server::poll(int64_t* tickets, me_info* infos, int max, int* count) {
  int c = 0;
  while (c < max && !done_.empty()) {
    Request* r = done_.front();
    done_.erase(done_.begin());
    if (tickets) tickets[c] = r->ticket;
    if (infos) infos[c] = r->info;
    delete r;
    ++c;
  }
  if (count) *count = c;
  return ME_OK;
}

}  // namespace me

struct me_server {
  me::Server* s;
};

extern "C" {

void me_server_opts_default(me_server_opts* so) {
  if (!so) return;
  so->mem_budget = 0;
  so->max_active = 256;
  so->workspace = nullptr;
  me_opts_default(&so->opts);
}

int me_server_create(const me_server_opts* so, void* stream, me_server** out) {
  if (!out) return ME_ERR_INVALID_ARG;
  *out = nullptr;
  me_server_opts o;
  if (so) o = *so; else me_server_opts_default(&o);
  if (o.max_active < 1 || !me::opts_valid(o.opts) || o.opts.product != ME_PRODUCT_FP64)
    return ME_ERR_INVALID_ARG;
  // a region must hold at least the tables and the work-list areas
  if (o.workspace && o.mem_budget < ((size_t)4 << 20)) return ME_ERR_WORKSPACE;
  auto* h = new (std::nothrow) me_server();
  if (!h) return ME_ERR_HIP;
  h->s = new (std::nothrow) me::Server(o, (hipStream_t)stream);
  if (!h->s) {
    delete h;
    return ME_ERR_HIP;
  }
  const int st = h->s->init();
  if (st < 0) {
    delete h->s;
    delete h;
    return st;
  }
  *out = h;
  return ME_OK;
}

int me_server_request_bytes(const me_csr* W, int K, void* stream, size_t* bytes) {
  if (!W || !bytes || K < 1 || K > me::kMaxBlockCols) return ME_ERR_INVALID_ARG;
  *bytes = 0;
  int64_t tb = 0;
  ME_TRY_STATUS(me::two_hop_bound(W, (hipStream_t)stream, &tb));
  *bytes = me::request_bytes(W->n, W->nnz, tb, K);
  return ME_OK;
}

int me_server_submit(me_server* s, const me_csr* W, int K, double tol, double* X,
                     double* lambda, int64_t* ticket) {
  if (!s) return ME_ERR_INVALID_ARG;
  return s->s->submit(W, K, tol, X, lambda, ticket);
}

int me_server_step(me_server* s, int* in_flight) {
  if (!s) return ME_ERR_INVALID_ARG;
  return s->s->step(in_flight);
}

int me_server_poll(me_server* s, int64_t* tickets, me_info* infos, int max, int* count) {
  if (!s || max < 0) return ME_ERR_INVALID_ARG;
  return s->s->poll(tickets, infos, max, count);
}

void me_server_destroy(me_server* s) {
  if (!s) return;
  delete s->s;
  delete s;
}

}  // extern "C"
