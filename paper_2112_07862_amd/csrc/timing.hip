// Diagnostic kernel timing: HIP events recorded around the launches of one
// kernel kind on the stream that launches them, summed when a solve ends.
// A run of back-to-back launches of the kind is bracketed by one event pair
// (an event record between two kernels costs several microseconds of GPU
// time, so per-launch pairs would distort what they measure).
// Launches that found the solve already converged (early exit) are dropped
// so that the totals cover only launches that did the work.
#include <mutex>
#include <vector>

#include "common.h"

namespace me {

namespace {
struct Pending {
  hipEvent_t a, b;
  double bytes;
  int phase, tag, launches;
};
struct KTimer {
  std::mutex mu;
  int kind = 0;
  int phase = 0;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};
KTimer& kt() {
  static KTimer t;
  return t;
}
hipEvent_t take_event(KTimer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

int ktimer_kind() { return kt().kind; }

int ktimer_new_phase() {
  std::lock_guard<std::mutex> l(kt().mu);
  return ++kt().phase;
}

KScope::KScope(int kind, hipStream_t s, double bytes, int tag, int launches)
    : on(false), s_(s) {
  KTimer& t = kt();
  if (t.kind == 0 || kind != t.kind) return;
  std::lock_guard<std::mutex> l(t.mu);
  a_ = take_event(t);
  b_ = take_event(t);
  if (!a_ || !b_) return;
  on = true;
  bytes_ = bytes;
  tag_ = tag;
  launches_ = launches;
  phase_ = t.phase;
  (void)hipEventRecord(a_, s_);
}

KScope::~KScope() {
  if (!on) return;
  (void)hipEventRecord(b_, s_);
  KTimer& t = kt();
  std::lock_guard<std::mutex> l(t.mu);
  t.pending.push_back({a_, b_, bytes_, phase_, tag_, launches_});
}

// Launches of `phase` with tag > last_real did no work (early exit).
void ktimer_drop_after(int phase, int last_real) {
  KTimer& t = kt();
  std::lock_guard<std::mutex> l(t.mu);
  std::vector<Pending> keep;
  for (auto& p : t.pending) {
    if (p.phase == phase && p.tag > last_real) {
      t.pool.push_back(p.a);
      t.pool.push_back(p.b);
    } else {
      keep.push_back(p);
    }
  }
  t.pending.swap(keep);
}

// Call after the stream has been synchronised.
void ktimer_collect() {
  KTimer& t = kt();
  std::lock_guard<std::mutex> l(t.mu);
  for (auto& p : t.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      t.ms += ms;
      t.bytes += p.bytes;
      t.launches += p.launches;
    }
    t.pool.push_back(p.a);
    t.pool.push_back(p.b);
  }
  t.pending.clear();
}

}  // namespace me

extern "C" int me_kernel_timing(int kind) {
  using namespace me;
  KTimer& t = kt();
  std::lock_guard<std::mutex> l(t.mu);
  if (kind < 0 || kind > 4) return ME_ERR_INVALID_ARG;
  t.kind = kind;
  t.launches = 0;
  t.ms = 0.0;
  t.bytes = 0.0;
  return ME_OK;
}

extern "C" int me_kernel_timing_read(int64_t* launches, double* total_ms, double* bytes) {
  using namespace me;
  KTimer& t = kt();
  std::lock_guard<std::mutex> l(t.mu);
  if (launches) *launches = t.launches;
  if (total_ms) *total_ms = t.ms;
  if (bytes) *bytes = t.bytes;
  return ME_OK;
}
