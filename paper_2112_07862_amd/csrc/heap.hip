// Device memory of the library's calls (DevHeap, declared in common.h).
#include <algorithm>

#include "common.h"

namespace me {

DevHeap::DevHeap(void* base, size_t bytes) {
  // the region's first byte is aligned up to kHeapAlign
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t a = (b + kHeapAlign - 1) & ~(uintptr_t)(kHeapAlign - 1);
  const size_t skip = (size_t)(a - b);
  if (!base || bytes <= skip) {
    base_ = reinterpret_cast<char*>(base);  // a region with no room
    cap_ = 0;
    region_ = true;
    return;
  }
  base_ = reinterpret_cast<char*>(a);
  cap_ = (bytes - skip) & ~(size_t)(kHeapAlign - 1);
  region_ = true;
  if (cap_ > 0) free_[0] = cap_;
}

int DevHeap::alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  const size_t need = round(bytes > 0 ? bytes : 1);
  if (!region_) {
    ME_TRY(hipMallocAsync(p, need, s));
    return ME_OK;
  }
  std::lock_guard<std::mutex> lk(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[off + need] = len - need;
    live_[off] = need;
    hw_ = std::max(hw_, off + need);
    *p = base_ + off;
    return ME_OK;
  }
  return ME_ERR_WORKSPACE;
}

void DevHeap::put_back(size_t off, size_t len) {
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && off + len == nx->first) {  // merge with the next range
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {  // and with the previous one
      pv->second += len;
      return;
    }
  }
  free_[off] = len;
}

void DevHeap::release(void* p, hipStream_t s) {
  if (!p) return;
  if (!region_) {
    (void)hipFreeAsync(p, s);
    return;
  }
  std::lock_guard<std::mutex> lk(mu_);
  const size_t off = (size_t)(reinterpret_cast<char*>(p) - base_);
  auto it = live_.find(off);
  if (it == live_.end()) return;
  const size_t len = it->second;
  live_.erase(it);
  put_back(off, len);
}

void DevHeap::release_later(void* p, hipStream_t s) {
  if (!p) return;
  if (!region_) {
    (void)hipFreeAsync(p, s);
    return;
  }
  std::lock_guard<std::mutex> lk(mu_);
  later_.push_back(p);
}

void DevHeap::quiesce() {
  if (!region_) return;
  std::vector<void*> v;
  {
    std::lock_guard<std::mutex> lk(mu_);
    v.swap(later_);
  }
  for (void* p : v) release(p, nullptr);
}

bool DevHeap::owns(const void* p) const {
  if (!region_ || !p) return false;
  const char* c = reinterpret_cast<const char*>(p);
  return c >= base_ && c < base_ + cap_;
}

size_t DevHeap::largest_free() {
  if (!region_) return SIZE_MAX;
  std::lock_guard<std::mutex> lk(mu_);
  size_t m = 0;
  for (const auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

}  // namespace me
