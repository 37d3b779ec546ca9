// me_embed_noalloc: the embedding solve of me_embed for callers that cannot
// allocate device memory.  Its workspace is a file-scope device array of
// the library, so the call makes no allocation of any kind; each device the
// library runs on holds its own copy until the process ends.
#include <mutex>

#include "common.h"

using namespace me;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;

// Device memory of me_embed_noalloc.  In host code this name stands for the
// symbol, not a device address: the address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
std::mutex g_in_use[kMaxDevices];   // one call at a time per device

// The address of this device's copy of `scratch` (looked up once per
// device, with the device current) and the device's call lock.
int scratch_for_device(void** ptr, std::mutex** lock) {
  int dev = 0;
  ME_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return ME_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ME_ERR_HIP;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  *lock = &g_in_use[dev];
  return ME_OK;
}

}  // namespace

extern "C" {

size_t me_embed_noalloc_max_bytes(void) { return kScratchBytes; }

int me_embed_noalloc(const me_graph_ops* ops, int K, double tol, const me_opts* opts,
                     const double* X0, double* X, double* lambda, me_info* info,
                     void* stream) {
  if (!ops || K < 1 || K > kMaxBlockCols) return ops ? ME_ERR_K_RANGE : ME_ERR_INVALID_ARG;
  me_opts o;
  if (opts) o = *opts; else me_opts_default(&o);
  if (!opts_valid(o)) return ME_ERR_INVALID_ARG;
  if (embed_workspace_bytes(ops->g.n, K, &o) > kScratchBytes) return ME_ERR_WORKSPACE;
  void* ptr = nullptr;
  std::mutex* lock = nullptr;
  ME_TRY_STATUS(scratch_for_device(&ptr, &lock));
  // the call synchronises its stream before returning, so holding the lock
  // for the call keeps two calls from sharing the array
  std::lock_guard<std::mutex> lk(*lock);
  return embed(ops->g, K, tol, &o, X0, ptr, kScratchBytes, X, lambda, info,
               (hipStream_t)stream);
}

}  // extern "C"
