// Fixed device scratch of the allocation-free sampling entry point
// (mctrg_sample_batched_noalloc): the ESP tables of the draw live in one
// file-scope device array instead of a per-call allocation.  Each device the
// library runs on holds its own copy of the array until the process ends; its
// address is looked up once per device, with that device current, and kept.
#include <mutex>

#include "mctrg_internal.h"

namespace mctrg {

namespace {
constexpr size_t kNoAllocDoubles = size_t(8) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

size_t noalloc_scratch_doubles() { return kNoAllocDoubles; }

hipError_t noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace mctrg
