// Fixed device workspace of the allocation-free adjoint entry point
// (rd_adjoint_step_noalloc): one statically sized array per GPU, held by
// the process from the first use on that GPU until it exits. Its device
// address is looked up once per device and cached; host code never passes
// the array's own name (a host-side stand-in) to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rd_noalloc.h"

namespace {

static __device__ __align__(256) unsigned char scratch[rd::kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace rd {

hipError_t noalloc_scratch(void** ptr) {
  *ptr = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace rd
