// Fixed device scratch for the entry point that allocates nothing
// (logm_forward_noalloc): one file-scope array per device, its address looked up
// once per device with that device current.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace logm {
namespace {

// The workspace of a logm of an n x n real matrix, n <= kNoallocMaxN; every call
// on a device shares that device's copy.
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace logm
