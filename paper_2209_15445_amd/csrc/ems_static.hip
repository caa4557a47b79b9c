// ems_static.hip -- the library's static device workspace.
//
// ems_create_static runs a context in this array instead of a workspace the
// caller allocates, for callers that cannot allocate device memory (code
// under graph capture, tight serving loops, harnesses that forbid it).  Each
// GPU the library runs on holds its own copy of the array, at its own
// address, from the loading of the library's code until the process ends.
// The host only ever uses the address that hipGetSymbolAddress returns for
// the current device: the array's name in host code stands for a host-side
// shadow, not for device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ems_runtime.hpp"

namespace ems {

namespace {

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxStaticDevices];  // device address of each GPU's copy

}  // namespace

hipError_t static_workspace(int dev, void** p) {
  if (dev < 0 || dev >= kMaxStaticDevices || !p) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // once per device, with that device current
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!q || reinterpret_cast<uintptr_t>(q) % 256) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = q;
  }
  *p = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace ems
