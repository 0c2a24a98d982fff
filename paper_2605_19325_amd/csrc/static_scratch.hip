// Fixed device scratch for the allocation-free product entry point
// (enmf_xv_static): one file-scope device array per GPU, sized once for the
// life of the process.  Host code never passes the array's name to a kernel
// or copy: the per-device address comes from hipGetSymbolAddress, taken once
// per device at context creation with that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "enmf_internal.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[enmf::kStaticScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace enmf {

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(g_lock);
  if (g_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_ptr[device] = p;
  if (cur != device) (void)hipSetDevice(cur);
  return e == hipSuccess && !p ? hipErrorInvalidSymbol : e;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> guard(g_lock);
  return g_ptr[device];
}

}  // namespace enmf
