// Fixed device scratch for sipg_schwarz_noalloc: the per-subdomain
// corrections of one Schwarz step live in a file-scope device array instead
// of a buffer the context allocates, so that callers which cannot allocate
// device memory at call time still get a weighted Schwarz correction.
//
// The array's name is a host-side stand-in in host code, not a device
// address: its address on each device is obtained once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels.  Every call on a device shares that device's array;
// calls that overlap on one device race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace sipg {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_addr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_addr[device];
}

}  // namespace sipg
