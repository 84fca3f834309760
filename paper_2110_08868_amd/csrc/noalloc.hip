// Point location without device allocation: mak_legendre_noalloc runs the
// same grid build and location kernels as mak_legendre, with every buffer they
// need (sorted sites, grid, weight bounds, staging, scan temporaries, status)
// carved from one file-scope device array instead of the context's
// workspace, for callers that cannot allocate device memory.
//
// The array is a static __device__ object: each device the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host that name is only a stand-in, not a
// device address); it resolves the copy's device address once per device
// with hipGetSymbolAddress (at mak_create, with that device current) and
// uses that address.  Every call on a device shares the one array: calls that
// overlap on one device (different streams or threads) race, and each call
// leaves its contents behind; the kernels clear what must start at zero
// (cell counts, status word) themselves.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/mak.h"
#include "engine.h"

namespace mak {

constexpr size_t kNoAllocBytes = size_t(64) << 20;

namespace {

__device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Resolve this device's copy of the array (the device must be current).
// Returns false when the address cannot be obtained.
bool noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return true;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return false;
  }
  g_ptr[device] = ptr;
  return true;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

size_t noalloc_capacity() { return kNoAllocBytes; }

}  // namespace mak
