// Fixed device scratch for the sweep entry point that allocates nothing
// (mm_sweep_noalloc).  The array lives in the library's code object, one copy
// per device, for the life of the process.  Host code never uses its name as
// an address: the device address of each device's copy is looked up once per
// device with hipGetSymbolAddress (at context creation, with that device
// current) and that pointer is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace mm {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices] = {};
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_setup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;  // caller makes it current
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  *out = g_ptr[device];
  return g_err[device];
}

}  // namespace mm
