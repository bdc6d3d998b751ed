// Device-resident scratch of the allocation-free product (hdf_matvec_noalloc):
// a file-scope device array of fixed size, one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address: its
// device address is resolved once per device, with that device current, and
// kept here; every kernel argument or copy that needs the memory uses it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace hdf {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(void** p) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = q;
  }
  *p = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace hdf
