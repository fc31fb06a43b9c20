// Device-runtime helpers of the C ABI (kept out of lb_api.hip so that its host
// logic can be built and checked without a GPU, with these stubbed): the
// current device, and the per-GPU static scratch of lb_adjoint_run_static.
//
// The static scratch: device memory for the
// two padded FP64 adjoint buffers that callers who cannot allocate do not
// pass in.  Each GPU the library runs on holds its own copy of the array for
// the life of the process.  In host code `scratch` names a host-side
// stand-in, never the device memory: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device (with that device current) and kept.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "d2q37_launch.h"

namespace d2q37 {

static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_address[kMaxDevices] = {};

}  // namespace

hipError_t current_device(int* dev) { return hipGetDevice(dev); }

hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_address[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return hipErrorInvalidValue;
    g_address[dev] = ptr;
  }
  *out = g_address[dev];
  return hipSuccess;
}

}  // namespace d2q37
