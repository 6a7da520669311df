// The library's static column scratch: a fixed-size device array that every
// GPU the library runs on holds until the process ends. It serves
// fftb_sphere_to_grid_static, the entry point for callers that cannot
// allocate device memory at call time. Host code never passes the array's
// name to a kernel: the name is only a host-side stand-in. Each device's copy
// has its own address, looked up once per device with hipGetSymbolAddress
// (with that device current) and kept here.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/fftb.h"

static __device__ __align__(256) unsigned char scratch[FFTB_STATIC_SCRATCH_BYTES];

namespace fftb {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// clear n 16-byte words (a fill kernel rather than a memset node, so that a
// caller may capture the call in a graph)
__global__ void __launch_bounds__(256) zero16(uint4* p, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}
}  // namespace

// Device address of the current device's copy of the static scratch.
hipError_t static_scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

// Clear the first `bytes` (a multiple of 16) of the scratch at device address p.
hipError_t launch_zero_scratch(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  const int grid = static_cast<int>(blocks < 2048 ? blocks : 2048);
  hipLaunchKernelGGL(zero16, dim3(grid), dim3(256), 0, st, static_cast<uint4*>(p), n);
  return hipGetLastError();
}

}  // namespace fftb
