// Memory-bandwidth references for the measurements (not on any solve path):
// a streaming copy, a read-only pass and a write-only pass over a caller's
// buffer in 16-byte vectors with non-temporal accesses, each a grid-stride
// loop over a fixed grid of four 256-thread blocks per CU.  The read pass
// keeps its loads alive with a sum that is stored only if it equals a value
// the data cannot produce.
#include "lib.h"

namespace dirac {

namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_probe_copy(const vf4* __restrict__ a, vf4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ void __launch_bounds__(256) k_probe_read(const vf4* __restrict__ a, vf4* __restrict__ sink, size_t n) {
  vf4 s = {0.f, 0.f, 0.f, 0.f};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += __builtin_nontemporal_load(a + i);
  if (s.x + s.y + s.z + s.w == -1.2345e30f) sink[0] = s;
}

__global__ void __launch_bounds__(256) k_probe_write(vf4* __restrict__ b, size_t n) {
  const vf4 v = {1.f, 2.f, 3.f, 4.f};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(v, b + i);
}

}  // namespace

}  // namespace dirac

using namespace dirac;

extern "C" int dirac_bandwidth_probe(int32_t kind, const void* src, void* dst, int64_t bytes, void* stream) {
  clear_error();
  if (kind < 0 || kind > 2) return set_error(DIRAC_EINVAL, "dirac_bandwidth_probe: kind must be 0, 1 or 2");
  if (bytes <= 0 || bytes % 16) return set_error(DIRAC_EINVAL, "dirac_bandwidth_probe: bytes must be a positive multiple of 16");
  if (dst == nullptr || (kind != 2 && src == nullptr))
    return set_error(DIRAC_EINVAL, "dirac_bandwidth_probe: NULL buffer");
  if ((((uintptr_t)src | (uintptr_t)dst) & 15u) != 0)
    return set_error(DIRAC_EINVAL, "dirac_bandwidth_probe: buffers must be 16-byte aligned");
  if (kind == 0) {
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return set_error(DIRAC_EINVAL, "dirac_bandwidth_probe: buffers overlap");
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  const size_t n = (size_t)bytes / 16;
  const dim3 grid(4 * cus), block(256);
  hipStream_t st = (hipStream_t)stream;
  const vf4* a = (const vf4*)src;
  vf4* b = (vf4*)dst;
  if (kind == 0) hipLaunchKernelGGL(k_probe_copy, grid, block, 0, st, a, b, n);
  else if (kind == 1) hipLaunchKernelGGL(k_probe_read, grid, block, 0, st, a, b, n);
  else hipLaunchKernelGGL(k_probe_write, grid, block, 0, st, b, n);
  return hip_status(hipGetLastError(), "bandwidth probe launch");
}
