// Utility kernels: cache flush for timing (writes a buffer larger than L2 + MALL).
#include <hip/hip_runtime.h>

namespace {
__global__ __launch_bounds__(256) void flush_kernel(uint4* buf, size_t n, unsigned v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    buf[i] = make_uint4(v, v + 1u, v + 2u, v + 3u);
}
}  // namespace

extern "C" hipError_t coot_flush_launch(void* buf, size_t bytes, unsigned v, hipStream_t s) {
  const size_t n = bytes / sizeof(uint4);
  hipLaunchKernelGGL(flush_kernel, dim3(2048), dim3(256), 0, s, (uint4*)buf, n, v);
  return hipGetLastError();
}
