// Utility kernels: cache flush for timing.  It streams through a buffer larger than
// L2 + the Infinity Cache, reading it (a written buffer would leave dirty lines whose
// write-back the next, timed kernel would pay for); each thread folds what it read
// into one word of a small per-thread slot area at the buffer's start, so the reads
// cannot be dropped and almost nothing is left dirty.
#include <hip/hip_runtime.h>

namespace {
__global__ __launch_bounds__(256) void flush_kernel(uint4* buf, size_t n, unsigned v) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nt = (size_t)gridDim.x * blockDim.x;
  unsigned x = v;
  for (size_t i = nt + tid; i < n; i += nt) {
    const uint4 q = buf[i];
    x ^= q.x ^ q.y ^ q.z ^ q.w;
  }
  reinterpret_cast<unsigned*>(buf)[tid] = x;
}
}  // namespace

extern "C" hipError_t coot_flush_launch(void* buf, size_t bytes, unsigned v, hipStream_t s) {
  const size_t n = bytes / sizeof(uint4);
  hipLaunchKernelGGL(flush_kernel, dim3(2048), dim3(256), 0, s, (uint4*)buf, n, v);
  return hipGetLastError();
}
