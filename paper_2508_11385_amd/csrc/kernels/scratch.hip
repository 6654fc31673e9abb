// Device scratch of the allocation-free reduction entry point (coot_reduce_noalloc):
// one file-scope array per device, holding the partial results that coot_reduce
// otherwise keeps in workspaces from the caller's allocator.  In host code the
// array's name is a host-side stand-in, not a device address; the address each
// device gives it is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "core.h"

namespace {
static __device__ __align__(256) unsigned char scratch[coot::kNoallocScratchBytes];

std::mutex& scratch_mutex() {
  static std::mutex m;
  return m;
}
std::vector<void*>& scratch_ptrs() {  // indexed by device ordinal; NULL = not looked up yet
  static std::vector<void*> v;
  return v;
}
}  // namespace

namespace coot {

void* noalloc_scratch() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> g(scratch_mutex());
  auto& v = scratch_ptrs();
  if ((size_t)dev >= v.size()) v.resize((size_t)dev + 1, nullptr);
  if (!v[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(COOT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    v[dev] = p;
  }
  return v[dev];
}

}  // namespace coot
