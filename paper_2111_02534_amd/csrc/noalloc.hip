// Device scratch for the allocation-free entry point (tp3b_block_orth_noalloc):
// a fixed-size array in the library's own device memory, so that callers that
// cannot allocate (code under graph capture, serving loops, harnesses that
// forbid hipMalloc) still get the block orthogonalisation's partial sums and
// small factors somewhere.  Each GPU the library runs on holds its own copy of
// the array until the process ends; every call on a GPU shares it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace tp3b {

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
static double* g_scratch_dev[64] = {nullptr};
static std::mutex g_scratch_mu;

hipError_t static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace tp3b
