// Device memory of the allocation-free Fock build (fsim_fock_build_noalloc):
// its J' and K' half-sum accumulators live in one file-scope device array,
// so that the entry point itself allocates nothing.  Each GPU the library
// runs on holds its own copy of the array (2 x FSIM_NOALLOC_MAX_PACKED FP64,
// 32 MiB) until the process ends.
//
// In host code `scratch` only names a host-side stand-in: its device address
// differs per GPU and is taken once per device with hipGetSymbolAddress,
// with that device current, when a context is created there.  Host code uses
// only the resolved pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace fsim {

static __device__ __align__(256) double scratch[2 * NOALLOC_MAX_PACKED];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_resolve(double **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = (double *)p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace fsim
