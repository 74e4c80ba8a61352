// Allocation-free Fock build (noalloc.hip): J' and K' accumulators of at most
// NOALLOC_MAX_PACKED elements each in a file-scope device array.
#pragma once

#include <hip/hip_runtime.h>

namespace fsim {

constexpr long long NOALLOC_MAX_PACKED = 1LL << 21;
// Device address of the array on the current device (resolved with
// hipGetSymbolAddress once per device).
hipError_t noalloc_scratch_resolve(double **out);

}  // namespace fsim
