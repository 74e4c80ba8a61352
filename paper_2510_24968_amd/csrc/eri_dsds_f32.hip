// (ds|ds) class kernels, FP32 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_dsds_f32(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<2, 0, 2, 0, float>(store, variant, wpb, a, s);
}

}  // namespace fsim
