// (ds|pp) class kernels, FP32 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_dspp_f32(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<2, 0, 1, 1, float>(store, variant, wpb, a, s);
}

}  // namespace fsim
