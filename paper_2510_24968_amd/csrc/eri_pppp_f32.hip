// (pp|pp) class kernels, FP32 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_pppp_f32(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<1, 1, 1, 1, float>(store, variant, wpb, a, s);
}

}  // namespace fsim
