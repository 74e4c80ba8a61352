// (ps|ss) class kernels, FP32 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_psss_f32(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<1, 0, 0, 0, float>(store, variant, wpb, a, s);
}

}  // namespace fsim
