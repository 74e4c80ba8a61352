// (dd|pp) class kernels, FP64 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_ddpp_f64(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<2, 2, 1, 1, double>(store, variant, wpb, a, s);
}

}  // namespace fsim
