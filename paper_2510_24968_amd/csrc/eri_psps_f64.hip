// (ps|ps) class kernels, FP64 arithmetic.
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_psps_f64(bool store, int variant, int wpb, const EriArgs &a,
                                 hipStream_t s) {
    return launch_class<1, 0, 1, 0, double>(store, variant, wpb, a, s);
}

}  // namespace fsim
