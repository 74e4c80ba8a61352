// Quartet-class dispatch: (bra pair class, ket pair class, precision) -> the
// explicit instantiation of launch_eri_unit compiled from eri_class.hip.
#include "fsim_internal.h"

namespace fsim {

template <int X, int Y>
static hipError_t unit(bool fp32, bool store, int variant, int wpb, const EriArgs &a,
                       hipStream_t s) {
    return fp32 ? launch_eri_unit<X, Y, true>(store, variant, wpb, a, s)
                : launch_eri_unit<X, Y, false>(store, variant, wpb, a, s);
}

hipError_t launch_eri(int bra_pc, int ket_pc, bool fp32, bool store, int variant, int wpb,
                      const EriArgs &a, hipStream_t s) {
#define FSIM_UNIT(X, Y) \
    case X * NPCLASS + Y: return unit<X, Y>(fp32, store, variant, wpb, a, s);
    switch (bra_pc * NPCLASS + ket_pc) {
        FSIM_UNIT(0, 0)
        FSIM_UNIT(1, 0) FSIM_UNIT(1, 1)
        FSIM_UNIT(2, 0) FSIM_UNIT(2, 1) FSIM_UNIT(2, 2)
        FSIM_UNIT(3, 0) FSIM_UNIT(3, 1) FSIM_UNIT(3, 2) FSIM_UNIT(3, 3)
        FSIM_UNIT(4, 0) FSIM_UNIT(4, 1) FSIM_UNIT(4, 2) FSIM_UNIT(4, 3) FSIM_UNIT(4, 4)
        FSIM_UNIT(5, 0) FSIM_UNIT(5, 1) FSIM_UNIT(5, 2) FSIM_UNIT(5, 3) FSIM_UNIT(5, 4)
        FSIM_UNIT(5, 5)
        default: return hipErrorInvalidValue;
    }
#undef FSIM_UNIT
}

}  // namespace fsim
