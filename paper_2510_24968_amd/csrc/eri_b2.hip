// Kernel instantiations for bra pair class 2 (l = 1, 1).
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_bra2(int ket_pc, bool fp32, bool store, const EriArgs &a, hipStream_t s) {
    switch (ket_pc) {
        case 0: return launch_class<1, 1, 0, 0>(fp32, store, a, s);
        case 1: return launch_class<1, 1, 1, 0>(fp32, store, a, s);
        case 2: return launch_class<1, 1, 1, 1>(fp32, store, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsim
