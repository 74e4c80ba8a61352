// Kernel instantiations for bra pair class 4 (l = 2, 1).
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_bra4(int ket_pc, bool fp32, bool store, const EriArgs &a, hipStream_t s) {
    switch (ket_pc) {
        case 0: return launch_class<2, 1, 0, 0>(fp32, store, a, s);
        case 1: return launch_class<2, 1, 1, 0>(fp32, store, a, s);
        case 2: return launch_class<2, 1, 1, 1>(fp32, store, a, s);
        case 3: return launch_class<2, 1, 2, 0>(fp32, store, a, s);
        case 4: return launch_class<2, 1, 2, 1>(fp32, store, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsim
