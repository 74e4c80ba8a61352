// Kernel instantiations for bra pair class 5 (l = 2, 2).
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_bra5(int ket_pc, bool fp32, bool store, const EriArgs &a, hipStream_t s) {
    switch (ket_pc) {
        case 0: return launch_class<2, 2, 0, 0>(fp32, store, a, s);
        case 1: return launch_class<2, 2, 1, 0>(fp32, store, a, s);
        case 2: return launch_class<2, 2, 1, 1>(fp32, store, a, s);
        case 3: return launch_class<2, 2, 2, 0>(fp32, store, a, s);
        case 4: return launch_class<2, 2, 2, 1>(fp32, store, a, s);
        case 5: return launch_class<2, 2, 2, 2>(fp32, store, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsim
