// Kernel instantiations for bra pair class 0 (l = 0, 0).
#include "eri_kernels.h"

namespace fsim {

hipError_t launch_eri_bra0(int ket_pc, bool fp32, bool store, const EriArgs &a, hipStream_t s) {
    switch (ket_pc) {
        case 0: return launch_class<0, 0, 0, 0>(fp32, store, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsim
