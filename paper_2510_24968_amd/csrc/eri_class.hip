// ERI kernels of one quartet class and precision.  The build compiles this
// file once per (bra pair class FSIM_BRA, ket pair class FSIM_KET, FSIM_FP32)
// so that the 42 instantiations of eri_kernels.h build in parallel; each
// object defines one explicit instantiation of launch_eri_unit.
#include "eri_kernels.h"

#if !defined(FSIM_BRA) || !defined(FSIM_KET) || !defined(FSIM_FP32)
#error "compile with -DFSIM_BRA=<0..5> -DFSIM_KET=<0..FSIM_BRA> -DFSIM_FP32=<0|1>"
#endif

namespace fsim {

template <int X, int Y, bool F32>
hipError_t launch_eri_unit(bool store, int variant, int wpb, const EriArgs &a, hipStream_t s) {
    static_assert(X >= Y && X < NPCLASS, "bra pair class must be >= ket pair class");
    using T = std::conditional_t<F32, float, double>;
    return launch_class<pc_l1(X), pc_l2(X), pc_l1(Y), pc_l2(Y), T>(store, variant, wpb, a, s);
}

template hipError_t launch_eri_unit<FSIM_BRA, FSIM_KET, (FSIM_FP32 != 0)>(bool, int, int,
                                                                          const EriArgs &,
                                                                          hipStream_t);

}  // namespace fsim
