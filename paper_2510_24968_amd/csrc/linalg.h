// Small FP64 matrix kernels of the Fock assembly and the SCF step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fsim {

constexpr int DIIS_MAX = 16;
struct DiisPtrs {
    const double *m[DIIS_MAX];
    double c[DIIS_MAX];
};

hipError_t fill(double *x, size_t n, double v, hipStream_t s);
hipError_t assemble_fock(int N, const double *Jh, const double *Kh, const double *H, double *F,
                         double *J, double *K, hipStream_t s);
hipError_t dot3(size_t n, const double *A, const double *B, const double *C, double w, double *out,
                hipStream_t s);
hipError_t diff2(size_t n, const double *A, const double *B, double *out, hipStream_t s);
hipError_t antisym(int N, const double *A, double *E, hipStream_t s);
hipError_t scale_cols(int N, const double *U, const double *w, double *out, hipStream_t s);
hipError_t inv_sqrt(int n, const double *sv, double *w, hipStream_t s);
hipError_t lincomb(size_t n, int m, const DiisPtrs &P, double *out, hipStream_t s);

}  // namespace fsim
