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
hipError_t fill_int(int *x, size_t n, int v, hipStream_t s);
// dst[i] = sum_{k < ncopy} src[k * stride + i] for i < n
hipError_t sum_copies(size_t n, int ncopy, const double *src, size_t stride, double *dst,
                      hipStream_t s);
hipError_t assemble_fock(int N, const double *Jh, const double *Kh, const double *H, double *F,
                         double *J, double *K, hipStream_t s);
hipError_t dot3(size_t n, const double *A, const double *B, const double *C, double w, double *out,
                hipStream_t s);
hipError_t diff2(size_t n, const double *A, const double *B, double *out, hipStream_t s);
hipError_t antisym(int N, const double *A, double *E, hipStream_t s);
hipError_t scale_cols(int N, const double *U, const double *w, double *out, hipStream_t s);
hipError_t inv_sqrt(int n, const double *sv, double *w, hipStream_t s);
hipError_t lincomb(size_t n, int m, const DiisPtrs &P, double *out, hipStream_t s);

// ---- packed per-molecule blocks (batched contexts) ----
// A batch keeps each molecule's N_m x N_m matrix at packed offset mol_off[m]
// ("packed"), or zero-padded to N_max x N_max at m * N_max^2 ("padded").
struct MolLayout {
    int nmol = 1, nmax = 0;
    const long long *off = nullptr;   // [nmol]
    const int *n = nullptr;           // [nmol]
};
hipError_t assemble_fock_packed(const MolLayout &L, const double *Jh, const double *Kh,
                                const double *H, double *F, double *J, double *K, hipStream_t s);
// J = Jref + Jh + Jh^T, K = Kref + Kh + Kh^T, F = H + J - K/2 per block (F may
// be NULL; J may alias Jref, K may alias Kref)
hipError_t assemble_delta(const MolLayout &L, const double *Jh, const double *Kh, const double *H,
                          const double *Jref, const double *Kref, double *F, double *J, double *K,
                          hipStream_t s);
// out = (A + A^T) / 2 (N x N; out must not alias A)
hipError_t symmetrize(int N, const double *A, double *out, hipStream_t s);
// J = (Jr + Jr^T)/2, K = (Kr + Kr^T)/2, F = H + J - K/2 (N x N; outputs may be
// NULL and must not alias Jr, Kr)
hipError_t assemble_sym(int N, const double *Jr, const double *Kr, const double *H, double *F,
                        double *J, double *K, hipStream_t s);
// one molecule: dD = D - Dref and M[a * ns + b] = max |dD| over shell block
// (a, b), by bit-pattern atomics on M (which must hold zeros on entry)
hipError_t delta_blockmax(int N, const double *D, const double *Dref, double *dD,
                          const int *bf_shell, int ns, double *M, hipStream_t s);
// E[m] += w * sum_block A (B + C)
hipError_t dot3_packed(const MolLayout &L, const double *A, const double *B, const double *C,
                       double w, double *E, hipStream_t s);
// padded <- packed, with `diag` on the padding diagonal
hipError_t pad_blocks(const MolLayout &L, const double *packed, double *padded, double diag,
                      hipStream_t s);
hipError_t unpad_blocks(const MolLayout &L, const double *padded, double *packed, hipStream_t s);
// padded: set the padding diagonal i >= N_m to big * (1 + i), padding off-diagonals to 0
hipError_t pad_diag(const MolLayout &L, double *padded, double big, hipStream_t s);
// padded column-major C: zero columns j >= nocc[m]
hipError_t mask_cols(const MolLayout &L, const int *nocc, double *C, hipStream_t s);
// padded: E[m] = A[m] - A[m]^T
hipError_t antisym_padded(const MolLayout &L, const double *A, double *E, hipStream_t s);
// out[m] += sum (A - B)^2 over the padded block
hipError_t diff2_padded(const MolLayout &L, const double *A, const double *B, double *out,
                        hipStream_t s);
// out[m * cnt + k] = <E_new[m], hist_k[m]> for k < cnt (hist: DiisPtrs.m[k], padded)
hipError_t dots_padded(const MolLayout &L, const double *Enew, const DiisPtrs &hist, int cnt,
                       double *out, hipStream_t s);
// out[m] = sum_k coef[m * cnt + k] hist_k[m]
hipError_t lincomb_padded(const MolLayout &L, const DiisPtrs &hist, int cnt, const double *coef,
                          double *out, hipStream_t s);
// padded column-major: out[m] = U[m] diag(w[m * N_max .. ])
hipError_t scale_cols_padded(const MolLayout &L, const double *U, const double *w, double *out,
                             hipStream_t s);

}  // namespace fsim
