// Small FP64 matrix kernels of the Fock assembly and the SCF step.
#include "linalg.h"

namespace fsim {

__global__ void k_fill(double *x, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_fill_int(int *x, size_t n, int v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_sum_copies(size_t n, int ncopy, const double *__restrict__ src, size_t stride,
                             double *dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int k = 0; k < ncopy; ++k) v += src[k * stride + i];
        dst[i] = v;
    }
}

// J = J' + J'^T, K = K' + K'^T, F = H + J - K/2 (Eq. fock, G = J - K/2).
__global__ void k_assemble_fock(int N, const double *__restrict__ Jh, const double *__restrict__ Kh,
                                const double *__restrict__ H, double *F, double *J, double *K) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / N, j = x - i * N, xt = j * N + i;
        const double jj = Jh[x] + Jh[xt], kk = Kh[x] + Kh[xt];
        if (F) F[x] = H[x] + jj - 0.5 * kk;
        if (J) J[x] = jj;
        if (K) K[x] = kk;
    }
}

// Block-reduced sum of w * sum_x A[x] * (B[x] + C[x]) (C may be NULL) into *out.
__global__ void k_dot3(size_t n, const double *__restrict__ A, const double *__restrict__ B,
                       const double *__restrict__ C, double w, double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n;
         x += (size_t)gridDim.x * blockDim.x)
        s += A[x] * (B[x] + (C ? C[x] : 0.0));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, w * red[0]);
}

// sum (A - B)^2 into *out
__global__ void k_diff2(size_t n, const double *__restrict__ A, const double *__restrict__ B,
                        double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n;
         x += (size_t)gridDim.x * blockDim.x) {
        const double d = A[x] - B[x];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// E = A - A^T (column- or row-major alike)
__global__ void k_antisym(int N, const double *__restrict__ A, double *E) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / N, j = x - i * N;
        E[x] = A[x] - A[j * N + i];
    }
}

// column j of U scaled by w[j] (column-major U)
__global__ void k_scale_cols(int N, const double *__restrict__ U, const double *__restrict__ w,
                             double *out) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t j = x / N;
        out[x] = U[x] * w[j];
    }
}

__global__ void k_inv_sqrt(int n, const double *__restrict__ s, double *w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 1.0 / sqrt(s[i]);
}

// out = sum_k c[k] * M_k  (up to 16 matrices)
__global__ void k_lincomb(size_t n, int m, DiisPtrs P, double *out) {
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n;
         x += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += P.c[k] * P.m[k][x];
        out[x] = s;
    }
}

// ---------------------------------------------------------------------------
// packed / padded per-molecule kernels: grid.y runs over molecules
// ---------------------------------------------------------------------------
__global__ void k_assemble_packed(MolLayout L, const double *__restrict__ Jh,
                                  const double *__restrict__ Kh, const double *__restrict__ H,
                                  double *F, double *J, double *K) {
    const int m = blockIdx.y, n = L.n[m];
    const size_t base = L.off[m], n2 = (size_t)n * n;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / n, j = x - i * n;
        const size_t a = base + x, at = base + j * n + i;
        const double jj = Jh[a] + Jh[at], kk = Kh[a] + Kh[at];
        if (F) F[a] = H[a] + jj - 0.5 * kk;
        if (J) J[a] = jj;
        if (K) K[a] = kk;
    }
}

// Incremental build: J = Jref + J'_d + J'_d^T, K = Kref + K'_d + K'_d^T,
// F = H + J - K/2 (J may alias Jref and K may alias Kref).
__global__ void k_assemble_delta(MolLayout L, const double *__restrict__ Jh,
                                 const double *__restrict__ Kh, const double *__restrict__ H,
                                 const double *Jref, const double *Kref, double *F, double *J,
                                 double *K) {
    const int m = blockIdx.y, n = L.n[m];
    const size_t base = L.off[m], n2 = (size_t)n * n;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / n, j = x - i * n;
        const size_t a = base + x, at = base + j * n + i;
        const double jj = Jref[a] + (Jh[a] + Jh[at]), kk = Kref[a] + (Kh[a] + Kh[at]);
        if (F) F[a] = H[a] + jj - 0.5 * kk;
        J[a] = jj;
        K[a] = kk;
    }
}

// out = (A + A^T) / 2 (out must not alias A)
__global__ void k_symmetrize(int N, const double *__restrict__ A, double *__restrict__ out) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / N, j = x - i * N;
        out[x] = 0.5 * (A[x] + A[j * N + i]);
    }
}

// J = (Jr + Jr^T)/2, K = (Kr + Kr^T)/2, F = H + J - K/2 (J, K, F may be NULL;
// none may alias Jr or Kr)
__global__ void k_assemble_sym(int N, const double *__restrict__ Jr, const double *__restrict__ Kr,
                               const double *__restrict__ H, double *F, double *J, double *K) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / N, j = x - i * N, t = j * N + i;
        const double jj = 0.5 * (Jr[x] + Jr[t]), kk = 0.5 * (Kr[x] + Kr[t]);
        if (F) F[x] = H[x] + jj - 0.5 * kk;
        if (J) J[x] = jj;
        if (K) K[x] = kk;
    }
}

// dD = D - Dref and, per shell pair (a, b), M[a * ns + b] = max |dD| over the
// block (non-negative doubles order like their bit patterns; M starts at 0).
__global__ void k_delta_blockmax(int N, const double *__restrict__ D,
                                 const double *__restrict__ Dref, double *dD,
                                 const int *__restrict__ bf_shell, int ns,
                                 unsigned long long *M) {
    const size_t n2 = (size_t)N * N;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / N, j = x - i * N;
        const double v = D[x] - Dref[x];
        dD[x] = v;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
        unsigned long long *slot = M + (size_t)bf_shell[i] * ns + bf_shell[j];
        if (bits > *slot) atomicMax(slot, bits);
    }
}

__global__ void k_dot3_packed(MolLayout L, const double *__restrict__ A,
                              const double *__restrict__ B, const double *__restrict__ C, double w,
                              double *E) {
    __shared__ double red[256];
    const int m = blockIdx.y, n = L.n[m];
    const size_t base = L.off[m], n2 = (size_t)n * n;
    double acc = 0.0;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x)
        acc += A[base + x] * (B[base + x] + (C ? C[base + x] : 0.0));
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&E[m], w * red[0]);
}

__global__ void k_pad(MolLayout L, const double *__restrict__ packed, double *padded, double diag) {
    const int m = blockIdx.y, n = L.n[m], M = L.nmax;
    const size_t M2 = (size_t)M * M;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(x / M), j = (int)(x - (size_t)i * M);
        double v;
        if (i < n && j < n) v = packed[L.off[m] + (size_t)i * n + j];
        else v = (i == j) ? diag : 0.0;
        padded[(size_t)m * M2 + x] = v;
    }
}

__global__ void k_unpad(MolLayout L, const double *__restrict__ padded, double *packed) {
    const int m = blockIdx.y, n = L.n[m], M = L.nmax;
    const size_t n2 = (size_t)n * n;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < n2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / n, j = x - i * n;
        packed[L.off[m] + x] = padded[(size_t)m * M * M + i * M + j];
    }
}

__global__ void k_pad_diag(MolLayout L, double *padded, double big) {
    const int m = blockIdx.y, n = L.n[m], M = L.nmax;
    const size_t M2 = (size_t)M * M;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(x / M), j = (int)(x - (size_t)i * M);
        if (i >= n || j >= n) padded[(size_t)m * M2 + x] = (i == j) ? big * (1.0 + i) : 0.0;
    }
}

__global__ void k_mask_cols(MolLayout L, const int *__restrict__ nocc, double *C) {
    const int m = blockIdx.y, M = L.nmax;
    const size_t M2 = (size_t)M * M;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)(x / M);   // column-major: column index is the slow one
        if (col >= nocc[m]) C[(size_t)m * M2 + x] = 0.0;
    }
}

__global__ void k_antisym_padded(MolLayout L, const double *__restrict__ A, double *E) {
    const int m = blockIdx.y, M = L.nmax;
    const size_t M2 = (size_t)M * M, base = (size_t)m * M2;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        const size_t i = x / M, j = x - i * M;
        E[base + x] = A[base + x] - A[base + j * M + i];
    }
}

__global__ void k_diff2_padded(MolLayout L, const double *__restrict__ A,
                               const double *__restrict__ B, double *out) {
    __shared__ double red[256];
    const int m = blockIdx.y, M = L.nmax;
    const size_t M2 = (size_t)M * M, base = (size_t)m * M2;
    double acc = 0.0;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        const double d = A[base + x] - B[base + x];
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&out[m], red[0]);
}

// grid: (blocks, nmol, cnt)
__global__ void k_dots_padded(MolLayout L, const double *__restrict__ En, DiisPtrs H, int cnt,
                              double *out) {
    __shared__ double red[256];
    const int m = blockIdx.y, k = blockIdx.z, M = L.nmax;
    const size_t M2 = (size_t)M * M, base = (size_t)m * M2;
    const double *__restrict__ Hk = H.m[k];
    double acc = 0.0;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x)
        acc += En[base + x] * Hk[base + x];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&out[(size_t)m * cnt + k], red[0]);
}

__global__ void k_lincomb_padded(MolLayout L, DiisPtrs H, int cnt, const double *__restrict__ coef,
                                 double *out) {
    const int m = blockIdx.y, M = L.nmax;
    const size_t M2 = (size_t)M * M, base = (size_t)m * M2;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int k = 0; k < cnt; ++k) v += coef[(size_t)m * cnt + k] * H.m[k][base + x];
        out[base + x] = v;
    }
}

__global__ void k_scale_cols_padded(MolLayout L, const double *__restrict__ U,
                                    const double *__restrict__ w, double *out) {
    const int m = blockIdx.y, M = L.nmax;
    const size_t M2 = (size_t)M * M, base = (size_t)m * M2;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < M2;
         x += (size_t)gridDim.x * blockDim.x)
        out[base + x] = U[base + x] * w[(size_t)m * M + x / M];
}

static inline dim3 grid_mol(size_t per_mol, int nmol, int z = 1) {
    size_t b = (per_mol + 255) / 256;
    if (b > 64) b = 64;
    if (b < 1) b = 1;
    return dim3((unsigned)b, (unsigned)nmol, (unsigned)z);
}

hipError_t assemble_fock_packed(const MolLayout &L, const double *Jh, const double *Kh,
                                const double *H, double *F, double *J, double *K, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_packed, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0,
                       s, L, Jh, Kh, H, F, J, K);
    return hipGetLastError();
}
hipError_t dot3_packed(const MolLayout &L, const double *A, const double *B, const double *C,
                       double w, double *E, hipStream_t s) {
    hipLaunchKernelGGL(k_dot3_packed, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s,
                       L, A, B, C, w, E);
    return hipGetLastError();
}
hipError_t pad_blocks(const MolLayout &L, const double *packed, double *padded, double diag,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_pad, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s, L,
                       packed, padded, diag);
    return hipGetLastError();
}
hipError_t unpad_blocks(const MolLayout &L, const double *padded, double *packed, hipStream_t s) {
    hipLaunchKernelGGL(k_unpad, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s, L,
                       padded, packed);
    return hipGetLastError();
}
hipError_t pad_diag(const MolLayout &L, double *padded, double big, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_diag, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s, L,
                       padded, big);
    return hipGetLastError();
}
hipError_t mask_cols(const MolLayout &L, const int *nocc, double *C, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_cols, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s, L,
                       nocc, C);
    return hipGetLastError();
}
hipError_t antisym_padded(const MolLayout &L, const double *A, double *E, hipStream_t s) {
    hipLaunchKernelGGL(k_antisym_padded, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0,
                       s, L, A, E);
    return hipGetLastError();
}
hipError_t diff2_padded(const MolLayout &L, const double *A, const double *B, double *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_diff2_padded, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0, s,
                       L, A, B, out);
    return hipGetLastError();
}
hipError_t dots_padded(const MolLayout &L, const double *Enew, const DiisPtrs &hist, int cnt,
                       double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dots_padded, grid_mol((size_t)L.nmax * L.nmax, L.nmol, cnt), dim3(256),
                       0, s, L, Enew, hist, cnt, out);
    return hipGetLastError();
}
hipError_t lincomb_padded(const MolLayout &L, const DiisPtrs &hist, int cnt, const double *coef,
                          double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb_padded, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0,
                       s, L, hist, cnt, coef, out);
    return hipGetLastError();
}

hipError_t scale_cols_padded(const MolLayout &L, const double *U, const double *w, double *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols_padded, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256),
                       0, s, L, U, w, out);
    return hipGetLastError();
}

static inline dim3 grid_for(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t fill(double *x, size_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}
hipError_t fill_int(int *x, size_t n, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, grid_for(n), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}
hipError_t sum_copies(size_t n, int ncopy, const double *src, size_t stride, double *dst,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_sum_copies, grid_for(n), dim3(256), 0, s, n, ncopy, src, stride, dst);
    return hipGetLastError();
}
hipError_t assemble_fock(int N, const double *Jh, const double *Kh, const double *H, double *F,
                         double *J, double *K, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_fock, grid_for((size_t)N * N), dim3(256), 0, s, N, Jh, Kh, H, F,
                       J, K);
    return hipGetLastError();
}
hipError_t assemble_delta(const MolLayout &L, const double *Jh, const double *Kh, const double *H,
                          const double *Jref, const double *Kref, double *F, double *J, double *K,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_delta, grid_mol((size_t)L.nmax * L.nmax, L.nmol), dim3(256), 0,
                       s, L, Jh, Kh, H, Jref, Kref, F, J, K);
    return hipGetLastError();
}
hipError_t symmetrize(int N, const double *A, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_symmetrize, grid_for((size_t)N * N), dim3(256), 0, s, N, A, out);
    return hipGetLastError();
}
hipError_t assemble_sym(int N, const double *Jr, const double *Kr, const double *H, double *F,
                        double *J, double *K, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_sym, grid_for((size_t)N * N), dim3(256), 0, s, N, Jr, Kr, H, F,
                       J, K);
    return hipGetLastError();
}
hipError_t delta_blockmax(int N, const double *D, const double *Dref, double *dD,
                          const int *bf_shell, int ns, double *M, hipStream_t s) {
    hipLaunchKernelGGL(k_delta_blockmax, grid_for((size_t)N * N), dim3(256), 0, s, N, D, Dref, dD,
                       bf_shell, ns, (unsigned long long *)M);
    return hipGetLastError();
}
hipError_t dot3(size_t n, const double *A, const double *B, const double *C, double w, double *out,
                hipStream_t s) {
    hipLaunchKernelGGL(k_dot3, grid_for(n), dim3(256), 0, s, n, A, B, C, w, out);
    return hipGetLastError();
}
hipError_t diff2(size_t n, const double *A, const double *B, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diff2, grid_for(n), dim3(256), 0, s, n, A, B, out);
    return hipGetLastError();
}
hipError_t antisym(int N, const double *A, double *E, hipStream_t s) {
    hipLaunchKernelGGL(k_antisym, grid_for((size_t)N * N), dim3(256), 0, s, N, A, E);
    return hipGetLastError();
}
hipError_t scale_cols(int N, const double *U, const double *w, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols, grid_for((size_t)N * N), dim3(256), 0, s, N, U, w, out);
    return hipGetLastError();
}
hipError_t inv_sqrt(int n, const double *sv, double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_inv_sqrt, dim3((n + 255) / 256), dim3(256), 0, s, n, sv, w);
    return hipGetLastError();
}
hipError_t lincomb(size_t n, int m, const DiisPtrs &P, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, grid_for(n), dim3(256), 0, s, n, m, P, out);
    return hipGetLastError();
}

}  // namespace fsim
