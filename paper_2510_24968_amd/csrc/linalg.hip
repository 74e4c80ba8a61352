// Small FP64 matrix kernels of the Fock assembly and the SCF step.
#include "linalg.h"

namespace fsim {

__global__ void k_fill(double *x, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
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
hipError_t assemble_fock(int N, const double *Jh, const double *Kh, const double *H, double *F,
                         double *J, double *K, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_fock, grid_for((size_t)N * N), dim3(256), 0, s, N, Jh, Kh, H, F,
                       J, K);
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
