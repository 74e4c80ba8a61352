// BF16 matrix-core kernels of the learned initial-guess network: a GEMM on
// v_mfma_f32_16x16x16bf16_1k with FP32 accumulation (optional transposes,
// split-K with FP32 atomics, fused bias + ReLU epilogue), and the elementwise
// pieces of training (ReLU backward, bias gradient, MSE loss and gradient,
// Adam with FP32 master weights, FP32 -> BF16 rounding).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/fsim.h"

namespace fsim {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even FP32 -> BF16 (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GT = 64;    // block tile (M and N)
constexpr int GK = 16;    // K step (one MFMA)

// C[M x N] (+)= op(A)[M x K] op(B)[K x N]; A, B BF16 row-major with leading
// dimensions lda, ldb (op = transpose when ta / tb).  256 threads = 4 waves,
// each wave owns a 32 x 32 quarter of the 64 x 64 tile (2 x 2 MFMA tiles).
// grid.z splits K; with splits > 1 the partial sums are added atomically
// into C (which the caller zeroes) and the epilogue must be plain.
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A,
                                                   int lda, int ta, const uint16_t *__restrict__ B,
                                                   int ldb, int tb, float *C, int ldc,
                                                   uint16_t *Cb, const float *__restrict__ bias,
                                                   int relu, int atomic) {
    __shared__ uint16_t As[GT][GK + 2];   // [m][k]
    __shared__ uint16_t Bs[GK][GT + 2];   // [k][n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kper = (K + gridDim.z - 1) / gridDim.z;
    const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        // stage the 64 x 16 slice of op(A) and the 16 x 64 slice of op(B)
        for (int e = tid; e < GT * GK; e += 256) {
            const int r = e / GK, k = e % GK;
            const int gm = m0 + r, gk = k0 + k;
            uint16_t v = 0;
            if (gm < M && gk < kend) v = ta ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[r][k] = v;
            const int k2 = e / GT, c = e % GT;
            const int gn = n0 + c, gk2 = k0 + k2;
            uint16_t w = 0;
            if (gn < N && gk2 < kend) w = tb ? B[(size_t)gn * ldb + gk2] : B[(size_t)gk2 * ldb + gn];
            Bs[k2][c] = w;
        }
        __syncthreads();
        // lane layout of the 16x16x16 MFMA: A row = lane % 16, k = 4 (lane / 16) + j;
        // B column = lane % 16, k = 4 (lane / 16) + j
        const int r16 = lane & 15, kq = (lane >> 4) * 4;
        bf16x4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[i][j] = (short)As[wm + 16 * i + r16][kq + j];
                b[i][j] = (short)Bs[kq + j][wn + 16 * i + r16];
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result layout: column = lane % 16, rows 4 (lane / 16) + q
    const int c16 = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gm = m0 + wm + 16 * i + rq + q, gn = n0 + wn + 16 * j + c16;
                if (gm >= M || gn >= N) continue;
                float v = acc[i][j][q];
                if (atomic) {
                    atomicAdd(&C[(size_t)gm * ldc + gn], v);
                    continue;
                }
                if (bias) v += bias[gn];
                if (relu) v = v > 0.f ? v : 0.f;
                if (C) C[(size_t)gm * ldc + gn] = v;
                if (Cb) Cb[(size_t)gm * ldc + gn] = f2bf(v);
            }
}

__global__ void k_f2bf(size_t n, const float *__restrict__ x, uint16_t *y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// dH <- dH * (H > 0) (FP32), and its BF16 copy
__global__ void k_relu_bwd(size_t n, const float *__restrict__ H, float *dH, uint16_t *dHb) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float g = H[i] > 0.f ? dH[i] : 0.f;
        dH[i] = g;
        if (dHb) dHb[i] = f2bf(g);
    }
}

// db[j] = sum_i dY[i][j]
__global__ void k_bias_grad(int n, int m, const float *__restrict__ dY, float *db) {
    const int j = blockIdx.x;
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += dY[(size_t)i * m + j];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[j] = red[0];
}

// masked MSE: loss += sum mask (Y - T)^2 / count;  dY = 2 mask (Y - T) / count
__global__ void k_mse(size_t n, const float *__restrict__ Y, const float *__restrict__ T,
                      const float *__restrict__ mask, float inv_count, float *dY, float *loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float d = (Y[i] - T[i]) * mask[i];
        s += d * d;
        dY[i] = 2.f * d * inv_count;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv_count);
}

// Adam on FP32 master weights, then the BF16 copy
__global__ void k_adam(size_t n, float *w, const float *__restrict__ g, float *m1, float *m2,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *wb) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.f - b1) * gi, b = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float v = w[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
        w[i] = v;
        if (wb) wb[i] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------
// Fused inference of the three-layer guess network.  One block of 4 waves
// takes 32 rows through all three layers; the BF16 hidden activations stay
// in LDS and are rounded exactly where the layered GEMMs round them, and the
// K loop runs in the same 16-wide MFMA steps in the same order, so the
// output equals the layered forward pass bit for bit.  Weights come from
// global memory (L2-resident, read by every block) pre-packed in MFMA
// fragment order: one 8-byte load per lane per 16 x 16 B fragment.
// ---------------------------------------------------------------------------
constexpr int FR = 32;                          // rows per block
constexpr int FIN = 64, FH = 256, FOUT = 36;
constexpr int FXP = FIN + 4, FHP = FH + 4;      // LDS row pitches (BF16): 8-byte rows, skewed banks

// Packed fragment layout of a K x N BF16 matrix (row-major, ld = N): for K
// step s (16 rows) and column tile t (16 columns), lane l holds rows
// 16 s + 4 (l / 16) + j, j < 4, of column 16 t + l % 16 (zero past N):
// Wp[((s * ntile + t) * 64 + l) * 4 + j].
__global__ void k_pack_frag(int K, int N, const uint16_t *__restrict__ W, uint16_t *Wp) {
    const int ntile = (N + 15) / 16;
    const size_t total = (size_t)(K / 16) * ntile * 256;
    for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < total;
         x += (size_t)gridDim.x * blockDim.x) {
        const int j = x & 3, l = (x >> 2) & 63;
        const size_t st = x >> 8;
        const int t = (int)(st % ntile), sk = (int)(st / ntile);
        const int k = 16 * sk + 4 * (l >> 4) + j, n = 16 * t + (l & 15);
        Wp[x] = n < N ? W[(size_t)k * N + n] : (uint16_t)0;
    }
}

// acc[i][c] += A[row0 + 16 i .., 0..K) W[0..K, 16 (t0 + c) ..) for the
// wave's NRT row tiles and NCT column tiles; A in LDS (pitch in BF16).
template <int K, int NRT, int NCT>
__device__ __forceinline__ void frag_mma(const uint16_t *As, int pitch, int row0,
                                         const uint16_t *__restrict__ Wp, int ntile, int t0,
                                         f32x4 (&acc)[NRT][NCT]) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < NRT; ++i)
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x4 *__restrict__ wf = (const bf16x4 *)Wp + (size_t)t0 * 64 + lane;
#pragma unroll 2
    for (int s = 0; s < K / 16; ++s) {
        bf16x4 a[NRT], b[NCT];
#pragma unroll
        for (int i = 0; i < NRT; ++i)
            a[i] = *(const bf16x4 *)(As + (row0 + 16 * i + r16) * pitch + 16 * s + kq);
#pragma unroll
        for (int c = 0; c < NCT; ++c) b[c] = wf[((size_t)s * ntile + c) * 64];
#pragma unroll
        for (int i = 0; i < NRT; ++i)
#pragma unroll
            for (int c = 0; c < NCT; ++c)
                acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[c], acc[i][c], 0, 0, 0);
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(int n, const uint16_t *__restrict__ X,
                                                     const uint16_t *__restrict__ W1p,
                                                     const float *__restrict__ b1,
                                                     const uint16_t *__restrict__ W2p,
                                                     const float *__restrict__ b2,
                                                     const uint16_t *__restrict__ W3p,
                                                     const float *__restrict__ b3, float *Y) {
    __shared__ __align__(16) uint16_t xs[FR * FXP];
    __shared__ __align__(16) uint16_t h1[FR * FHP];
    __shared__ __align__(16) uint16_t h2[FR * FHP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * FR;
    const int c16 = lane & 15, rq = (lane >> 4) * 4;
    // input tile, 8 bytes per access; rows past n are zero
    for (int e = tid; e < FR * (FIN / 4); e += 256) {
        const int r = e / (FIN / 4), c4 = e % (FIN / 4);
        uint2 v = {0u, 0u};
        if (m0 + r < n) v = *(const uint2 *)(X + (size_t)(m0 + r) * FIN + 4 * c4);
        *(uint2 *)(xs + r * FXP + 4 * c4) = v;
    }
    __syncthreads();
    // hidden layers: wave w owns columns [64 w, 64 w + 64) of all 32 rows
    auto hidden = [&](const uint16_t *in, int pitch_in, const uint16_t *Wp, const float *bias,
                      uint16_t *out, auto kdim) {
        constexpr int K = decltype(kdim)::value;
        f32x4 acc[FR / 16][4];
        frag_mma<K, FR / 16, 4>(in, pitch_in, 0, Wp, FH / 16, 4 * wave, acc);
#pragma unroll
        for (int i = 0; i < FR / 16; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = 64 * wave + 16 * c + c16;
                const float bc = bias[col];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = acc[i][c][q] + bc;
                    v = v > 0.f ? v : 0.f;
                    out[(16 * i + rq + q) * FHP + col] = f2bf(v);
                }
            }
    };
    hidden(xs, FXP, W1p, b1, h1, std::integral_constant<int, FIN>{});
    __syncthreads();
    hidden(h1, FHP, W2p, b2, h2, std::integral_constant<int, FH>{});
    __syncthreads();
    // output layer: waves 0 and 1 take one 16-row tile each, 3 column tiles
    if (wave < FR / 16) {
        f32x4 acc[1][3];
        frag_mma<FH, 1, 3>(h2, FHP, 16 * wave, W3p, 3, 0, acc);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int col = 16 * c + c16;
            if (col >= FOUT) continue;
            const float bc = b3[col];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + 16 * wave + rq + q;
                if (row < n) Y[(size_t)row * FOUT + col] = acc[0][c][q] + bc;
            }
        }
    }
}

static inline dim3 grid1(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

}  // namespace fsim

using namespace fsim;

extern "C" fsim_status fsim_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A,
                                      int32_t lda, int32_t ta, const uint16_t *B, int32_t ldb,
                                      int32_t tb, float *C, int32_t ldc, uint16_t *Cb,
                                      const float *bias, int32_t relu, int32_t ksplit,
                                      void *stream) {
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || (!C && !Cb)) return FSIM_EINVAL;
    if (ksplit < 1) ksplit = 1;
    if (ksplit > 1 && (!C || Cb || bias || relu)) return FSIM_EINVAL;
    dim3 g((N + GT - 1) / GT, (M + GT - 1) / GT, ksplit);
    hipLaunchKernelGGL(k_gemm_bf16, g, dim3(256), 0, (hipStream_t)stream, M, N, K, A, lda, ta, B,
                       ldb, tb, C, ldc, Cb, bias, relu, ksplit > 1 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_f32_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream) {
    if (n < 0 || (n > 0 && (!x || !y))) return FSIM_EINVAL;
    if (n == 0) return FSIM_OK;
    hipLaunchKernelGGL(k_f2bf, grid1(n), dim3(256), 0, (hipStream_t)stream, (size_t)n, x, y);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_relu_backward(int64_t n, const float *H, float *dH, uint16_t *dHb,
                                          void *stream) {
    if (n <= 0 || !H || !dH) return FSIM_EINVAL;
    hipLaunchKernelGGL(k_relu_bwd, grid1(n), dim3(256), 0, (hipStream_t)stream, (size_t)n, H, dH, dHb);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_bias_grad(int32_t n, int32_t m, const float *dY, float *db,
                                      void *stream) {
    if (n <= 0 || m <= 0 || !dY || !db) return FSIM_EINVAL;
    hipLaunchKernelGGL(k_bias_grad, dim3(m), dim3(256), 0, (hipStream_t)stream, n, m, dY, db);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_mse(int64_t n, const float *Y, const float *T, const float *mask,
                                float inv_count, float *dY, float *loss, void *stream) {
    if (n <= 0 || !Y || !T || !mask || !dY || !loss) return FSIM_EINVAL;
    hipLaunchKernelGGL(k_mse, grid1(n), dim3(256), 0, (hipStream_t)stream, (size_t)n, Y, T, mask,
                       inv_count, dY, loss);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_adam(int64_t n, float *w, const float *g, float *m1, float *m2,
                                 float lr, float b1, float b2, float eps, int32_t step,
                                 uint16_t *wb, void *stream) {
    if (n <= 0 || !w || !g || !m1 || !m2 || step < 1) return FSIM_EINVAL;
    float pb1 = 1.f, pb2 = 1.f;
    for (int i = 0; i < step; ++i) {
        pb1 *= b1;
        pb2 *= b2;
    }
    const float c1 = 1.f / (1.f - pb1), c2 = 1.f / (1.f - pb2);
    hipLaunchKernelGGL(k_adam, grid1(n), dim3(256), 0, (hipStream_t)stream, (size_t)n, w, g, m1,
                       m2, lr, b1, b2, eps, c1, c2, wb);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_mlp_pack(int32_t K, int32_t N, const uint16_t *W, uint16_t *Wp,
                                     void *stream) {
    if (K <= 0 || K % 16 || N <= 0 || !W || !Wp) return FSIM_EINVAL;
    if ((uintptr_t)Wp & 7) return FSIM_EINVAL;      // read back as 8-byte fragments
    const size_t total = (size_t)(K / 16) * ((N + 15) / 16) * 256;
    hipLaunchKernelGGL(k_pack_frag, grid1(total), dim3(256), 0, (hipStream_t)stream, K, N, W, Wp);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}

extern "C" fsim_status fsim_mlp_forward(int32_t n, const uint16_t *X, const uint16_t *W1p,
                                        const float *b1, const uint16_t *W2p, const float *b2,
                                        const uint16_t *W3p, const float *b3, float *Y,
                                        void *stream) {
    if (n < 0) return FSIM_EINVAL;
    if (n == 0) return FSIM_OK;
    if (!X || !W1p || !b1 || !W2p || !b2 || !W3p || !b3 || !Y) return FSIM_EINVAL;
    // the kernel reads X rows and weight fragments 8 bytes at a time
    for (const void *q : {(const void *)X, (const void *)W1p, (const void *)W2p, (const void *)W3p})
        if ((uintptr_t)q & 7) return FSIM_EINVAL;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + FR - 1) / FR), dim3(256), 0, (hipStream_t)stream,
                       n, X, W1p, b1, W2p, b2, W3p, b3, Y);
    return hipGetLastError() == hipSuccess ? FSIM_OK : FSIM_EHIP;
}
