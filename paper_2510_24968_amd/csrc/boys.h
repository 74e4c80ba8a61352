// Boys function F_n(T) = int_0^1 exp(-T t^2) t^(2n) dt on the device
// (definition in Sec. 2.3.3; the paper gives no evaluation method).
//
// Grid T_k = k * BOYS_DT, k < BOYS_NT.  A class kernel of total angular
// momentum L stages the orders L .. L+7 of the FP64 grid into LDS, each
// pre-divided by j!, so that
//     F_L(T) = sum_j F_{L+j}(T_k) (T_k - T)^j / j!       (dF_n/dT = -F_{n+1})
// is one 8-term Horner polynomial in (T_k - T) about the nearest grid point,
// and the lower orders follow from the downward recursion
//     F_{n-1} = (2 T F_n + exp(-T)) / (2n - 1).
// For T >= BOYS_TMAX, F_0 = sqrt(pi / T) / 2 (erfc(sqrt T) < 1e-16 there)
// and the upward recursion F_{n+1} = ((2n + 1) F_n - exp(-T)) / (2T), which
// is stable for 2T > 2n + 1.  Everything here is FP64 except the Taylor
// step of boys_eval_mixed (FP32 tiles).
#pragma once

#include "fsim_internal.h"

namespace fsim {

__host__ __device__ constexpr double inv_factorial(int j) {
    double f = 1.0;
    for (int k = 2; k <= j; ++k) f *= k;
    return 1.0 / f;
}

// LDS footprint of one staged table, in doubles.
constexpr int BOYS_LDS = BOYS_NT * BOYS_NTAYLOR;

__device__ inline void boys_stage(double *lds, const double *__restrict__ g, int L) {
    for (int i = threadIdx.x; i < BOYS_LDS; i += blockDim.x) {
        int k = i / BOYS_NTAYLOR, j = i - k * BOYS_NTAYLOR;
        double s = 1.0;
        for (int m = 2; m <= j; ++m) s *= m;
        lds[i] = g[k * BOYS_NORD + L + j] / s;
    }
}

// Large-T branch shared by the evaluators: F_0 = sqrt(pi)/2 / sqrt(T) and
// the upward recursion with 1/(2T) taken from the same reciprocal square
// root (a product of two roundings instead of a division).
template <int L>
__device__ __forceinline__ void boys_large_t(double T, double e, double *F) {
    const double rs = rsqrt(T);
    F[0] = 0.88622692545275801365 * rs;
    if constexpr (L > 0) {
        const double h = 0.5 * rs * rs;
#pragma unroll
        for (int n = 0; n < L; ++n) F[n + 1] = ((2 * n + 1) * F[n] - e) * h;
    }
}

// Optional exp column after the staged grid: exp(-T_k) at T_k = k * BOYS_DT
// for k < BOYS_NE (T up to 100; beyond it exp(-T) < 4e-44 is taken as 0).
// exp(-T) = exp(-T_k) * exp(T_k - T) with the second factor from its Taylor
// series through d^8/8! (|T_k - T| <= 0.05, so the truncation is below 6e-18
// relative): eight FMAs and one LDS read instead of the library exponential.
constexpr int BOYS_NE = 1001;
constexpr int BOYS_LDS_E = BOYS_LDS + BOYS_NE;

__device__ inline void boys_stage_exp(double *lds) {
    for (int i = threadIdx.x; i < BOYS_NE; i += blockDim.x) lds[BOYS_LDS + i] = exp(-i * BOYS_DT);
}

__device__ __forceinline__ double boys_exp_tab(double T, const double *etab) {
    constexpr double TE = (BOYS_NE - 1) * BOYS_DT;
    const double Tc = fmin(T, TE);
    const int k = __double2int_rn(Tc * BOYS_INV_DT);
    const double d = k * BOYS_DT - Tc;
    double p = inv_factorial(8);
#pragma unroll
    for (int j = 7; j >= 0; --j) p = fma(p, d, inv_factorial(j));
    return T <= TE ? etab[k] * p : 0.0;
}

// F_0..F_L at T from a table staged for order L (with the exp column when
// ET).  exp(-T), which both branches need for L > 0, is evaluated once ahead
// of the branch: the lanes of a wave often take both branches, which would
// otherwise run it twice.
template <int L, bool ET = false>
__device__ __forceinline__ void boys_eval(double T, const double *tab, double *F) {
    double e = 0.0;
    if constexpr (L > 0) e = ET ? boys_exp_tab(T, tab + BOYS_LDS) : exp(-T);
    if (T < BOYS_TMAX) {
        const int k = __double2int_rn(T * BOYS_INV_DT);
        const double d = k * BOYS_DT - T;
        const double *c = tab + k * BOYS_NTAYLOR;
        double f = c[BOYS_NTAYLOR - 1];
#pragma unroll
        for (int j = BOYS_NTAYLOR - 2; j >= 0; --j) f = fma(f, d, c[j]);
        F[L] = f;
        if constexpr (L > 0) {
            const double t2 = 2.0 * T;
#pragma unroll
            for (int n = L; n > 0; --n) F[n - 1] = fma(t2, F[n], e) * (1.0 / (2 * n - 1));
        }
    } else {
        boys_large_t<L>(T, e, F);
    }
}

// Evaluation for the FP32 tiles (quartets whose Schwarz bound is below the
// FP32 threshold).  Only the small-T Taylor step runs in FP32: the same grid
// rounded to FP32 and 5 Taylor terms (truncation at most 0.05^5/5! relative
// to F_L, below FP32 rounding), which gives F_L to FP32 accuracy.  The
// downward recursion to F_0..F_{L-1} and the whole large-T branch
// (asymptotic F_0 and the upward recursion) stay FP64; the caller rounds
// the R^n_000 sources to FP32 afterwards.
constexpr int BOYS_NTAYLOR32 = 5;
constexpr int BOYS_LDS32 = BOYS_NT * BOYS_NTAYLOR32;

__device__ inline void boys_stage32(float *lds, const double *__restrict__ g, int L) {
    for (int i = threadIdx.x; i < BOYS_LDS32; i += blockDim.x) {
        int k = i / BOYS_NTAYLOR32, j = i - k * BOYS_NTAYLOR32;
        double s = 1.0;
        for (int m = 2; m <= j; ++m) s *= m;
        lds[i] = (float)(g[k * BOYS_NORD + L + j] / s);
    }
}

template <int L>
__device__ __forceinline__ void boys_eval_mixed(double T, const float *tab, double *F) {
    double e = 0.0;
    if constexpr (L > 0) e = exp(-T);
    if (T < BOYS_TMAX) {
        const float Tf = (float)T;
        const int k = __float2int_rn(Tf * (float)BOYS_INV_DT);
        const float d = k * (float)BOYS_DT - Tf;
        const float *c = tab + k * BOYS_NTAYLOR32;
        float f = c[BOYS_NTAYLOR32 - 1];
#pragma unroll
        for (int j = BOYS_NTAYLOR32 - 2; j >= 0; --j) f = fmaf(f, d, c[j]);
        F[L] = (double)f;
        if constexpr (L > 0) {
            const double t2 = 2.0 * T;
#pragma unroll
            for (int n = L; n > 0; --n) F[n - 1] = fma(t2, F[n], e) * (1.0 / (2 * n - 1));
        }
    } else {
        boys_large_t<L>(T, e, F);
    }
}

// Runtime-L variant reading the full global grid (setup kernels only).
__device__ inline void boys_eval_rt(int L, double T, const double *__restrict__ g, double *F) {
    if (T < BOYS_TMAX) {
        const int k = __double2int_rn(T * BOYS_INV_DT);
        const double d = k * BOYS_DT - T;
        double f = 0.0;
        for (int j = BOYS_NTAYLOR - 1; j >= 0; --j)
            f = fma(f, d, g[k * BOYS_NORD + L + j] * inv_factorial(j));
        F[L] = f;
        const double e = exp(-T), t2 = 2.0 * T;
        for (int n = L; n > 0; --n) F[n - 1] = (t2 * F[n] + e) / (2 * n - 1);
    } else {
        F[0] = 0.88622692545275801365 * rsqrt(T);
        const double e = exp(-T), h = 0.5 / T;
        for (int n = 0; n < L; ++n) F[n + 1] = ((2 * n + 1) * F[n] - e) * h;
    }
}

}  // namespace fsim
