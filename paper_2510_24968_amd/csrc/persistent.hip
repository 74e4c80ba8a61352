// One resident launch per Fock build and precision over every s/p quartet
// class: a global queue of (class, tile) work items, heaviest class first,
// served by an atomic tile counter.  Each wave takes the next tile and runs
// the ket-outer tile body of that class (eri_kernels.h), so the launch
// stays resident across classes and molecules instead of draining and
// refilling the GPU once per class.  The Boys grid in LDS holds every order
// the s/p classes need (L <= 4, Taylor terms up to L + 7) as raw F_n(T_k);
// the 1/j! of each Taylor term is applied at evaluation.
#include "eri_kernels.h"

namespace fsim {

constexpr int PERSIST_NR = 12;     // FP64 orders 0..11 (L <= 4, 8 Taylor terms)
constexpr int PERSIST_NR32 = 9;    // FP32 Taylor step: orders 0..8 (5 terms)

struct BoysRaw64 {
    const double *tab;   // [BOYS_NT][PERSIST_NR]
    template <int L>
    __device__ __forceinline__ void eval(double T, double *F) const {
        static_assert(L + BOYS_NTAYLOR <= PERSIST_NR, "order outside the persistent grid");
        double e = 0.0;
        if constexpr (L > 0) e = exp(-T);
        if (T < BOYS_TMAX) {
            const int k = __double2int_rn(T * BOYS_INV_DT);
            const double d = k * BOYS_DT - T;
            const double *c = tab + k * PERSIST_NR + L;
            double f = c[BOYS_NTAYLOR - 1] * inv_factorial(BOYS_NTAYLOR - 1);
#pragma unroll
            for (int j = BOYS_NTAYLOR - 2; j >= 0; --j) f = fma(f, d, c[j] * inv_factorial(j));
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
};

// FP32 tiles: only the Taylor step in FP32 (as boys_eval_mixed)
struct BoysRawMixed {
    const float *tab;    // [BOYS_NT][PERSIST_NR32]
    template <int L>
    __device__ __forceinline__ void eval(double T, double *F) const {
        static_assert(L + BOYS_NTAYLOR32 <= PERSIST_NR32, "order outside the persistent grid");
        double e = 0.0;
        if constexpr (L > 0) e = exp(-T);
        if (T < BOYS_TMAX) {
            const float Tf = (float)T;
            const int k = __float2int_rn(Tf * (float)BOYS_INV_DT);
            const float d = k * (float)BOYS_DT - Tf;
            const float *c = tab + k * PERSIST_NR32 + L;
            float f = c[BOYS_NTAYLOR32 - 1] * (float)inv_factorial(BOYS_NTAYLOR32 - 1);
#pragma unroll
            for (int j = BOYS_NTAYLOR32 - 2; j >= 0; --j)
                f = fmaf(f, d, c[j] * (float)inv_factorial(j));
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
};

// queue slot -> (bra pair class, ket pair class), heaviest first
__host__ __device__ constexpr int persist_bra(int slot) {
    return slot == 0 ? 2 : slot == 1 ? 2 : slot == 2 ? 1 : slot == 3 ? 2 : slot == 4 ? 1 : 0;
}
__host__ __device__ constexpr int persist_ket(int slot) {
    return slot == 0 ? 2 : slot == 1 ? 1 : slot == 2 ? 1 : slot == 3 ? 0 : slot == 4 ? 0 : 0;
}

template <int SLOT, typename T, typename BP>
__device__ __forceinline__ void persist_tile(const PersistArgs &p, int tile, const BP &bp,
                                             double *sp) {
    constexpr int X = persist_bra(SLOT), Y = persist_ket(SLOT);
    constexpr int LA = pc_l1(X), LB = pc_l2(X), LC = pc_l1(Y), LD = pc_l2(Y);
    constexpr int B = PERSIST_BUDGET;
    ko_tile<LA, LB, LC, LD, T, false, chunk_a(LA, LB, LC, LD, B), chunk_cd(LA, LB, LC, LD, B)>(
        p.cls[SLOT], tile, bp, sp);
}

// Segment item: the block's waves split the segment's tiles, adding K' into
// the LDS rows, which are flushed once the block is done with it.
template <int SLOT, typename T, typename BP>
__device__ __forceinline__ void persist_segment(const PersistArgs &p, int sg, const BP &bp,
                                                double *sp, double *krow) {
    constexpr int X = persist_bra(SLOT), Y = persist_ket(SLOT);
    constexpr int LA = pc_l1(X), LB = pc_l2(X), LC = pc_l1(Y), LD = pc_l2(Y);
    constexpr int B = PERSIST_BUDGET;
    const EriArgs &a = p.cls[SLOT];
    const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
    const int t0 = a.tl.seg_t0[sg], nt = a.tl.seg_nt[sg];
    for (int t = t0 + wave; t < t0 + nt; t += wpb)
        ko_tile<LA, LB, LC, LD, T, false, chunk_a(LA, LB, LC, LD, B), chunk_cd(LA, LB, LC, LD, B)>(
            a, __builtin_amdgcn_readfirstlane(t), bp, sp, krow, true);
    __syncthreads();
    const long long xoff = a.xcd_stride ? xcd_index() * a.xcd_stride : 0;
    segment_flush<ncart(LA), ncart(LB)>(a, krow, xoff, sg);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_eri_persistent(PersistArgs p) {
    constexpr bool F32 = std::is_same<T, float>::value;
    constexpr int NR = F32 ? PERSIST_NR32 : PERSIST_NR;
    __shared__ std::conditional_t<F32, float, double> tab[BOYS_NT * NR];
    extern __shared__ __align__(16) unsigned char stage_lds[];
    for (int i = threadIdx.x; i < BOYS_NT * NR; i += blockDim.x)
        tab[i] = p.boys[(i / NR) * BOYS_NORD + i % NR];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    double *__restrict__ sp = (double *)(stage_lds + (size_t)(threadIdx.x >> 6) * p.stage_bytes);
    using BP = std::conditional_t<F32, BoysRawMixed, BoysRaw64>;
    const BP bp{tab};
    const int total = p.start[PERSIST_SLOTS];
    if (p.kn > 0) {
        // segment items, one per block at a time; the rows (6 of kn doubles,
        // the pp bras' count) follow the 4 staging slices
        double *__restrict__ krow = (double *)(stage_lds + (size_t)4 * p.stage_bytes);
        __shared__ int item;
        for (int x = threadIdx.x; x < 6 * p.kn; x += blockDim.x) krow[x] = 0.0;
        while (true) {
            __syncthreads();   // the rows are clear and every thread has read the last item
            if (threadIdx.x == 0) item = atomicAdd(p.counter, 1);
            __syncthreads();
            const int q = item;
            if (q >= total) break;   // the same q in every thread of the block
            int slot = 0;
            while (slot + 1 < PERSIST_SLOTS && q >= p.start[slot + 1]) ++slot;
            const int sg = q - p.start[slot];
            switch (slot) {
                case 0: persist_segment<0, T>(p, sg, bp, sp, krow); break;
                case 1: persist_segment<1, T>(p, sg, bp, sp, krow); break;
                case 2: persist_segment<2, T>(p, sg, bp, sp, krow); break;
                case 3: persist_segment<3, T>(p, sg, bp, sp, krow); break;
                case 4: persist_segment<4, T>(p, sg, bp, sp, krow); break;
                default: persist_segment<5, T>(p, sg, bp, sp, krow); break;
            }
        }
        return;
    }
    while (true) {
        int q = 0;
        if (lane == 0) q = atomicAdd(p.counter, 1);
        q = __builtin_amdgcn_readfirstlane(__shfl(q, 0, 64));
        if (q >= total) break;   // every wave reaches this once the queue is drained
        int slot = 0;
        while (slot + 1 < PERSIST_SLOTS && q >= p.start[slot + 1]) ++slot;
        const int tile = q - p.start[slot];
        switch (slot) {
            case 0: persist_tile<0, T>(p, tile, bp, sp); break;
            case 1: persist_tile<1, T>(p, tile, bp, sp); break;
            case 2: persist_tile<2, T>(p, tile, bp, sp); break;
            case 3: persist_tile<3, T>(p, tile, bp, sp); break;
            case 4: persist_tile<4, T>(p, tile, bp, sp); break;
            default: persist_tile<5, T>(p, tile, bp, sp); break;
        }
    }
}

hipError_t launch_persistent(bool fp32, const PersistArgs &pin, hipStream_t s) {
    if (pin.start[PERSIST_SLOTS] <= 0) return hipSuccess;
    PersistArgs p = pin;
    if (p.kn > 0) {
        // segment items need the rows beside the Boys grid and the staging
        // slices; otherwise tile items with global K' atomics
        const size_t stat = (size_t)BOYS_NT * (fp32 ? PERSIST_NR32 * sizeof(float)
                                                    : PERSIST_NR * sizeof(double));
        const size_t need_lds =
            stat + (size_t)4 * p.stage_bytes + (size_t)6 * p.kn * sizeof(double);
        if (need_lds > LDS_PER_CU) {
            p.kn = 0;
            for (int k = 0; k < PERSIST_SLOTS; ++k) {
                p.cls[k].kn = 0;
                p.start[k + 1] = p.start[k] + p.cls[k].tl.ntile;
            }
        }
    }
    // resident grid: as many blocks as fit on the device at once (queried
    // once per kernel and LDS size), never more than one per 4 tiles
    static int cached[2][2] = {{0, 0}, {0, 0}};   // [fp32] -> (dynamic LDS, blocks per CU)
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t dyn = (size_t)4 * p.stage_bytes + (size_t)6 * p.kn * sizeof(double);
    int per_cu = 0;
    if (cached[fp32][0] == (int)dyn && cached[fp32][1] > 0) {
        per_cu = cached[fp32][1];
    } else {
        e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eri_persistent<float>, 256, dyn)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eri_persistent<double>, 256, dyn);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        cached[fp32][0] = (int)dyn;
        cached[fp32][1] = per_cu;
    }
    int blocks = per_cu * ncu;
    // tile items: one per wave; segment items: one per block
    const int need = p.kn > 0 ? p.start[PERSIST_SLOTS] : (p.start[PERSIST_SLOTS] + 3) / 4;
    if (blocks > need) blocks = need;
    if (fp32)
        hipLaunchKernelGGL(k_eri_persistent<float>, dim3(blocks), dim3(256), dyn, s, p);
    else
        hipLaunchKernelGGL(k_eri_persistent<double>, dim3(blocks), dim3(256), dyn, s, p);
    return hipGetLastError();
}

}  // namespace fsim
