// Conventional (stored-integral) Fock build: the data path of the paper's
// own implementation (Sec. 3.3: the unique integrals are computed once and
// kept; every SCF iteration's G build runs over the stored values).  Here the
// Fock-build kernels write every kept quartet's contracted block once, in
// tile order, and each later build streams them back from HBM and digests
// them with the density (Eq. fock) -- no integral is recomputed.
//
// Store layout of one quartet class: tile t (one bra pair x up to 64 kets of
// the class's FP64 tile list), component e = ((i NB + j) NC + k) ND + l of the
// block, lane (ket) x:  store[(t * NE + e) * 64 + x], NE = NA NB NC ND, so a
// wave reads each component as one coalesced 512-byte line.
#include "eri_kernels.h"

namespace fsim {

// chunk of the block held per lane while digesting: at most 48 values
__host__ __device__ constexpr int digest_chunk_cd(int la, int lb, int lc, int ld) {
    int ca = ncart(la), cdc = ncart(lc) * ncart(ld);
    while (ca * ncart(lb) * cdc > 48) {
        if (cdc > 1) cdc = (cdc + 1) / 2;
        else if (ca > 1) ca = (ca + 1) / 2;
        else break;
    }
    return cdc;
}
__host__ __device__ constexpr int digest_chunk_a(int la, int lb, int lc, int ld) {
    int ca = ncart(la), cdc = ncart(lc) * ncart(ld);
    while (ca * ncart(lb) * cdc > 48) {
        if (cdc > 1) cdc = (cdc + 1) / 2;
        else if (ca > 1) ca = (ca + 1) / 2;
        else break;
    }
    return ca;
}

// SEG: segment mode as in the lane kernels (blocks of 8 waves over segments
// of one bra's tiles, the bra's K' rows in LDS, a.kn doubles per row).
template <int LA, int LB, int LC, int LD, bool SEG>
__global__ __launch_bounds__(SEG ? 512 : 256) void k_digest_stored(EriArgs a) {
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NCD = NC * ND, NE = NA * NB * NCD;
    constexpr int CA = digest_chunk_a(LA, LB, LC, LD), CDC = digest_chunk_cd(LA, LB, LC, LD);
    constexpr int NCHA = (NA + CA - 1) / CA, NCHCD = (NCD + CDC - 1) / CDC;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long xoff = a.xcd_stride ? xcd_index() * a.xcd_stride : 0;
    auto tile_body = [&](const int tile, double *__restrict__ krow,
                         const bool kl) __attribute__((always_inline)) {
        const int b = tile_bra(a.tl, tile);
        const int bra = __builtin_amdgcn_readfirstlane(a.tl.bra[b]);
        const int k0 = a.tl.ket_lo[b] + (tile - a.tl.tile_start[b]) * TILE;
        int ket = k0 + lane;
        const bool active = ket < a.tl.ket_hi[b];
        if (!active) ket = k0;
        const int mol = __builtin_amdgcn_readfirstlane(a.bra.mol[bra]);
        const long long mbase = a.mol_off[mol];
        const int N = a.mol_n[mol];
        const double *__restrict__ D = a.D + mbase;
        double *__restrict__ Jh = a.Jh + xoff + mbase;
        double *__restrict__ Kh = a.Kh + xoff + mbase;
        const int f1 = __builtin_amdgcn_readfirstlane(a.bra.bf1[bra]);
        const int f2 = __builtin_amdgcn_readfirstlane(a.bra.bf2[bra]);
        const int f3 = a.ket.bf1[ket], f4 = a.ket.bf2[ket];
        double fac = active ? 1.0 : 0.0;
        if (a.bra.sh1[bra] == a.bra.sh2[bra]) fac *= 0.5;
        if (a.ket.sh1[ket] == a.ket.sh2[ket]) fac *= 0.5;
        if (a.same_class && ket == bra) fac *= 0.5;
        const double *__restrict__ src = a.out + (size_t)tile * NE * 64 + lane;
        static_for<NCHA * NCHCD>([&](auto ch_) {
            constexpr int ch = decltype(ch_)::value;
            constexpr int A0 = (ch / NCHCD) * CA, A1 = cmin(A0 + CA, NA);
            constexpr int CD0 = (ch % NCHCD) * CDC, CD1 = cmin(CD0 + CDC, NCD);
            constexpr int NABc = (A1 - A0) * NB, NCDc = CD1 - CD0;
            double out[NABc][NCDc];
            static_for<NABc>([&](auto abl_) {
                constexpr int abl = decltype(abl_)::value;
                static_for<NCDc>([&](auto cdl_) {
                    constexpr int cdl = decltype(cdl_)::value;
                    constexpr int e = (A0 * NB + abl) * NCD + CD0 + cdl;
                    // idle lanes hold nothing in the store
                    out[abl][cdl] = active ? src[(size_t)e * 64] : 0.0;
                });
            });
            digest_chunk<LA, LB, LC, LD, double, A0, A1, CD0, CD1>(out, D, Jh, Kh, N, f1, f2, f3,
                                                                   f4, fac, active, krow, a.kn,
                                                                   kl);
        });
    };
    if constexpr (SEG) {
        extern __shared__ __align__(16) unsigned char row_lds[];
        double *__restrict__ krow = (double *)row_lds;
        run_segments<NA, NB>(a, krow, xoff, [&](int t) __attribute__((always_inline)) {
            tile_body(t, krow, true);
        });
    } else {
        for (int tile0 = blockIdx.x * wpb + (threadIdx.x >> 6); tile0 < a.tl.ntile;
             tile0 += gridDim.x * wpb)
            tile_body(__builtin_amdgcn_readfirstlane(tile0), nullptr, false);
    }
}

template <int X, int Y>
static hipError_t launch_digest(int wpb, const EriArgs &a, hipStream_t s) {
    if (a.tl.ntile <= 0) return hipSuccess;
    constexpr int LA = pc_l1(X), LB = pc_l2(X), LC = pc_l1(Y), LD = pc_l2(Y);
    if (a.kn > 0 && a.tl.nseg > 0) {
        EriArgs b = a;
        b.stage_bytes = 0;
        int blocks = 0;
        size_t dyn = 0;
        auto seg = k_digest_stored<LA, LB, LC, LD, true>;
        if (segment_fit<LA, LB>((const void *)seg, 8, b, blocks, dyn)) {
            hipLaunchKernelGGL(seg, dim3(blocks), dim3(512), dyn, s, b);
            return hipGetLastError();
        }
    }
    if (wpb < 1 || wpb > 4) wpb = 4;
    int blocks = (a.tl.ntile + wpb - 1) / wpb;
    if (blocks > 8192) blocks = 8192;
    EriArgs b = a;
    b.kn = 0;
    hipLaunchKernelGGL((k_digest_stored<LA, LB, LC, LD, false>), dim3(blocks), dim3(64 * wpb), 0,
                       s, b);
    return hipGetLastError();
}

hipError_t launch_digest_stored(int bra_pc, int ket_pc, int wpb, const EriArgs &a,
                                hipStream_t s) {
#define FSIM_DIGEST(X, Y) \
    case X * NPCLASS + Y: return launch_digest<X, Y>(wpb, a, s);
    switch (bra_pc * NPCLASS + ket_pc) {
        FSIM_DIGEST(0, 0)
        FSIM_DIGEST(1, 0) FSIM_DIGEST(1, 1)
        FSIM_DIGEST(2, 0) FSIM_DIGEST(2, 1) FSIM_DIGEST(2, 2)
        FSIM_DIGEST(3, 0) FSIM_DIGEST(3, 1) FSIM_DIGEST(3, 2) FSIM_DIGEST(3, 3)
        FSIM_DIGEST(4, 0) FSIM_DIGEST(4, 1) FSIM_DIGEST(4, 2) FSIM_DIGEST(4, 3) FSIM_DIGEST(4, 4)
        FSIM_DIGEST(5, 0) FSIM_DIGEST(5, 1) FSIM_DIGEST(5, 2) FSIM_DIGEST(5, 3) FSIM_DIGEST(5, 4)
        FSIM_DIGEST(5, 5)
        default: return hipErrorInvalidValue;
    }
#undef FSIM_DIGEST
}

}  // namespace fsim
