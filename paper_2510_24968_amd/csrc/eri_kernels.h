// McMurchie-Davidson electron-repulsion kernels for one quartet class
// (bra pair class (LA, LB), ket pair class (LC, LD)), with the on-the-fly
// J/K digest of Eq. fock or a plain store of the contracted block.
//
// Per primitive quartet (bra primitive pair i, ket primitive pair j):
//   alpha = p q / (p + q),  R_PQ = P - Q,  T = alpha |R_PQ|^2
//   F_0..F_L(T)                                  (Boys, boys.h)
//   R^n_000 = (-2 alpha)^n F_n(T) / sqrt(p + q)  (Eq. Rn-definition, source;
//             the 1/sqrt(p+q) of the ERI prefactor rides along linearly)
//   R^0_tuv by Eq. R-recursion, in place
//   W_{tuv,cd} = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R^0_{t+tau,u+nu,v+phi}
//   (ab|cd)   += sum_{tuv} E^{ab}_{tuv} W_{tuv,cd}
// which is Eq. eri-tensor-contracted evaluated through the intermediate
// J_{tuv,k} of Sec. 2.5.  The pair tables carry the contraction
// coefficients and sqrt(2 pi^(5/2)) / p (resp. / q) of the prefactor of
// Eq. twoe-final, so the sum is already the contracted integral.
//
// Digest of a canonical quartet (ab|cd) with value v and degeneracy factor
// f = (1/2)^[a=b] (1/2)^[c=d] (1/2)^[ab=cd] into half-sums J', K':
//   J'_ab += 2 f v D_cd   J'_cd += 2 f v D_ab
//   K'_ac += f v D_bd     K'_bc += f v D_ad   K'_ad += f v D_bc   K'_bd += f v D_ac
// so that J = J' + J'^T and K = K' + K'^T (the eight permutational images of
// every canonical quartet then count once).
#pragma once

#include <type_traits>
#include <utility>

#include "boys.h"
#include "fsim_internal.h"

namespace fsim {

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (N > 0) static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename T>
__device__ __forceinline__ const T *etab(const PairTable &t);
template <>
__device__ __forceinline__ const double *etab<double>(const PairTable &t) { return t.E; }
template <>
__device__ __forceinline__ const float *etab<float>(const PairTable &t) { return t.Ef; }

// Index (0..7) of the XCD the calling wave runs on, from the XCC_ID
// hardware register (bits 3:0).
__device__ __forceinline__ int xcd_index() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// In-place Hermite Coulomb recursion: on entry src[n] = R^n_000; on exit
// r[hidx(t,u,v)] = R^0_tuv for t + u + v <= L.  At step n the totals are
// rewritten from high to low, so every R^{n+1} value is read before its slot
// is overwritten.
template <int L, typename T>
__device__ __forceinline__ void hermite_r(const T *src, T X, T Y, T Z, T *r) {
    r[0] = src[L];
    static_for<L>([&](auto m_) {
        constexpr int n = L - 1 - decltype(m_)::value;
        static_for<L - n>([&](auto k_) {
            constexpr int s = L - n - decltype(k_)::value;
            constexpr int base = s == 0 ? 0 : nherm(s - 1);
            static_for<nherm(s) - base>([&](auto q_) {
                constexpr int id = base + decltype(q_)::value;
                constexpr int t = hidx_t(id), u = hidx_u(id), v = hidx_v(id);
                if constexpr (t > 0) {
                    if constexpr (t > 1)
                        r[id] = X * r[hidx(t - 1, u, v)] + T(t - 1) * r[hidx(t - 2, u, v)];
                    else
                        r[id] = X * r[hidx(t - 1, u, v)];
                } else if constexpr (u > 0) {
                    if constexpr (u > 1)
                        r[id] = Y * r[hidx(t, u - 1, v)] + T(u - 1) * r[hidx(t, u - 2, v)];
                    else
                        r[id] = Y * r[hidx(t, u - 1, v)];
                } else {
                    if constexpr (v > 1)
                        r[id] = Z * r[hidx(t, u, v - 1)] + T(v - 1) * r[hidx(t, u, v - 2)];
                    else
                        r[id] = Z * r[hidx(t, u, v - 1)];
                }
            });
        });
        r[0] = src[n];
    });
}

// Locate the tile's bra and ket range (Fock mode).  tile_start is the
// prefix sum of tiles per bra; the search is wave-uniform.
__device__ __forceinline__ int tile_bra(const TileList &tl, int tile) {
    int lo = 0, hi = tl.nbra - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tl.tile_start[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ===========================================================================
// Kernel A: one lane per contracted quartet, everything unrolled at compile
// time.  A wave owns a tile (one bra pair, up to 64 consecutive kets), so the
// bra's exponents, centre and Hermite tensor are wave-uniform and the ket
// tables are read with unit stride across lanes.
//
// Loop order (the intermediate J_{tuv,k} of Sec. 2.5, summed over the ket
// primitives before the bra contraction):
//   for each bra primitive pair i:
//       W_{tuv,cd} = sum over ket primitive pairs j of (-1)^{..} E^{cd}_j R^0_ij
//       (ab|cd)   += sum_tuv E^{ab}_i W_{tuv,cd}
// The block is produced in chunks of CA bra components a and CDC ket
// component pairs cd, so that block, W and R^0 fit in registers; each chunk
// re-evaluates the Boys function and R^0 and is digested when complete.
// ===========================================================================
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// live values per lane of a chunk: block + W + R^0
__host__ __device__ constexpr int lane_live(int la, int lb, int lc, int ld, int ca, int cdc) {
    return ca * ncart(lb) * cdc + nherm(la + lb) * cdc + nherm(la + lb + lc + ld);
}
// chunk sizes: halve the cd range, then the a range, until the live set fits
__host__ __device__ constexpr int chunk_cd(int la, int lb, int lc, int ld, int limit) {
    int ca = ncart(la), cdc = ncart(lc) * ncart(ld);
    while (lane_live(la, lb, lc, ld, ca, cdc) > limit) {
        if (cdc > 1) cdc = (cdc + 1) / 2;
        else if (ca > 1) ca = (ca + 1) / 2;
        else break;
    }
    return cdc;
}
__host__ __device__ constexpr int chunk_a(int la, int lb, int lc, int ld, int limit) {
    int ca = ncart(la), cdc = ncart(lc) * ncart(ld);
    while (lane_live(la, lb, lc, ld, ca, cdc) > limit) {
        if (cdc > 1) cdc = (cdc + 1) / 2;
        else if (ca > 1) ca = (ca + 1) / 2;
        else break;
    }
    return ca;
}
__host__ __device__ constexpr int n_chunks(int la, int lb, int lc, int ld, int limit) {
    const int ca = chunk_a(la, lb, lc, ld, limit), cdc = chunk_cd(la, lb, lc, ld, limit);
    return ((ncart(la) + ca - 1) / ca) * ((ncart(lc) * ncart(ld) + cdc - 1) / cdc);
}

// Digest of one chunk of a lane's block (components a in [A0, A1), ket
// component pairs in [CD0, CD1)) into the half-sums of Eq. fock:
// J'_ab += 2 v D_cd (wave-reduced), J'_cd += 2 v D_ab, K'_ac += v D_bd,
// K'_bc += v D_ad, K'_ad += v D_bc, K'_bd += v D_ac (fac: degeneracy factor,
// 0 for an idle lane).
//
// With kl, the K' terms go to the block's LDS rows instead (krow: row x < NA
// is K'_{f1 + x, .}, row NA + y is K'_{f2 + y, .}, kn doubles per row),
// which the kernel flushes to global memory once per segment of tiles.
template <int LA, int LB, int LC, int LD, typename T, int A0, int A1, int CD0, int CD1>
__device__ __forceinline__ void digest_chunk(const T (&out)[(A1 - A0) * ncart(LB)][CD1 - CD0],
                                             const double *__restrict__ D, double *__restrict__ Jh,
                                             double *__restrict__ Kh, int N, int f1, int f2, int f3,
                                             int f4, double fac, bool active,
                                             double *__restrict__ krow = nullptr, int kn = 0,
                                             bool kl = false) {
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAc = A1 - A0, NABc = NAc * NB, NCDc = CD1 - CD0;
    const int lane = threadIdx.x & 63;
    // J'_ab (partial over this chunk's cd): pre-reduced over the wave
    static_for<NABc>([&](auto abl_) {
        constexpr int abl = decltype(abl_)::value;
        constexpr int ia = A0 + abl / NB, ib = abl % NB;
        double sum = 0.0;
        static_for<NCDc>([&](auto cdl_) {
            constexpr int cdl = decltype(cdl_)::value;
            constexpr int ic = (CD0 + cdl) / ND, id = (CD0 + cdl) % ND;
            sum += (double)out[abl][cdl] * D[(size_t)(f3 + ic) * N + f4 + id];
        });
        sum = wave_sum(2.0 * fac * sum);
        if (lane == 0) atomicAdd(&Jh[(size_t)(f1 + ia) * N + f2 + ib], sum);
    });
    if (active) {
        // J'_cd (partial over this chunk's a)
        static_for<NCDc>([&](auto cdl_) {
            constexpr int cdl = decltype(cdl_)::value;
            constexpr int ic = (CD0 + cdl) / ND, id = (CD0 + cdl) % ND;
            double sum = 0.0;
            static_for<NABc>([&](auto abl_) {
                constexpr int abl = decltype(abl_)::value;
                constexpr int ia = A0 + abl / NB, ib = abl % NB;
                sum += (double)out[abl][cdl] * D[(size_t)(f1 + ia) * N + f2 + ib];
            });
            atomicAdd(&Jh[(size_t)(f3 + ic) * N + f4 + id], 2.0 * fac * sum);
        });
        // K'_xc for x in {a (with D_bd), b (with D_ad)} and every c in the chunk
        static_for<NC>([&](auto c_) {
            constexpr int ic = decltype(c_)::value;
            constexpr bool has_c = ic * ND + ND > CD0 && ic * ND < CD1;
            if constexpr (has_c) {
                static_for<NAc>([&](auto al_) {
                    constexpr int al = decltype(al_)::value;
                    double sum = 0.0;
                    static_for<NB>([&](auto b_) {
                        constexpr int ib = decltype(b_)::value;
                        static_for<ND>([&](auto d_) {
                            constexpr int id = decltype(d_)::value;
                            constexpr int cd = ic * ND + id;
                            if constexpr (cd >= CD0 && cd < CD1)
                                sum += (double)out[al * NB + ib][cd - CD0] *
                                       D[(size_t)(f2 + ib) * N + f4 + id];
                        });
                    });
                    if (kl) atomicAdd(&krow[(A0 + al) * kn + f3 + ic], fac * sum);
                    else atomicAdd(&Kh[(size_t)(f1 + A0 + al) * N + f3 + ic], fac * sum);
                });
                static_for<NB>([&](auto b_) {
                    constexpr int ib = decltype(b_)::value;
                    double sum = 0.0;
                    static_for<NAc>([&](auto al_) {
                        constexpr int al = decltype(al_)::value;
                        static_for<ND>([&](auto d_) {
                            constexpr int id = decltype(d_)::value;
                            constexpr int cd = ic * ND + id;
                            if constexpr (cd >= CD0 && cd < CD1)
                                sum += (double)out[al * NB + ib][cd - CD0] *
                                       D[(size_t)(f1 + A0 + al) * N + f4 + id];
                        });
                    });
                    if (kl) atomicAdd(&krow[(NA + ib) * kn + f3 + ic], fac * sum);
                    else atomicAdd(&Kh[(size_t)(f2 + ib) * N + f3 + ic], fac * sum);
                });
            }
        });
        // K'_xd for x in {a (with D_bc), b (with D_ac)} and every d in the chunk
        static_for<ND>([&](auto d_) {
            constexpr int id = decltype(d_)::value;
            constexpr bool has_d = [] {
                for (int c = 0; c < NC; ++c)
                    if (c * ND + id >= CD0 && c * ND + id < CD1) return true;
                return false;
            }();
            if constexpr (has_d) {
                static_for<NAc>([&](auto al_) {
                    constexpr int al = decltype(al_)::value;
                    double sum = 0.0;
                    static_for<NB>([&](auto b_) {
                        constexpr int ib = decltype(b_)::value;
                        static_for<NC>([&](auto c_) {
                            constexpr int ic = decltype(c_)::value;
                            constexpr int cd = ic * ND + id;
                            if constexpr (cd >= CD0 && cd < CD1)
                                sum += (double)out[al * NB + ib][cd - CD0] *
                                       D[(size_t)(f2 + ib) * N + f3 + ic];
                        });
                    });
                    if (kl) atomicAdd(&krow[(A0 + al) * kn + f4 + id], fac * sum);
                    else atomicAdd(&Kh[(size_t)(f1 + A0 + al) * N + f4 + id], fac * sum);
                });
                static_for<NB>([&](auto b_) {
                    constexpr int ib = decltype(b_)::value;
                    double sum = 0.0;
                    static_for<NAc>([&](auto al_) {
                        constexpr int al = decltype(al_)::value;
                        static_for<NC>([&](auto c_) {
                            constexpr int ic = decltype(c_)::value;
                            constexpr int cd = ic * ND + id;
                            if constexpr (cd >= CD0 && cd < CD1)
                                sum += (double)out[al * NB + ib][cd - CD0] *
                                       D[(size_t)(f1 + A0 + al) * N + f3 + ic];
                        });
                    });
                    if (kl) atomicAdd(&krow[(NA + ib) * kn + f4 + id], fac * sum);
                    else atomicAdd(&Kh[(size_t)(f2 + ib) * N + f4 + id], fac * sum);
                });
            }
        });
    }
}

// Segment mode of the lane kernels (Fock builds): the block takes whole
// segments, each a run of tiles of one bra record, and its waves split the
// segment's tiles.  The K' terms of a quartet all lie in the rows of the
// bra's functions (K'_ac, K'_ad in the rows of a, K'_bc, K'_bd in those of
// b), so they are added into the block's LDS copy of those rows; after a
// block barrier the non-zero entries go to global K' with one atomic each
// and the rows are cleared.  krow: (NA + NB) rows of a.kn doubles.
// The block's rows after segment sg: non-zero entries added to global K'
// and cleared (every thread of the block takes part; no barriers inside).
template <int NA, int NB>
__device__ __forceinline__ void segment_flush(const EriArgs &a, double *__restrict__ krow,
                                              long long xoff, int sg) {
    constexpr int NR = NA + NB;
    const int kn = a.kn;
    const int bra = a.tl.bra[a.tl.seg_rec[sg]];
    const int mol = a.bra.mol[bra];
    const int N = a.mol_n[mol];
    const int f1 = a.bra.bf1[bra], f2 = a.bra.bf2[bra];
    double *__restrict__ Kh = a.Kh + xoff + a.mol_off[mol];
    for (int x = threadIdx.x; x < NR * N; x += blockDim.x) {
        const int r = x / N, col = x - r * N;
        const double v = krow[r * kn + col];
        if (v != 0.0) {
            atomicAdd(&Kh[(size_t)(r < NA ? f1 + r : f2 + r - NA) * N + col], v);
            krow[r * kn + col] = 0.0;
        }
    }
}

template <int NA, int NB, typename Body>
__device__ __forceinline__ void run_segments(const EriArgs &a, double *__restrict__ krow,
                                             long long xoff, Body &&body) {
    constexpr int NR = NA + NB;
    const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
    for (int x = threadIdx.x; x < NR * a.kn; x += blockDim.x) krow[x] = 0.0;
    __syncthreads();
    for (int sg = blockIdx.x; sg < a.tl.nseg; sg += gridDim.x) {
        const int t0 = a.tl.seg_t0[sg], nt = a.tl.seg_nt[sg];
        for (int t = t0 + wave; t < t0 + nt; t += wpb) body(__builtin_amdgcn_readfirstlane(t));
        __syncthreads();
        segment_flush<NA, NB>(a, krow, xoff, sg);
        __syncthreads();
    }
}

// Minimum waves per SIMD the lane kernel is compiled for.  d bras with a
// live set of up to 128 FP64 values are held to two resident waves (256
// registers each); every other kernel is left to the compiler, which
// measured faster for the s and p bras.
__host__ __device__ constexpr int lane_min_waves(int la, int lb, int lc, int ld, int ca, int cdc) {
    return la == 2 && lane_live(la, lb, lc, ld, ca, cdc) <= 128 ? 2 : 1;
}

// Blocks of the lane kernel in segment mode: 8 waves where the kernel is held
// to two waves per SIMD (two blocks' worth of registers per CU), else 4.
__host__ __device__ constexpr int seg_waves(int la, int lb, int lc, int ld, int ca, int cdc) {
    return lane_min_waves(la, lb, lc, ld, ca, cdc) == 2 ? 8 : 4;
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE, int CA, int CDC, bool SEG>
__global__ __launch_bounds__(SEG ? 64 * seg_waves(LA, LB, LC, LD, CA, CDC) : 256,
                             lane_min_waves(LA, LB, LC, LD, CA, CDC)) void k_eri_lane(EriArgs a) {
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NCD = NC * ND, NHAB = nherm(LAB), NH = nherm(L);
    constexpr int NEB = n_entries(LA, LB), NEK = n_entries(LC, LD);
    constexpr int NCHA = (NA + CA - 1) / CA, NCHCD = (NCD + CDC - 1) / CDC;
    // Boys grid in LDS: FP64 for FP64 tiles, FP32 (5 terms, the Taylor step
    // only) for FP32 tiles
    constexpr bool F32 = std::is_same<T, float>::value;
    __shared__ std::conditional_t<F32, float, double> tab[F32 ? BOYS_LDS32 : BOYS_LDS];
    extern __shared__ __align__(16) unsigned char stage_lds[];
    if constexpr (F32) boys_stage32(tab, a.boys, L);
    else boys_stage(tab, a.boys, L);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int ntile = STORE ? a.st_ntile : a.tl.ntile;
    const T *__restrict__ Eb = etab<T>(a.bra);
    const T *__restrict__ Ek = etab<T>(a.ket);
    const size_t nb = a.bra.n, nk = a.ket.n;
    // The bra pair is the same for the whole wave.  For d bras (large Hermite
    // boxes, re-read in every chunk) its primitive data are copied once per
    // tile (or per group of ks primitive pairs) into this wave's LDS slice and
    // read back as broadcasts; s and p bras read them from global memory,
    // which measured faster for their small boxes.
    constexpr bool STAGE = LA == 2;
    const int ks = STAGE ? a.stage_prims : 1 << 20;
    double *__restrict__ sp = (double *)(stage_lds + (size_t)(threadIdx.x >> 6) * a.stage_bytes);
    T *__restrict__ se = (T *)(sp + 4 * ks);
    auto stage = [&](int bra_, int i0, int cnt) {
        for (int x = lane; x < cnt * 4; x += 64) {
            const int s = x >> 2, f = x & 3;
            sp[x] = f == 0 ? a.bra.p[(size_t)(i0 + s) * nb + bra_]
                           : a.bra.P[((size_t)(i0 + s) * 3 + f - 1) * nb + bra_];
        }
        for (int x = lane; x < cnt * NEB; x += 64)
            se[x] = Eb[((size_t)i0 * NEB + x) * nb + bra_];
        // the wave's own LDS writes complete before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // per-XCD private J'/K' copies keep each cache line's atomics on one XCD
    const long long xoff = (!STORE && a.xcd_stride) ? xcd_index() * a.xcd_stride : 0;

    // one tile; kl: K' rows into the block's LDS rows krow (segment mode)
    auto tile_body = [&](const int tile, double *__restrict__ krow,
                         const bool kl) __attribute__((always_inline)) {
        int bra, ket;
        bool active;
        if constexpr (STORE) {
            bra = __builtin_amdgcn_readfirstlane(a.st_bra[tile]);
            ket = a.st_ket[tile * 64 + lane];
            active = ket >= 0;
            if (!active) ket = 0;
        } else {
            const int b = tile_bra(a.tl, tile);
            bra = __builtin_amdgcn_readfirstlane(a.tl.bra[b]);
            const int k0 = a.tl.ket_lo[b] + (tile - a.tl.tile_start[b]) * TILE;
            ket = k0 + lane;
            active = ket < a.tl.ket_hi[b];
            if (!active) ket = k0;
        }
        const int nbp = __builtin_amdgcn_readfirstlane(a.bra.nprim[bra]);
        const int nkp = active ? a.ket.nprim[ket] : 0;
        const bool all_staged = nbp <= ks;
        if (STAGE && all_staged) stage(bra, 0, nbp);
        // the quartet's molecule block (bra and ket pairs share the molecule)
        const int mol = __builtin_amdgcn_readfirstlane(a.bra.mol[bra]);
        const long long mbase = STORE ? 0 : a.mol_off[mol];
        const int N = STORE ? 0 : a.mol_n[mol];
        const double *__restrict__ D = STORE ? nullptr : a.D + mbase;
        double *__restrict__ Jh = STORE ? nullptr : a.Jh + xoff + mbase;
        double *__restrict__ Kh = STORE ? nullptr : a.Kh + xoff + mbase;
        int f1 = 0, f2 = 0, f3 = 0, f4 = 0;
        double fac = 0.0;
        long long soff = 0;
        int st0 = 0, st1 = 0, st2 = 0, st3 = 0;
        if constexpr (STORE) {
            if (active) {
                const size_t q = (size_t)tile * 64 + lane;
                soff = a.st_off[q];
                st0 = a.st_stride[q * 4 + 0];
                st1 = a.st_stride[q * 4 + 1];
                st2 = a.st_stride[q * 4 + 2];
                st3 = a.st_stride[q * 4 + 3];
            }
        } else {
            f1 = __builtin_amdgcn_readfirstlane(a.bra.bf1[bra]);
            f2 = __builtin_amdgcn_readfirstlane(a.bra.bf2[bra]);
            f3 = a.ket.bf1[ket];
            f4 = a.ket.bf2[ket];
            fac = active ? 1.0 : 0.0;
            if (a.bra.sh1[bra] == a.bra.sh2[bra]) fac *= 0.5;
            if (a.ket.sh1[ket] == a.ket.sh2[ket]) fac *= 0.5;
            if (a.same_class && ket == bra) fac *= 0.5;
        }

        static_for<NCHA * NCHCD>([&](auto ch_) {
            constexpr int ch = decltype(ch_)::value;
            constexpr int A0 = (ch / NCHCD) * CA, A1 = cmin(A0 + CA, NA);
            constexpr int CD0 = (ch % NCHCD) * CDC, CD1 = cmin(CD0 + CDC, NCD);
            constexpr int NAc = A1 - A0, NABc = NAc * NB, NCDc = CD1 - CD0;
            T out[NABc][NCDc];
#pragma unroll
            for (int x = 0; x < NABc; ++x)
#pragma unroll
                for (int y = 0; y < NCDc; ++y) out[x][y] = T(0);

            for (int i = 0; i < nbp; ++i) {
                int il = i;
                if (STAGE && !all_staged) {
                    il = i % ks;
                    if (il == 0) stage(bra, i, nbp - i < ks ? nbp - i : ks);
                }
                const double p = STAGE ? sp[il * 4 + 0] : a.bra.p[(size_t)i * nb + bra];
                const double Px = STAGE ? sp[il * 4 + 1] : a.bra.P[((size_t)i * 3 + 0) * nb + bra];
                const double Py = STAGE ? sp[il * 4 + 2] : a.bra.P[((size_t)i * 3 + 1) * nb + bra];
                const double Pz = STAGE ? sp[il * 4 + 3] : a.bra.P[((size_t)i * 3 + 2) * nb + bra];
                T W[NCDc][NHAB];
#pragma unroll
                for (int x = 0; x < NCDc; ++x)
#pragma unroll
                    for (int h = 0; h < NHAB; ++h) W[x][h] = T(0);
                // d bras: ket primitive data, including this chunk's Hermite box
                // entries, loaded one primitive ahead of use (s and p bras load
                // them in place, which measured faster)
                constexpr int EK0 = box_off(LC, LD, CD0);
                constexpr int EK1 = CD1 < NCD ? box_off(LC, LD, CD1) : NEK;
                constexpr int NEKC = STAGE ? EK1 - EK0 : 1;
                double qn = 0.0, Kxn = 0.0, Kyn = 0.0, Kzn = 0.0;
                T ekn[NEKC];
                auto kload = [&](int j_) {
                    qn = a.ket.p[(size_t)j_ * nk + ket];
                    Kxn = a.ket.P[((size_t)j_ * 3 + 0) * nk + ket];
                    Kyn = a.ket.P[((size_t)j_ * 3 + 1) * nk + ket];
                    Kzn = a.ket.P[((size_t)j_ * 3 + 2) * nk + ket];
                    if constexpr (STAGE) {
                        const T *__restrict__ ekp = Ek + (size_t)j_ * NEK * nk + ket;
#pragma unroll
                        for (int e = 0; e < NEKC; ++e) ekn[e] = ekp[(size_t)(EK0 + e) * nk];
                    }
                };
                if (STAGE && nkp > 0) kload(0);
                for (int j = 0; j < nkp; ++j) {
                    if (!STAGE) kload(j);
                    const double q = qn;
                    const double X = Px - Kxn, Y = Py - Kyn, Z = Pz - Kzn;
                    T ekc[NEKC];
#pragma unroll
                    for (int e = 0; e < NEKC; ++e) ekc[e] = ekn[e];
                    if (STAGE && j + 1 < nkp) kload(j + 1);
                    // 1/sqrt(p+q) once; 1/(p+q) and alpha = pq/(p+q) from it
                    T src[L + 1];
                    if constexpr (F32) {
                        // FP32 tile: FP32 Taylor step, FP64 recursion and
                        // prefactor, sources rounded to FP32
                        const double rs = rsqrt(p + q);
                        const double alpha = p * q * (rs * rs);
                        double F[L + 1];
                        boys_eval_mixed<L>(alpha * (X * X + Y * Y + Z * Z), tab, F);
                        double m = rs;
#pragma unroll
                        for (int n = 0; n <= L; ++n) {
                            src[n] = (float)(F[n] * m);
                            m *= -2.0 * alpha;
                        }
                    } else {
                        const double rs = rsqrt(p + q);
                        const double alpha = p * q * (rs * rs);
                        double F[L + 1];
                        boys_eval<L>(alpha * (X * X + Y * Y + Z * Z), tab, F);
                        double m = rs;
#pragma unroll
                        for (int n = 0; n <= L; ++n) {
                            src[n] = T(F[n] * m);
                            m *= -2.0 * alpha;
                        }
                    }
                    T r[NH];
                    hermite_r<L, T>(src, T(X), T(Y), T(Z), r);
                    const T *__restrict__ ek = Ek + (size_t)j * NEK * nk + ket;
                    static_for<NCDc>([&](auto cdl_) {
                        constexpr int cdl = decltype(cdl_)::value;
                        constexpr int cd = CD0 + cdl;
                        constexpr int bx = box_dim(LC, LD, cd, 0), by = box_dim(LC, LD, cd, 1),
                                      bz = box_dim(LC, LD, cd, 2);
                        constexpr int eo = box_off(LC, LD, cd);
                        static_for<bx + 1>([&](auto ta_) {
                            constexpr int ta = decltype(ta_)::value;
                            static_for<by + 1>([&](auto nu_) {
                                constexpr int nu = decltype(nu_)::value;
                                static_for<bz + 1>([&](auto ph_) {
                                    constexpr int ph = decltype(ph_)::value;
                                    constexpr int e = eo + (ta * (by + 1) + nu) * (bz + 1) + ph;
                                    T ev;
                                    if constexpr (STAGE) ev = ekc[e - EK0];
                                    else ev = ek[(size_t)e * nk];
                                    if constexpr ((ta + nu + ph) & 1) ev = -ev;
                                    static_for<NHAB>([&](auto h_) {
                                        constexpr int h = decltype(h_)::value;
                                        constexpr int ri = hidx(hidx_t(h) + ta, hidx_u(h) + nu,
                                                                hidx_v(h) + ph);
                                        W[cdl][h] = fma(ev, r[ri], W[cdl][h]);
                                    });
                                });
                            });
                        });
                    });
                }
                // bra contraction, once per bra primitive pair
                const T *__restrict__ eb = STAGE ? se + il * NEB : Eb + (size_t)i * NEB * nb + bra;
                const size_t es = STAGE ? 1 : nb;
                static_for<NABc>([&](auto abl_) {
                    constexpr int abl = decltype(abl_)::value;
                    constexpr int ab = (A0 + abl / NB) * NB + abl % NB;
                    constexpr int ax = box_dim(LA, LB, ab, 0), ay = box_dim(LA, LB, ab, 1),
                                  az = box_dim(LA, LB, ab, 2);
                    constexpr int ao = box_off(LA, LB, ab);
                    static_for<ax + 1>([&](auto t_) {
                        constexpr int t = decltype(t_)::value;
                        static_for<ay + 1>([&](auto u_) {
                            constexpr int u = decltype(u_)::value;
                            static_for<az + 1>([&](auto v_) {
                                constexpr int v = decltype(v_)::value;
                                constexpr int e = ao + (t * (ay + 1) + u) * (az + 1) + v;
                                const T ebv = eb[e * es];
                                static_for<NCDc>([&](auto cdl_) {
                                    constexpr int cdl = decltype(cdl_)::value;
                                    out[abl][cdl] = fma(ebv, W[cdl][hidx(t, u, v)], out[abl][cdl]);
                                });
                            });
                        });
                    });
                });
            }

            if constexpr (STORE) {
                if (active) {
                    static_for<NABc>([&](auto abl_) {
                        constexpr int abl = decltype(abl_)::value;
                        constexpr int ia = A0 + abl / NB, ib = abl % NB;
                        static_for<NCDc>([&](auto cdl_) {
                            constexpr int cdl = decltype(cdl_)::value;
                            constexpr int ic = (CD0 + cdl) / ND, id = (CD0 + cdl) % ND;
                            a.out[soff + ia * st0 + ib * st1 + ic * st2 + id * st3] =
                                (double)out[abl][cdl];
                        });
                    });
                }
            } else {
                digest_chunk<LA, LB, LC, LD, T, A0, A1, CD0, CD1>(out, D, Jh, Kh, N, f1, f2, f3, f4,
                                                                  fac, active, krow, a.kn, kl);
            }
        });
    };
    if constexpr (SEG && !STORE) {
        double *__restrict__ krow = (double *)(stage_lds + (size_t)wpb * a.stage_bytes);
        run_segments<NA, NB>(a, krow, xoff, [&](int t) __attribute__((always_inline)) {
            tile_body(t, krow, true);
        });
    } else {
        for (int tile0 = blockIdx.x * wpb + (threadIdx.x >> 6); tile0 < ntile;
             tile0 += gridDim.x * wpb)
            tile_body(__builtin_amdgcn_readfirstlane(tile0), nullptr, false);
    }
}

// ===========================================================================
// Kernel A, ket-outer order (ss, ps, pp and ds bras; Fock or store mode).  The same lane-per-
// quartet tiles as k_eri_lane, with the primitive loops swapped: each ket
// primitive's data are loaded once and held in registers while the bra
// primitives (staged in LDS for the whole wave) run inside, and the bra
// contraction is applied per primitive quartet:
//   V_{tuv,cd} = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R^0_{t+tau,u+nu,v+phi}
//   (ab|cd)   += sum_tuv E^{ab}_{tuv} V_{tuv,cd}
// This trades the once-per-bra-primitive bra step for one per primitive
// quartet (cheap for small bra boxes) against loading every ket primitive
// once per quartet instead of once per bra primitive.
// ===========================================================================
// Boys-function providers of the ket-outer tile body: the class kernels
// stage the grid pre-divided for their own order L (boys.h); the persistent
// kernel stages raw F_n(T_k) for every order its classes need.
template <bool ET>
struct BoysStaged64 {
    const double *tab;
    template <int L>
    __device__ __forceinline__ void eval(double T, double *F) const { boys_eval<L, ET>(T, tab, F); }
};
struct BoysStagedMixed {
    const float *tab;
    template <int L>
    __device__ __forceinline__ void eval(double T, double *F) const {
        boys_eval_mixed<L>(T, tab, F);
    }
};

// One tile (one bra pair x up to 64 kets) of the ket-outer kernel.  sp: this
// wave's LDS slice for the staged bra primitives (4 + n_entries values each,
// a.stage_prims of them).
template <int LA, int LB, int LC, int LD, typename T, bool STORE, int CA, int CDC, typename BP>
__device__ __forceinline__ void ko_tile(const EriArgs &a, const int tile, const BP &bp,
                                        double *__restrict__ sp, double *__restrict__ krow = nullptr,
                                        bool kl = false) {
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NCD = NC * ND, NHAB = nherm(LAB), NH = nherm(L);
    constexpr int NEB = n_entries(LA, LB), NEK = n_entries(LC, LD);
    constexpr int NCHA = (NA + CA - 1) / CA, NCHCD = (NCD + CDC - 1) / CDC;
    constexpr bool F32 = std::is_same<T, float>::value;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ Eb = etab<T>(a.bra);
    const T *__restrict__ Ek = etab<T>(a.ket);
    const size_t nb = a.bra.n, nk = a.ket.n;
    const long long xoff = (!STORE && a.xcd_stride) ? xcd_index() * a.xcd_stride : 0;
    T *__restrict__ se = (T *)(sp + 4 * a.stage_prims);
    int bra, ket;
    bool active;
    if constexpr (STORE) {
        bra = __builtin_amdgcn_readfirstlane(a.st_bra[tile]);
        ket = a.st_ket[tile * 64 + lane];
        active = ket >= 0;
        if (!active) ket = 0;
    } else {
        const int b = tile_bra(a.tl, tile);
        bra = __builtin_amdgcn_readfirstlane(a.tl.bra[b]);
        const int k0 = a.tl.ket_lo[b] + (tile - a.tl.tile_start[b]) * TILE;
        ket = k0 + lane;
        active = ket < a.tl.ket_hi[b];
        if (!active) ket = k0;
    }
    const int nbp = __builtin_amdgcn_readfirstlane(a.bra.nprim[bra]);
    const int nkp = active ? a.ket.nprim[ket] : 0;
    const int mol = __builtin_amdgcn_readfirstlane(a.bra.mol[bra]);
    const long long mbase = STORE ? 0 : a.mol_off[mol];
    const int N = STORE ? 0 : a.mol_n[mol];
    const double *__restrict__ D = STORE ? nullptr : a.D + mbase;
    double *__restrict__ Jh = STORE ? nullptr : a.Jh + xoff + mbase;
    double *__restrict__ Kh = STORE ? nullptr : a.Kh + xoff + mbase;
    const int f1 = __builtin_amdgcn_readfirstlane(a.bra.bf1[bra]);
    const int f2 = __builtin_amdgcn_readfirstlane(a.bra.bf2[bra]);
    const int f3 = a.ket.bf1[ket], f4 = a.ket.bf2[ket];
    double fac = active ? 1.0 : 0.0;
    if (a.bra.sh1[bra] == a.bra.sh2[bra]) fac *= 0.5;
    if (a.ket.sh1[ket] == a.ket.sh2[ket]) fac *= 0.5;
    if (a.same_class && ket == bra) fac *= 0.5;
    long long soff = 0;
    int st0 = 0, st1 = 0, st2 = 0, st3 = 0;
    if constexpr (STORE) {
        if (active) {
            const size_t q = (size_t)tile * 64 + lane;
            soff = a.st_off[q];
            st0 = a.st_stride[q * 4 + 0];
            st1 = a.st_stride[q * 4 + 1];
            st2 = a.st_stride[q * 4 + 2];
            st3 = a.st_stride[q * 4 + 3];
        }
    }

    // stage the bra primitives: p, P (4 doubles) and the Hermite boxes
    for (int x = lane; x < nbp * 4; x += 64) {
        const int s = x >> 2, f = x & 3;
        sp[x] = f == 0 ? a.bra.p[(size_t)s * nb + bra] : a.bra.P[((size_t)s * 3 + f - 1) * nb + bra];
    }
    for (int x = lane; x < nbp * NEB; x += 64) se[x] = Eb[(size_t)x * nb + bra];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    static_for<NCHA * NCHCD>([&](auto ch_) {
        constexpr int ch = decltype(ch_)::value;
        constexpr int A0 = (ch / NCHCD) * CA, A1 = cmin(A0 + CA, NA);
        constexpr int CD0 = (ch % NCHCD) * CDC, CD1 = cmin(CD0 + CDC, NCD);
        constexpr int NAc = A1 - A0, NABc = NAc * NB, NCDc = CD1 - CD0;
        constexpr int EK0 = box_off(LC, LD, CD0);
        constexpr int EK1 = CD1 < NCD ? box_off(LC, LD, CD1) : NEK;
        T out[NABc][NCDc];
#pragma unroll
        for (int x = 0; x < NABc; ++x)
#pragma unroll
            for (int y = 0; y < NCDc; ++y) out[x][y] = T(0);

        for (int j = 0; j < nkp; ++j) {
            // this ket primitive, held across the bra primitives
            const double q = a.ket.p[(size_t)j * nk + ket];
            const double Kx = a.ket.P[((size_t)j * 3 + 0) * nk + ket];
            const double Ky = a.ket.P[((size_t)j * 3 + 1) * nk + ket];
            const double Kz = a.ket.P[((size_t)j * 3 + 2) * nk + ket];
            T ek[EK1 - EK0];
            const T *__restrict__ ekp = Ek + (size_t)j * NEK * nk + ket;
#pragma unroll
            for (int e = EK0; e < EK1; ++e) {
                T ev = ekp[(size_t)e * nk];
                ek[e - EK0] = ev;
            }
            for (int i = 0; i < nbp; ++i) {
                // bras with small Hermite boxes (ss, ps) read this
                // primitive's box entries here, in one batch with its p and
                // P, instead of one LDS round trip per pair of entries in
                // the bra step below
                constexpr bool EPRE = NEB <= 8;
                T ebr[EPRE ? NEB : 1];
                if constexpr (EPRE) {
#pragma unroll
                    for (int e = 0; e < NEB; ++e) ebr[e] = se[i * NEB + e];
                }
                const double p = sp[i * 4 + 0];
                const double X = sp[i * 4 + 1] - Kx, Y = sp[i * 4 + 2] - Ky,
                             Z = sp[i * 4 + 3] - Kz;
                T src[L + 1];
                if constexpr (F32) {
                    // FP32 tile: FP32 Taylor step, FP64 recursion and
                    // prefactor, sources rounded to FP32
                    const double rs = rsqrt(p + q);
                    const double alpha = p * q * (rs * rs);
                    double F[L + 1];
                    bp.template eval<L>(alpha * (X * X + Y * Y + Z * Z), F);
                    double m = rs;
#pragma unroll
                    for (int n = 0; n <= L; ++n) {
                        src[n] = (float)(F[n] * m);
                        m *= -2.0 * alpha;
                    }
                } else {
                    const double rs = rsqrt(p + q);
                    const double alpha = p * q * (rs * rs);
                    double F[L + 1];
                    bp.template eval<L>(alpha * (X * X + Y * Y + Z * Z), F);
                    double m = rs;
#pragma unroll
                    for (int n = 0; n <= L; ++n) {
                        src[n] = T(F[n] * m);
                        m *= -2.0 * alpha;
                    }
                }
                T r[NH];
                hermite_r<L, T>(src, T(X), T(Y), T(Z), r);
                // ket step for this primitive quartet
                T V[NCDc][NHAB];
                static_for<NCDc>([&](auto cdl_) {
                    constexpr int cdl = decltype(cdl_)::value;
                    constexpr int cd = CD0 + cdl;
                    constexpr int bx = box_dim(LC, LD, cd, 0), by = box_dim(LC, LD, cd, 1),
                                  bz = box_dim(LC, LD, cd, 2);
                    constexpr int eo = box_off(LC, LD, cd);
                    static_for<NHAB>([&](auto h_) { V[cdl][decltype(h_)::value] = T(0); });
                    static_for<bx + 1>([&](auto ta_) {
                        constexpr int ta = decltype(ta_)::value;
                        static_for<by + 1>([&](auto nu_) {
                            constexpr int nu = decltype(nu_)::value;
                            static_for<bz + 1>([&](auto ph_) {
                                constexpr int ph = decltype(ph_)::value;
                                constexpr int e = eo + (ta * (by + 1) + nu) * (bz + 1) + ph;
                                T ev = ek[e - EK0];
                                if constexpr ((ta + nu + ph) & 1) ev = -ev;
                                static_for<NHAB>([&](auto h_) {
                                    constexpr int h = decltype(h_)::value;
                                    constexpr int ri = hidx(hidx_t(h) + ta, hidx_u(h) + nu,
                                                            hidx_v(h) + ph);
                                    V[cdl][h] = fma(ev, r[ri], V[cdl][h]);
                                });
                            });
                        });
                    });
                });
                // bra step for this primitive quartet (boxes from LDS)
                const T *__restrict__ eb = se + i * NEB;
                static_for<NABc>([&](auto abl_) {
                    constexpr int abl = decltype(abl_)::value;
                    constexpr int ab = (A0 + abl / NB) * NB + abl % NB;
                    constexpr int ax = box_dim(LA, LB, ab, 0), ay = box_dim(LA, LB, ab, 1),
                                  az = box_dim(LA, LB, ab, 2);
                    constexpr int ao = box_off(LA, LB, ab);
                    static_for<ax + 1>([&](auto t_) {
                        constexpr int t = decltype(t_)::value;
                        static_for<ay + 1>([&](auto u_) {
                            constexpr int u = decltype(u_)::value;
                            static_for<az + 1>([&](auto v_) {
                                constexpr int v = decltype(v_)::value;
                                constexpr int e = ao + (t * (ay + 1) + u) * (az + 1) + v;
                                const T ebv = EPRE ? ebr[EPRE ? e : 0] : eb[e];
                                static_for<NCDc>([&](auto cdl_) {
                                    constexpr int cdl = decltype(cdl_)::value;
                                    out[abl][cdl] = fma(ebv, V[cdl][hidx(t, u, v)], out[abl][cdl]);
                                });
                            });
                        });
                    });
                });
            }
        }
        if constexpr (STORE) {
            if (active) {
                static_for<NABc>([&](auto abl_) {
                    constexpr int abl = decltype(abl_)::value;
                    constexpr int ia = A0 + abl / NB, ib = abl % NB;
                    static_for<NCDc>([&](auto cdl_) {
                        constexpr int cdl = decltype(cdl_)::value;
                        constexpr int ic = (CD0 + cdl) / ND, id = (CD0 + cdl) % ND;
                        a.out[soff + ia * st0 + ib * st1 + ic * st2 + id * st3] =
                            (double)out[abl][cdl];
                    });
                });
            }
        } else {
            digest_chunk<LA, LB, LC, LD, T, A0, A1, CD0, CD1>(out, D, Jh, Kh, N, f1, f2, f3,
                                                              f4, fac, active, krow, a.kn, kl);
        }
    });
}

// Blocks of the ket-outer kernel in segment mode: 12 waves for the s/p
// classes of total angular momentum 2, whose ~150 registers allow three
// waves per SIMD; 4 (one per SIMD, AGPRs available) for FP64 (ds|pp),
// which at two waves per SIMD spills to scratch; 8 (two per SIMD)
// otherwise.
__host__ __device__ constexpr int ko_seg_waves(int la, int lb, int lc, int ld, bool f64) {
    return la <= 1 && la + lb + lc + ld == 2 ? 12
                                             : (f64 && la == 2 && lc == 1 && ld == 1 ? 4 : 8);
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE, int CA, int CDC, bool SEG>
__global__ __launch_bounds__(SEG ? 64 * ko_seg_waves(LA, LB, LC, LD, !std::is_same<T, float>::value)
                                 : 256)
void k_eri_lane_ko(EriArgs a) {
    constexpr int L = LA + LB + LC + LD;
    // Boys grid in LDS: FP64 for FP64 tiles, FP32 (5 terms, the Taylor step
    // only) for FP32 tiles. FP64 tiles of s and p bras in segment mode add
    // the exp column (the d bras keep that LDS for their K' rows; launches
    // over tiles measured slower with it).
    constexpr bool F32 = std::is_same<T, float>::value;
    constexpr bool ET = !F32 && LA <= 1 && SEG;
    __shared__ std::conditional_t<F32, float, double>
        tab[F32 ? BOYS_LDS32 : (ET ? BOYS_LDS_E : BOYS_LDS)];
    extern __shared__ __align__(16) unsigned char stage_lds[];
    if constexpr (F32) boys_stage32(tab, a.boys, L);
    else boys_stage(tab, a.boys, L);
    if constexpr (ET) boys_stage_exp(tab);
    __syncthreads();
    const int wpb = blockDim.x >> 6;
    const int ntile = STORE ? a.st_ntile : a.tl.ntile;
    // every bra primitive of the tile is staged (the launch checks kmax fits)
    double *__restrict__ sp = (double *)(stage_lds + (size_t)(threadIdx.x >> 6) * a.stage_bytes);
    using BP = std::conditional_t<F32, BoysStagedMixed, BoysStaged64<ET>>;
    const BP bp{tab};
    if constexpr (SEG && !STORE) {
        // segment mode: the block's waves share the bra's K' rows
        double *__restrict__ krow = (double *)(stage_lds + (size_t)wpb * a.stage_bytes);
        const long long xoff = a.xcd_stride ? xcd_index() * a.xcd_stride : 0;
        run_segments<ncart(LA), ncart(LB)>(a, krow, xoff, [&](int t) __attribute__((always_inline)) {
            ko_tile<LA, LB, LC, LD, T, STORE, CA, CDC>(a, t, bp, sp, krow, true);
        });
    } else {
        for (int tile0 = blockIdx.x * wpb + (threadIdx.x >> 6); tile0 < ntile;
             tile0 += gridDim.x * wpb)
            ko_tile<LA, LB, LC, LD, T, STORE, CA, CDC>(a, __builtin_amdgcn_readfirstlane(tile0),
                                                       bp, sp);
    }
}

// ===========================================================================
// Kernel B: one wave per contracted quartet for the high-L classes (d shells).
// R^0 is built level by level in LDS with the lanes over Hermite triples,
// W_{tuv,cd} is accumulated over ket primitives with the lanes over
// (tuv, cd), and the block with the lanes over (ab, cd).
// ===========================================================================
template <int LA, int LB, int LC, int LD, typename T, bool STORE>
__global__ __launch_bounds__(64) void k_eri_wave(EriArgs a) {
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND, NHAB = nherm(LAB), NH = nherm(L);
    constexpr int NEB = n_entries(LA, LB), NEK = n_entries(LC, LD);
    constexpr int NW = NHAB * NCD, NWL = (NW + 63) / 64;
    constexpr int NO = NAB * NCD, NOL = (NO + 63) / 64;
    constexpr int NRL = (NH + 63) / 64;
    __shared__ double tab[BOYS_LDS];
    __shared__ T rbuf[2][NH];
    __shared__ T wl[NW];
    __shared__ T ebl[NEB], ekl[NEK];
    // digest staging: density elements D_ab, D_cd, D_bd, D_ad, D_bc, D_ac
    // (offsets DO_*) and the J'/K' targets (offsets TG_*)
    constexpr int DO_CD = NAB, DO_BD = DO_CD + NCD, DO_AD = DO_BD + NB * ND,
                  DO_BC = DO_AD + NA * ND, DO_AC = DO_BC + NB * NC, NDEN = DO_AC + NA * NC;
    constexpr int TG_JCD = NAB, TG_KAC = TG_JCD + NCD, TG_KBC = TG_KAC + NA * NC,
                  TG_KAD = TG_KBC + NB * NC, TG_KBD = TG_KAD + NA * ND, NTGT = TG_KBD + NB * ND;
    __shared__ double blk[STORE ? 1 : NO];
    __shared__ double den[STORE ? 1 : NDEN];
    boys_stage(tab, a.boys, L);
    const int lane = threadIdx.x;

    // per-lane decode of the owned Hermite triples, W entries and block entries
    int rt[NRL], ru[NRL], rv[NRL];
#pragma unroll
    for (int k = 0; k < NRL; ++k) {
        const int id = lane + 64 * k < NH ? lane + 64 * k : 0;
        rt[k] = hidx_t(id);
        ru[k] = hidx_u(id);
        rv[k] = hidx_v(id);
    }
    int wt[NWL], wu[NWL], wv[NWL], wcd[NWL], wbx[NWL], wby[NWL], wbz[NWL], wo[NWL];
#pragma unroll
    for (int k = 0; k < NWL; ++k) {
        const int e = lane + 64 * k < NW ? lane + 64 * k : 0;
        const int h = e / NCD, cd = e % NCD;
        wt[k] = hidx_t(h);
        wu[k] = hidx_u(h);
        wv[k] = hidx_v(h);
        wcd[k] = cd;
        wbx[k] = box_dim(LC, LD, cd, 0);
        wby[k] = box_dim(LC, LD, cd, 1);
        wbz[k] = box_dim(LC, LD, cd, 2);
        wo[k] = box_off(LC, LD, cd);
    }
    int oab[NOL], ocd[NOL], obx[NOL], oby[NOL], obz[NOL], oo[NOL];
#pragma unroll
    for (int k = 0; k < NOL; ++k) {
        const int e = lane + 64 * k < NO ? lane + 64 * k : 0;
        oab[k] = e / NCD;
        ocd[k] = e % NCD;
        obx[k] = box_dim(LA, LB, oab[k], 0);
        oby[k] = box_dim(LA, LB, oab[k], 1);
        obz[k] = box_dim(LA, LB, oab[k], 2);
        oo[k] = box_off(LA, LB, oab[k]);
    }
    __syncthreads();

    const int ntile = STORE ? a.st_ntile : a.tl.ntile;
    const T *__restrict__ Eb = etab<T>(a.bra);
    const T *__restrict__ Ek = etab<T>(a.ket);
    const size_t nb = a.bra.n, nk = a.ket.n;

    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        int bra, k0 = 0, k1 = 0;
        if constexpr (STORE) {
            bra = a.st_bra[tile];
            k1 = 64;
        } else {
            const int b = tile_bra(a.tl, tile);
            bra = a.tl.bra[b];
            k0 = a.tl.ket_lo[b] + (tile - a.tl.tile_start[b]) * TILE;
            k1 = min(k0 + TILE, a.tl.ket_hi[b]);
        }
        const int nbp = a.bra.nprim[bra];
        for (int kk = k0; kk < k1; ++kk) {
            int ket = kk;
            if constexpr (STORE) {
                ket = a.st_ket[tile * 64 + kk];
                if (ket < 0) continue;
            }
            const int nkp = a.ket.nprim[ket];
            T o[NOL];
#pragma unroll
            for (int k = 0; k < NOL; ++k) o[k] = T(0);
            for (int i = 0; i < nbp; ++i) {
                const double p = a.bra.p[i * nb + bra];
                const double Px = a.bra.P[(i * 3 + 0) * nb + bra];
                const double Py = a.bra.P[(i * 3 + 1) * nb + bra];
                const double Pz = a.bra.P[(i * 3 + 2) * nb + bra];
                for (int e = lane; e < NEB; e += 64) ebl[e] = Eb[((size_t)i * NEB + e) * nb + bra];
                T w[NWL];
#pragma unroll
                for (int k = 0; k < NWL; ++k) w[k] = T(0);
                for (int j = 0; j < nkp; ++j) {
                    const double q = a.ket.p[j * nk + ket];
                    const double X = Px - a.ket.P[(j * 3 + 0) * nk + ket];
                    const double Y = Py - a.ket.P[(j * 3 + 1) * nk + ket];
                    const double Z = Pz - a.ket.P[(j * 3 + 2) * nk + ket];
                    const double pq = p + q, alpha = p * q / pq;
                    double F[L + 1];
                    boys_eval<L>(alpha * (X * X + Y * Y + Z * Z), tab, F);
                    T src[L + 1];
                    double m = 1.0 / sqrt(pq);
#pragma unroll
                    for (int n = 0; n <= L; ++n) {
                        src[n] = T(F[n] * m);
                        m *= -2.0 * alpha;
                    }
                    for (int e = lane; e < NEK; e += 64)
                        ekl[e] = Ek[((size_t)j * NEK + e) * nk + ket];
                    // R^0 level by level (level n holds totals <= L - n)
                    int cur = 0;
                    if (lane == 0) rbuf[0][0] = src[L];
                    __syncthreads();
                    for (int n = L - 1; n >= 0; --n) {
                        const int nxt = cur ^ 1, cnt = nherm(L - n);
                        const T Xt = T(X), Yt = T(Y), Zt = T(Z);
#pragma unroll
                        for (int k = 0; k < NRL; ++k) {
                            const int id = lane + 64 * k;
                            if (id < cnt) {
                                const int t = rt[k], u = ru[k], v = rv[k];
                                T val;
                                if (id == 0) val = src[n];
                                else if (t > 0)
                                    val = Xt * rbuf[cur][hidx(t - 1, u, v)] +
                                          (t > 1 ? T(t - 1) * rbuf[cur][hidx(t - 2, u, v)] : T(0));
                                else if (u > 0)
                                    val = Yt * rbuf[cur][hidx(t, u - 1, v)] +
                                          (u > 1 ? T(u - 1) * rbuf[cur][hidx(t, u - 2, v)] : T(0));
                                else
                                    val = Zt * rbuf[cur][hidx(t, u, v - 1)] +
                                          (v > 1 ? T(v - 1) * rbuf[cur][hidx(t, u, v - 2)] : T(0));
                                rbuf[nxt][id] = val;
                            }
                        }
                        cur = nxt;
                        __syncthreads();
                    }
                    const T *R = rbuf[cur];
#pragma unroll
                    for (int k = 0; k < NWL; ++k) {
                        if (lane + 64 * k < NW) {
                            T acc = w[k];
                            int e = wo[k];
                            for (int ta = 0; ta <= wbx[k]; ++ta)
                                for (int nu = 0; nu <= wby[k]; ++nu)
                                    for (int ph = 0; ph <= wbz[k]; ++ph, ++e) {
                                        const T ev = ((ta + nu + ph) & 1) ? -ekl[e] : ekl[e];
                                        acc += ev * R[hidx(wt[k] + ta, wu[k] + nu, wv[k] + ph)];
                                    }
                            w[k] = acc;
                        }
                    }
                    __syncthreads();
                }
#pragma unroll
                for (int k = 0; k < NWL; ++k)
                    if (lane + 64 * k < NW) wl[lane + 64 * k] = w[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NOL; ++k) {
                    if (lane + 64 * k < NO) {
                        T acc = o[k];
                        int e = oo[k];
                        for (int t = 0; t <= obx[k]; ++t)
                            for (int u = 0; u <= oby[k]; ++u)
                                for (int v = 0; v <= obz[k]; ++v, ++e)
                                    acc += ebl[e] * wl[hidx(t, u, v) * NCD + ocd[k]];
                        o[k] = acc;
                    }
                }
                __syncthreads();
            }
            // write out or digest
            if constexpr (STORE) {
                const size_t q = (size_t)tile * 64 + kk;
                const long long off = a.st_off[q];
                const int s0 = a.st_stride[q * 4 + 0], s1 = a.st_stride[q * 4 + 1],
                          s2 = a.st_stride[q * 4 + 2], s3 = a.st_stride[q * 4 + 3];
#pragma unroll
                for (int k = 0; k < NOL; ++k) {
                    if (lane + 64 * k < NO) {
                        const int ia = oab[k] / NB, ib = oab[k] % NB, ic = ocd[k] / ND,
                                  id = ocd[k] % ND;
                        a.out[off + ia * s0 + ib * s1 + ic * s2 + id * s3] = (double)o[k];
                    }
                }
            } else {
                const int mol = a.bra.mol[bra];
                const long long mbase = a.mol_off[mol];
                const int N = a.mol_n[mol];
                const double *__restrict__ D = a.D + mbase;
                const long long xoff = a.xcd_stride ? xcd_index() * a.xcd_stride : 0;
                double *__restrict__ Jh = a.Jh + xoff + mbase;
                double *__restrict__ Kh = a.Kh + xoff + mbase;
                const int f1 = a.bra.bf1[bra], f2 = a.bra.bf2[bra];
                const int f3 = a.ket.bf1[ket], f4 = a.ket.bf2[ket];
                double fac = 1.0;
                if (a.bra.sh1[bra] == a.bra.sh2[bra]) fac *= 0.5;
                if (a.ket.sh1[ket] == a.ket.sh2[ket]) fac *= 0.5;
                if (a.same_class && ket == bra) fac *= 0.5;
                // Reduce before scattering: the scaled block and the density
                // elements it meets go to LDS, then every J'/K' target element
                // is summed once and added with a single atomic (adding each
                // block element separately would put up to NCD lanes of one
                // instruction on the same address).
#pragma unroll
                for (int k = 0; k < NOL; ++k)
                    if (lane + 64 * k < NO) blk[lane + 64 * k] = fac * (double)o[k];
                for (int x = lane; x < NDEN; x += 64) {
                    size_t r, c;
                    if (x < DO_CD) { r = f1 + x / NB; c = f2 + x % NB; }
                    else if (x < DO_BD) { r = f3 + (x - DO_CD) / ND; c = f4 + (x - DO_CD) % ND; }
                    else if (x < DO_AD) { r = f2 + (x - DO_BD) / ND; c = f4 + (x - DO_BD) % ND; }
                    else if (x < DO_BC) { r = f1 + (x - DO_AD) / ND; c = f4 + (x - DO_AD) % ND; }
                    else if (x < DO_AC) { r = f2 + (x - DO_BC) / NC; c = f3 + (x - DO_BC) % NC; }
                    else { r = f1 + (x - DO_AC) / NC; c = f3 + (x - DO_AC) % NC; }
                    den[x] = D[r * N + c];
                }
                __syncthreads();
                for (int t = lane; t < NTGT; t += 64) {
                    double sum = 0.0;
                    size_t r, c;
                    if (t < TG_JCD) {   // J'_ab += 2 sum_cd v D_cd
                        for (int cd = 0; cd < NCD; ++cd) sum += blk[t * NCD + cd] * den[DO_CD + cd];
                        sum *= 2.0;
                        r = f1 + t / NB;
                        c = f2 + t % NB;
                        atomicAdd(&Jh[r * N + c], sum);
                    } else if (t < TG_KAC) {   // J'_cd += 2 sum_ab v D_ab
                        const int cd = t - TG_JCD;
                        for (int ab = 0; ab < NAB; ++ab) sum += blk[ab * NCD + cd] * den[ab];
                        sum *= 2.0;
                        r = f3 + cd / ND;
                        c = f4 + cd % ND;
                        atomicAdd(&Jh[r * N + c], sum);
                    } else if (t < TG_KBC) {   // K'_ac += sum_bd v D_bd
                        const int ia = (t - TG_KAC) / NC, ic = (t - TG_KAC) % NC;
                        for (int ib = 0; ib < NB; ++ib)
                            for (int id = 0; id < ND; ++id)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_BD + ib * ND + id];
                        atomicAdd(&Kh[(size_t)(f1 + ia) * N + f3 + ic], sum);
                    } else if (t < TG_KAD) {   // K'_bc += sum_ad v D_ad
                        const int ib = (t - TG_KBC) / NC, ic = (t - TG_KBC) % NC;
                        for (int ia = 0; ia < NA; ++ia)
                            for (int id = 0; id < ND; ++id)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_AD + ia * ND + id];
                        atomicAdd(&Kh[(size_t)(f2 + ib) * N + f3 + ic], sum);
                    } else if (t < TG_KBD) {   // K'_ad += sum_bc v D_bc
                        const int ia = (t - TG_KAD) / ND, id = (t - TG_KAD) % ND;
                        for (int ib = 0; ib < NB; ++ib)
                            for (int ic = 0; ic < NC; ++ic)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_BC + ib * NC + ic];
                        atomicAdd(&Kh[(size_t)(f1 + ia) * N + f4 + id], sum);
                    } else {   // K'_bd += sum_ac v D_ac
                        const int ib = (t - TG_KBD) / ND, id = (t - TG_KBD) % ND;
                        for (int ia = 0; ia < NA; ++ia)
                            for (int ic = 0; ic < NC; ++ic)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_AC + ia * NC + ic];
                        atomicAdd(&Kh[(size_t)(f2 + ib) * N + f4 + id], sum);
                    }
                }
                __syncthreads();
            }
        }
    }
}

// ===========================================================================
// Kernel C: one wave per contracted quartet with both E.R.E steps on the
// matrix cores (16x16x4 MFMA, FP64 or FP32).  Per primitive quartet,
//   W[h_ab][cd] += sum_{h_cd} R^0[h_ab + h_cd] Et[h_cd][cd]     (step 1)
// with Et the ket Hermite entries carrying (-1)^{tau+nu+phi} (zero outside a
// component pair's box); per bra primitive pair,
//   (ab|cd)     += sum_{h_ab} E[ab][h_ab] W[h_ab][cd]            (step 2).
// Both are dense products over the Hermite index, the J_{tuv,k} form of
// Sec. 2.5 (Eq. eri-tensor-contracted) written as matrix products.
// Operand layout of v_mfma_{f64,f32}_16x16x4 (lane l): A[l % 16][l / 16],
// B[l / 16][l % 16]; accumulator v of lane l holds D[l / 16 + 4 v][l % 16]
// for FP64 and D[4 (l / 16) + v][l % 16] for FP32.
// ===========================================================================
typedef double mfma_v4d __attribute__((ext_vector_type(4)));
typedef float mfma_v4f __attribute__((ext_vector_type(4)));
template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<double> {
    using acc = mfma_v4d;
    static __device__ __forceinline__ acc mma(double x, double y, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MfmaOp<float> {
    using acc = mfma_v4f;
    static __device__ __forceinline__ acc mma(float x, float y, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// F_0..F_L at T from the FP64 grid in global memory (wave-uniform reads).
template <int L>
__device__ __forceinline__ void boys_eval_global(double T, const double *__restrict__ g, double *F) {
    if (T < BOYS_TMAX) {
        const int k = __double2int_rn(T * BOYS_INV_DT);
        const double d = k * BOYS_DT - T;
        const double *c = g + k * BOYS_NORD + L;
        double f = c[BOYS_NTAYLOR - 1] * inv_factorial(BOYS_NTAYLOR - 1);
#pragma unroll
        for (int j = BOYS_NTAYLOR - 2; j >= 0; --j) f = fma(f, d, c[j] * inv_factorial(j));
        F[L] = f;
        if constexpr (L > 0) {
            const double e = exp(-T), t2 = 2.0 * T;
#pragma unroll
            for (int n = L; n > 0; --n) F[n - 1] = fma(t2, F[n], e) * (1.0 / (2 * n - 1));
        }
    } else {
        F[0] = 0.88622692545275801365 * rsqrt(T);
        if constexpr (L > 0) {
            const double e = exp(-T), h = 0.5 / T;
#pragma unroll
            for (int n = 0; n < L; ++n) F[n + 1] = ((2 * n + 1) * F[n] - e) * h;
        }
    }
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE>
__global__ __launch_bounds__(64) void k_eri_mfma(EriArgs a) {
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND;
    constexpr int NHAB = nherm(LAB), NHCD = nherm(LCD), NH = nherm(L);
    constexpr int NEB = n_entries(LA, LB), NEK = n_entries(LC, LD);
    constexpr int MT1 = (NHAB + 15) / 16, NT = (NCD + 15) / 16, KS1 = (NHCD + 3) / 4;
    constexpr int MT2 = (NAB + 15) / 16, KS2 = (NHAB + 3) / 4;
    constexpr int KR = KS1 * 4, NC16 = NT * 16, MR2 = MT2 * 16, KR2 = KS2 * 4;
    constexpr int NO = NAB * NCD, NRL = (NH + 63) / 64;
    using M = MfmaOp<T>;
    using acc_t = typename M::acc;
    // digest staging (as kernel B): density blocks and J'/K' targets
    constexpr int DO_CD = NAB, DO_BD = DO_CD + NCD, DO_AD = DO_BD + NB * ND,
                  DO_BC = DO_AD + NA * ND, DO_AC = DO_BC + NB * NC, NDEN = DO_AC + NA * NC;
    constexpr int TG_JCD = NAB, TG_KAC = TG_JCD + NCD, TG_KBC = TG_KAC + NA * NC,
                  TG_KAD = TG_KBC + NB * NC, TG_KBD = TG_KAD + NA * ND, NTGT = TG_KBD + NB * ND;
    constexpr int NWST = (KR2 * NC16 * (int)sizeof(T) + 7) / 8;   // W staging, in doubles
    constexpr int NU = STORE ? NWST : (NWST > NO ? NWST : NO);
    __shared__ T rbuf[2][NH];
    __shared__ T ekl[NEK], ebl[NEB];
    constexpr int MR1 = MT1 * 16;
    __shared__ short rmap[MR1][KR];    // R^0 index of (h_ab, h_cd), -1 in the padding
    __shared__ short kmap[KR][NC16];   // +-(ket entry + 1) with the Hermite sign, 0 outside
    __shared__ short bmap[MR2][KR2];   // bra entry + 1, 0 outside
    __shared__ double ubuf[NU];        // W staging, then the scaled block for the digest
    __shared__ double den[STORE ? 1 : NDEN];
    T *wst = (T *)ubuf;
    const int lane = threadIdx.x;

    for (int x = lane; x < KR * NC16; x += 64) {
        const int k = x / NC16, n = x % NC16;
        int val = 0;
        if (k < NHCD && n < NCD) {
            const int t = hidx_t(k), u = hidx_u(k), v = hidx_v(k);
            const int bx = box_dim(LC, LD, n, 0), by = box_dim(LC, LD, n, 1),
                      bz = box_dim(LC, LD, n, 2);
            if (t <= bx && u <= by && v <= bz) {
                const int e = box_off(LC, LD, n) + (t * (by + 1) + u) * (bz + 1) + v;
                val = ((t + u + v) & 1) ? -(e + 1) : e + 1;
            }
        }
        kmap[k][n] = (short)val;
    }
    for (int x = lane; x < MR2 * KR2; x += 64) {
        const int m = x / KR2, k = x % KR2;
        int val = 0;
        if (m < NAB && k < NHAB) {
            const int t = hidx_t(k), u = hidx_u(k), v = hidx_v(k);
            const int bx = box_dim(LA, LB, m, 0), by = box_dim(LA, LB, m, 1),
                      bz = box_dim(LA, LB, m, 2);
            if (t <= bx && u <= by && v <= bz)
                val = box_off(LA, LB, m) + (t * (by + 1) + u) * (bz + 1) + v + 1;
        }
        bmap[m][k] = (short)val;
    }
    for (int x = lane; x < MR1 * KR; x += 64) {
        const int r = x / KR, k = x % KR;
        rmap[r][k] = (short)((r < NHAB && k < NHCD)
                                 ? hidx(hidx_t(r) + hidx_t(k), hidx_u(r) + hidx_u(k),
                                        hidx_v(r) + hidx_v(k))
                                 : -1);
    }
    // level decode of the R recursion (as kernel B)
    int rt[NRL], ru[NRL], rv[NRL];
#pragma unroll
    for (int k = 0; k < NRL; ++k) {
        const int id = lane + 64 * k < NH ? lane + 64 * k : 0;
        rt[k] = hidx_t(id);
        ru[k] = hidx_u(id);
        rv[k] = hidx_v(id);
    }
    __syncthreads();

    const int ntile = STORE ? a.st_ntile : a.tl.ntile;
    const T *__restrict__ Eb = etab<T>(a.bra);
    const T *__restrict__ Ek = etab<T>(a.ket);
    const size_t nb = a.bra.n, nk = a.ket.n;

    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        int bra, k0 = 0, k1 = 0;
        if constexpr (STORE) {
            bra = a.st_bra[tile];
            k1 = 64;
        } else {
            const int b = tile_bra(a.tl, tile);
            bra = a.tl.bra[b];
            k0 = a.tl.ket_lo[b] + (tile - a.tl.tile_start[b]) * TILE;
            k1 = min(k0 + TILE, a.tl.ket_hi[b]);
        }
        const int nbp = a.bra.nprim[bra];
        for (int kk = k0; kk < k1; ++kk) {
            int ket = kk;
            if constexpr (STORE) {
                ket = a.st_ket[tile * 64 + kk];
                if (ket < 0) continue;
            }
            const int nkp = a.ket.nprim[ket];
            acc_t o[MT2][NT];
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) o[mt][nt] = acc_t{};
            for (int i = 0; i < nbp; ++i) {
                const double p = a.bra.p[i * nb + bra];
                const double Px = a.bra.P[(i * 3 + 0) * nb + bra];
                const double Py = a.bra.P[(i * 3 + 1) * nb + bra];
                const double Pz = a.bra.P[(i * 3 + 2) * nb + bra];
                for (int e = lane; e < NEB; e += 64) ebl[e] = Eb[((size_t)i * NEB + e) * nb + bra];
                acc_t w[MT1][NT];
#pragma unroll
                for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) w[mt][nt] = acc_t{};
                for (int j = 0; j < nkp; ++j) {
                    const double q = a.ket.p[j * nk + ket];
                    const double X = Px - a.ket.P[(j * 3 + 0) * nk + ket];
                    const double Y = Py - a.ket.P[(j * 3 + 1) * nk + ket];
                    const double Z = Pz - a.ket.P[(j * 3 + 2) * nk + ket];
                    const double pq = p + q, alpha = p * q / pq;
                    double F[L + 1];
                    boys_eval_global<L>(alpha * (X * X + Y * Y + Z * Z), a.boys, F);
                    T src[L + 1];
                    double m = 1.0 / sqrt(pq);
#pragma unroll
                    for (int n = 0; n <= L; ++n) {
                        src[n] = T(F[n] * m);
                        m *= -2.0 * alpha;
                    }
                    for (int e = lane; e < NEK; e += 64)
                        ekl[e] = Ek[((size_t)j * NEK + e) * nk + ket];
                    // R^0 level by level (level n holds totals <= L - n)
                    int cur = 0;
                    if (lane == 0) rbuf[0][0] = src[L];
                    __syncthreads();
                    for (int n = L - 1; n >= 0; --n) {
                        const int nxt = cur ^ 1, cnt = nherm(L - n);
                        const T Xt = T(X), Yt = T(Y), Zt = T(Z);
#pragma unroll
                        for (int k = 0; k < NRL; ++k) {
                            const int id = lane + 64 * k;
                            if (id < cnt) {
                                const int t = rt[k], u = ru[k], v = rv[k];
                                T val;
                                if (id == 0) val = src[n];
                                else if (t > 0)
                                    val = Xt * rbuf[cur][hidx(t - 1, u, v)] +
                                          (t > 1 ? T(t - 1) * rbuf[cur][hidx(t - 2, u, v)] : T(0));
                                else if (u > 0)
                                    val = Yt * rbuf[cur][hidx(t, u - 1, v)] +
                                          (u > 1 ? T(u - 1) * rbuf[cur][hidx(t, u - 2, v)] : T(0));
                                else
                                    val = Zt * rbuf[cur][hidx(t, u, v - 1)] +
                                          (v > 1 ? T(v - 1) * rbuf[cur][hidx(t, u, v - 2)] : T(0));
                                rbuf[nxt][id] = val;
                            }
                        }
                        cur = nxt;
                        __syncthreads();
                    }
                    const T *R = rbuf[cur];
                    // step 1 on the matrix cores (K steps not unrolled: the
                    // operands of one step are loaded just before its MFMAs)
#pragma unroll 1
                    for (int ks = 0; ks < KS1; ++ks) {
                        T bv[NT];
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            const int mk = kmap[4 * ks + (lane >> 4)][16 * nt + (lane & 15)];
                            bv[nt] = mk == 0 ? T(0) : (mk > 0 ? ekl[mk - 1] : -ekl[-mk - 1]);
                        }
#pragma unroll
                        for (int mt = 0; mt < MT1; ++mt) {
                            const int ri = rmap[16 * mt + (lane & 15)][4 * ks + (lane >> 4)];
                            const T av = ri >= 0 ? R[ri] : T(0);
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt) w[mt][nt] = M::mma(av, bv[nt], w[mt][nt]);
                        }
                    }
                    __syncthreads();   // rbuf and ekl are rewritten by the next ket primitive
                }
                // W to LDS in the B-operand order of step 2 (rows h_ab < KR2)
#pragma unroll
                for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r = 16 * mt + M::row(lane, v);
                            if (r < KR2) wst[r * NC16 + 16 * nt + (lane & 15)] = w[mt][nt][v];
                        }
                __syncthreads();
                // step 2 on the matrix cores
#pragma unroll 1
                for (int ks = 0; ks < KS2; ++ks) {
                    T bv[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        bv[nt] = wst[(4 * ks + (lane >> 4)) * NC16 + 16 * nt + (lane & 15)];
#pragma unroll
                    for (int mt = 0; mt < MT2; ++mt) {
                        const int mb = bmap[16 * mt + (lane & 15)][4 * ks + (lane >> 4)];
                        const T av = mb ? ebl[mb - 1] : T(0);
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) o[mt][nt] = M::mma(av, bv[nt], o[mt][nt]);
                    }
                }
                __syncthreads();   // wst and ebl are rewritten by the next bra primitive
            }
            if constexpr (STORE) {
                const size_t qq = (size_t)tile * 64 + kk;
                const long long off = a.st_off[qq];
                const int s0 = a.st_stride[qq * 4 + 0], s1 = a.st_stride[qq * 4 + 1],
                          s2 = a.st_stride[qq * 4 + 2], s3 = a.st_stride[qq * 4 + 3];
#pragma unroll
                for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int ab = 16 * mt + M::row(lane, v), cd = 16 * nt + (lane & 15);
                            if (ab < NAB && cd < NCD)
                                a.out[off + (ab / NB) * s0 + (ab % NB) * s1 + (cd / ND) * s2 +
                                      (cd % ND) * s3] = (double)o[mt][nt][v];
                        }
            } else {
                const int mol = a.bra.mol[bra];
                const long long mbase = a.mol_off[mol];
                const int N = a.mol_n[mol];
                const double *__restrict__ D = a.D + mbase;
                const long long xoff = a.xcd_stride ? xcd_index() * a.xcd_stride : 0;
                double *__restrict__ Jh = a.Jh + xoff + mbase;
                double *__restrict__ Kh = a.Kh + xoff + mbase;
                const int f1 = a.bra.bf1[bra], f2 = a.bra.bf2[bra];
                const int f3 = a.ket.bf1[ket], f4 = a.ket.bf2[ket];
                double fac = 1.0;
                if (a.bra.sh1[bra] == a.bra.sh2[bra]) fac *= 0.5;
                if (a.ket.sh1[ket] == a.ket.sh2[ket]) fac *= 0.5;
                if (a.same_class && ket == bra) fac *= 0.5;
                double *blk = ubuf;
#pragma unroll
                for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int ab = 16 * mt + M::row(lane, v), cd = 16 * nt + (lane & 15);
                            if (ab < NAB && cd < NCD) blk[ab * NCD + cd] = fac * (double)o[mt][nt][v];
                        }
                for (int x = lane; x < NDEN; x += 64) {
                    size_t r, c;
                    if (x < DO_CD) { r = f1 + x / NB; c = f2 + x % NB; }
                    else if (x < DO_BD) { r = f3 + (x - DO_CD) / ND; c = f4 + (x - DO_CD) % ND; }
                    else if (x < DO_AD) { r = f2 + (x - DO_BD) / ND; c = f4 + (x - DO_BD) % ND; }
                    else if (x < DO_BC) { r = f1 + (x - DO_AD) / ND; c = f4 + (x - DO_AD) % ND; }
                    else if (x < DO_AC) { r = f2 + (x - DO_BC) / NC; c = f3 + (x - DO_BC) % NC; }
                    else { r = f1 + (x - DO_AC) / NC; c = f3 + (x - DO_AC) % NC; }
                    den[x] = D[r * N + c];
                }
                __syncthreads();
                for (int t = lane; t < NTGT; t += 64) {
                    double sum = 0.0;
                    if (t < TG_JCD) {   // J'_ab += 2 sum_cd v D_cd
#pragma unroll 2
                        for (int cd = 0; cd < NCD; ++cd) sum += blk[t * NCD + cd] * den[DO_CD + cd];
                        atomicAdd(&Jh[(size_t)(f1 + t / NB) * N + f2 + t % NB], 2.0 * sum);
                    } else if (t < TG_KAC) {   // J'_cd += 2 sum_ab v D_ab
                        const int cd = t - TG_JCD;
#pragma unroll 2
                        for (int ab = 0; ab < NAB; ++ab) sum += blk[ab * NCD + cd] * den[ab];
                        atomicAdd(&Jh[(size_t)(f3 + cd / ND) * N + f4 + cd % ND], 2.0 * sum);
                    } else if (t < TG_KBC) {   // K'_ac += sum_bd v D_bd
                        const int ia = (t - TG_KAC) / NC, ic = (t - TG_KAC) % NC;
#pragma unroll 1
                        for (int ib = 0; ib < NB; ++ib)
                            for (int id = 0; id < ND; ++id)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_BD + ib * ND + id];
                        atomicAdd(&Kh[(size_t)(f1 + ia) * N + f3 + ic], sum);
                    } else if (t < TG_KAD) {   // K'_bc += sum_ad v D_ad
                        const int ib = (t - TG_KBC) / NC, ic = (t - TG_KBC) % NC;
#pragma unroll 1
                        for (int ia = 0; ia < NA; ++ia)
                            for (int id = 0; id < ND; ++id)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_AD + ia * ND + id];
                        atomicAdd(&Kh[(size_t)(f2 + ib) * N + f3 + ic], sum);
                    } else if (t < TG_KBD) {   // K'_ad += sum_bc v D_bc
                        const int ia = (t - TG_KAD) / ND, id = (t - TG_KAD) % ND;
#pragma unroll 1
                        for (int ib = 0; ib < NB; ++ib)
                            for (int ic = 0; ic < NC; ++ic)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_BC + ib * NC + ic];
                        atomicAdd(&Kh[(size_t)(f1 + ia) * N + f4 + id], sum);
                    } else {   // K'_bd += sum_ac v D_ac
                        const int ib = (t - TG_KBD) / ND, id = (t - TG_KBD) % ND;
#pragma unroll 1
                        for (int ia = 0; ia < NA; ++ia)
                            for (int ic = 0; ic < NC; ++ic)
                                sum += blk[(ia * NB + ib) * NCD + ic * ND + id] * den[DO_AC + ia * NC + ic];
                        atomicAdd(&Kh[(size_t)(f2 + ib) * N + f4 + id], sum);
                    }
                }
                __syncthreads();   // blk and den are rewritten by the next quartet
            }
        }
    }
}

// Launch variants.  Variants 0..2 fix the per-lane register budget of kernel
// A (live block + W + R^0 values; the chunking follows from it); variant 3 is
// kernel B; variant 4 is kernel A in ket-outer order (bras with small
// Hermite boxes: ss, ps, pp, ds; other classes run the default variant).  A budget whose chunking does not
// fit, or needs more than MAX_CHUNKS chunks, falls back to kernel B.  The
// autotuner picks a variant and the waves per block for every class and
// precision.
constexpr int NVARIANT = 7;
constexpr int VARIANT_WAVE = 3;
constexpr int VARIANT_KO = 4;
constexpr int VARIANT_WIDE = 5;   // kernel A at 192 live values, where 160 does not fit
constexpr int VARIANT_MFMA = 6;   // kernel C (matrix cores), classes with a d bra
constexpr int DEFAULT_VARIANT = 1;
__host__ __device__ constexpr int variant_budget(int v) {
    return v == 0 ? 96 : (v == 1 ? 128 : (v == 2 ? 160 : (v == VARIANT_WIDE ? 192 : 0)));
}
constexpr int MAX_CHUNKS = 24;

// LDS per wave for the staged bra primitives of the lane kernel, and the
// most the ket-outer kernel may stage (all primitives of the bra)
constexpr int STAGE_BYTES = 3072;
constexpr int KO_STAGE_MAX = 8192;
// the ket-outer kernel serves bra classes with small Hermite boxes (ss, ps,
// pp, ds: 1, 6, 33, 21 entries), whose per-quartet bra step is cheap
constexpr int KO_MAX_BRA_BOX = 33;

template <int LA, int LB, int LC, int LD, int BUDGET>
__host__ __device__ constexpr bool lane_fits() {
    return BUDGET > 0 &&
           lane_live(LA, LB, LC, LD, chunk_a(LA, LB, LC, LD, BUDGET),
                     chunk_cd(LA, LB, LC, LD, BUDGET)) <= BUDGET &&
           n_chunks(LA, LB, LC, LD, BUDGET) <= MAX_CHUNKS;
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE>
void launch_wave_kernel(int ntile, const EriArgs &a, hipStream_t s) {
    int blocks = ntile;
    if (blocks > 32768) blocks = 32768;
    hipLaunchKernelGGL((k_eri_wave<LA, LB, LC, LD, T, STORE>), dim3(blocks), dim3(64), 0, s, a);
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE>
void launch_mfma_kernel(int ntile, const EriArgs &a, hipStream_t s) {
    int blocks = ntile;
    if (blocks > 32768) blocks = 32768;
    hipLaunchKernelGGL((k_eri_mfma<LA, LB, LC, LD, T, STORE>), dim3(blocks), dim3(64), 0, s, a);
}

// LDS of one workgroup on gfx950.
constexpr size_t LDS_PER_CU = 160 * 1024;

// Segment mode of a lane-kernel launch (waves_per_block = 8 in a Fock build
// with a.kn > 0 and a segment list): W-wave blocks over segments, the
// dynamic LDS holding the W staging slices and the bra's K' rows.  False
// (the caller then launches the tile-mode kernel with kn = 0) when the rows
// do not fit next to the kernel's static LDS.
template <int LA, int LB>
bool segment_fit(const void *kernel, int W, EriArgs &b, int &blocks, size_t &dyn) {
    if (b.kn <= 0 || b.tl.nseg <= 0) return false;
    const size_t rows = (size_t)(ncart(LA) + ncart(LB)) * b.kn * sizeof(double);
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    dyn = (size_t)W * b.stage_bytes + rows;
    if (fa.sharedSizeBytes + dyn > LDS_PER_CU) return false;
    blocks = b.tl.nseg < 8192 ? b.tl.nseg : 8192;
    return true;
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE, int BUDGET>
void launch_budget(int ntile, int wpb, const EriArgs &a, hipStream_t s) {
    if constexpr (lane_fits<LA, LB, LC, LD, BUDGET>()) {
        constexpr int CA = chunk_a(LA, LB, LC, LD, BUDGET), CDC = chunk_cd(LA, LB, LC, LD, BUDGET);
        int blocks = (ntile + wpb - 1) / wpb;
        if (blocks > 8192) blocks = 8192;
        // LDS stage of the bra primitives: up to STAGE_BYTES per wave
        constexpr int per_prim = 4 * (int)sizeof(double) + n_entries(LA, LB) * (int)sizeof(T);
        EriArgs b = a;
        b.stage_prims = STAGE_BYTES / per_prim < 1 ? 1 : STAGE_BYTES / per_prim;
        if (b.stage_prims > a.bra.kmax) b.stage_prims = a.bra.kmax > 0 ? a.bra.kmax : 1;
        b.stage_bytes = LA == 2 ? (b.stage_prims * per_prim + 15) / 16 * 16 : 0;
        if constexpr (!STORE) {
            if (wpb == 8) {
                constexpr int W = seg_waves(LA, LB, LC, LD, CA, CDC);
                auto seg = k_eri_lane<LA, LB, LC, LD, T, false, CA, CDC, true>;
                int sblocks = 0;
                size_t dyn = 0;
                if (segment_fit<LA, LB>((const void *)seg, W, b, sblocks, dyn)) {
                    hipLaunchKernelGGL(seg, dim3(sblocks), dim3(64 * W), dyn, s, b);
                    return;
                }
            }
        }
        b.kn = 0;
        const int w = wpb > 4 ? 4 : wpb;
        blocks = (ntile + w - 1) / w;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL((k_eri_lane<LA, LB, LC, LD, T, STORE, CA, CDC, false>), dim3(blocks),
                           dim3(64 * w), (size_t)w * b.stage_bytes, s, b);
    } else {
        launch_wave_kernel<LA, LB, LC, LD, T, STORE>(ntile, a, s);
    }
}

template <int LA, int LB, int LC, int LD, typename T, bool STORE>
void launch_ko(int ntile, int wpb, const EriArgs &a, hipStream_t s) {
    constexpr int BUDGET = variant_budget(DEFAULT_VARIANT);
    if constexpr (n_entries(LA, LB) <= KO_MAX_BRA_BOX && lane_fits<LA, LB, LC, LD, BUDGET>()) {
        constexpr int CA = chunk_a(LA, LB, LC, LD, BUDGET), CDC = chunk_cd(LA, LB, LC, LD, BUDGET);
        constexpr int per_prim = 4 * (int)sizeof(double) + n_entries(LA, LB) * (int)sizeof(T);
        const int kmax = a.bra.kmax > 0 ? a.bra.kmax : 1;
        if (kmax * per_prim <= KO_STAGE_MAX) {
            EriArgs b = a;
            b.stage_prims = kmax;
            b.stage_bytes = (kmax * per_prim + 15) / 16 * 16;
            if constexpr (!STORE) {
                if (wpb == 8) {
                    auto seg = k_eri_lane_ko<LA, LB, LC, LD, T, false, CA, CDC, true>;
                    constexpr int W =
                        ko_seg_waves(LA, LB, LC, LD, !std::is_same<T, float>::value);
                    int sblocks = 0;
                    size_t dyn = 0;
                    if (segment_fit<LA, LB>((const void *)seg, W, b, sblocks, dyn)) {
                        hipLaunchKernelGGL(seg, dim3(sblocks), dim3(64 * W), dyn, s, b);
                        return;
                    }
                }
            }
            b.kn = 0;
            const int w = wpb > 4 ? 4 : wpb;
            int blocks = (ntile + w - 1) / w;
            if (blocks > 8192) blocks = 8192;
            hipLaunchKernelGGL((k_eri_lane_ko<LA, LB, LC, LD, T, STORE, CA, CDC, false>),
                               dim3(blocks), dim3(64 * w), (size_t)w * b.stage_bytes, s, b);
            return;
        }
    }
    launch_budget<LA, LB, LC, LD, T, STORE, BUDGET>(ntile, wpb, a, s);
}

// One variant in Fock mode (STORE = false) or store mode (the same kernel
// code writing the contracted blocks out instead of digesting them).
template <int LA, int LB, int LC, int LD, typename T, bool STORE>
void launch_variant(int ntile, int variant, int wpb, const EriArgs &a, hipStream_t s) {
    switch (variant) {
        case 0: launch_budget<LA, LB, LC, LD, T, STORE, variant_budget(0)>(ntile, wpb, a, s); break;
        case 1: launch_budget<LA, LB, LC, LD, T, STORE, variant_budget(1)>(ntile, wpb, a, s); break;
        case 2: launch_budget<LA, LB, LC, LD, T, STORE, variant_budget(2)>(ntile, wpb, a, s); break;
        case VARIANT_KO: launch_ko<LA, LB, LC, LD, T, STORE>(ntile, wpb, a, s); break;
        case VARIANT_WIDE:
            // a 192-value lane kernel for the classes whose smallest chunk
            // exceeds 160 live values, or that need fewer chunks at 192
            // ((ds|pp), (dp|pp), (dp|ds): each chunk re-evaluates Boys and
            // R, and these run at one wave per SIMD either way); every other
            // class runs variant 2
            if constexpr (!lane_fits<LA, LB, LC, LD, variant_budget(2)>() ||
                          (lane_fits<LA, LB, LC, LD, variant_budget(VARIANT_WIDE)>() &&
                           n_chunks(LA, LB, LC, LD, variant_budget(VARIANT_WIDE)) <
                               n_chunks(LA, LB, LC, LD, variant_budget(2))))
                launch_budget<LA, LB, LC, LD, T, STORE, variant_budget(VARIANT_WIDE)>(ntile, wpb, a, s);
            else
                launch_budget<LA, LB, LC, LD, T, STORE, variant_budget(2)>(ntile, wpb, a, s);
            break;
        case VARIANT_MFMA:
            // the matrix-core kernel serves classes with a d bra; the others
            // run the wave kernel
            if constexpr (LA == 2) launch_mfma_kernel<LA, LB, LC, LD, T, STORE>(ntile, a, s);
            else launch_wave_kernel<LA, LB, LC, LD, T, STORE>(ntile, a, s);
            break;
        default: launch_wave_kernel<LA, LB, LC, LD, T, STORE>(ntile, a, s); break;
    }
}

template <int LA, int LB, int LC, int LD, typename T>
hipError_t launch_class(bool store, int variant, int wpb, const EriArgs &a, hipStream_t s) {
    const int ntile = store ? a.st_ntile : a.tl.ntile;
    if (ntile <= 0) return hipSuccess;
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8) wpb = 4;
    if (store) launch_variant<LA, LB, LC, LD, T, true>(ntile, variant, wpb, a, s);
    else launch_variant<LA, LB, LC, LD, T, false>(ntile, variant, wpb, a, s);
    return hipGetLastError();
}

}  // namespace fsim
