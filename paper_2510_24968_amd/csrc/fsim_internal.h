// Internal declarations of libfsim: compile-time index algebra of Cartesian
// and Hermite components, device-side table layouts and kernel launch
// records.  Shared by the HIP sources of the library only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace fsim {

constexpr int LMAX = 2;                // s, p, Cartesian d
constexpr int LTOT_MAX = 4 * LMAX;     // highest L of a shell quartet
constexpr int MAXPRIM = 8;             // primitives per shell
constexpr int NPCLASS = 6;             // pair classes ss ps pp ds dp dd

// ---- Boys-function grid ------------------------------------------------
// F_n(T_k) is tabulated at T_k = k * BOYS_DT for k < BOYS_NT and
// n < BOYS_NORD; below BOYS_TMAX a class of total L evaluates F_L by an
// 8-term Taylor expansion about the nearest grid point (|dT| <= 0.05, so the
// truncation error is below dT^8 / 8! ~ 1e-15 relative) and the lower orders
// by the downward recursion; from BOYS_TMAX on, F_0 = sqrt(pi / T) / 2 and
// the upward recursion (exact up to erfc(6) ~ 2e-17).
constexpr double BOYS_DT = 0.1;
constexpr double BOYS_INV_DT = 10.0;
constexpr double BOYS_TMAX = 36.0;
constexpr int BOYS_NT = 361;
constexpr int BOYS_NTAYLOR = 8;
constexpr int BOYS_NORD = LTOT_MAX + BOYS_NTAYLOR;   // orders 0..15

// ---- component algebra -------------------------------------------------
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int nherm(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

// Cartesian exponent of component c of a shell with angular momentum l in
// direction dir (0 = x, 1 = y, 2 = z); components run lx descending, then ly
// descending.
__host__ __device__ constexpr int cart_exp(int l, int c, int dir) {
    int k = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == c) return dir == 0 ? x : (dir == 1 ? y : l - x - y);
            ++k;
        }
    return 0;
}

// Linear index of the Hermite triple (t, u, v): graded by s = t + u + v, so
// the first nherm(L) slots hold every triple of total <= L for any L.
__host__ __device__ constexpr int hidx(int t, int u, int v) {
    int s = t + u + v, a = u + v;
    return s * (s + 1) * (s + 2) / 6 + a * (a + 1) / 2 + v;
}
__host__ __device__ constexpr int hidx_t(int i) {
    int s = 0;
    while (nherm(s) <= i) ++s;
    int r = i - (s == 0 ? 0 : nherm(s - 1));
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= r) ++a;
    return s - a;
}
__host__ __device__ constexpr int hidx_v(int i) {
    int s = 0;
    while (nherm(s) <= i) ++s;
    int r = i - (s == 0 ? 0 : nherm(s - 1));
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= r) ++a;
    return r - a * (a + 1) / 2;
}
__host__ __device__ constexpr int hidx_u(int i) {
    int s = 0;
    while (nherm(s) <= i) ++s;
    return s - hidx_t(i) - hidx_v(i);
}

// Hermite box of the component pair cp = c1 * ncart(l2) + c2 of a shell pair
// (l1, l2): E^{c1 c2}_{tuv} is non-zero only for t <= bx, u <= by, v <= bz.
__host__ __device__ constexpr int box_dim(int l1, int l2, int cp, int dir) {
    return cart_exp(l1, cp / ncart(l2), dir) + cart_exp(l2, cp % ncart(l2), dir);
}
__host__ __device__ constexpr int box_size(int l1, int l2, int cp) {
    return (box_dim(l1, l2, cp, 0) + 1) * (box_dim(l1, l2, cp, 1) + 1) *
           (box_dim(l1, l2, cp, 2) + 1);
}
// Offset of component pair cp's box in the per-primitive-pair entry list.
__host__ __device__ constexpr int box_off(int l1, int l2, int cp) {
    int o = 0;
    for (int k = 0; k < cp; ++k) o += box_size(l1, l2, k);
    return o;
}
// Entries per primitive pair of class (l1, l2).
__host__ __device__ constexpr int n_entries(int l1, int l2) {
    return box_off(l1, l2, ncart(l1) * ncart(l2));
}

__host__ __device__ constexpr int pclass(int l1, int l2) {   // l1 >= l2
    return l1 * (l1 + 1) / 2 + l2;
}
__host__ __device__ constexpr int pc_l1(int pc) { return pc < 1 ? 0 : (pc < 3 ? 1 : 2); }
__host__ __device__ constexpr int pc_l2(int pc) { return pc - pclass(pc_l1(pc), 0); }
inline int pclass_l1(int pc) { return pc_l1(pc); }
inline int pclass_l2(int pc) { return pc_l2(pc); }

// ---- device tables -------------------------------------------------------
// One shell-pair class (l1 >= l2).  Pairs are stored column-wise (pair index
// fastest) so that lanes handling consecutive pairs read consecutive words.
// Each primitive pair slot k < kmax holds the product exponent p, the centre
// P and the Hermite box entries
//   E[k][e][pair] = c1 c2 n1 n2 sqrt(2) pi^(5/4) / p * E^{i1 j1}_t E^{i2 j2}_u E^{i3 j3}_v
// (contraction coefficients, component normalisation and the pair's share of
// the ERI prefactor 2 pi^(5/2) / (p q sqrt(p + q)) folded in).
struct PairTable {
    int n = 0;        // pairs
    int kmax = 0;     // primitive-pair slots
    int ne = 0;       // box entries per primitive pair
    int l1 = 0, l2 = 0;
    int *sh1 = nullptr, *sh2 = nullptr;   // shell indices (l(sh1) >= l(sh2))
    int *bf1 = nullptr, *bf2 = nullptr;   // first basis function of each shell (in its molecule)
    int *mol = nullptr;                   // molecule of the pair (batched contexts)
    int *nprim = nullptr;                 // primitive pairs in use
    double *Q = nullptr;                  // Schwarz factor
    double *p = nullptr;                  // [kmax][n]
    double *P = nullptr;                  // [kmax][3][n]
    double *E = nullptr;                  // [kmax][ne][n]
    float *Ef = nullptr;                  // FP32 copy of E
};

// Tile lists of one quartet class and precision: bra pair b owns the ket
// range [ket_lo[b], ket_hi[b]) cut into tiles of TILE kets.
struct TileList {
    int nbra = 0;
    int ntile = 0;
    int64_t nquartet = 0;
    int *tile_start = nullptr;   // [nbra + 1]
    int *bra = nullptr;          // [nbra]
    int *ket_lo = nullptr;       // [nbra]
    int *ket_hi = nullptr;       // [nbra]
    // segments (Fock builds with K' rows in LDS): segment s is the tiles
    // [seg_t0[s], seg_t0[s] + seg_nt[s]) of bra record seg_rec[s], at most
    // the class's segment length of them; nseg = 0: no segments
    int nseg = 0;
    int *seg_rec = nullptr, *seg_t0 = nullptr, *seg_nt = nullptr;
};

constexpr int TILE = 64;        // kets per wave tile (one per lane)
constexpr int SEG_TILES = 64;   // default tiles per segment (tuned per class)

struct EriArgs {
    PairTable bra, ket;
    int same_class;
    // Fock mode
    TileList tl;
    const double *D;        // packed per-molecule blocks (one block for a single molecule)
    double *Jh;
    double *Kh;
    // > 0: Jh and Kh each hold one copy per XCD, xcd_stride elements apart,
    // and a wave adds into the copy of the XCD it runs on (0: one copy)
    long long xcd_stride;
    // lane kernels: each wave stages up to stage_prims primitive pairs of its
    // bra (p, P, Hermite boxes) in stage_bytes of dynamic LDS
    int stage_prims, stage_bytes;
    int nbf;
    const long long *mol_off;   // [nmol] offset of each molecule's N_m x N_m block
    const int *mol_n;           // [nmol] N_m
    // store mode: tile t has bra st_bra[t]; lane l evaluates ket st_ket[t*64+l]
    // (-1 = idle) and writes component (i,j,k,l) to
    // out[st_off + i*s0 + j*s1 + k*s2 + l*s3]
    int st_ntile;
    const int *st_bra;
    const int *st_ket;
    const long long *st_off;
    const int *st_stride;   // [4 per task]
    double *out;
    const double *boys;     // [BOYS_NT][BOYS_NORD]
    // > 0: segment mode of the lane kernels, the K' rows of each segment's
    // bra accumulate in LDS, kn doubles per row (the largest N_m); the
    // dynamic LDS holds (ncart(la) + ncart(lb)) * kn doubles after the
    // waves' staging slices.  0: every K' term is a global atomic.
    int kn;
};


// setup kernels (setup.hip)
hipError_t launch_boys_table(double *tab, hipStream_t s);
struct ShellsDev {
    int nshell = 0, natom = 0, nmol = 1;
    double *xyz = nullptr;     // [nshell][3] centre of each shell
    int *l = nullptr, *nprim = nullptr, *prim0 = nullptr;
    int *bf0 = nullptr;        // first basis function of the shell within its molecule
    int *mol = nullptr;        // molecule of the shell
    int *mol_atom0 = nullptr, *mol_natom = nullptr;   // [nmol] atom range
    int *mol_bf0 = nullptr;    // [nmol] first global basis function
    int *mol_n = nullptr;      // [nmol] N_m
    long long *mol_off = nullptr;   // [nmol] packed block offset
    double *exps = nullptr;
    double *coef = nullptr;    // normalised (radial norm x contraction renorm)
    double *atom_xyz = nullptr;
    double *atom_Z = nullptr;
};
hipError_t launch_shell_norm(const ShellsDev &sh, hipStream_t s);
hipError_t launch_build_pairs(const ShellsDev &sh, PairTable &t, const int *pair_sh1,
                              const int *pair_sh2, hipStream_t s);
// Drop the primitive pairs of every pair whose Schwarz bound times
// qmax_mol[mol] is below tau_prim, compacting the slots in place (setup.hip).
hipError_t launch_prim_screen(PairTable &t, const double *qmax_mol, double tau_prim,
                              hipStream_t s);
hipError_t launch_one_electron_impl(const ShellsDev &sh, const double *boys, int nmax,
                                    const int *bf_shell, const int *bf_comp, double *S,
                                    double *T, double *V, hipStream_t s);
// one quartet class and precision (eri_class.hip, compiled per class)
template <int X, int Y, bool F32>
hipError_t launch_eri_unit(bool store, int variant, int wpb, const EriArgs &a, hipStream_t s);
// Persistent launch over the s/p quartet classes (persistent.hip): queue
// slot k holds the tiles (or segments) of class (persist_bra(k) | persist_ket(k)), slots
// 0..5 = (pp|pp) (pp|ps) (ps|ps) (pp|ss) (ps|ss) (ss|ss); start[k] is the
// first queue position of slot k, start[6] the total.  *counter must be 0
// at launch.  Every slot's stage_prims x (4 + n_entries) FP64/T values must
// fit stage_bytes, the per-wave LDS slice.
constexpr int PERSIST_SLOTS = 6;
constexpr int PERSIST_BUDGET = 128;   // lane-kernel live-value budget of the tile bodies
struct PersistArgs {
    EriArgs cls[PERSIST_SLOTS];
    int start[PERSIST_SLOTS + 1];
    int *counter;
    int stage_bytes;
    const double *boys;
    // > 0: queue items are segments (start[] counts segments), each taken
    // by a whole block that keeps its bra's K' rows in LDS (kn doubles per
    // row, as EriArgs::kn, which every slot's record carries too); 0: items
    // are tiles taken by single waves, K' terms added globally
    int kn;
};
hipError_t launch_persistent(bool fp32, const PersistArgs &p, hipStream_t s);
// digest of stored blocks (stored.hip): a.out = the class's store, a.tl its
// FP64 tile list
hipError_t launch_digest_stored(int bra_pc, int ket_pc, int wpb, const EriArgs &a,
                                hipStream_t s);
// quartet-class dispatch (eri_dispatch.hip); bra_pc >= ket_pc
hipError_t launch_eri(int bra_pc, int ket_pc, bool fp32, bool store, int variant, int wpb,
                      const EriArgs &a, hipStream_t s);
constexpr int ERI_NVARIANT = 7;   // kernel-A budgets 96/128/160, kernel B, kernel A ket-outer,
                                  // kernel A at 192 (classes that do not fit 160),
                                  // kernel C on the matrix cores (d bras)
constexpr int ERI_VARIANT_WAVE = 3;
constexpr int ERI_VARIANT_KO = 4;
constexpr int ERI_VARIANT_WIDE = 5;
constexpr int ERI_VARIANT_MFMA = 6;
constexpr int ERI_DEFAULT_VARIANT = 1;

}  // namespace fsim
