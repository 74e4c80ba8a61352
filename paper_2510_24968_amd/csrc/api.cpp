// Host side of libfsim: the C ABI of include/fsim.h, input validation, the
// context (device tables and buffers), Schwarz screening and quartet work
// lists, the Fock-build launch sequence and the SCF step.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fsim.h"
#include "fsim_internal.h"
#include "linalg.h"
#include "noalloc.h"

using namespace fsim;

static thread_local std::string g_err;

static fsim_status fail(fsim_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FSIM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)
#define BLASCHK(expr)                                                                      \
    do {                                                                                   \
        rocblas_status e_ = (expr);                                                        \
        if (e_ != rocblas_status_success)                                                  \
            return fail(FSIM_EHIP, std::string(#expr) + ": rocblas status " +             \
                                       std::to_string((int)e_));                           \
    } while (0)
#define STCHK(expr)                                                                        \
    do {                                                                                   \
        fsim_status s_ = (expr);                                                           \
        if (s_ != FSIM_OK) return s_;                                                      \
    } while (0)

namespace {

// Quartet work lists of one class pair: FP64-mode list, and the two parts
// of the mixed-mode split.
struct ListStats {
    int64_t nq = 0, npq = 0;
    double flops = 0.0, flops_exec = 0.0;
};
// Host copy of a tile list's bra records and ket ranges.
struct HostList {
    std::vector<int> bra, lo, hi;
};
struct ClassLists {
    TileList all64, mix64, mix32;
    ListStats s64, sm64, sm32;
    // incremental builds: host copies of the three lists (all64, mix64,
    // mix32) and lists of the same bra records with density-screened ket
    // ends (own tile_start / ket_hi; bra and ket_lo shared)
    HostList host[3];
    TileList delta[3];
    std::vector<int> dstart[3], dhi[3];
    std::vector<int> dseg[3];   // segments of the delta lists: rec, t0, nt (3 arrays)
    int64_t dnq[3] = {0, 0, 0};
    // device capacity of each list's segment arrays (segments of the
    // smallest segment size, SEG_MIN tiles)
    int segcap[3] = {0, 0, 0};
};

// Segment sizes the tuning may choose (tiles per segment).
constexpr int SEG_MIN = 16, SEG_MAX = 512;
static bool valid_seg(int n) { return n >= SEG_MIN && n <= SEG_MAX && (n & (n - 1)) == 0; }

// Segments of at most seg tiles over the tile ranges of a list's bra records
// (tile starts st[0..nbra]) into host arrays rec/t0/nt; returns the count.
static size_t cut_segments(const std::vector<int> &st, int seg, int *rec, int *t0, int *nt) {
    size_t ns = 0;
    for (size_t r = 0; r + 1 < st.size(); ++r)
        for (int t = st[r]; t < st[r + 1]; t += seg) {
            rec[ns] = (int)r;
            t0[ns] = t;
            nt[ns] = std::min(seg, st[r + 1] - t);
            ++ns;
        }
    return ns;
}

struct DevPool {
    std::vector<void *> ptrs;
    template <typename T>
    hipError_t alloc(T **p, size_t n) {
        *p = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc((void **)p, n * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release(void *p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            hipFree(p);
            ptrs.erase(it);
        }
    }
    void clear() {
        for (void *p : ptrs) hipFree(p);
        ptrs.clear();
    }
};

}  // namespace

struct fsim_ctx {
    int device = 0;
    fsim_options opt{};
    int natom = 0, nshell = 0, nbf = 0, nelec = 0, nocc = 0;
    std::vector<double> xyz, Z, exps, coefs;
    std::vector<int> sh_atom, sh_l, sh_nprim, sh_prim0, sh_bf0, sh_mol;
    double enuc = 0.0;

    // molecules (one for fsim_ctx_create, many for fsim_batch_create): each
    // keeps its N_m x N_m matrices at a packed offset
    int nmol = 1, nmax = 0;
    long long packed = 0;
    std::vector<int> mol_n, mol_nocc, mol_bf0, mol_atom0, mol_natom, mol_shell0, mol_nshell;
    std::vector<long long> mol_off;
    std::vector<double> mol_enuc;
    int *d_mol_n = nullptr, *d_nocc = nullptr;
    long long *d_mol_off = nullptr;
    double *Emol = nullptr;           // [nmol] electronic energies of the last build
    std::vector<double> Emol_host;
    // batched SCF (nmol > 1): zero-padded N_max x N_max blocks
    double *pS = nullptr, *pX = nullptr, *pH = nullptr, *pF = nullptr, *pD = nullptr,
           *pT1 = nullptr, *pT2 = nullptr, *pEig = nullptr, *pErr = nullptr, *pRed = nullptr;
    std::vector<double *> pdF, pdE;
    std::vector<double> Bb;            // [nmol][m][m]
    std::vector<double> Eprev_mol;
    std::vector<fsim_scf_info> mol_info;
    // s/p quartet classes in one persistent launch per precision part (tile
    // counters: one per part)
    bool persistent = false;
    int *pcounter = nullptr;
    // lane-kernel launches accumulate each bra's K' rows in LDS over
    // segments of its tiles (default), or add every K' term globally
    bool krow_lds = true;
    // tiles per segment, per class and precision (tuning)
    int segt[NPCLASS][NPCLASS][2];
    // captured Fock build (hipGraph), one per precision
    bool graph_enabled = false;
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipEvent_t gev[2] = {nullptr, nullptr};
    double *gD = nullptr, *gF = nullptr;

    DevPool pool;        // lives as long as the context
    DevPool screen_pool; // replaced by every screen
    ShellsDev sh;
    double *boys = nullptr;
    double *S = nullptr, *H = nullptr, *X = nullptr;

    // all pairs (canonical order) and the screened, Q-sorted pairs
    PairTable all[NPCLASS];
    std::vector<int> all_s1[NPCLASS], all_s2[NPCLASS];
    std::map<long long, std::pair<int, int>> pair_lookup;   // (s1*nshell+s2) -> (pc, index)
    PairTable kept[NPCLASS];
    std::vector<double> Qkept[NPCLASS];
    bool screened = false;
    double tau = 0.0, tau32 = 0.0;
    // primitive-pair screening threshold applied by the next screen (0: off)
    // and each kept pair's primitive pairs in use after it
    double tau_prim = 0.0;
    std::vector<int> kept_np[NPCLASS];
    ClassLists lists[NPCLASS][NPCLASS];
    fsim_screen_stats stats{};
    std::vector<double> Qmat;

    // work buffers
    double *Jh = nullptr, *Kh = nullptr, *F = nullptr, *Dn = nullptr, *T1 = nullptr, *T2 = nullptr;
    // per-XCD private J'/K' accumulators (NXCD copies of each), summed after the build
    bool xcd_private = true;
    double *priv = nullptr;
    // accumulators of fsim_fock_build_noalloc: this device's copy of the
    // library's static array (2 x NOALLOC_MAX_PACKED), resolved at create
    double *noalloc = nullptr;
    // incremental builds (one molecule): shell of each basis function,
    // D - Dref, per-shell-pair max |D - Dref| (device and host), the kept
    // pairs' shells per class
    int *d_bf_shell = nullptr;
    double *dD = nullptr, *Mblk = nullptr;
    std::vector<double> Mhost;
    std::vector<int> kept_s1[NPCLASS], kept_s2[NPCLASS];
    // spherical basis (one molecule): the caller's matrices are nscf x nscf
    // over real solid harmonic d functions; the kernels work on the nbf
    // Cartesian functions, with T (nbf x nscf, row-major) between the two
    bool sph = false;
    int nscf = 0;
    double *Tsph = nullptr, *Dc = nullptr, *Jc = nullptr, *Kc = nullptr, *Wsph = nullptr;
    // conventional mode: every kept quartet's block stored once (FP64, tile
    // order) and digested by later builds instead of being recomputed
    DevPool store_pool;
    bool stored = false;
    double *store = nullptr;
    long long store_off[NPCLASS][NPCLASS] = {};
    int64_t store_bytes = 0;
    // SCF with incremental builds: full build every inc_every steps, the
    // reference density and its J, K
    int inc_every = 0, inc_count = 0;
    bool inc_have = false;
    double inc_tau = 0.0;   // density-weighted threshold (<= 0: the screen's tau)
    double *Dref = nullptr, *Jref = nullptr, *Kref = nullptr;
    double *eig = nullptr, *ework = nullptr, *scal = nullptr;
    int *dinfo = nullptr;
    rocblas_handle blas = nullptr;

    // launch settings per (bra class, ket class, fp32)
    int variant[NPCLASS][NPCLASS][2];
    int wpb[NPCLASS][NPCLASS][2];
    double tuned_ms[NPCLASS][NPCLASS][2];

    // per-launch profiling
    bool profiling = false;
    std::vector<hipEvent_t> ev;
    std::vector<fsim_class_profile> prof;

    // DIIS and step state
    std::vector<double *> dF, dE;
    int diis_count = 0, diis_next = 0;
    std::vector<double> Bm;   // [m*m]
    int iter = 0;
    bool have_prev = false;
    double E_prev = 0.0;
};

static void drop_graphs(fsim_ctx *c);

static int ncart_h(int l) { return (l + 1) * (l + 2) / 2; }

static MolLayout layout_of(const fsim_ctx *c) {
    MolLayout L;
    L.nmol = c->nmol;
    L.nmax = c->nmax;
    L.off = c->d_mol_off;
    L.n = c->d_mol_n;
    return L;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static fsim_status alloc_table(DevPool &pool, PairTable &t, int l1, int l2, int n, int kmax) {
    t = PairTable{};
    t.l1 = l1;
    t.l2 = l2;
    t.n = n;
    t.kmax = kmax;
    t.ne = n_entries(l1, l2);
    if (n == 0) return FSIM_OK;
    HIPCHK(pool.alloc(&t.sh1, n));
    HIPCHK(pool.alloc(&t.sh2, n));
    HIPCHK(pool.alloc(&t.bf1, n));
    HIPCHK(pool.alloc(&t.bf2, n));
    HIPCHK(pool.alloc(&t.nprim, n));
    HIPCHK(pool.alloc(&t.mol, n));
    HIPCHK(pool.alloc(&t.Q, n));
    HIPCHK(pool.alloc(&t.p, (size_t)kmax * n));
    HIPCHK(pool.alloc(&t.P, (size_t)kmax * 3 * n));
    HIPCHK(pool.alloc(&t.E, (size_t)kmax * t.ne * n));
    HIPCHK(pool.alloc(&t.Ef, (size_t)kmax * t.ne * n));
    return FSIM_OK;
}

static fsim_status build_table(fsim_ctx *c, DevPool &pool, PairTable &t, int pc,
                               const std::vector<int> &s1, const std::vector<int> &s2) {
    const int l1 = pclass_l1(pc), l2 = pclass_l2(pc);
    int kmax = 1;
    for (size_t i = 0; i < s1.size(); ++i)
        kmax = std::max(kmax, c->sh_nprim[s1[i]] * c->sh_nprim[s2[i]]);
    STCHK(alloc_table(pool, t, l1, l2, (int)s1.size(), kmax));
    if (t.n == 0) return FSIM_OK;
    int *d1 = nullptr, *d2 = nullptr;
    HIPCHK(hipMalloc(&d1, sizeof(int) * t.n));
    HIPCHK(hipMalloc(&d2, sizeof(int) * t.n));
    HIPCHK(hipMemcpy(d1, s1.data(), sizeof(int) * t.n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d2, s2.data(), sizeof(int) * t.n, hipMemcpyHostToDevice));
    HIPCHK(launch_build_pairs(c->sh, t, d1, d2, nullptr));
    HIPCHK(hipDeviceSynchronize());
    hipFree(d1);
    hipFree(d2);
    return FSIM_OK;
}

// Column-major GEMM C = op(A) op(B) (all N x N here except the density step).
static fsim_status gemm(rocblas_handle h, bool ta, bool tb, int m, int n, int k, double alpha,
                        const double *A, int lda, const double *B, int ldb, double beta,
                        double *C, int ldc) {
    BLASCHK(rocblas_dgemm(h, ta ? rocblas_operation_transpose : rocblas_operation_none,
                          tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k,
                          &alpha, A, lda, B, ldb, &beta, C, ldc));
    return FSIM_OK;
}

// Symmetric eigen-decomposition in place (column-major, ascending).
static fsim_status syevd(fsim_ctx *c, double *A, double *w, hipStream_t s) {
    BLASCHK(rocblas_set_stream(c->blas, s));
    BLASCHK(rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_upper, c->nscf, A,
                             c->nscf, w, c->ework, c->dinfo));
    return FSIM_OK;
}

// D = 2 C_occ C_occ^T with C = X V, V the eigenvectors of X^T F X.
static fsim_status density_from_fock(fsim_ctx *c, const double *Fm, double *Dout, hipStream_t s) {
    const int N = c->nscf;
    BLASCHK(rocblas_set_stream(c->blas, s));
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, Fm, N, c->X, N, 0.0, c->T1, N));   // F X
    STCHK(gemm(c->blas, true, false, N, N, N, 1.0, c->X, N, c->T1, N, 0.0, c->T2, N));  // X^T F X
    STCHK(syevd(c, c->T2, c->eig, s));
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->X, N, c->T2, N, 0.0, c->T1, N));  // C
    STCHK(gemm(c->blas, false, true, N, N, c->nocc, 2.0, c->T1, N, c->T1, N, 0.0, Dout, N));
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Spherical basis (Sec. 2.1.1: each real solid harmonic Gaussian is a fixed
// combination of Cartesian Gaussians of degree l, with coefficients S^{lm}).
// Integrals over spherical functions are the Cartesian ones contracted with
// those coefficients on every index, so with T (Cartesian x spherical):
//   S' = T^T S T,  H' = T^T H T,  J'(D') = T^T J(T D' T^T) T  (and K').
// rocBLAS is column-major: the row-major T (nbf x nscf) is the column-major
// Tcm = T^T (nscf x nbf, ld nscf); the symmetric matrices read the same in
// either order.
// ---------------------------------------------------------------------------

// Racah-normalised real solid harmonics of a d shell on its Cartesian
// components (xx, xy, xz, yy, yz, zz), m = -2..2:
//   sqrt3 xy, sqrt3 yz, zz - (xx + yy)/2, sqrt3 xz, sqrt3/2 (xx - yy)
static void d_solid_harmonics(double (&t)[6][5]) {
    const double r3 = std::sqrt(3.0);
    const double c[5][6] = {{0, r3, 0, 0, 0, 0},
                            {0, 0, 0, 0, r3, 0},
                            {-0.5, 0, 0, -0.5, 0, 1.0},
                            {0, 0, r3, 0, 0, 0},
                            {r3 / 2, 0, 0, -r3 / 2, 0, 0}};
    // the Cartesian functions are of unit norm: x^a y^b z^c e^{-ar^2} is
    // sqrt((2a-1)!! (2b-1)!! (2c-1)!!) times the unit function (up to a
    // factor common to the shell): sqrt3 for xx, yy, zz, 1 for the others
    const double w[6] = {r3, 1.0, 1.0, r3, 1.0, r3};
    for (int q = 0; q < 6; ++q)
        for (int m = 0; m < 5; ++m) t[q][m] = c[m][q] * w[q];
}

// Ms = T^T Mc T (nscf x nscf, not symmetrised) through Wsph
static fsim_status sph_from_cart(fsim_ctx *c, const double *Mc, double *Ms) {
    const int Nc = c->nbf, Ns = c->nscf;
    STCHK(gemm(c->blas, false, true, Nc, Ns, Nc, 1.0, Mc, Nc, c->Tsph, Ns, 0.0, c->Wsph, Nc));
    STCHK(gemm(c->blas, false, false, Ns, Ns, Nc, 1.0, c->Tsph, Ns, c->Wsph, Nc, 0.0, Ms, Ns));
    return FSIM_OK;
}

// Mc = T Ms T^T (nbf x nbf, not symmetrised) through Wsph
static fsim_status cart_from_sph(fsim_ctx *c, const double *Ms, double *Mc) {
    const int Nc = c->nbf, Ns = c->nscf;
    STCHK(gemm(c->blas, false, false, Ns, Nc, Ns, 1.0, Ms, Ns, c->Tsph, Ns, 0.0, c->Wsph, Ns));
    STCHK(gemm(c->blas, true, false, Nc, Nc, Ns, 1.0, c->Tsph, Ns, c->Wsph, Ns, 0.0, Mc, Nc));
    return FSIM_OK;
}

// Build T from the Cartesian overlap in c->S (each spherical d function
// rescaled to unit self-overlap), then S, H <- T^T S T, T^T H T.
static fsim_status spherical_setup(fsim_ctx *c, DevPool &pool) {
    const int Nc = c->nbf;
    int Ns = 0;
    for (int l : c->sh_l) Ns += l == 2 ? 5 : ncart_h(l);
    c->nscf = Ns;
    c->sph = true;
    std::vector<double> S((size_t)Nc * Nc);
    HIPCHK(hipMemcpy(S.data(), c->S, sizeof(double) * S.size(), hipMemcpyDeviceToHost));
    std::vector<double> T((size_t)Nc * Ns, 0.0);
    double td[6][5];
    d_solid_harmonics(td);
    int c0 = 0, s0 = 0;
    for (int l : c->sh_l) {
        const int nc = ncart_h(l);
        if (l < 2) {
            for (int q = 0; q < nc; ++q) T[(size_t)(c0 + q) * Ns + s0 + q] = 1.0;
            s0 += nc;
        } else {
            for (int m = 0; m < 5; ++m) {
                double nrm = 0.0;
                for (int p = 0; p < 6; ++p)
                    for (int q = 0; q < 6; ++q)
                        nrm += td[p][m] * S[(size_t)(c0 + p) * Nc + c0 + q] * td[q][m];
                for (int q = 0; q < 6; ++q)
                    T[(size_t)(c0 + q) * Ns + s0 + m] = td[q][m] / std::sqrt(nrm);
            }
            s0 += 5;
        }
        c0 += nc;
    }
    HIPCHK(pool.alloc(&c->Tsph, T.size()));
    HIPCHK(pool.alloc(&c->Dc, (size_t)Nc * Nc));
    HIPCHK(pool.alloc(&c->Jc, (size_t)Nc * Nc));
    HIPCHK(pool.alloc(&c->Kc, (size_t)Nc * Nc));
    HIPCHK(pool.alloc(&c->Wsph, (size_t)Nc * Ns));
    HIPCHK(hipMemcpy(c->Tsph, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice));
    BLASCHK(rocblas_set_stream(c->blas, nullptr));
    STCHK(sph_from_cart(c, c->S, c->T1));
    HIPCHK(symmetrize(Ns, c->T1, c->S, nullptr));
    STCHK(sph_from_cart(c, c->H, c->T1));
    HIPCHK(symmetrize(Ns, c->T1, c->H, nullptr));
    HIPCHK(hipDeviceSynchronize());
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" const char *fsim_last_error(void) { return g_err.c_str(); }
extern "C" const char *fsim_version(void) { return "fsim-mi355x 0.1 (gfx950)"; }

static fsim_status validate(const fsim_basis *b, const fsim_options *o) {
    if (!b || !o) return fail(FSIM_EINVAL, "basis and options must not be NULL");
    if (b->natom <= 0 || b->nshell <= 0) return fail(FSIM_EINVAL, "natom and nshell must be > 0");
    if (!b->xyz || !b->Z || !b->shell_atom || !b->shell_l || !b->shell_nprim ||
        !b->shell_prim0 || !b->exps || !b->coefs)
        return fail(FSIM_EINVAL, "a basis array pointer is NULL");
    for (int i = 0; i < 3 * b->natom; ++i)
        if (!std::isfinite(b->xyz[i])) return fail(FSIM_EINVAL, "non-finite coordinate");
    for (int a = 0; a < b->natom; ++a)
        if (!std::isfinite(b->Z[a]) || b->Z[a] < 0) return fail(FSIM_EINVAL, "bad nuclear charge");
    int nbf = 0;
    for (int s = 0; s < b->nshell; ++s) {
        if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->natom)
            return fail(FSIM_EINVAL, "shell_atom out of range at shell " + std::to_string(s));
        if (b->shell_l[s] < 0 || b->shell_l[s] > LMAX)
            return fail(FSIM_EINVAL, "shell_l must be 0..2 (shell " + std::to_string(s) + ")");
        if (b->shell_nprim[s] < 1 || b->shell_nprim[s] > MAXPRIM)
            return fail(FSIM_EINVAL, "shell_nprim must be 1..8 (shell " + std::to_string(s) + ")");
        if (b->shell_prim0[s] < 0) return fail(FSIM_EINVAL, "negative shell_prim0");
        for (int k = 0; k < b->shell_nprim[s]; ++k) {
            const double e = b->exps[b->shell_prim0[s] + k], d = b->coefs[b->shell_prim0[s] + k];
            if (!(e > 0) || !std::isfinite(e)) return fail(FSIM_EINVAL, "exponent must be > 0");
            if (!std::isfinite(d)) return fail(FSIM_EINVAL, "non-finite contraction coefficient");
        }
        nbf += ncart_h(b->shell_l[s]);
    }
    if (b->nelec <= 0 || (b->nelec & 1) || b->nelec > 2 * nbf)
        return fail(FSIM_EINVAL, "nelec must be even and in 2..2N");
    if (o->tau_screen < 0 || o->tau_fp32 < 0 || !std::isfinite(o->tau_screen) ||
        !std::isfinite(o->tau_fp32))
        return fail(FSIM_EINVAL, "thresholds must be finite and >= 0");
    if (o->diis_m < 0 || o->diis_m > DIIS_MAX) return fail(FSIM_EINVAL, "diis_m must be 0..16");
    if (o->spherical != 0 && o->spherical != 1) return fail(FSIM_EINVAL, "spherical must be 0 or 1");
    return FSIM_OK;
}

static fsim_status batched_orthogonaliser(fsim_ctx *c, hipStream_t s);

// Context over nmol molecules.  Shells, pairs and quartets never mix
// molecules; every matrix is kept per molecule at a packed offset.
static fsim_status create_impl(const fsim_basis *mols, int nmol, const fsim_options *o,
                               fsim_ctx **out) {
    if (!out) return fail(FSIM_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!mols || nmol < 1) return fail(FSIM_EINVAL, "need at least one molecule");
    for (int m = 0; m < nmol; ++m) {
        fsim_status v = validate(&mols[m], o);
        if (v != FSIM_OK) {
            if (nmol > 1) g_err = "molecule " + std::to_string(m) + ": " + g_err;
            return v;
        }
    }
    fsim_ctx *c = new fsim_ctx();
    auto cleanup = [&](fsim_status st) {
        fsim_ctx_destroy(c);
        return st;
    };
#define PCHK(expr)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return cleanup(fail(FSIM_ENOMEM, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)
#define HCHK(expr)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return cleanup(fail(FSIM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)
#define SCHK(expr)                                                                         \
    do {                                                                                   \
        fsim_status s_ = (expr);                                                           \
        if (s_ != FSIM_OK) return cleanup(s_);                                             \
    } while (0)
    HCHK(hipGetDevice(&c->device));
    HCHK(noalloc_scratch_resolve(&c->noalloc));
    c->opt = *o;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y < NPCLASS; ++Y)
            for (int f = 0; f < 2; ++f) {
                c->variant[X][Y][f] = ERI_DEFAULT_VARIANT;
                c->wpb[X][Y][f] = 8;
                c->segt[X][Y][f] = SEG_TILES;
                c->tuned_ms[X][Y][f] = 0.0;
            }
    c->nmol = nmol;
    // concatenate the molecules
    std::vector<int> bf_shell, bf_comp;
    int gbf = 0;
    for (int m = 0; m < nmol; ++m) {
        const fsim_basis *b = &mols[m];
        const int a0 = c->natom, s0 = c->nshell, p0 = (int)c->exps.size();
        c->mol_atom0.push_back(a0);
        c->mol_natom.push_back(b->natom);
        c->mol_shell0.push_back(s0);
        c->mol_nshell.push_back(b->nshell);
        c->mol_bf0.push_back(gbf);
        c->xyz.insert(c->xyz.end(), b->xyz, b->xyz + 3 * b->natom);
        c->Z.insert(c->Z.end(), b->Z, b->Z + b->natom);
        int np = 0;
        for (int k = 0; k < b->nshell; ++k) np = std::max(np, b->shell_prim0[k] + b->shell_nprim[k]);
        c->exps.insert(c->exps.end(), b->exps, b->exps + np);
        c->coefs.insert(c->coefs.end(), b->coefs, b->coefs + np);
        int nb = 0;
        for (int k = 0; k < b->nshell; ++k) {
            c->sh_atom.push_back(a0 + b->shell_atom[k]);
            c->sh_l.push_back(b->shell_l[k]);
            c->sh_nprim.push_back(b->shell_nprim[k]);
            c->sh_prim0.push_back(p0 + b->shell_prim0[k]);
            c->sh_bf0.push_back(nb);
            c->sh_mol.push_back(m);
            for (int q = 0; q < ncart_h(b->shell_l[k]); ++q) {
                bf_shell.push_back(s0 + k);
                bf_comp.push_back(q);
            }
            nb += ncart_h(b->shell_l[k]);
        }
        c->mol_n.push_back(nb);
        c->mol_nocc.push_back(b->nelec / 2);
        c->mol_off.push_back(c->packed);
        c->packed += (long long)nb * nb;
        c->nmax = std::max(c->nmax, nb);
        double en = 0.0;
        for (int A = 0; A < b->natom; ++A)
            for (int B = 0; B < A; ++B) {
                const double dx = b->xyz[3 * A] - b->xyz[3 * B], dy = b->xyz[3 * A + 1] - b->xyz[3 * B + 1],
                             dz = b->xyz[3 * A + 2] - b->xyz[3 * B + 2];
                en += b->Z[A] * b->Z[B] / std::sqrt(dx * dx + dy * dy + dz * dz);
            }
        c->mol_enuc.push_back(en);
        c->enuc += en;
        c->natom += b->natom;
        c->nshell += b->nshell;
        c->nelec += b->nelec;
        gbf += nb;
    }
    c->nbf = nmol == 1 ? c->mol_n[0] : gbf;
    c->nocc = c->nelec / 2;
    const int nprim_tot = (int)c->exps.size();
    const size_t P = (size_t)c->packed;

    // shells and molecules on the device
    std::vector<double> shxyz(3 * c->nshell);
    for (int k = 0; k < c->nshell; ++k)
        for (int d = 0; d < 3; ++d) shxyz[3 * k + d] = c->xyz[3 * c->sh_atom[k] + d];
    ShellsDev &sh = c->sh;
    sh.nshell = c->nshell;
    sh.natom = c->natom;
    sh.nmol = nmol;
    PCHK(c->pool.alloc(&sh.xyz, 3 * c->nshell));
    PCHK(c->pool.alloc(&sh.l, c->nshell));
    PCHK(c->pool.alloc(&sh.nprim, c->nshell));
    PCHK(c->pool.alloc(&sh.prim0, c->nshell));
    PCHK(c->pool.alloc(&sh.bf0, c->nshell));
    PCHK(c->pool.alloc(&sh.mol, c->nshell));
    PCHK(c->pool.alloc(&sh.exps, nprim_tot));
    PCHK(c->pool.alloc(&sh.coef, nprim_tot));
    PCHK(c->pool.alloc(&sh.atom_xyz, 3 * c->natom));
    PCHK(c->pool.alloc(&sh.atom_Z, c->natom));
    PCHK(c->pool.alloc(&sh.mol_atom0, nmol));
    PCHK(c->pool.alloc(&sh.mol_natom, nmol));
    PCHK(c->pool.alloc(&sh.mol_bf0, nmol));
    PCHK(c->pool.alloc(&sh.mol_n, nmol));
    PCHK(c->pool.alloc(&sh.mol_off, nmol));
    auto up = [&](void *d, const void *h, size_t bytes) {
        return hipMemcpy(d, h, bytes, hipMemcpyHostToDevice);
    };
    HCHK(up(sh.xyz, shxyz.data(), sizeof(double) * shxyz.size()));
    HCHK(up(sh.l, c->sh_l.data(), sizeof(int) * c->nshell));
    HCHK(up(sh.nprim, c->sh_nprim.data(), sizeof(int) * c->nshell));
    HCHK(up(sh.prim0, c->sh_prim0.data(), sizeof(int) * c->nshell));
    HCHK(up(sh.bf0, c->sh_bf0.data(), sizeof(int) * c->nshell));
    HCHK(up(sh.mol, c->sh_mol.data(), sizeof(int) * c->nshell));
    HCHK(up(sh.exps, c->exps.data(), sizeof(double) * nprim_tot));
    HCHK(up(sh.coef, c->coefs.data(), sizeof(double) * nprim_tot));
    HCHK(up(sh.atom_xyz, c->xyz.data(), sizeof(double) * 3 * c->natom));
    HCHK(up(sh.atom_Z, c->Z.data(), sizeof(double) * c->natom));
    HCHK(up(sh.mol_atom0, c->mol_atom0.data(), sizeof(int) * nmol));
    HCHK(up(sh.mol_natom, c->mol_natom.data(), sizeof(int) * nmol));
    HCHK(up(sh.mol_bf0, c->mol_bf0.data(), sizeof(int) * nmol));
    HCHK(up(sh.mol_n, c->mol_n.data(), sizeof(int) * nmol));
    HCHK(up(sh.mol_off, c->mol_off.data(), sizeof(long long) * nmol));
    c->d_mol_n = sh.mol_n;
    c->d_mol_off = sh.mol_off;
    PCHK(c->pool.alloc(&c->d_nocc, nmol));
    HCHK(up(c->d_nocc, c->mol_nocc.data(), sizeof(int) * nmol));
    PCHK(c->pool.alloc(&c->Emol, nmol));
    HCHK(launch_shell_norm(sh, nullptr));
    PCHK(c->pool.alloc(&c->boys, (size_t)BOYS_NT * BOYS_NORD));
    HCHK(launch_boys_table(c->boys, nullptr));

    // every shell pair within a molecule, oriented so that l(s1) >= l(s2)
    for (int m = 0; m < nmol; ++m) {
        const int s0 = c->mol_shell0[m], ns = c->mol_nshell[m];
        for (int a = s0; a < s0 + ns; ++a)
            for (int bb = s0; bb <= a; ++bb) {
                int s1 = a, s2 = bb;
                if (c->sh_l[s1] < c->sh_l[s2]) std::swap(s1, s2);
                const int pc = pclass(c->sh_l[s1], c->sh_l[s2]);
                c->pair_lookup[(long long)s1 * c->nshell + s2] = {pc, (int)c->all_s1[pc].size()};
                c->all_s1[pc].push_back(s1);
                c->all_s2[pc].push_back(s2);
            }
    }
    for (int pc = 0; pc < NPCLASS; ++pc)
        SCHK(build_table(c, c->pool, c->all[pc], pc, c->all_s1[pc], c->all_s2[pc]));

    // packed matrices and Fock work buffers
    PCHK(c->pool.alloc(&c->S, P));
    PCHK(c->pool.alloc(&c->H, P));
    PCHK(c->pool.alloc(&c->X, P));
    PCHK(c->pool.alloc(&c->Jh, P));
    PCHK(c->pool.alloc(&c->Kh, P));
    PCHK(c->pool.alloc(&c->F, P));
    PCHK(c->pool.alloc(&c->Dn, P));
    PCHK(c->pool.alloc(&c->T1, P));
    PCHK(c->pool.alloc(&c->T2, P));
    PCHK(c->pool.alloc(&c->scal, 8));
    PCHK(c->pool.alloc(&c->dinfo, std::max(4, nmol)));
    if (rocblas_create_handle(&c->blas) != rocblas_status_success)
        return cleanup(fail(FSIM_EHIP, "rocblas_create_handle failed"));

    // one-electron matrices, one packed block per molecule
    const int Ntot = gbf;
    int *dbs = nullptr, *dbc = nullptr;
    PCHK(c->pool.alloc(&dbs, Ntot));
    PCHK(c->pool.alloc(&dbc, Ntot));
    HCHK(up(dbs, bf_shell.data(), sizeof(int) * Ntot));
    HCHK(up(dbc, bf_comp.data(), sizeof(int) * Ntot));
    HCHK(launch_one_electron_impl(sh, c->boys, c->nmax, dbs, dbc, c->S, c->T1, c->T2, nullptr));
    HCHK(hipMemcpy(c->H, c->T1, sizeof(double) * P, hipMemcpyDeviceToDevice));
    {
        const double one = 1.0;
        if (rocblas_daxpy(c->blas, (int)P, &one, c->T2, 1, c->H, 1) != rocblas_status_success)
            return cleanup(fail(FSIM_EHIP, "rocblas_daxpy failed"));
    }
    if (nmol == 1) {
        // incremental builds read the shell of every basis function
        c->d_bf_shell = dbs;
        PCHK(c->pool.alloc(&c->dD, P));
        PCHK(c->pool.alloc(&c->Mblk, (size_t)c->nshell * c->nshell));
        c->Mhost.assign((size_t)c->nshell * c->nshell, 0.0);
    } else {
        c->pool.release(dbs);
    }
    c->pool.release(dbc);

    c->nscf = c->nbf;
    if (o->spherical) {
        if (nmol != 1)
            return cleanup(fail(FSIM_EINVAL, "spherical basis sets are for one-molecule contexts"));
        SCHK(spherical_setup(c, c->pool));
    }
    const int m_hist = std::max(1, c->opt.diis_m);
    if (nmol == 1) {
        const int N = c->nscf;
        const size_t N2 = (size_t)N * N;
        PCHK(c->pool.alloc(&c->eig, N));
        PCHK(c->pool.alloc(&c->ework, N));
        // X = U s^-1/2 U^T
        HCHK(hipMemcpy(c->T1, c->S, sizeof(double) * N2, hipMemcpyDeviceToDevice));
        SCHK(syevd(c, c->T1, c->eig, nullptr));
        std::vector<double> sv(N);
        HCHK(hipMemcpy(sv.data(), c->eig, sizeof(double) * N, hipMemcpyDeviceToHost));
        if (!(sv[0] > 1e-10))
            return cleanup(fail(FSIM_EINVAL, "overlap matrix is (near) singular: lowest eigenvalue " +
                                                 std::to_string(sv[0])));
        HCHK(inv_sqrt(N, c->eig, c->ework, nullptr));
        HCHK(scale_cols(N, c->T1, c->ework, c->T2, nullptr));
        SCHK(gemm(c->blas, false, true, N, N, N, 1.0, c->T2, N, c->T1, N, 0.0, c->X, N));
        c->dF.resize(m_hist, nullptr);
        c->dE.resize(m_hist, nullptr);
        for (int k = 0; k < m_hist; ++k) {
            PCHK(c->pool.alloc(&c->dF[k], N2));
            PCHK(c->pool.alloc(&c->dE[k], N2));
        }
        c->Bm.assign((size_t)m_hist * m_hist, 0.0);
    } else {
        const size_t M2 = (size_t)c->nmax * c->nmax, B = M2 * nmol;
        PCHK(c->pool.alloc(&c->pS, B));
        PCHK(c->pool.alloc(&c->pX, B));
        PCHK(c->pool.alloc(&c->pH, B));
        PCHK(c->pool.alloc(&c->pF, B));
        PCHK(c->pool.alloc(&c->pD, B));
        PCHK(c->pool.alloc(&c->pT1, B));
        PCHK(c->pool.alloc(&c->pT2, B));
        PCHK(c->pool.alloc(&c->pErr, B));
        PCHK(c->pool.alloc(&c->pEig, (size_t)c->nmax * nmol));
        PCHK(c->pool.alloc(&c->ework, (size_t)c->nmax * nmol));
        PCHK(c->pool.alloc(&c->pRed, (size_t)nmol * (DIIS_MAX + 2)));
        c->pdF.resize(m_hist, nullptr);
        c->pdE.resize(m_hist, nullptr);
        for (int k = 0; k < m_hist; ++k) {
            PCHK(c->pool.alloc(&c->pdF[k], B));
            PCHK(c->pool.alloc(&c->pdE[k], B));
        }
        c->Bb.assign((size_t)nmol * m_hist * m_hist, 0.0);
        SCHK(batched_orthogonaliser(c, nullptr));
    }
    HCHK(hipDeviceSynchronize());
    c->Eprev_mol.assign(nmol, 0.0);
    c->mol_info.assign(nmol, fsim_scf_info{});
    c->Emol_host.assign(nmol, 0.0);
#undef PCHK
#undef HCHK
#undef SCHK
    *out = c;
    return FSIM_OK;
}

extern "C" fsim_status fsim_ctx_create(const fsim_basis *b, const fsim_options *o, fsim_ctx **out) {
    return create_impl(b, 1, o, out);
}

extern "C" fsim_status fsim_batch_create(const fsim_basis *mols, int32_t nmol,
                                         const fsim_options *o, fsim_ctx **out) {
    return create_impl(mols, nmol, o, out);
}

// Batched X_m = U_m s_m^-1/2 U_m^T on zero-padded blocks (identity padding).
static fsim_status batched_orthogonaliser(fsim_ctx *c, hipStream_t s) {
    const MolLayout L = layout_of(c);
    const int M = c->nmax;
    const long long M2 = (long long)M * M;
    HIPCHK(pad_blocks(L, c->S, c->pS, 1.0, s));
    HIPCHK(pad_blocks(L, c->H, c->pH, 0.0, s));
    HIPCHK(hipMemcpyAsync(c->pT1, c->pS, sizeof(double) * M2 * c->nmol, hipMemcpyDeviceToDevice, s));
    BLASCHK(rocblas_set_stream(c->blas, s));
    BLASCHK(rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper, M,
                                             c->pT1, M, M2, c->pEig, M, c->ework, M, c->dinfo,
                                             c->nmol));
    std::vector<double> ev((size_t)M * c->nmol);
    HIPCHK(hipMemcpy(ev.data(), c->pEig, sizeof(double) * ev.size(), hipMemcpyDeviceToHost));
    for (int m = 0; m < c->nmol; ++m)
        if (!(ev[(size_t)m * M] > 1e-10))
            return fail(FSIM_EINVAL, "molecule " + std::to_string(m) +
                                         ": overlap matrix is (near) singular");
    HIPCHK(inv_sqrt(M * c->nmol, c->pEig, c->ework, s));
    HIPCHK(scale_cols_padded(L, c->pT1, c->ework, c->pT2, s));
    const double one = 1.0, zero = 0.0;
    BLASCHK(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none,
                                          rocblas_operation_transpose, M, M, M, &one, c->pT2, M,
                                          M2, c->pT1, M, M2, &zero, c->pX, M, M2, c->nmol));
    HIPCHK(unpad_blocks(L, c->pX, c->X, s));
    return FSIM_OK;
}

extern "C" fsim_status fsim_ctx_destroy(fsim_ctx *c) {
    if (!c) return FSIM_OK;
    hipDeviceSynchronize();
    if (c->blas) rocblas_destroy_handle(c->blas);
    for (int p = 0; p < 2; ++p) {
        if (c->gexec[p]) hipGraphExecDestroy(c->gexec[p]);
        if (c->gev[p]) hipEventDestroy(c->gev[p]);
    }
    if (c->gstream) hipStreamDestroy(c->gstream);
    for (auto &e : c->ev) hipEventDestroy(e);
    c->store_pool.clear();
    c->screen_pool.clear();
    c->pool.clear();
    delete c;
    return FSIM_OK;
}

extern "C" fsim_status fsim_nbf(const fsim_ctx *c, int32_t *nbf, int32_t *nshell) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (nbf) *nbf = c->nscf;
    if (nshell) *nshell = c->nshell;
    return FSIM_OK;
}

extern "C" fsim_status fsim_nuclear_repulsion(const fsim_ctx *c, double *e) {
    if (!c || !e) return fail(FSIM_EINVAL, "NULL argument");
    *e = c->enuc;
    return FSIM_OK;
}

extern "C" fsim_status fsim_one_electron(fsim_ctx *c, double *S, double *H, double *X, void *stream) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes =
        sizeof(double) * (c->nmol == 1 ? (size_t)c->nscf * c->nscf : (size_t)c->packed);
    if (S) HIPCHK(hipMemcpyAsync(S, c->S, bytes, hipMemcpyDeviceToDevice, s));
    if (H) HIPCHK(hipMemcpyAsync(H, c->H, bytes, hipMemcpyDeviceToDevice, s));
    if (X) HIPCHK(hipMemcpyAsync(X, c->X, bytes, hipMemcpyDeviceToDevice, s));
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Stored-block evaluation (used by the Schwarz screen and fsim_eri_quartets)
// ---------------------------------------------------------------------------

namespace {
struct StoreTask {
    int bra, ket;
    long long off;
    int st[4];
};
}  // namespace

// Run the store kernels for tasks grouped by (bra class, ket class) on the
// all-pairs tables: with tuned, each class runs the kernel variant and block
// shape its Fock build uses (the same kernel code writing blocks out instead
// of digesting them); otherwise the default variant.
static fsim_status run_store(fsim_ctx *c, std::vector<StoreTask> (&tasks)[NPCLASS][NPCLASS],
                             double *out, bool fp32, bool tuned, hipStream_t s) {
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            auto &tv = tasks[X][Y];
            if (tv.empty()) continue;
            std::stable_sort(tv.begin(), tv.end(),
                             [](const StoreTask &a, const StoreTask &b) { return a.bra < b.bra; });
            std::vector<int> tbra, tket;
            std::vector<long long> toff;
            std::vector<int> tst;
            size_t i = 0;
            while (i < tv.size()) {
                const int b = tv[i].bra;
                size_t j = i;
                while (j < tv.size() && tv[j].bra == b && j - i < 64) ++j;
                tbra.push_back(b);
                for (size_t k = 0; k < 64; ++k) {
                    if (i + k < j) {
                        tket.push_back(tv[i + k].ket);
                        toff.push_back(tv[i + k].off);
                        for (int d = 0; d < 4; ++d) tst.push_back(tv[i + k].st[d]);
                    } else {
                        tket.push_back(-1);
                        toff.push_back(0);
                        for (int d = 0; d < 4; ++d) tst.push_back(0);
                    }
                }
                i = j;
            }
            int *dbra = nullptr, *dket = nullptr, *dst = nullptr;
            long long *doff = nullptr;
            HIPCHK(hipMalloc(&dbra, sizeof(int) * tbra.size()));
            HIPCHK(hipMalloc(&dket, sizeof(int) * tket.size()));
            HIPCHK(hipMalloc(&doff, sizeof(long long) * toff.size()));
            HIPCHK(hipMalloc(&dst, sizeof(int) * tst.size()));
            HIPCHK(hipMemcpyAsync(dbra, tbra.data(), sizeof(int) * tbra.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(dket, tket.data(), sizeof(int) * tket.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(doff, toff.data(), sizeof(long long) * toff.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(dst, tst.data(), sizeof(int) * tst.size(), hipMemcpyHostToDevice, s));
            EriArgs a{};
            a.bra = c->all[X];
            a.ket = c->all[Y];
            a.same_class = X == Y;
            a.st_ntile = (int)tbra.size();
            a.st_bra = dbra;
            a.st_ket = dket;
            a.st_off = doff;
            a.st_stride = dst;
            a.out = out;
            a.boys = c->boys;
            a.nbf = c->nbf;
            const int f = fp32 ? 1 : 0;
            HIPCHK(launch_eri(X, Y, fp32, true, tuned ? c->variant[X][Y][f] : ERI_DEFAULT_VARIANT,
                              tuned ? c->wpb[X][Y][f] : 4, a, s));
            HIPCHK(hipStreamSynchronize(s));
            hipFree(dbra);
            hipFree(dket);
            hipFree(doff);
            hipFree(dst);
        }
    return FSIM_OK;
}

extern "C" fsim_status fsim_eri_quartets(fsim_ctx *c, int64_t n, const int32_t *q,
                                         const int64_t *offsets, double *out, fsim_precision prec,
                                         void *stream) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(FSIM_EINVAL, "negative quartet count");
    if (n == 0) return FSIM_OK;
    if (!q || !offsets || !out) return fail(FSIM_EINVAL, "NULL argument");
    std::vector<StoreTask> tasks[NPCLASS][NPCLASS];
    for (int64_t i = 0; i < n; ++i) {
        int sh[4];
        for (int d = 0; d < 4; ++d) {
            sh[d] = q[4 * i + d];
            if (sh[d] < 0 || sh[d] >= c->nshell)
                return fail(FSIM_EINVAL, "shell index out of range in quartet " + std::to_string(i));
        }
        if (offsets[i] < 0) return fail(FSIM_EINVAL, "negative offset");
        int n_[4];
        for (int d = 0; d < 4; ++d) n_[d] = ncart_h(c->sh_l[sh[d]]);
        const int u[4] = {n_[1] * n_[2] * n_[3], n_[2] * n_[3], n_[3], 1};
        // locate the two pairs and the stride of each stored component slot
        int pc[2], idx[2], stv[2][2];
        for (int h = 0; h < 2; ++h) {
            const int x = sh[2 * h], y = sh[2 * h + 1];
            auto it = c->pair_lookup.find((long long)x * c->nshell + y);
            bool swapped = false;
            if (it == c->pair_lookup.end()) {
                it = c->pair_lookup.find((long long)y * c->nshell + x);
                swapped = true;
            }
            if (it == c->pair_lookup.end()) return fail(FSIM_EINVAL, "internal: pair not found");
            pc[h] = it->second.first;
            idx[h] = it->second.second;
            stv[h][0] = swapped ? u[2 * h + 1] : u[2 * h];
            stv[h][1] = swapped ? u[2 * h] : u[2 * h + 1];
        }
        StoreTask t;
        t.off = offsets[i];
        int bh = 0, kh = 1;
        if (pc[0] < pc[1]) std::swap(bh, kh);
        t.bra = idx[bh];
        t.ket = idx[kh];
        t.st[0] = stv[bh][0];
        t.st[1] = stv[bh][1];
        t.st[2] = stv[kh][0];
        t.st[3] = stv[kh][1];
        tasks[pc[bh]][pc[kh]].push_back(t);
    }
    return run_store(c, tasks, out, prec == FSIM_MIXED, true, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Schwarz screening and work lists
// ---------------------------------------------------------------------------

// Flop models of one class (FMA = 2), as per-primitive-quartet,
// per-bra-primitive-pair and per-contracted-quartet terms.
struct FlopModel {
    double prim, bra, quartet;
};
static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
// Reference model: dense Hermite sets.  Per primitive quartet 25 (setup) +
// 30 + 3(L+1) (Boys) + 2 C(L+4,4) (R) + 2 C(Lab+3,3) C(Lcd+3,3) n_cart(cd)
// (step 1); per bra primitive pair 2 C(Lab+3,3) n_cart(ab) n_cart(cd)
// (step 2); per contracted quartet 6 n_cart(abcd) FMAs of digest.
static FlopModel flop_model(int la, int lb, int lc, int ld) {
    const int L = la + lb + lc + ld, lab = la + lb, lcd = lc + ld;
    const double nab = ncart_h(la) * ncart_h(lb), ncd = ncart_h(lc) * ncart_h(ld);
    FlopModel m;
    m.prim = 25.0 + 30.0 + 3.0 * (L + 1) + 2.0 * binom(L + 4, 4) +
             2.0 * binom(lab + 3, 3) * binom(lcd + 3, 3) * ncd;
    m.bra = 2.0 * binom(lab + 3, 3) * nab * ncd;
    m.quartet = 12.0 * nab * ncd;
    return m;
}
// What the kernels execute (without chunk recomputation): only the nonzero
// Hermite box entries of each component pair, and the R recursion's own count.
static FlopModel flop_model_exec(int la, int lb, int lc, int ld) {
    const int L = la + lb + lc + ld;
    double rec = 0;
    for (int n = 0; n < L; ++n)
        for (int s = 1; s <= L - n; ++s) rec += (s + 1) * (s + 2) / 2;
    FlopModel m;
    m.prim = 60.0 + 3.0 * (L + 1) + 2.0 * rec + 2.0 * n_entries(lc, ld) * nherm(la + lb);
    m.bra = 2.0 * n_entries(la, lb) * ncart_h(lc) * ncart_h(ld);
    m.quartet = 12.0 * ncart_h(la) * ncart_h(lb) * ncart_h(lc) * ncart_h(ld);
    return m;
}

static fsim_status upload_list(DevPool &pool, TileList &tl, const std::vector<int> &bra,
                               const std::vector<int> &lo, const std::vector<int> &hi, int seg,
                               int *segcap) {
    tl = TileList{};
    tl.nbra = (int)bra.size();
    std::vector<int> start(bra.size() + 1, 0);
    int64_t nq = 0;
    for (size_t i = 0; i < bra.size(); ++i) {
        const int nk = hi[i] - lo[i];
        nq += nk;
        const long long ns = (long long)start[i] + (nk + TILE - 1) / TILE;
        if (ns > 0x7fffffffLL) return fail(FSIM_ENOMEM, "too many tiles for one quartet class");
        start[i + 1] = (int)ns;
    }
    tl.ntile = start.back();
    tl.nquartet = nq;
    if (tl.nbra == 0) return FSIM_OK;
    HIPCHK(pool.alloc(&tl.tile_start, start.size()));
    HIPCHK(pool.alloc(&tl.bra, bra.size()));
    HIPCHK(pool.alloc(&tl.ket_lo, bra.size()));
    HIPCHK(pool.alloc(&tl.ket_hi, bra.size()));
    HIPCHK(hipMemcpy(tl.tile_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tl.bra, bra.data(), sizeof(int) * bra.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tl.ket_lo, lo.data(), sizeof(int) * bra.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tl.ket_hi, hi.data(), sizeof(int) * bra.size(), hipMemcpyHostToDevice));
    // segments of at most seg tiles, each within one bra record; the device
    // arrays hold the segments of the smallest size, so that a later tuning
    // may cut them again (set_segments)
    size_t cap = 0;
    for (size_t i = 0; i < bra.size(); ++i) cap += (start[i + 1] - start[i] + SEG_MIN - 1) / SEG_MIN;
    *segcap = (int)cap;
    std::vector<int> h(3 * cap);
    tl.nseg = (int)cut_segments(start, seg, h.data(), h.data() + cap, h.data() + 2 * cap);
    HIPCHK(pool.alloc(&tl.seg_rec, cap));
    HIPCHK(pool.alloc(&tl.seg_t0, cap));
    HIPCHK(pool.alloc(&tl.seg_nt, cap));
    HIPCHK(hipMemcpy(tl.seg_rec, h.data(), sizeof(int) * tl.nseg, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tl.seg_t0, h.data() + cap, sizeof(int) * tl.nseg, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tl.seg_nt, h.data() + 2 * cap, sizeof(int) * tl.nseg, hipMemcpyHostToDevice));
    return FSIM_OK;
}

// Tile starts of a host list (bra records with ket ranges [lo, hi)).
static std::vector<int> tile_starts(const std::vector<int> &lo, const std::vector<int> &hi) {
    std::vector<int> st(lo.size() + 1, 0);
    for (size_t i = 0; i < lo.size(); ++i) st[i + 1] = st[i] + (hi[i] - lo[i] + TILE - 1) / TILE;
    return st;
}

extern "C" fsim_status fsim_schwarz_screen(fsim_ctx *c, double tau, double tau32, double *Q_out,
                                           fsim_screen_stats *stats) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (!(tau >= 0) || !(tau32 >= 0) || !std::isfinite(tau) || !std::isfinite(tau32))
        return fail(FSIM_EINVAL, "thresholds must be finite and >= 0");
    if (Q_out && c->nmol != 1) return fail(FSIM_EINVAL, "Q_out is only available for one molecule");
    const int ns = c->nshell;
    // diagonal integrals (ab|ab) of every pair
    std::vector<StoreTask> tasks[NPCLASS][NPCLASS];
    std::vector<long long> base(NPCLASS + 1, 0);
    for (int pc = 0; pc < NPCLASS; ++pc) {
        const int n1 = ncart_h(pclass_l1(pc)), n2 = ncart_h(pclass_l2(pc));
        const long long bs = (long long)n1 * n2 * n1 * n2;
        base[pc + 1] = base[pc] + bs * c->all[pc].n;
        for (int i = 0; i < c->all[pc].n; ++i) {
            StoreTask t;
            t.bra = t.ket = i;
            t.off = base[pc] + bs * i;
            t.st[0] = n2 * n1 * n2;
            t.st[1] = n1 * n2;
            t.st[2] = n2;
            t.st[3] = 1;
            tasks[pc][pc].push_back(t);
        }
    }
    double *dblk = nullptr;
    HIPCHK(hipMalloc(&dblk, sizeof(double) * std::max<long long>(1, base[NPCLASS])));
    STCHK(run_store(c, tasks, dblk, false, false, nullptr));
    std::vector<double> blk(base[NPCLASS]);
    HIPCHK(hipMemcpy(blk.data(), dblk, sizeof(double) * blk.size(), hipMemcpyDeviceToHost));
    hipFree(dblk);
    if (c->nmol == 1) c->Qmat.assign((size_t)ns * ns, 0.0);
    std::vector<double> Qpair[NPCLASS];
    std::vector<double> Qmax(c->nmol, 0.0);
    for (int pc = 0; pc < NPCLASS; ++pc) {
        const int n1 = ncart_h(pclass_l1(pc)), n2 = ncart_h(pclass_l2(pc));
        const long long bs = (long long)n1 * n2 * n1 * n2;
        Qpair[pc].resize(c->all[pc].n);
        for (int i = 0; i < c->all[pc].n; ++i) {
            double mx = 0.0;
            for (int x = 0; x < n1; ++x)
                for (int y = 0; y < n2; ++y) {
                    const double v = blk[base[pc] + bs * i + ((x * n2 + y) * n1 + x) * n2 + y];
                    mx = std::max(mx, v);
                }
            const double qv = std::sqrt(mx);
            Qpair[pc][i] = qv;
            const int s1 = c->all_s1[pc][i], s2 = c->all_s2[pc][i];
            Qmax[c->sh_mol[s1]] = std::max(Qmax[c->sh_mol[s1]], qv);
            if (c->nmol == 1) {
                c->Qmat[(size_t)s1 * ns + s2] = qv;
                c->Qmat[(size_t)s2 * ns + s1] = qv;
            }
        }
    }
    // kept pairs per class, ordered by (molecule, Q descending); each
    // molecule owns a contiguous segment of every class table
    drop_graphs(c);
    c->store_pool.clear();
    c->stored = false;
    c->store = nullptr;
    c->store_bytes = 0;
    c->screen_pool.clear();
    c->screened = false;
    fsim_screen_stats S{};
    for (int pc = 0; pc < NPCLASS; ++pc) S.shell_pairs += c->all[pc].n;
    std::vector<int> order[NPCLASS];
    std::vector<int> kmol[NPCLASS];                 // molecule of each kept pair
    std::vector<int> seg[NPCLASS];                  // [nmol + 1] segment starts
    for (int pc = 0; pc < NPCLASS; ++pc) {
        auto molof = [&](int i) { return c->sh_mol[c->all_s1[pc][i]]; };
        for (int i = 0; i < c->all[pc].n; ++i)
            if (Qpair[pc][i] * Qmax[molof(i)] >= tau) order[pc].push_back(i);
        std::stable_sort(order[pc].begin(), order[pc].end(), [&](int a, int b) {
            const int ma = molof(a), mb = molof(b);
            if (ma != mb) return ma < mb;
            return Qpair[pc][a] > Qpair[pc][b];
        });
        std::vector<int> &s1 = c->kept_s1[pc], &s2 = c->kept_s2[pc];
        s1.clear();
        s2.clear();
        c->Qkept[pc].clear();
        seg[pc].assign(c->nmol + 1, 0);
        for (int i : order[pc]) {
            s1.push_back(c->all_s1[pc][i]);
            s2.push_back(c->all_s2[pc][i]);
            c->Qkept[pc].push_back(Qpair[pc][i]);
            kmol[pc].push_back(molof(i));
            seg[pc][molof(i) + 1]++;
        }
        for (int m = 0; m < c->nmol; ++m) seg[pc][m + 1] += seg[pc][m];
        STCHK(build_table(c, c->screen_pool, c->kept[pc], pc, s1, s2));
        if (c->kept[pc].n)
            HIPCHK(hipMemcpy(c->kept[pc].Q, c->Qkept[pc].data(), sizeof(double) * c->kept[pc].n,
                             hipMemcpyHostToDevice));
        S.pairs_kept += c->kept[pc].n;
        std::vector<int> &np = c->kept_np[pc];
        np.resize(s1.size());
        for (size_t i = 0; i < s1.size(); ++i) np[i] = c->sh_nprim[s1[i]] * c->sh_nprim[s2[i]];
        for (int v : np) S.prim_pairs_total += v;
        if (c->tau_prim > 0 && c->kept[pc].n) {
            double *dq = nullptr;
            HIPCHK(hipMalloc(&dq, sizeof(double) * c->nmol));
            HIPCHK(hipMemcpy(dq, Qmax.data(), sizeof(double) * c->nmol, hipMemcpyHostToDevice));
            HIPCHK(launch_prim_screen(c->kept[pc], dq, c->tau_prim, nullptr));
            HIPCHK(hipDeviceSynchronize());
            hipFree(dq);
            HIPCHK(hipMemcpy(np.data(), c->kept[pc].nprim, sizeof(int) * np.size(),
                             hipMemcpyDeviceToHost));
        }
        for (int v : np) S.prim_pairs_kept += v;
    }
    // canonical quartets: per molecule, npair_m (npair_m + 1) / 2
    {
        std::vector<long long> np(c->nmol, 0);
        for (int pc = 0; pc < NPCLASS; ++pc)
            for (int i = 0; i < c->all[pc].n; ++i) np[c->sh_mol[c->all_s1[pc][i]]]++;
        for (int m = 0; m < c->nmol; ++m) S.quartets_total += np[m] * (np[m] + 1) / 2;
    }
    // work lists
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const auto &Qb = c->Qkept[X], &Qk = c->Qkept[Y];
            std::vector<int> b64, lo64, hi64, bm64, lom64, him64, bm32, lom32, him32;
            const int la = pclass_l1(X), lb = pclass_l2(X), lc = pclass_l1(Y), ld = pclass_l2(Y);
            const FlopModel fm = flop_model(la, lb, lc, ld), fx = flop_model_exec(la, lb, lc, ld);
            for (int i = 0; i < (int)Qb.size(); ++i) {
                const double qi = Qb[i];
                const int m = kmol[X][i];
                const int k0 = seg[Y][m], k1 = seg[Y][m + 1];
                // kets of the same molecule with qi * Q_j >= tau (Q descending)
                int lo = k0, hi = k1;
                while (lo < hi) {
                    const int mid = (lo + hi) / 2;
                    if (qi * Qk[mid] >= tau) lo = mid + 1;
                    else hi = mid;
                }
                int n = lo;
                if (X == Y) n = std::min(n, i + 1);
                if (n <= k0) continue;
                int split = n;
                if (tau32 > 0) {
                    int l2 = k0, h2 = n;
                    while (l2 < h2) {
                        const int mid = (l2 + h2) / 2;
                        if (qi * Qk[mid] >= tau32) l2 = mid + 1;
                        else h2 = mid;
                    }
                    split = l2;
                }
                b64.push_back(i);
                lo64.push_back(k0);
                hi64.push_back(n);
                if (split > k0) {
                    bm64.push_back(i);
                    lom64.push_back(k0);
                    him64.push_back(split);
                }
                if (n > split) {
                    bm32.push_back(i);
                    lom32.push_back(split);
                    him32.push_back(n);
                }
                S.quartets_fp64 += split - k0;
                S.quartets_fp32 += n - split;
            }
            ClassLists &cl = c->lists[X][Y];
            STCHK(upload_list(c->screen_pool, cl.all64, b64, lo64, hi64, c->segt[X][Y][0],
                              &cl.segcap[0]));
            STCHK(upload_list(c->screen_pool, cl.mix64, bm64, lom64, him64, c->segt[X][Y][0],
                              &cl.segcap[1]));
            STCHK(upload_list(c->screen_pool, cl.mix32, bm32, lom32, him32, c->segt[X][Y][1],
                              &cl.segcap[2]));
            cl.host[0] = HostList{b64, lo64, hi64};
            cl.host[1] = HostList{bm64, lom64, him64};
            cl.host[2] = HostList{bm32, lom32, him32};
            const TileList *full[3] = {&cl.all64, &cl.mix64, &cl.mix32};
            for (int k = 0; k < 3; ++k) {
                TileList &d = cl.delta[k];
                d = *full[k];
                d.ntile = 0;
                d.nquartet = 0;
                // density-screened ket ends change the tiles: segments are
                // cut again for every build, at most as many as the full list's
                d.nseg = 0;
                d.seg_rec = d.seg_t0 = d.seg_nt = nullptr;
                cl.dseg[k].assign(3 * (size_t)cl.segcap[k], 0);
                cl.dnq[k] = 0;
                cl.dstart[k].assign(d.nbra + 1, 0);
                cl.dhi[k] = cl.host[k].lo;
                if (d.nbra == 0) continue;
                HIPCHK(c->screen_pool.alloc(&d.tile_start, (size_t)d.nbra + 1));
                HIPCHK(c->screen_pool.alloc(&d.ket_hi, (size_t)d.nbra));
                if (cl.segcap[k] > 0) {
                    HIPCHK(c->screen_pool.alloc(&d.seg_rec, (size_t)cl.segcap[k]));
                    HIPCHK(c->screen_pool.alloc(&d.seg_t0, (size_t)cl.segcap[k]));
                    HIPCHK(c->screen_pool.alloc(&d.seg_nt, (size_t)cl.segcap[k]));
                }
            }
            S.quartets_kept += cl.all64.nquartet;
            // primitive quartets: sum over kept quartets of K_bra * K_ket
            // (primitive pairs in use: after primitive-pair screening, if on)
            const std::vector<int> &kb = c->kept_np[X], &kk = c->kept_np[Y];
            std::vector<long long> kpre(kk.size() + 1, 0);
            for (size_t j = 0; j < kk.size(); ++j) kpre[j + 1] = kpre[j] + kk[j];
            cl.s64 = cl.sm64 = cl.sm32 = ListStats{};
            auto tally = [&](ListStats &ls, const std::vector<int> &bb, const std::vector<int> &lo,
                             const std::vector<int> &hi) {
                for (size_t t = 0; t < bb.size(); ++t) {
                    const long long nk = hi[t] - lo[t];
                    const long long pq = (long long)kb[bb[t]] * (kpre[hi[t]] - kpre[lo[t]]);
                    const double bp = (double)kb[bb[t]] * nk;   // bra primitive pairs x kets
                    ls.npq += pq;
                    ls.flops += fm.prim * pq + fm.bra * bp + fm.quartet * nk;
                    ls.flops_exec += fx.prim * pq + fx.bra * bp + fx.quartet * nk;
                }
            };
            tally(cl.s64, b64, lo64, hi64);
            tally(cl.sm64, bm64, lom64, him64);
            tally(cl.sm32, bm32, lom32, him32);
            S.prim_quartets_kept += cl.s64.npq;
            S.flops_fp64 += cl.s64.flops;
            S.flops_mixed_fp64 += cl.sm64.flops;
            S.flops_mixed_fp32 += cl.sm32.flops;
            cl.s64.nq = cl.all64.nquartet;
            cl.sm64.nq = cl.mix64.nquartet;
            cl.sm32.nq = cl.mix32.nquartet;
        }
    if (tau32 <= 0) {
        S.quartets_fp64 = S.quartets_kept;
        S.quartets_fp32 = 0;
    }
    c->tau = tau;
    c->tau32 = tau32;
    c->stats = S;
    c->screened = true;
    c->inc_have = false;
    if (Q_out)
        HIPCHK(hipMemcpy(Q_out, c->Qmat.data(), sizeof(double) * ns * ns, hipMemcpyHostToDevice));
    if (stats) *stats = S;
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Fock build
// ---------------------------------------------------------------------------

// Enqueue the class kernels and the Fock assembly for density D into F (J, K
// optional) on stream s.  No host synchronisation, no memset: this is the
// sequence a graph captures.
// Captured Fock builds bake in kernel variants and buffers: drop them when
// either changes.
static void drop_graphs(fsim_ctx *c) {
    for (int p = 0; p < 2; ++p)
        if (c->gexec[p]) {
            hipGraphExecDestroy(c->gexec[p]);
            c->gexec[p] = nullptr;
        }
}

static constexpr int NXCD = 8;   // XCDs of an MI355X

// Persistent queue slots (as persistent.hip orders them) and the class record
// the profile uses for the persistent launch.
static int persist_slot_bra(int k) { return k <= 1 || k == 3 ? 2 : (k == 5 ? 0 : 1); }
static int persist_slot_ket(int k) { return k == 0 ? 2 : (k == 1 || k == 2 ? 1 : 0); }
static int persist_slot_of(int X, int Y) {
    for (int k = 0; k < PERSIST_SLOTS; ++k)
        if (persist_slot_bra(k) == X && persist_slot_ket(k) == Y) return k;
    return -1;
}
static constexpr int PERSIST_PROFILE_CLASS = NPCLASS;
static constexpr int KO_STAGE_BYTES_MAX = 8192;   // per-wave LDS stage of a ket-outer tile

// acc (optional): one shared pair of J'/K' accumulators to use instead of
// the context's own (the allocation-free entry point).
struct AccPair {
    double *J, *K;
};

// dref (optional): an incremental build over the density-screened lists;
// D is then D - Dref and J, K (required) become Jref + J[D], Kref + K[D].
struct DeltaRefs {
    const double *J, *K;
};

static fsim_status enqueue_build(fsim_ctx *c, const double *D, double *F, double *J, double *K,
                                 bool mixed, std::vector<fsim_class_profile> *prof,
                                 hipStream_t s, const AccPair *acc = nullptr,
                                 const DeltaRefs *dref = nullptr) {
    const size_t P = (size_t)c->packed;
    const bool xp = !acc && c->xcd_private && c->priv;
    double *Jsum = acc ? acc->J : c->Jh, *Ksum = acc ? acc->K : c->Kh;
    double *Jacc = xp ? c->priv : Jsum;
    double *Kacc = xp ? c->priv + NXCD * P : Ksum;
    if (xp) {
        HIPCHK(fill(c->priv, 2 * NXCD * P, 0.0, s));
    } else {
        HIPCHK(fill(Jsum, P, 0.0, s));
        HIPCHK(fill(Ksum, P, 0.0, s));
    }
    int nev = 0;
    // s/p classes through the persistent queue kernel when every one of them
    // fits its per-wave LDS stage (the stored-integral digest has its own kernel)
    int pstage = 0;
    bool persist = c->persistent && !(c->stored && !dref);
    if (persist) {
        for (int k = 0; k < PERSIST_SLOTS; ++k) {
            const int X = persist_slot_bra(k);
            const int per_prim = 32 + n_entries(pclass_l1(X), pclass_l2(X)) * 8;   // FP64 boxes
            const int bytes = std::max(1, c->kept[X].kmax) * per_prim;
            pstage = std::max(pstage, (bytes + 15) / 16 * 16);
        }
        persist = pstage <= KO_STAGE_BYTES_MAX;
    }
    PersistArgs pa[2];
    bool have_pa[2] = {false, false};
    const int maxn = *std::max_element(c->mol_n.begin(), c->mol_n.end());
    if (persist) HIPCHK(fill_int(c->pcounter, 2, 0, s));
    // heaviest classes (highest L) first
    for (int X = NPCLASS - 1; X >= 0; --X)
        for (int Y = X; Y >= 0; --Y) {
            ClassLists &cl = c->lists[X][Y];
            const int slot = persist ? persist_slot_of(X, Y) : -1;
            for (int part = 0; part < (mixed ? 2 : 1); ++part) {
                const int li = mixed ? 1 + part : 0;
                const TileList &tl = dref ? cl.delta[li]
                                          : (mixed ? (part == 0 ? cl.mix64 : cl.mix32) : cl.all64);
                if (slot >= 0) {
                    // queued for the persistent launch of this part
                    PersistArgs &q = pa[part];
                    if (!have_pa[part]) {
                        q = PersistArgs{};
                        have_pa[part] = true;
                    }
                    EriArgs &a = q.cls[slot];
                    a = EriArgs{};
                    a.bra = c->kept[X];
                    a.ket = c->kept[Y];
                    a.same_class = X == Y;
                    a.tl = tl;
                    a.D = D;
                    a.Jh = Jacc;
                    a.Kh = Kacc;
                    a.xcd_stride = xp ? (long long)P : 0;
                    a.nbf = c->nbf;
                    a.mol_off = c->d_mol_off;
                    a.mol_n = c->d_mol_n;
                    a.boys = c->boys;
                    a.stage_prims = std::max(1, c->kept[X].kmax);
                    a.stage_bytes = pstage;
                    continue;
                }
                if (tl.ntile == 0) continue;
                if (prof) {
                    const ListStats &ls = mixed ? (part == 0 ? cl.sm64 : cl.sm32) : cl.s64;
                    // delta lists: model counts scaled by the evaluated share
                    const double share = dref ? (double)cl.dnq[li] / std::max<int64_t>(1, ls.nq) : 1.0;
                    fsim_class_profile pr{};
                    pr.bra_class = X;
                    pr.ket_class = Y;
                    pr.fp32 = mixed && part == 1;
                    pr.tiles = tl.ntile;
                    pr.quartets = dref ? cl.dnq[li] : ls.nq;
                    pr.prim_quartets = (int64_t)(ls.npq * share);
                    pr.flops = ls.flops * share;
                    pr.flops_exec = ls.flops_exec * share;
                    prof->push_back(pr);
                    HIPCHK(hipEventRecord(c->ev[nev++], s));
                }
                EriArgs a{};
                a.bra = c->kept[X];
                a.ket = c->kept[Y];
                a.same_class = X == Y;
                a.tl = tl;
                a.D = D;
                a.Jh = Jacc;
                a.Kh = Kacc;
                a.xcd_stride = xp ? (long long)P : 0;
                a.nbf = c->nbf;
                a.mol_off = c->d_mol_off;
                a.mol_n = c->d_mol_n;
                a.boys = c->boys;
                a.kn = c->krow_lds && tl.nseg > 0 ? maxn : 0;
                const int f32 = mixed && part == 1;
                if (c->stored && !dref) {
                    a.out = c->store + c->store_off[X][Y];
                    HIPCHK(launch_digest_stored(X, Y, 4, a, s));
                } else {
                    HIPCHK(launch_eri(X, Y, f32, false, c->variant[X][Y][f32], c->wpb[X][Y][f32],
                                      a, s));
                }
                if (prof) HIPCHK(hipEventRecord(c->ev[nev++], s));
            }
        }
    for (int part = 0; part < 2; ++part) {
        if (!have_pa[part]) continue;
        PersistArgs &q = pa[part];
        q.start[0] = 0;
        int64_t nq = 0, npq = 0;
        double fl = 0.0, flx = 0.0;
        // segment items (blocks of 4 waves keep K' rows in LDS) where the
        // segments average at least 16 tiles, 4 per wave of a block; tile
        // items taken by single waves otherwise.  Measured on the
        // 1024-molecule C/H batch (5.8 tiles per segment): 682 ms per FP64
        // build with segment items, 614 ms with tile items, the waves of a
        // block idling at the ends of its short segments.
        long long qt = 0, qs = 0;
        for (int k = 0; k < PERSIST_SLOTS; ++k) {
            qt += q.cls[k].tl.ntile;
            qs += q.cls[k].tl.nseg;
        }
        q.kn = c->krow_lds && qs > 0 && qt >= 16 * qs ? maxn : 0;
        for (int k = 0; k < PERSIST_SLOTS; ++k) {
            q.cls[k].kn = q.kn;
            q.start[k + 1] = q.start[k] + (q.kn > 0 ? q.cls[k].tl.nseg : q.cls[k].tl.ntile);
            const ClassLists &cl = c->lists[persist_slot_bra(k)][persist_slot_ket(k)];
            const int li = mixed ? 1 + part : 0;
            const ListStats &ls = mixed ? (part == 0 ? cl.sm64 : cl.sm32) : cl.s64;
            const double share = dref ? (double)cl.dnq[li] / std::max<int64_t>(1, ls.nq) : 1.0;
            nq += dref ? cl.dnq[li] : ls.nq;
            npq += (int64_t)(ls.npq * share);
            fl += ls.flops * share;
            flx += ls.flops_exec * share;
        }
        if (q.start[PERSIST_SLOTS] == 0) continue;
        q.counter = c->pcounter + part;
        q.stage_bytes = pstage;
        q.boys = c->boys;
        if (prof) {
            fsim_class_profile pr{};
            pr.bra_class = PERSIST_PROFILE_CLASS;
            pr.ket_class = PERSIST_PROFILE_CLASS;
            pr.fp32 = mixed && part == 1;
            pr.tiles = q.start[PERSIST_SLOTS];
            pr.quartets = nq;
            pr.prim_quartets = npq;
            pr.flops = fl;
            pr.flops_exec = flx;
            prof->push_back(pr);
            HIPCHK(hipEventRecord(c->ev[nev++], s));
        }
        HIPCHK(launch_persistent(mixed && part == 1, q, s));
        if (prof) HIPCHK(hipEventRecord(c->ev[nev++], s));
    }
    if (xp) {
        HIPCHK(sum_copies(P, NXCD, c->priv, P, Jsum, s));
        HIPCHK(sum_copies(P, NXCD, c->priv + NXCD * P, P, Ksum, s));
    }
    if (dref)
        HIPCHK(assemble_delta(layout_of(c), Jsum, Ksum, c->H, dref->J, dref->K, F, J, K, s));
    else
        HIPCHK(assemble_fock_packed(layout_of(c), Jsum, Ksum, c->H, F, J, K, s));
    return FSIM_OK;
}

// E_elec = 1/2 Tr[D (H + F)] summed over the molecules (synchronises s).
static fsim_status electronic_energy(fsim_ctx *c, const double *D, const double *F, double *E,
                                     hipStream_t s) {
    HIPCHK(fill(c->Emol, c->nmol, 0.0, s));
    HIPCHK(dot3_packed(layout_of(c), D, c->H, F, 0.5, c->Emol, s));
    HIPCHK(hipMemcpyAsync(c->Emol_host.data(), c->Emol, sizeof(double) * c->nmol,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double e = 0.0;
    for (double v : c->Emol_host) e += v;
    *E = e;
    return FSIM_OK;
}

// Spherical context: D' -> D = T D' T^T, Cartesian J, K by the class
// kernels, J' = T^T J T, K' = T^T K T, F' = H' + J' - K'/2 (no graph replay).
static fsim_status fock_build_sph(fsim_ctx *c, const double *D, double *F, double *J, double *K,
                                  double *E_elec, bool mixed, hipStream_t s) {
    const int Ns = c->nscf;
    BLASCHK(rocblas_set_stream(c->blas, s));
    STCHK(cart_from_sph(c, D, c->T1));
    HIPCHK(symmetrize(c->nbf, c->T1, c->Dc, s));
    if (c->profiling && c->ev.empty()) {
        c->ev.resize(2 * 2 * NPCLASS * NPCLASS);
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
    }
    if (c->xcd_private && !c->priv) HIPCHK(c->pool.alloc(&c->priv, 2 * NXCD * (size_t)c->packed));
    std::vector<fsim_class_profile> prof;
    STCHK(enqueue_build(c, c->Dc, nullptr, c->Jc, c->Kc, mixed, c->profiling ? &prof : nullptr, s));
    if (c->profiling) {
        HIPCHK(hipStreamSynchronize(s));
        for (size_t k = 0; k < prof.size(); ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
            prof[k].ms = ms;
        }
        c->prof = prof;
    }
    STCHK(sph_from_cart(c, c->Jc, c->T1));
    STCHK(sph_from_cart(c, c->Kc, c->T2));
    HIPCHK(assemble_sym(Ns, c->T1, c->T2, c->H, F, J, K, s));
    if (E_elec) {
        if (!F) return fail(FSIM_EINVAL, "E_elec needs F");
        HIPCHK(fill(c->Emol, 1, 0.0, s));
        HIPCHK(dot3((size_t)Ns * Ns, D, c->H, F, 0.5, c->Emol, s));
        HIPCHK(hipMemcpyAsync(c->Emol_host.data(), c->Emol, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *E_elec = c->Emol_host[0];
    }
    return FSIM_OK;
}

static fsim_status fock_build(fsim_ctx *c, const double *D, double *F, double *J, double *K,
                              double *E_elec, fsim_precision prec, hipStream_t s) {
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before a Fock build");
    if (!D) return fail(FSIM_EINVAL, "D must not be NULL");
    if (c->sph)
        return fock_build_sph(c, D, F, J, K, E_elec, prec == FSIM_MIXED && c->tau32 > 0 && !c->stored,
                              s);
    const size_t P = (size_t)c->packed;
    // a store holds FP64 blocks of every kept quartet: its builds digest those
    const bool mixed = prec == FSIM_MIXED && c->tau32 > 0 && !c->stored;
    if (c->profiling && c->ev.empty()) {
        c->ev.resize(2 * 2 * NPCLASS * NPCLASS);
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
    }
    if (c->xcd_private && !c->priv) HIPCHK(c->pool.alloc(&c->priv, 2 * NXCD * P));
    const bool use_graph = c->graph_enabled && !c->profiling && !J && !K && F;
    if (use_graph) {
        const int g = mixed ? 1 : 0;
        if (!c->gstream) {
            HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
            for (auto &e : c->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            HIPCHK(c->pool.alloc(&c->gD, P));
            HIPCHK(c->pool.alloc(&c->gF, P));
        }
        // order the internal stream after the caller's work
        HIPCHK(hipEventRecord(c->gev[0], s));
        HIPCHK(hipStreamWaitEvent(c->gstream, c->gev[0], 0));
        HIPCHK(hipMemcpyAsync(c->gD, D, sizeof(double) * P, hipMemcpyDeviceToDevice, c->gstream));
        if (!c->gexec[g]) {
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
            fsim_status st = enqueue_build(c, c->gD, c->gF, nullptr, nullptr, mixed, nullptr,
                                           c->gstream);
            hipError_t ec = hipStreamEndCapture(c->gstream, &graph);
            if (st != FSIM_OK) {
                if (graph) hipGraphDestroy(graph);
                return st;
            }
            HIPCHK(ec);
            hipError_t ei = hipGraphInstantiate(&c->gexec[g], graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            HIPCHK(ei);
        }
        HIPCHK(hipGraphLaunch(c->gexec[g], c->gstream));
        HIPCHK(hipMemcpyAsync(F, c->gF, sizeof(double) * P, hipMemcpyDeviceToDevice, c->gstream));
        HIPCHK(hipEventRecord(c->gev[1], c->gstream));
        HIPCHK(hipStreamWaitEvent(s, c->gev[1], 0));
    } else {
        std::vector<fsim_class_profile> prof;
        STCHK(enqueue_build(c, D, F, J, K, mixed, c->profiling ? &prof : nullptr, s));
        if (c->profiling) {
            HIPCHK(hipStreamSynchronize(s));
            for (size_t k = 0; k < prof.size(); ++k) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
                prof[k].ms = ms;
            }
            c->prof = prof;
        }
    }
    if (E_elec) {
        if (!F) return fail(FSIM_EINVAL, "E_elec needs F");
        STCHK(electronic_energy(c, D, F, E_elec, s));
    }
    return FSIM_OK;
}

extern "C" fsim_status fsim_fock_build(fsim_ctx *c, const double *D, double *F, double *J, double *K,
                                       double *E_elec, fsim_precision prec, void *stream) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    hipStream_t s = (hipStream_t)stream;
    double *Fo = F;
    if (!Fo && E_elec) Fo = c->F;
    return fock_build(c, D, Fo, J, K, E_elec, prec, s);
}

extern "C" fsim_status fsim_fock_build_noalloc(fsim_ctx *c, const double *D, double *F, double *J,
                                               double *K, double *E_elec, fsim_precision prec,
                                               void *stream) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (!D) return fail(FSIM_EINVAL, "D must not be NULL");
    if (c->packed > NOALLOC_MAX_PACKED)
        return fail(FSIM_EINVAL, "fsim_fock_build_noalloc: the packed matrix size " +
                                     std::to_string(c->packed) + " exceeds the maximum " +
                                     std::to_string(NOALLOC_MAX_PACKED) +
                                     " (N <= 1448 for one molecule); use fsim_fock_build");
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before a Fock build");
    if (!c->noalloc) return fail(FSIM_ESTATE, "no device scratch for this context's device");
    if (c->sph) return fail(FSIM_EINVAL, "fsim_fock_build_noalloc takes Cartesian contexts only");
    hipStream_t s = (hipStream_t)stream;
    double *Fo = F;
    if (!Fo && E_elec) Fo = c->F;   // context-owned, allocated at create
    const AccPair acc{c->noalloc, c->noalloc + NOALLOC_MAX_PACKED};
    STCHK(enqueue_build(c, D, Fo, J, K, prec == FSIM_MIXED && c->tau32 > 0, nullptr, s, &acc));
    if (E_elec) STCHK(electronic_energy(c, D, Fo, E_elec, s));
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Conventional mode: integrals computed once, digested by every build
// ---------------------------------------------------------------------------

extern "C" fsim_status fsim_store_eris(fsim_ctx *c, int32_t enable, int64_t *bytes) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    drop_graphs(c);
    c->store_pool.clear();
    c->stored = false;
    c->store = nullptr;
    c->store_bytes = 0;
    if (bytes) *bytes = 0;
    if (!enable) return FSIM_OK;
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before storing integrals");
    // sizes: every tile of the FP64 lists, NE components x 64 lanes
    long long total = 0;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const long long ne = (long long)ncart_h(pclass_l1(X)) * ncart_h(pclass_l2(X)) *
                                 ncart_h(pclass_l1(Y)) * ncart_h(pclass_l2(Y));
            c->store_off[X][Y] = total;
            total += (long long)c->lists[X][Y].all64.ntile * ne * TILE;
        }
    size_t freeb = 0, totb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totb));
    const double need = (double)total * sizeof(double);
    if (need > 0.9 * (double)freeb)
        return fail(FSIM_ENOMEM, "stored integrals need " + std::to_string(need / 1e9) +
                                     " GB, more than 90% of the free device memory (" +
                                     std::to_string(freeb / 1e9) + " GB)");
    HIPCHK(c->store_pool.alloc(&c->store, (size_t)std::max(1LL, total)));
    // one store launch per class over its tiles, with the class's tuned FP64
    // kernel; task arrays are built per class on the host
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const ClassLists &cl = c->lists[X][Y];
            const HostList &h = cl.host[0];
            const int nt = cl.all64.ntile;
            if (nt == 0) continue;
            const int nb = ncart_h(pclass_l2(X)), nc = ncart_h(pclass_l1(Y)),
                      nd = ncart_h(pclass_l2(Y));
            const long long ne = (long long)ncart_h(pclass_l1(X)) * nb * nc * nd;
            std::vector<int> tbra(nt), tket((size_t)nt * TILE, -1), tst((size_t)nt * TILE * 4, 0);
            std::vector<long long> toff((size_t)nt * TILE, 0);
            int t = 0;
            for (size_t r = 0; r < h.bra.size(); ++r)
                for (int k0 = h.lo[r]; k0 < h.hi[r]; k0 += TILE, ++t) {
                    tbra[t] = h.bra[r];
                    for (int l = 0; l < TILE && k0 + l < h.hi[r]; ++l) {
                        const size_t q = (size_t)t * TILE + l;
                        tket[q] = k0 + l;
                        toff[q] = c->store_off[X][Y] + (long long)t * ne * TILE + l;
                        tst[4 * q + 0] = nb * nc * nd * TILE;
                        tst[4 * q + 1] = nc * nd * TILE;
                        tst[4 * q + 2] = nd * TILE;
                        tst[4 * q + 3] = TILE;
                    }
                }
            if (t != nt) return fail(FSIM_ESTATE, "internal: tile count mismatch while storing");
            int *dbra = nullptr, *dket = nullptr, *dst = nullptr;
            long long *doff = nullptr;
            DevPool tmp;
            HIPCHK(tmp.alloc(&dbra, tbra.size()));
            HIPCHK(tmp.alloc(&dket, tket.size()));
            HIPCHK(tmp.alloc(&doff, toff.size()));
            HIPCHK(tmp.alloc(&dst, tst.size()));
            HIPCHK(hipMemcpy(dbra, tbra.data(), sizeof(int) * tbra.size(), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(dket, tket.data(), sizeof(int) * tket.size(), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(doff, toff.data(), sizeof(long long) * toff.size(), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(dst, tst.data(), sizeof(int) * tst.size(), hipMemcpyHostToDevice));
            EriArgs a{};
            a.bra = c->kept[X];
            a.ket = c->kept[Y];
            a.same_class = X == Y;
            a.st_ntile = nt;
            a.st_bra = dbra;
            a.st_ket = dket;
            a.st_off = doff;
            a.st_stride = dst;
            a.out = c->store;
            a.boys = c->boys;
            a.nbf = c->nbf;
            HIPCHK(launch_eri(X, Y, false, true, c->variant[X][Y][0], c->wpb[X][Y][0], a, nullptr));
            HIPCHK(hipDeviceSynchronize());
            tmp.clear();
        }
    c->stored = true;
    c->store_bytes = total * (int64_t)sizeof(double);
    if (bytes) *bytes = c->store_bytes;
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Incremental (difference-density) Fock build
// ---------------------------------------------------------------------------

// Density-screened ket ends for every tile list, from M (host, per shell
// pair max |dD|).  A kept quartet (ab|cd) reads dD only in the blocks ab, cd,
// ac, ad, bc and bd, each bounded by max(m_ab, M_cd, R_c, R_d) with R_x the
// largest M in shell row x and m_ab = max(M_ab, R_a, R_b).  With the kets of a
// class Q-sorted, w_k = Q_k max(M_cd, R_c, R_d) and its suffix maximum SW_k,
// every ket j >= k of bra i has Q_i Q_j max|dD blocks| <= Q_i max(SW_k,
// m_i Q_k); the first k where that falls below thr ends the bra's range, so
// only quartets whose density-weighted bound is below thr are skipped.
static fsim_status delta_lists(fsim_ctx *c, double thr, hipStream_t s, int64_t *nq_total) {
    const int ns = c->nshell;
    const std::vector<double> &M = c->Mhost;
    std::vector<double> R(ns, 0.0);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) R[a] = std::max(R[a], M[(size_t)a * ns + b]);
    std::vector<double> mpair[NPCLASS], SW[NPCLASS];
    for (int pc = 0; pc < NPCLASS; ++pc) {
        const size_t n = c->Qkept[pc].size();
        mpair[pc].resize(n);
        SW[pc].assign(n + 1, 0.0);
        for (size_t k = 0; k < n; ++k) {
            const int x = c->kept_s1[pc][k], y = c->kept_s2[pc][k];
            mpair[pc][k] = std::max(M[(size_t)x * ns + y], std::max(R[x], R[y]));
        }
        for (size_t k = n; k-- > 0;)
            SW[pc][k] = std::max(SW[pc][k + 1], c->Qkept[pc][k] * mpair[pc][k]);
    }
    int64_t total = 0;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            ClassLists &cl = c->lists[X][Y];
            const std::vector<double> &Qb = c->Qkept[X], &Qk = c->Qkept[Y];
            for (int li = 0; li < 3; ++li) {
                const HostList &h = cl.host[li];
                TileList &d = cl.delta[li];
                std::vector<int> &st = cl.dstart[li], &hi = cl.dhi[li];
                int64_t nq = 0;
                for (size_t r = 0; r < h.bra.size(); ++r) {
                    const int i = h.bra[r];
                    const double qi = Qb[i], mi = mpair[X][i];
                    int lo = h.lo[r], up = h.hi[r];
                    // first ket whose bound (and every later one's) is below tau
                    while (lo < up) {
                        const int k = (lo + up) / 2;
                        if (qi * std::max(SW[Y][k], mi * Qk[k]) >= thr) lo = k + 1;
                        else up = k;
                    }
                    hi[r] = lo;
                    const int nk = lo - h.lo[r];
                    nq += nk;
                    st[r + 1] = st[r] + (nk + TILE - 1) / TILE;
                }
                d.ntile = h.bra.empty() ? 0 : st.back();
                d.nquartet = nq;
                cl.dnq[li] = nq;
                // segments over the new tile ranges, at the class's segment size
                // (never more than the capacity, cut at the smallest size over
                // the full ranges)
                const size_t cap = cl.dseg[li].size() / 3;
                int *srec = cl.dseg[li].data(), *st0 = srec + cap, *snt = st0 + cap;
                const size_t ns = cap > 0 ? cut_segments(st, c->segt[X][Y][li == 2 ? 1 : 0],
                                                         srec, st0, snt)
                                          : 0;
                d.nseg = (int)ns;
                if (!h.bra.empty()) {
                    HIPCHK(hipMemcpyAsync(d.tile_start, st.data(), sizeof(int) * st.size(),
                                          hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(d.ket_hi, hi.data(), sizeof(int) * hi.size(),
                                          hipMemcpyHostToDevice, s));
                    if (ns > 0) {
                        HIPCHK(hipMemcpyAsync(d.seg_rec, srec, sizeof(int) * ns,
                                              hipMemcpyHostToDevice, s));
                        HIPCHK(hipMemcpyAsync(d.seg_t0, st0, sizeof(int) * ns,
                                              hipMemcpyHostToDevice, s));
                        HIPCHK(hipMemcpyAsync(d.seg_nt, snt, sizeof(int) * ns,
                                              hipMemcpyHostToDevice, s));
                    }
                }
                if (li == 0) total += nq;
            }
        }
    *nq_total = total;
    return FSIM_OK;
}

static fsim_status fock_build_delta_impl(fsim_ctx *c, const double *D, const double *Dref,
                                         const double *Jref, const double *Kref, double *F,
                                         double *J, double *K, double *E_elec, double tau_delta,
                                         int64_t *quartets, fsim_precision prec, hipStream_t s) {
    if (c->nmol != 1) return fail(FSIM_EINVAL, "incremental builds are for one-molecule contexts");
    if (c->sph) return fail(FSIM_EINVAL, "incremental builds take Cartesian contexts only");
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before a Fock build");
    if (!D || !Dref || !Jref || !Kref || !J || !K)
        return fail(FSIM_EINVAL, "D, D_ref, J_ref, K_ref, J and K must not be NULL");
    if (E_elec && !F) return fail(FSIM_EINVAL, "E_elec needs F");
    if (!std::isfinite(tau_delta)) return fail(FSIM_EINVAL, "tau_delta must be finite");
    const double thr = tau_delta > 0 ? tau_delta : c->tau;
    const bool mixed = prec == FSIM_MIXED && c->tau32 > 0;
    const int N = c->nbf, ns = c->nshell;
    HIPCHK(fill(c->Mblk, (size_t)ns * ns, 0.0, s));
    HIPCHK(delta_blockmax(N, D, Dref, c->dD, c->d_bf_shell, ns, c->Mblk, s));
    HIPCHK(hipMemcpyAsync(c->Mhost.data(), c->Mblk, sizeof(double) * c->Mhost.size(),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t nq = 0;
    STCHK(delta_lists(c, thr, s, &nq));
    if (mixed) {
        nq = 0;
        for (int X = 0; X < NPCLASS; ++X)
            for (int Y = 0; Y <= X; ++Y) nq += c->lists[X][Y].dnq[1] + c->lists[X][Y].dnq[2];
    }
    if (c->profiling && c->ev.empty()) {
        c->ev.resize(2 * 2 * NPCLASS * NPCLASS);
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
    }
    if (c->xcd_private && !c->priv) HIPCHK(c->pool.alloc(&c->priv, 2 * NXCD * (size_t)c->packed));
    std::vector<fsim_class_profile> prof;
    const DeltaRefs dref{Jref, Kref};
    STCHK(enqueue_build(c, c->dD, F, J, K, mixed, c->profiling ? &prof : nullptr, s, nullptr,
                        &dref));
    if (c->profiling) {
        HIPCHK(hipStreamSynchronize(s));
        for (size_t k = 0; k < prof.size(); ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
            prof[k].ms = ms;
        }
        c->prof = prof;
    }
    if (quartets) *quartets = nq;
    if (E_elec) STCHK(electronic_energy(c, D, F, E_elec, s));
    return FSIM_OK;
}

extern "C" fsim_status fsim_fock_build_delta(fsim_ctx *c, const double *D, const double *Dref,
                                             const double *Jref, const double *Kref, double *F,
                                             double *J, double *K, double *E_elec,
                                             double tau_delta, int64_t *quartets,
                                             fsim_precision prec, void *stream) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    return fock_build_delta_impl(c, D, Dref, Jref, Kref, F, J, K, E_elec, tau_delta, quartets,
                                 prec, (hipStream_t)stream);
}

extern "C" fsim_status fsim_set_incremental(fsim_ctx *c, int32_t rebuild_every, double tau_delta) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (rebuild_every < 0) return fail(FSIM_EINVAL, "rebuild_every must be >= 0");
    if (!std::isfinite(tau_delta)) return fail(FSIM_EINVAL, "tau_delta must be finite");
    c->inc_tau = tau_delta;
    if (rebuild_every > 0 && c->nmol != 1)
        return fail(FSIM_EINVAL, "incremental builds are for one-molecule contexts");
    if (rebuild_every > 0 && c->sph)
        return fail(FSIM_EINVAL, "incremental builds take Cartesian contexts only");
    if (rebuild_every > 0 && !c->Dref) {
        const size_t P = (size_t)c->packed;
        HIPCHK(c->pool.alloc(&c->Dref, P));
        HIPCHK(c->pool.alloc(&c->Jref, P));
        HIPCHK(c->pool.alloc(&c->Kref, P));
    }
    c->inc_every = rebuild_every;
    c->inc_have = false;
    c->inc_count = 0;
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_profiling(fsim_ctx *c, int32_t enable) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    c->profiling = enable != 0;
    return FSIM_OK;
}

extern "C" fsim_status fsim_get_class_profile(fsim_ctx *c, fsim_class_profile *out, int32_t cap,
                                          int32_t *count) {
    if (!c || !count) return fail(FSIM_EINVAL, "NULL argument");
    *count = (int32_t)c->prof.size();
    if (out)
        for (int32_t k = 0; k < cap && k < *count; ++k) out[k] = c->prof[k];
    return FSIM_OK;
}

// Cut every full tile list's segments again at its class's segment size
// (after a tuning change); the device arrays hold segments of the smallest
// size, so they always fit.  Synchronous copies: not for graph capture.
static fsim_status set_segments(fsim_ctx *c) {
    if (!c->screened) return FSIM_OK;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            ClassLists &cl = c->lists[X][Y];
            TileList *tls[3] = {&cl.all64, &cl.mix64, &cl.mix32};
            for (int k = 0; k < 3; ++k) {
                TileList &tl = *tls[k];
                const size_t cap = (size_t)cl.segcap[k];
                if (tl.nbra == 0 || cap == 0) continue;
                const std::vector<int> st = tile_starts(cl.host[k].lo, cl.host[k].hi);
                std::vector<int> h(3 * cap);
                tl.nseg = (int)cut_segments(st, c->segt[X][Y][k == 2 ? 1 : 0], h.data(),
                                            h.data() + cap, h.data() + 2 * cap);
                HIPCHK(hipMemcpy(tl.seg_rec, h.data(), sizeof(int) * tl.nseg,
                                 hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(tl.seg_t0, h.data() + cap, sizeof(int) * tl.nseg,
                                 hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(tl.seg_nt, h.data() + 2 * cap, sizeof(int) * tl.nseg,
                                 hipMemcpyHostToDevice));
            }
        }
    drop_graphs(c);
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_tuning(fsim_ctx *c, const fsim_tuning *t, int32_t n) {
    if (!c || (n > 0 && !t)) return fail(FSIM_EINVAL, "NULL argument");
    for (int32_t k = 0; k < n; ++k) {
        const fsim_tuning &r = t[k];
        if (r.bra_class < 0 || r.bra_class >= NPCLASS || r.ket_class < 0 ||
            r.ket_class > r.bra_class || (r.fp32 != 0 && r.fp32 != 1))
            return fail(FSIM_EINVAL, "tuning record names no quartet class");
        if (r.variant < 0 || r.variant >= ERI_NVARIANT)
            return fail(FSIM_EINVAL, "variant must be 0.." + std::to_string(ERI_NVARIANT - 1));
        if (r.waves_per_block != 1 && r.waves_per_block != 2 && r.waves_per_block != 4 &&
            r.waves_per_block != 8)
            return fail(FSIM_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
        if (r.seg_tiles != 0 && !valid_seg(r.seg_tiles))
            return fail(FSIM_EINVAL, "seg_tiles must be 0 or a power of 2 in 16..512");
    }
    bool seg_changed = false;
    for (int32_t k = 0; k < n; ++k) {
        const fsim_tuning &r = t[k];
        c->variant[r.bra_class][r.ket_class][r.fp32] = r.variant;
        c->wpb[r.bra_class][r.ket_class][r.fp32] = r.waves_per_block;
        c->tuned_ms[r.bra_class][r.ket_class][r.fp32] = r.ms;
        const int seg = r.seg_tiles ? r.seg_tiles : SEG_TILES;
        seg_changed |= c->segt[r.bra_class][r.ket_class][r.fp32] != seg;
        c->segt[r.bra_class][r.ket_class][r.fp32] = seg;
    }
    if (seg_changed) STCHK(set_segments(c));
    drop_graphs(c);
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_krow_lds(fsim_ctx *c, int32_t enable) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    c->krow_lds = enable != 0;
    drop_graphs(c);
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_prim_screen(fsim_ctx *c, double tau_prim) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (!(tau_prim >= 0) || !std::isfinite(tau_prim))
        return fail(FSIM_EINVAL, "tau_prim must be finite and >= 0");
    c->tau_prim = tau_prim;
    // the kept tables and work lists are rebuilt by the next screen
    drop_graphs(c);
    c->screened = false;
    c->inc_have = false;
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_persistent(fsim_ctx *c, int32_t enable) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (enable && !c->pcounter) HIPCHK(c->pool.alloc(&c->pcounter, 2));
    c->persistent = enable != 0;
    drop_graphs(c);
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_xcd_private(fsim_ctx *c, int32_t enable) {
    if (!c) return fail(FSIM_EINVAL, "NULL argument");
    c->xcd_private = enable != 0;
    drop_graphs(c);
    return FSIM_OK;
}

extern "C" fsim_status fsim_get_tuning(fsim_ctx *c, fsim_tuning *out, int32_t cap, int32_t *n) {
    if (!c || !n) return fail(FSIM_EINVAL, "NULL argument");
    int32_t k = 0;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y)
            for (int f = 0; f < 2; ++f) {
                if (out && k < cap) {
                    fsim_tuning r{};
                    r.bra_class = X;
                    r.ket_class = Y;
                    r.fp32 = f;
                    r.variant = c->variant[X][Y][f];
                    r.waves_per_block = c->wpb[X][Y][f];
                    r.seg_tiles = c->segt[X][Y][f];
                    r.kbra = c->screened ? c->kept[X].kmax : c->all[X].kmax;
                    r.kket = c->screened ? c->kept[Y].kmax : c->all[Y].kmax;
                    r.ms = c->tuned_ms[X][Y][f];
                    out[k] = r;
                }
                ++k;
            }
    *n = k;
    return FSIM_OK;
}

// Chunk count of the one-lane-per-quartet kernel for a class at a budget of
// live values (the kernels' rule: halve the ket pair range, then the bra
// range, until the chunk's accumulators, Hermite intermediates and R fit),
// and whether the budget is met within 24 chunks.
static int lane_chunks(int X, int Y, int limit, bool *fits) {
    const int la = pclass_l1(X), lb = pclass_l2(X), lc = pclass_l1(Y), ld = pclass_l2(Y);
    const int na = ncart(la), ncd = ncart(lc) * ncart(ld);
    auto live = [&](int ca, int cdc) {
        return ca * ncart(lb) * cdc + nherm(la + lb) * cdc + nherm(la + lb + lc + ld);
    };
    int ca = na, cdc = ncd;
    while (live(ca, cdc) > limit) {
        if (cdc > 1) cdc = (cdc + 1) / 2;
        else if (ca > 1) ca = (ca + 1) / 2;
        else break;
    }
    const int n = ((na + ca - 1) / ca) * ((ncd + cdc - 1) / cdc);
    *fits = live(ca, cdc) <= limit && n <= 24;
    return n;
}

// Variant 5 is a kernel of its own (192 live values) for the classes whose
// chunks do not fit 160 or that need fewer chunks at 192; elsewhere it runs
// variant 2 and is not worth timing.
static bool wide_distinct(int X, int Y) {
    bool f160 = false, f192 = false;
    const int n160 = lane_chunks(X, Y, 160, &f160), n192 = lane_chunks(X, Y, 192, &f192);
    return !f160 || (f192 && n192 < n160);
}

extern "C" fsim_status fsim_autotune(fsim_ctx *c, const double *D, fsim_precision prec,
                                     void *stream) {
    if (!c || !D) return fail(FSIM_EINVAL, "NULL argument");
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before autotuning");
    hipStream_t s = (hipStream_t)stream;
    const bool was = c->profiling, was_persistent = c->persistent;
    c->profiling = true;
    c->persistent = false;   // every class is timed in its own launch
    double best[NPCLASS][NPCLASS][2];
    int bv[NPCLASS][NPCLASS][2], bw[NPCLASS][NPCLASS][2];
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y < NPCLASS; ++Y)
            for (int f = 0; f < 2; ++f) {
                best[X][Y][f] = 1e300;
                bv[X][Y][f] = c->variant[X][Y][f];
                bw[X][Y][f] = c->wpb[X][Y][f];
            }
    // 8: segment mode (K' rows in LDS) for the lane kernels
    const int wpbs[4] = {1, 2, 4, 8};
    fsim_status st = FSIM_OK;
    // FSIM_AUTOTUNE_VERBOSE=1: one progress line per timed pass on stderr
    const char *vb = std::getenv("FSIM_AUTOTUNE_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    // one warm-up build
    st = fock_build(c, D, c->F, nullptr, nullptr, nullptr, prec, s);
    for (int v = 0; v < ERI_NVARIANT && st == FSIM_OK; ++v)
        for (int w = 0; w < 4 && st == FSIM_OK; ++w) {
            if ((v == ERI_VARIANT_WAVE || v == ERI_VARIANT_MFMA) && w > 0)
                continue;   // one block shape
            if (v == ERI_VARIANT_WIDE && w != 0 && w != 3)
                continue;   // one wave per block, or segment mode
            if (w == 3 && !c->krow_lds) continue;
            // the wave kernel is only a candidate for the high angular-momentum
            // classes (L >= 5), the ket-outer kernel only for the ss, ps, pp
            // and ds bras, and variant 5 only where it is a kernel of its own;
            // elsewhere those classes keep a lane variant during that pass and
            // are not scored in it
            const bool wave = v == ERI_VARIANT_WAVE, ko = v == ERI_VARIANT_KO,
                       wide = v == ERI_VARIANT_WIDE, mf = v == ERI_VARIANT_MFMA;
            auto Ltot = [](int X, int Y) {
                return pclass_l1(X) + pclass_l2(X) + pclass_l1(Y) + pclass_l2(Y);
            };
            for (int X = 0; X < NPCLASS; ++X)
                for (int Y = 0; Y < NPCLASS; ++Y)
                    for (int f = 0; f < 2; ++f) {
                        const bool cand = (!wave || Ltot(X, Y) >= 5) && (!ko || X <= 3) &&
                                          (!wide || wide_distinct(X, Y)) && (!mf || X >= 3);
                        c->variant[X][Y][f] = cand ? v : ERI_DEFAULT_VARIANT;
                        c->wpb[X][Y][f] = wpbs[w];
                    }
            st = fock_build(c, D, c->F, nullptr, nullptr, nullptr, prec, s);
            if (st != FSIM_OK) break;
            if (verbose) {
                double tot = 0.0;
                for (const auto &r : c->prof) tot += r.ms;
                std::fprintf(stderr, "[fsim_autotune] %s variant %d, %d waves/block: %.1f ms\n",
                             prec == FSIM_MIXED ? "mixed" : "fp64", v, wpbs[w], tot);
                std::fflush(stderr);
            }
            for (const auto &r : c->prof)
                if ((!wave || Ltot(r.bra_class, r.ket_class) >= 5) &&
                    (!ko || r.bra_class <= 3) &&
                    (!wide || wide_distinct(r.bra_class, r.ket_class)) &&
                    (!mf || r.bra_class >= 3) &&
                    r.ms < best[r.bra_class][r.ket_class][r.fp32]) {
                    best[r.bra_class][r.ket_class][r.fp32] = r.ms;
                    bv[r.bra_class][r.ket_class][r.fp32] = v;
                    bw[r.bra_class][r.ket_class][r.fp32] = wpbs[w];
                }
        }
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y < NPCLASS; ++Y)
            for (int f = 0; f < 2; ++f) {
                c->variant[X][Y][f] = bv[X][Y][f];
                c->wpb[X][Y][f] = bw[X][Y][f];
                if (best[X][Y][f] < 1e299) c->tuned_ms[X][Y][f] = best[X][Y][f];
            }
    // segment size of the classes that chose segment mode: every class at
    // its chosen variant, one build per size
    if (st == FSIM_OK && c->krow_lds) {
        const int sizes[4] = {32, 64, 128, 256};
        double sbest[NPCLASS][NPCLASS][2];
        int sz[NPCLASS][NPCLASS][2];
        for (int X = 0; X < NPCLASS; ++X)
            for (int Y = 0; Y < NPCLASS; ++Y)
                for (int f = 0; f < 2; ++f) {
                    sbest[X][Y][f] = 1e300;
                    sz[X][Y][f] = SEG_TILES;
                }
        for (int k = 0; k < 4 && st == FSIM_OK; ++k) {
            for (int X = 0; X < NPCLASS; ++X)
                for (int Y = 0; Y < NPCLASS; ++Y)
                    for (int f = 0; f < 2; ++f) c->segt[X][Y][f] = sizes[k];
            st = set_segments(c);
            if (st != FSIM_OK) break;
            st = fock_build(c, D, c->F, nullptr, nullptr, nullptr, prec, s);
            if (st != FSIM_OK) break;
            if (verbose) {
                double tot = 0.0;
                for (const auto &r : c->prof) tot += r.ms;
                std::fprintf(stderr, "[fsim_autotune] %s segments of %d tiles: %.1f ms\n",
                             prec == FSIM_MIXED ? "mixed" : "fp64", sizes[k], tot);
                std::fflush(stderr);
            }
            for (const auto &r : c->prof)
                if (r.bra_class < NPCLASS && bw[r.bra_class][r.ket_class][r.fp32] == 8 &&
                    r.ms < sbest[r.bra_class][r.ket_class][r.fp32]) {
                    sbest[r.bra_class][r.ket_class][r.fp32] = r.ms;
                    sz[r.bra_class][r.ket_class][r.fp32] = sizes[k];
                }
        }
        for (int X = 0; X < NPCLASS; ++X)
            for (int Y = 0; Y < NPCLASS; ++Y)
                for (int f = 0; f < 2; ++f) {
                    c->segt[X][Y][f] = sz[X][Y][f];
                    if (sbest[X][Y][f] < 1e299) c->tuned_ms[X][Y][f] = sbest[X][Y][f];
                }
        const fsim_status s2 = set_segments(c);
        if (st == FSIM_OK) st = s2;
    }
    c->profiling = was;
    c->persistent = was_persistent;
    drop_graphs(c);
    return st;
}

static fsim_status batched_density(fsim_ctx *c, const double *Fin, double *Dpad, hipStream_t s);

extern "C" fsim_status fsim_core_guess(fsim_ctx *c, double *D, void *stream) {
    if (!c || !D) return fail(FSIM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (c->nmol > 1) {
        STCHK(batched_density(c, c->pH, c->pD, s));
        HIPCHK(unpad_blocks(layout_of(c), c->pD, D, s));
        HIPCHK(hipStreamSynchronize(s));
        return FSIM_OK;
    }
    STCHK(density_from_fock(c, c->H, D, s));
    HIPCHK(hipStreamSynchronize(s));
    return FSIM_OK;
}

extern "C" fsim_status fsim_scf_reset(fsim_ctx *c) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    c->diis_count = 0;
    c->diis_next = 0;
    std::fill(c->Bm.begin(), c->Bm.end(), 0.0);
    std::fill(c->Bb.begin(), c->Bb.end(), 0.0);
    for (auto &r : c->mol_info) r = fsim_scf_info{};
    c->iter = 0;
    c->have_prev = false;
    c->inc_have = false;
    c->inc_count = 0;
    return FSIM_OK;
}

// Solve the bordered DIIS system (Sec. 3.2.1) for m stored pairs by Gaussian
// elimination with partial pivoting.  Returns false when it is singular.
static bool diis_solve(const std::vector<double> &B, int m, const std::vector<int> &slots,
                       int mstride, std::vector<double> &cvec) {
    const int n = m + 1;
    std::vector<double> A((size_t)n * n, 0.0), rhs(n, 0.0);
    double scale = 0.0;
    for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(B[(size_t)slots[i] * mstride + slots[i]]));
    if (!(scale > 0)) return false;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i * n + j] = B[(size_t)slots[i] * mstride + slots[j]] / scale;
        A[i * n + m] = -1.0;
        A[m * n + i] = -1.0;
    }
    A[m * n + m] = 0.0;
    rhs[m] = -1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
        if (std::fabs(A[piv * n + col]) < 1e-14) return false;
        if (piv != col) {
            for (int k = 0; k < n; ++k) std::swap(A[col * n + k], A[piv * n + k]);
            std::swap(rhs[col], rhs[piv]);
        }
        for (int r = col + 1; r < n; ++r) {
            const double f = A[r * n + col] / A[col * n + col];
            for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
            rhs[r] -= f * rhs[col];
        }
    }
    std::vector<double> x(n);
    for (int r = n - 1; r >= 0; --r) {
        double v = rhs[r];
        for (int k = r + 1; k < n; ++k) v -= A[r * n + k] * x[k];
        x[r] = v / A[r * n + r];
    }
    cvec.assign(x.begin(), x.begin() + m);
    for (double v : cvec)
        if (!std::isfinite(v)) return false;
    return true;
}

static fsim_status batched_scf_step(fsim_ctx *c, double *D, fsim_scf_info *info,
                                    fsim_precision prec, hipStream_t s);

extern "C" fsim_status fsim_scf_step(fsim_ctx *c, double *D, fsim_scf_info *info,
                                     fsim_precision prec, void *stream) {
    if (!c || !D || !info) return fail(FSIM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (c->nmol > 1) return batched_scf_step(c, D, info, prec, s);
    const int N = c->nscf;
    const size_t N2 = (size_t)N * N;
    double Eel = 0.0;
    int full = 1;
    int64_t nq = prec == FSIM_MIXED && c->tau32 > 0 ? c->stats.quartets_fp64 + c->stats.quartets_fp32
                                                    : c->stats.quartets_kept;
    if (c->inc_every > 0) {
        if (c->inc_have && c->inc_count < c->inc_every) {
            // F(D) = H + Jref + J[D - Dref] - (Kref + K[D - Dref]) / 2, in place
            STCHK(fock_build_delta_impl(c, D, c->Dref, c->Jref, c->Kref, c->F, c->Jref, c->Kref,
                                        &Eel, c->inc_tau, &nq, prec, s));
            full = 0;
            c->inc_count += 1;
        } else {
            STCHK(fock_build(c, D, c->F, c->Jref, c->Kref, &Eel, prec, s));
            c->inc_have = true;
            c->inc_count = 1;
        }
        HIPCHK(hipMemcpyAsync(c->Dref, D, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    } else {
        STCHK(fock_build(c, D, c->F, nullptr, nullptr, &Eel, prec, s));
    }
    BLASCHK(rocblas_set_stream(c->blas, s));
    // e = F D S - S D F = A - A^T with A = F D S (symmetric F, D, S)
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->F, N, D, N, 0.0, c->T1, N));
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->T1, N, c->S, N, 0.0, c->T2, N));
    const int m = (int)c->dF.size();
    const bool use_diis = c->opt.diis_m > 0;
    const int slot = c->diis_next;
    double *eslot = c->dE[slot];
    HIPCHK(antisym(N, c->T2, eslot, s));
    HIPCHK(hipMemcpyAsync(c->dF[slot], c->F, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    c->diis_next = (slot + 1) % m;
    c->diis_count = std::min(c->diis_count + 1, m);
    // new row of B
    std::vector<int> slots;
    for (int k = 0; k < c->diis_count; ++k) slots.push_back((slot - k + m) % m);
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < c->diis_count; ++k) {
        double v = 0.0;
        BLASCHK(rocblas_set_pointer_mode(c->blas, rocblas_pointer_mode_host));
        BLASCHK(rocblas_ddot(c->blas, (int)N2, eslot, 1, c->dE[slots[k]], 1, &v));
        c->Bm[(size_t)slot * m + slots[k]] = v;
        c->Bm[(size_t)slots[k] * m + slot] = v;
    }
    const double comm = std::sqrt(std::max(0.0, c->Bm[(size_t)slot * m + slot]));
    const double *Fuse = c->F;
    int used = 0;
    if (use_diis && c->diis_count >= 2) {
        std::vector<double> cv;
        if (diis_solve(c->Bm, c->diis_count, slots, m, cv)) {
            DiisPtrs P{};
            for (int k = 0; k < c->diis_count; ++k) {
                P.m[k] = c->dF[slots[k]];
                P.c[k] = cv[k];
            }
            // the J' half-sum buffer is free once F is assembled
            HIPCHK(lincomb(N2, c->diis_count, P, c->Jh, s));
            Fuse = c->Jh;
            used = 1;
        }
    }
    STCHK(density_from_fock(c, Fuse, c->Dn, s));
    HIPCHK(fill(c->scal + 2, 1, 0.0, s));
    HIPCHK(diff2(N2, c->Dn, D, c->scal + 2, s));
    double d2 = 0.0;
    HIPCHK(hipMemcpyAsync(&d2, c->scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(D, c->Dn, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    c->iter += 1;
    const double Etot = Eel + c->enuc;
    info->E_total = Etot;
    info->E_elec = Eel;
    info->dE = c->have_prev ? Etot - c->E_prev : 0.0;
    info->rms_dD = std::sqrt(d2) / N;
    info->comm_norm = comm;
    info->iter = c->iter;
    info->diis_used = used;
    info->full_build = full;
    info->quartets = nq;
    info->converged = info->rms_dD < c->opt.conv_rms_dD &&
                      (c->opt.conv_dE <= 0 || (c->have_prev && std::fabs(info->dE) < c->opt.conv_dE));
    c->have_prev = true;
    c->E_prev = Etot;
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Batched SCF (many molecules): zero-padded N_max blocks, strided-batched
// rocBLAS / rocSOLVER, DIIS per molecule.  The padding of X^T F X gets a
// large distinct diagonal, so its eigenvectors are never occupied and the
// real block's eigenproblem decouples exactly.
// ---------------------------------------------------------------------------
static fsim_status bgemm(fsim_ctx *c, bool ta, bool tb, int k, double alpha, const double *A,
                         const double *B, double beta, double *C) {
    const int M = c->nmax;
    const long long M2 = (long long)M * M;
    BLASCHK(rocblas_dgemm_strided_batched(
        c->blas, ta ? rocblas_operation_transpose : rocblas_operation_none,
        tb ? rocblas_operation_transpose : rocblas_operation_none, M, M, k, &alpha, A, M, M2, B, M,
        M2, &beta, C, M, M2, c->nmol));
    return FSIM_OK;
}

// Dpad = 2 C_occ C_occ^T with C = X V, V the eigenvectors of X^T Fin X
// (padded blocks).  Dpad may alias Fin; scratch pT1, pT2.
static fsim_status batched_density(fsim_ctx *c, const double *Fin, double *Dpad, hipStream_t s) {
    const MolLayout L = layout_of(c);
    const int M = c->nmax;
    const long long M2 = (long long)M * M;
    BLASCHK(rocblas_set_stream(c->blas, s));
    STCHK(bgemm(c, false, false, M, 1.0, Fin, c->pX, 0.0, c->pT1));      // F X
    STCHK(bgemm(c, true, false, M, 1.0, c->pX, c->pT1, 0.0, c->pT2));    // X^T F X
    HIPCHK(pad_diag(L, c->pT2, 1e3, s));
    BLASCHK(rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper, M,
                                             c->pT2, M, M2, c->pEig, M, c->ework, M, c->dinfo,
                                             c->nmol));
    STCHK(bgemm(c, false, false, M, 1.0, c->pX, c->pT2, 0.0, c->pT1));   // C = X V
    HIPCHK(mask_cols(L, c->d_nocc, c->pT1, s));
    STCHK(bgemm(c, false, true, M, 2.0, c->pT1, c->pT1, 0.0, Dpad));
    return FSIM_OK;
}

static fsim_status batched_scf_step(fsim_ctx *c, double *D, fsim_scf_info *info,
                                    fsim_precision prec, hipStream_t s) {
    const MolLayout L = layout_of(c);
    const int nm = c->nmol;
    double Etot_el = 0.0;
    STCHK(fock_build(c, D, c->F, nullptr, nullptr, &Etot_el, prec, s));
    HIPCHK(pad_blocks(L, c->F, c->pF, 0.0, s));
    HIPCHK(pad_blocks(L, D, c->pD, 0.0, s));
    BLASCHK(rocblas_set_stream(c->blas, s));
    // e = F D S - S D F per molecule
    STCHK(bgemm(c, false, false, c->nmax, 1.0, c->pF, c->pD, 0.0, c->pT1));
    STCHK(bgemm(c, false, false, c->nmax, 1.0, c->pT1, c->pS, 0.0, c->pT2));
    const int mh = (int)c->pdF.size();
    const int slot = c->diis_next;
    HIPCHK(antisym_padded(L, c->pT2, c->pdE[slot], s));
    HIPCHK(hipMemcpyAsync(c->pdF[slot], c->pF, sizeof(double) * (size_t)c->nmax * c->nmax * nm,
                          hipMemcpyDeviceToDevice, s));
    c->diis_next = (slot + 1) % mh;
    c->diis_count = std::min(c->diis_count + 1, mh);
    const int cnt = c->diis_count;
    std::vector<int> slots;
    for (int k = 0; k < cnt; ++k) slots.push_back((slot - k + mh) % mh);
    DiisPtrs H{};
    for (int k = 0; k < cnt; ++k) H.m[k] = c->pdE[slots[k]];
    HIPCHK(fill(c->pRed, (size_t)nm * cnt, 0.0, s));
    HIPCHK(dots_padded(L, c->pdE[slot], H, cnt, c->pRed, s));
    std::vector<double> dots((size_t)nm * cnt);
    HIPCHK(hipMemcpyAsync(dots.data(), c->pRed, sizeof(double) * dots.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> coef((size_t)nm * cnt, 0.0), comm(nm, 0.0);
    std::vector<int> used(nm, 0);
    for (int m = 0; m < nm; ++m) {
        double *Bmol = c->Bb.data() + (size_t)m * mh * mh;
        for (int k = 0; k < cnt; ++k) {
            Bmol[(size_t)slot * mh + slots[k]] = dots[(size_t)m * cnt + k];
            Bmol[(size_t)slots[k] * mh + slot] = dots[(size_t)m * cnt + k];
        }
        comm[m] = std::sqrt(std::max(0.0, Bmol[(size_t)slot * mh + slot]));
        coef[(size_t)m * cnt + 0] = 1.0;   // plain F unless DIIS applies
        if (c->opt.diis_m > 0 && cnt >= 2) {
            std::vector<double> Bv(Bmol, Bmol + (size_t)mh * mh), cv;
            if (diis_solve(Bv, cnt, slots, mh, cv)) {
                for (int k = 0; k < cnt; ++k) coef[(size_t)m * cnt + k] = cv[k];
                used[m] = 1;
            }
        }
    }
    DiisPtrs Fh{};
    for (int k = 0; k < cnt; ++k) Fh.m[k] = c->pdF[slots[k]];
    HIPCHK(hipMemcpyAsync(c->pRed, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, s));
    HIPCHK(lincomb_padded(L, Fh, cnt, c->pRed, c->pErr, s));
    STCHK(batched_density(c, c->pErr, c->pErr, s));          // new padded density in pErr
    HIPCHK(fill(c->pRed, nm, 0.0, s));
    HIPCHK(diff2_padded(L, c->pErr, c->pD, c->pRed, s));
    std::vector<double> d2(nm);
    HIPCHK(hipMemcpyAsync(d2.data(), c->pRed, sizeof(double) * nm, hipMemcpyDeviceToHost, s));
    HIPCHK(unpad_blocks(L, c->pErr, D, s));
    HIPCHK(hipStreamSynchronize(s));
    c->iter += 1;
    fsim_scf_info agg{};
    agg.iter = c->iter;
    agg.converged = 1;
    agg.full_build = 1;
    agg.quartets = prec == FSIM_MIXED && c->tau32 > 0 ? c->stats.quartets_fp64 + c->stats.quartets_fp32
                                                      : c->stats.quartets_kept;
    for (int m = 0; m < nm; ++m) {
        fsim_scf_info &r = c->mol_info[m];
        const double E = c->Emol_host[m] + c->mol_enuc[m];
        r.E_elec = c->Emol_host[m];
        r.dE = c->have_prev ? E - c->Eprev_mol[m] : 0.0;
        r.E_total = E;
        r.rms_dD = std::sqrt(d2[m]) / c->mol_n[m];
        r.comm_norm = comm[m];
        r.iter = c->iter;
        r.diis_used = used[m];
        r.full_build = 1;
        r.converged = r.rms_dD < c->opt.conv_rms_dD &&
                      (c->opt.conv_dE <= 0 || (c->have_prev && std::fabs(r.dE) < c->opt.conv_dE));
        c->Eprev_mol[m] = E;
        agg.E_total += E;
        agg.E_elec += r.E_elec;
        agg.dE += r.dE;
        agg.rms_dD = std::max(agg.rms_dD, r.rms_dD);
        agg.comm_norm = std::max(agg.comm_norm, r.comm_norm);
        agg.diis_used += r.diis_used;
        agg.converged = agg.converged && r.converged;
    }
    c->have_prev = true;
    c->E_prev = agg.E_total;
    *info = agg;
    return FSIM_OK;
}

extern "C" fsim_status fsim_batch_layout(const fsim_ctx *c, int32_t *nmol, int32_t *nbf,
                                         int64_t *offsets, double *enuc, int64_t *packed) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (nmol) *nmol = c->nmol;
    for (int m = 0; m < c->nmol; ++m) {
        if (nbf) nbf[m] = c->nmol == 1 ? c->nscf : c->mol_n[m];
        if (offsets) offsets[m] = c->mol_off[m];
        if (enuc) enuc[m] = c->mol_enuc[m];
    }
    if (packed) *packed = c->nmol == 1 ? (int64_t)c->nscf * c->nscf : c->packed;
    return FSIM_OK;
}

extern "C" fsim_status fsim_batch_energies(const fsim_ctx *c, double *E_elec) {
    if (!c || !E_elec) return fail(FSIM_EINVAL, "NULL argument");
    for (int m = 0; m < c->nmol; ++m) E_elec[m] = c->Emol_host[m];
    return FSIM_OK;
}

extern "C" fsim_status fsim_batch_scf_info(const fsim_ctx *c, fsim_scf_info *info) {
    if (!c || !info) return fail(FSIM_EINVAL, "NULL argument");
    if (c->nmol == 1) return fail(FSIM_ESTATE, "not a batched context");
    for (int m = 0; m < c->nmol; ++m) info[m] = c->mol_info[m];
    return FSIM_OK;
}

extern "C" fsim_status fsim_set_graph(fsim_ctx *c, int32_t enable) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    c->graph_enabled = enable != 0;
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// McWeeny purification (one molecule)
// ---------------------------------------------------------------------------
extern "C" fsim_status fsim_purify(fsim_ctx *c, double *D, int32_t iters, double *err_in,
                                   double *err_out, void *stream) {
    if (!c || !D) return fail(FSIM_EINVAL, "NULL argument");
    if (c->nmol != 1) return fail(FSIM_EINVAL, "purification is for one-molecule contexts");
    if (iters < 0) return fail(FSIM_EINVAL, "iters must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int N = c->nscf;
    const size_t N2 = (size_t)N * N;
    BLASCHK(rocblas_set_stream(c->blas, s));
    // work on P = D / 2 in Dn
    auto measure = [&](double *P, double &err) -> fsim_status {
        STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->S, N, P, N, 0.0, c->T1, N));   // S P
        STCHK(gemm(c->blas, false, false, N, N, N, 1.0, P, N, c->T1, N, 0.0, c->T2, N));  // P S P
        HIPCHK(fill(c->scal + 3, 2, 0.0, s));
        HIPCHK(diff2(N2, c->T2, P, c->scal + 3, s));
        HIPCHK(dot3(N2, P, P, nullptr, 1.0, c->scal + 4, s));
        double h[2];
        HIPCHK(hipMemcpyAsync(h, c->scal + 3, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        err = std::sqrt(h[0]) / std::max(std::sqrt(h[1]), 1e-300);
        return FSIM_OK;
    };
    HIPCHK(hipMemcpyAsync(c->Dn, D, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    {
        const double half = 0.5;
        BLASCHK(rocblas_dscal(c->blas, (int)N2, &half, c->Dn, 1));
    }
    double err = 0.0;
    STCHK(measure(c->Dn, err));
    if (err_in) *err_in = err;
    for (int it = 0; it < iters && err >= 1e-12 && std::isfinite(err); ++it) {
        // T2 = PSP, T1 = SP from measure; Jh = PSP S P; P <- 3 PSP - 2 PSPSP
        STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->T2, N, c->T1, N, 0.0, c->Jh, N));
        HIPCHK(hipMemcpyAsync(c->Dn, c->T2, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
        const double three = 3.0, mtwo = -2.0;
        BLASCHK(rocblas_dscal(c->blas, (int)N2, &three, c->Dn, 1));
        BLASCHK(rocblas_daxpy(c->blas, (int)N2, &mtwo, c->Jh, 1, c->Dn, 1));
        STCHK(measure(c->Dn, err));
    }
    if (err_out) *err_out = err;
    HIPCHK(hipMemcpyAsync(D, c->Dn, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    {
        const double two = 2.0;
        BLASCHK(rocblas_dscal(c->blas, (int)N2, &two, D, 1));
    }
    HIPCHK(hipStreamSynchronize(s));
    return FSIM_OK;
}
