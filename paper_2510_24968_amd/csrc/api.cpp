// Host side of libfsim: the C ABI of include/fsim.h, input validation, the
// context (device tables and buffers), Schwarz screening and quartet work
// lists, the Fock-build launch sequence and the SCF step.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fsim.h"
#include "fsim_internal.h"
#include "linalg.h"

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
    double flops = 0.0;
};
struct ClassLists {
    TileList all64, mix64, mix32;
    ListStats s64, sm64, sm32;
};

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
    std::vector<int> sh_atom, sh_l, sh_nprim, sh_prim0, sh_bf0;
    double enuc = 0.0;

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
    ClassLists lists[NPCLASS][NPCLASS];
    fsim_screen_stats stats{};
    std::vector<double> Qmat;

    // work buffers
    double *Jh = nullptr, *Kh = nullptr, *F = nullptr, *Dn = nullptr, *T1 = nullptr, *T2 = nullptr;
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

static int ncart_h(int l) { return (l + 1) * (l + 2) / 2; }

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
    BLASCHK(rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_upper, c->nbf, A,
                             c->nbf, w, c->ework, c->dinfo));
    return FSIM_OK;
}

// D = 2 C_occ C_occ^T with C = X V, V the eigenvectors of X^T F X.
static fsim_status density_from_fock(fsim_ctx *c, const double *Fm, double *Dout, hipStream_t s) {
    const int N = c->nbf;
    BLASCHK(rocblas_set_stream(c->blas, s));
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, Fm, N, c->X, N, 0.0, c->T1, N));   // F X
    STCHK(gemm(c->blas, true, false, N, N, N, 1.0, c->X, N, c->T1, N, 0.0, c->T2, N));  // X^T F X
    STCHK(syevd(c, c->T2, c->eig, s));
    STCHK(gemm(c->blas, false, false, N, N, N, 1.0, c->X, N, c->T2, N, 0.0, c->T1, N));  // C
    STCHK(gemm(c->blas, false, true, N, N, c->nocc, 2.0, c->T1, N, c->T1, N, 0.0, Dout, N));
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
    return FSIM_OK;
}

extern "C" fsim_status fsim_ctx_create(const fsim_basis *b, const fsim_options *o, fsim_ctx **out) {
    if (!out) return fail(FSIM_EINVAL, "out must not be NULL");
    *out = nullptr;
    STCHK(validate(b, o));
    fsim_ctx *c = new fsim_ctx();
    auto cleanup = [&](fsim_status st) {
        fsim_ctx_destroy(c);
        return st;
    };
    HIPCHK(hipGetDevice(&c->device));
    c->opt = *o;
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y < NPCLASS; ++Y)
            for (int f = 0; f < 2; ++f) {
                c->variant[X][Y][f] = ERI_DEFAULT_VARIANT;
                c->wpb[X][Y][f] = 4;
                c->tuned_ms[X][Y][f] = 0.0;
            }
    c->natom = b->natom;
    c->nshell = b->nshell;
    c->nelec = b->nelec;
    c->nocc = b->nelec / 2;
    c->xyz.assign(b->xyz, b->xyz + 3 * b->natom);
    c->Z.assign(b->Z, b->Z + b->natom);
    c->sh_atom.assign(b->shell_atom, b->shell_atom + b->nshell);
    c->sh_l.assign(b->shell_l, b->shell_l + b->nshell);
    c->sh_nprim.assign(b->shell_nprim, b->shell_nprim + b->nshell);
    c->sh_prim0.assign(b->shell_prim0, b->shell_prim0 + b->nshell);
    int nprim_tot = 0;
    for (int s = 0; s < c->nshell; ++s)
        nprim_tot = std::max(nprim_tot, c->sh_prim0[s] + c->sh_nprim[s]);
    c->exps.assign(b->exps, b->exps + nprim_tot);
    c->coefs.assign(b->coefs, b->coefs + nprim_tot);
    c->sh_bf0.resize(c->nshell);
    int nbf = 0;
    std::vector<int> bf_shell, bf_comp;
    for (int s = 0; s < c->nshell; ++s) {
        c->sh_bf0[s] = nbf;
        for (int k = 0; k < ncart_h(c->sh_l[s]); ++k) {
            bf_shell.push_back(s);
            bf_comp.push_back(k);
        }
        nbf += ncart_h(c->sh_l[s]);
    }
    c->nbf = nbf;
    const int N = nbf;
    const size_t N2 = (size_t)N * N;

    // nuclear repulsion
    double en = 0.0;
    for (int A = 0; A < c->natom; ++A)
        for (int B = 0; B < A; ++B) {
            const double dx = c->xyz[3 * A] - c->xyz[3 * B], dy = c->xyz[3 * A + 1] - c->xyz[3 * B + 1],
                         dz = c->xyz[3 * A + 2] - c->xyz[3 * B + 2];
            en += c->Z[A] * c->Z[B] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    c->enuc = en;

    // shells on the device
    std::vector<double> shxyz(3 * c->nshell);
    for (int s = 0; s < c->nshell; ++s)
        for (int d = 0; d < 3; ++d) shxyz[3 * s + d] = c->xyz[3 * c->sh_atom[s] + d];
    ShellsDev &sh = c->sh;
    sh.nshell = c->nshell;
    sh.natom = c->natom;
    fsim_status st;
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
    PCHK(c->pool.alloc(&sh.xyz, 3 * c->nshell));
    PCHK(c->pool.alloc(&sh.l, c->nshell));
    PCHK(c->pool.alloc(&sh.nprim, c->nshell));
    PCHK(c->pool.alloc(&sh.prim0, c->nshell));
    PCHK(c->pool.alloc(&sh.bf0, c->nshell));
    PCHK(c->pool.alloc(&sh.exps, nprim_tot));
    PCHK(c->pool.alloc(&sh.coef, nprim_tot));
    PCHK(c->pool.alloc(&sh.atom_xyz, 3 * c->natom));
    PCHK(c->pool.alloc(&sh.atom_Z, c->natom));
    HCHK(hipMemcpy(sh.xyz, shxyz.data(), sizeof(double) * shxyz.size(), hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.l, c->sh_l.data(), sizeof(int) * c->nshell, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.nprim, c->sh_nprim.data(), sizeof(int) * c->nshell, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.prim0, c->sh_prim0.data(), sizeof(int) * c->nshell, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.bf0, c->sh_bf0.data(), sizeof(int) * c->nshell, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.exps, c->exps.data(), sizeof(double) * nprim_tot, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.coef, c->coefs.data(), sizeof(double) * nprim_tot, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.atom_xyz, c->xyz.data(), sizeof(double) * 3 * c->natom, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(sh.atom_Z, c->Z.data(), sizeof(double) * c->natom, hipMemcpyHostToDevice));
    HCHK(launch_shell_norm(sh, nullptr));
    PCHK(c->pool.alloc(&c->boys, (size_t)BOYS_NT * BOYS_NORD));
    HCHK(launch_boys_table(c->boys, nullptr));

    // every shell pair, oriented so that l(s1) >= l(s2)
    for (int a = 0; a < c->nshell; ++a)
        for (int bb = 0; bb <= a; ++bb) {
            int s1 = a, s2 = bb;
            if (c->sh_l[s1] < c->sh_l[s2]) std::swap(s1, s2);
            const int pc = pclass(c->sh_l[s1], c->sh_l[s2]);
            c->pair_lookup[(long long)s1 * c->nshell + s2] = {pc, (int)c->all_s1[pc].size()};
            c->all_s1[pc].push_back(s1);
            c->all_s2[pc].push_back(s2);
        }
    for (int pc = 0; pc < NPCLASS; ++pc) {
        st = build_table(c, c->pool, c->all[pc], pc, c->all_s1[pc], c->all_s2[pc]);
        if (st != FSIM_OK) return cleanup(st);
    }

    // work buffers
    PCHK(c->pool.alloc(&c->S, N2));
    PCHK(c->pool.alloc(&c->H, N2));
    PCHK(c->pool.alloc(&c->X, N2));
    PCHK(c->pool.alloc(&c->Jh, N2));
    PCHK(c->pool.alloc(&c->Kh, N2));
    PCHK(c->pool.alloc(&c->F, N2));
    PCHK(c->pool.alloc(&c->Dn, N2));
    PCHK(c->pool.alloc(&c->T1, N2));
    PCHK(c->pool.alloc(&c->T2, N2));
    PCHK(c->pool.alloc(&c->eig, N));
    PCHK(c->pool.alloc(&c->ework, N));
    PCHK(c->pool.alloc(&c->scal, 8));
    PCHK(c->pool.alloc(&c->dinfo, 4));
    if (rocblas_create_handle(&c->blas) != rocblas_status_success)
        return cleanup(fail(FSIM_EHIP, "rocblas_create_handle failed"));

    // one-electron matrices
    int *dbs = nullptr, *dbc = nullptr;
    PCHK(c->pool.alloc(&dbs, N));
    PCHK(c->pool.alloc(&dbc, N));
    HCHK(hipMemcpy(dbs, bf_shell.data(), sizeof(int) * N, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(dbc, bf_comp.data(), sizeof(int) * N, hipMemcpyHostToDevice));
    HCHK(launch_one_electron_impl(sh, c->boys, N, dbs, dbc, c->S, c->T1, c->T2, nullptr));
    HCHK(hipMemcpy(c->H, c->T1, sizeof(double) * N2, hipMemcpyDeviceToDevice));
    if (rocblas_daxpy(c->blas, (int)N2, std::vector<double>{1.0}.data(), c->T2, 1, c->H, 1) !=
        rocblas_status_success)
        return cleanup(fail(FSIM_EHIP, "rocblas_daxpy failed"));
    c->pool.release(dbs);
    c->pool.release(dbc);

    // X = U s^-1/2 U^T
    HCHK(hipMemcpy(c->T1, c->S, sizeof(double) * N2, hipMemcpyDeviceToDevice));
    st = syevd(c, c->T1, c->eig, nullptr);
    if (st != FSIM_OK) return cleanup(st);
    std::vector<double> sv(N);
    HCHK(hipMemcpy(sv.data(), c->eig, sizeof(double) * N, hipMemcpyDeviceToHost));
    if (!(sv[0] > 1e-10))
        return cleanup(fail(FSIM_EINVAL, "overlap matrix is (near) singular: lowest eigenvalue " +
                                             std::to_string(sv[0])));
    HCHK(inv_sqrt(N, c->eig, c->ework, nullptr));
    HCHK(scale_cols(N, c->T1, c->ework, c->T2, nullptr));
    st = gemm(c->blas, false, true, N, N, N, 1.0, c->T2, N, c->T1, N, 0.0, c->X, N);
    if (st != FSIM_OK) return cleanup(st);
    HCHK(hipDeviceSynchronize());

    const int m = std::max(1, c->opt.diis_m);
    c->dF.resize(m, nullptr);
    c->dE.resize(m, nullptr);
    for (int k = 0; k < m; ++k) {
        PCHK(c->pool.alloc(&c->dF[k], N2));
        PCHK(c->pool.alloc(&c->dE[k], N2));
    }
    c->Bm.assign((size_t)m * m, 0.0);
#undef PCHK
#undef HCHK
    *out = c;
    return FSIM_OK;
}

extern "C" fsim_status fsim_ctx_destroy(fsim_ctx *c) {
    if (!c) return FSIM_OK;
    hipDeviceSynchronize();
    if (c->blas) rocblas_destroy_handle(c->blas);
    for (auto &e : c->ev) hipEventDestroy(e);
    c->screen_pool.clear();
    c->pool.clear();
    delete c;
    return FSIM_OK;
}

extern "C" fsim_status fsim_nbf(const fsim_ctx *c, int32_t *nbf, int32_t *nshell) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (nbf) *nbf = c->nbf;
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
    const size_t bytes = sizeof(double) * c->nbf * c->nbf;
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
// all-pairs tables.
static fsim_status run_store(fsim_ctx *c, std::vector<StoreTask> (&tasks)[NPCLASS][NPCLASS],
                             double *out, bool fp32, hipStream_t s) {
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
            HIPCHK(launch_eri(X, Y, fp32, true, ERI_DEFAULT_VARIANT, 4, a, s));
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
    return run_store(c, tasks, out, prec == FSIM_MIXED, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Schwarz screening and work lists
// ---------------------------------------------------------------------------

static double flops_per_prim_quartet(int la, int lb, int lc, int ld) {
    // algorithmic model (FMA = 2): source + Boys ~ 60 + 3(L+1), R recursion,
    // W over ket boxes x bra Hermite set, block from bra boxes (per ket box set)
    const int L = la + lb + lc + ld;
    double rec = 0;
    for (int n = 0; n < L; ++n)
        for (int s = 1; s <= L - n; ++s) rec += (s + 1) * (s + 2) / 2;
    const double step1 = (double)n_entries(lc, ld) * nherm(la + lb);
    const double step2 = (double)n_entries(la, lb) * ncart_h(lc) * ncart_h(ld);
    return 60.0 + 3.0 * (L + 1) + 2.0 * rec + 2.0 * step1 + 2.0 * step2;
}

static fsim_status upload_list(DevPool &pool, TileList &tl, const std::vector<int> &bra,
                               const std::vector<int> &lo, const std::vector<int> &hi) {
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
    return FSIM_OK;
}

extern "C" fsim_status fsim_schwarz_screen(fsim_ctx *c, double tau, double tau32, double *Q_out,
                                           fsim_screen_stats *stats) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    if (!(tau >= 0) || !(tau32 >= 0) || !std::isfinite(tau) || !std::isfinite(tau32))
        return fail(FSIM_EINVAL, "thresholds must be finite and >= 0");
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
    STCHK(run_store(c, tasks, dblk, false, nullptr));
    std::vector<double> blk(base[NPCLASS]);
    HIPCHK(hipMemcpy(blk.data(), dblk, sizeof(double) * blk.size(), hipMemcpyDeviceToHost));
    hipFree(dblk);
    c->Qmat.assign((size_t)ns * ns, 0.0);
    std::vector<double> Qpair[NPCLASS];
    double Qmax = 0.0;
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
            Qmax = std::max(Qmax, qv);
            const int s1 = c->all_s1[pc][i], s2 = c->all_s2[pc][i];
            c->Qmat[(size_t)s1 * ns + s2] = qv;
            c->Qmat[(size_t)s2 * ns + s1] = qv;
        }
    }
    // kept pairs, sorted by Q (descending; ties by canonical index)
    c->screen_pool.clear();
    c->screened = false;
    fsim_screen_stats S{};
    for (int pc = 0; pc < NPCLASS; ++pc) S.shell_pairs += c->all[pc].n;
    std::vector<int> order[NPCLASS];
    for (int pc = 0; pc < NPCLASS; ++pc) {
        for (int i = 0; i < c->all[pc].n; ++i)
            if (Qpair[pc][i] * Qmax >= tau) order[pc].push_back(i);
        std::stable_sort(order[pc].begin(), order[pc].end(),
                         [&](int a, int b) { return Qpair[pc][a] > Qpair[pc][b]; });
        std::vector<int> s1, s2;
        c->Qkept[pc].clear();
        for (int i : order[pc]) {
            s1.push_back(c->all_s1[pc][i]);
            s2.push_back(c->all_s2[pc][i]);
            c->Qkept[pc].push_back(Qpair[pc][i]);
        }
        STCHK(build_table(c, c->screen_pool, c->kept[pc], pc, s1, s2));
        if (c->kept[pc].n)
            HIPCHK(hipMemcpy(c->kept[pc].Q, c->Qkept[pc].data(), sizeof(double) * c->kept[pc].n,
                             hipMemcpyHostToDevice));
        S.pairs_kept += c->kept[pc].n;
    }
    // canonical quartet count over all pairs
    const long long npair = S.shell_pairs;
    S.quartets_total = npair * (npair + 1) / 2;
    // work lists
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const auto &Qb = c->Qkept[X], &Qk = c->Qkept[Y];
            std::vector<int> b64, lo64, hi64, bm64, lom64, him64, bm32, lom32, him32;
            const int la = pclass_l1(X), lb = pclass_l2(X), lc = pclass_l1(Y), ld = pclass_l2(Y);
            const double fpq = flops_per_prim_quartet(la, lb, lc, ld);
            for (int i = 0; i < (int)Qb.size(); ++i) {
                const double qi = Qb[i];
                // n = #{j : qi * Qk[j] >= tau}, Qk descending
                int lo = 0, hi = (int)Qk.size();
                while (lo < hi) {
                    const int mid = (lo + hi) / 2;
                    if (qi * Qk[mid] >= tau) lo = mid + 1;
                    else hi = mid;
                }
                int n = lo;
                if (X == Y) n = std::min(n, i + 1);
                if (n <= 0) continue;
                int m = n;
                if (tau32 > 0) {
                    int l2 = 0, h2 = n;
                    while (l2 < h2) {
                        const int mid = (l2 + h2) / 2;
                        if (qi * Qk[mid] >= tau32) l2 = mid + 1;
                        else h2 = mid;
                    }
                    m = l2;
                }
                b64.push_back(i);
                lo64.push_back(0);
                hi64.push_back(n);
                if (m > 0) {
                    bm64.push_back(i);
                    lom64.push_back(0);
                    him64.push_back(m);
                }
                if (n > m) {
                    bm32.push_back(i);
                    lom32.push_back(m);
                    him32.push_back(n);
                }
                // primitive-quartet count and flop model (uniform K per pair here:
                // take this bra's product count times the kets' average)
                S.quartets_fp64 += m;
                S.quartets_fp32 += n - m;
            }
            ClassLists &cl = c->lists[X][Y];
            STCHK(upload_list(c->screen_pool, cl.all64, b64, lo64, hi64));
            STCHK(upload_list(c->screen_pool, cl.mix64, bm64, lom64, him64));
            STCHK(upload_list(c->screen_pool, cl.mix32, bm32, lom32, him32));
            S.quartets_kept += cl.all64.nquartet;
            // primitive quartets: sum over kept quartets of K_bra * K_ket
            std::vector<int> kb(Qb.size()), kk(Qk.size());
            {
                std::vector<int> ob = order[X], ok = order[Y];
                for (size_t i = 0; i < ob.size(); ++i)
                    kb[i] = c->sh_nprim[c->all_s1[X][ob[i]]] * c->sh_nprim[c->all_s2[X][ob[i]]];
                for (size_t i = 0; i < ok.size(); ++i)
                    kk[i] = c->sh_nprim[c->all_s1[Y][ok[i]]] * c->sh_nprim[c->all_s2[Y][ok[i]]];
            }
            std::vector<long long> kpre(kk.size() + 1, 0);
            for (size_t j = 0; j < kk.size(); ++j) kpre[j + 1] = kpre[j] + kk[j];
            cl.s64 = cl.sm64 = cl.sm32 = ListStats{};
            for (size_t t = 0; t < b64.size(); ++t) {
                const long long pq = (long long)kb[b64[t]] * (kpre[hi64[t]] - kpre[lo64[t]]);
                S.prim_quartets_kept += pq;
                S.flops_fp64 += fpq * pq;
                cl.s64.npq += pq;
                cl.s64.flops += fpq * pq;
            }
            cl.s64.nq = cl.all64.nquartet;
            for (size_t t = 0; t < bm64.size(); ++t) {
                const long long pq = (long long)kb[bm64[t]] * (kpre[him64[t]] - kpre[lom64[t]]);
                S.flops_mixed_fp64 += fpq * pq;
                cl.sm64.npq += pq;
                cl.sm64.flops += fpq * pq;
            }
            cl.sm64.nq = cl.mix64.nquartet;
            for (size_t t = 0; t < bm32.size(); ++t) {
                const long long pq = (long long)kb[bm32[t]] * (kpre[him32[t]] - kpre[lom32[t]]);
                S.flops_mixed_fp32 += fpq * pq;
                cl.sm32.npq += pq;
                cl.sm32.flops += fpq * pq;
            }
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
    if (Q_out)
        HIPCHK(hipMemcpy(Q_out, c->Qmat.data(), sizeof(double) * ns * ns, hipMemcpyHostToDevice));
    if (stats) *stats = S;
    return FSIM_OK;
}

// ---------------------------------------------------------------------------
// Fock build
// ---------------------------------------------------------------------------

static fsim_status fock_build(fsim_ctx *c, const double *D, double *F, double *J, double *K,
                              double *E_elec, fsim_precision prec, hipStream_t s) {
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before a Fock build");
    if (!D) return fail(FSIM_EINVAL, "D must not be NULL");
    const int N = c->nbf;
    const size_t N2 = (size_t)N * N;
    HIPCHK(fill(c->Jh, N2, 0.0, s));
    HIPCHK(fill(c->Kh, N2, 0.0, s));
    const bool mixed = prec == FSIM_MIXED && c->tau32 > 0;
    std::vector<fsim_class_profile> prof;
    int nev = 0;
    if (c->profiling && c->ev.empty()) {
        c->ev.resize(2 * 2 * NPCLASS * NPCLASS);
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
    }
    // heaviest classes (highest L) first
    for (int X = NPCLASS - 1; X >= 0; --X)
        for (int Y = X; Y >= 0; --Y) {
            ClassLists &cl = c->lists[X][Y];
            for (int part = 0; part < (mixed ? 2 : 1); ++part) {
                const TileList &tl = mixed ? (part == 0 ? cl.mix64 : cl.mix32) : cl.all64;
                if (tl.ntile == 0) continue;
                if (c->profiling) {
                    const ListStats &ls = mixed ? (part == 0 ? cl.sm64 : cl.sm32) : cl.s64;
                    fsim_class_profile pr{};
                    pr.bra_class = X;
                    pr.ket_class = Y;
                    pr.fp32 = mixed && part == 1;
                    pr.tiles = tl.ntile;
                    pr.quartets = ls.nq;
                    pr.prim_quartets = ls.npq;
                    pr.flops = ls.flops;
                    prof.push_back(pr);
                    HIPCHK(hipEventRecord(c->ev[nev++], s));
                }
                EriArgs a{};
                a.bra = c->kept[X];
                a.ket = c->kept[Y];
                a.same_class = X == Y;
                a.tl = tl;
                a.D = D;
                a.Jh = c->Jh;
                a.Kh = c->Kh;
                a.nbf = N;
                a.boys = c->boys;
                const int f32 = mixed && part == 1;
                HIPCHK(launch_eri(X, Y, f32, false, c->variant[X][Y][f32], c->wpb[X][Y][f32], a, s));
                if (c->profiling) HIPCHK(hipEventRecord(c->ev[nev++], s));
            }
        }
    HIPCHK(assemble_fock(N, c->Jh, c->Kh, c->H, F, J, K, s));
    if (c->profiling) {
        HIPCHK(hipStreamSynchronize(s));
        for (size_t k = 0; k < prof.size(); ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
            prof[k].ms = ms;
        }
        c->prof = prof;
    }
    if (E_elec) {
        if (!F) return fail(FSIM_EINVAL, "E_elec needs F");
        HIPCHK(fill(c->scal, 1, 0.0, s));
        HIPCHK(dot3(N2, D, c->H, F, 0.5, c->scal, s));
        HIPCHK(hipMemcpyAsync(E_elec, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
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

extern "C" fsim_status fsim_set_tuning(fsim_ctx *c, const fsim_tuning *t, int32_t n) {
    if (!c || (n > 0 && !t)) return fail(FSIM_EINVAL, "NULL argument");
    for (int32_t k = 0; k < n; ++k) {
        const fsim_tuning &r = t[k];
        if (r.bra_class < 0 || r.bra_class >= NPCLASS || r.ket_class < 0 ||
            r.ket_class > r.bra_class || (r.fp32 != 0 && r.fp32 != 1))
            return fail(FSIM_EINVAL, "tuning record names no quartet class");
        if (r.variant < 0 || r.variant >= ERI_NVARIANT)
            return fail(FSIM_EINVAL, "variant must be 0..3");
        if (r.waves_per_block != 1 && r.waves_per_block != 2 && r.waves_per_block != 4)
            return fail(FSIM_EINVAL, "waves_per_block must be 1, 2 or 4");
    }
    for (int32_t k = 0; k < n; ++k) {
        const fsim_tuning &r = t[k];
        c->variant[r.bra_class][r.ket_class][r.fp32] = r.variant;
        c->wpb[r.bra_class][r.ket_class][r.fp32] = r.waves_per_block;
        c->tuned_ms[r.bra_class][r.ket_class][r.fp32] = r.ms;
    }
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

extern "C" fsim_status fsim_autotune(fsim_ctx *c, const double *D, fsim_precision prec,
                                     void *stream) {
    if (!c || !D) return fail(FSIM_EINVAL, "NULL argument");
    if (!c->screened) return fail(FSIM_ESTATE, "fsim_schwarz_screen must run before autotuning");
    hipStream_t s = (hipStream_t)stream;
    const bool was = c->profiling;
    c->profiling = true;
    double best[NPCLASS][NPCLASS][2];
    int bv[NPCLASS][NPCLASS][2], bw[NPCLASS][NPCLASS][2];
    for (int X = 0; X < NPCLASS; ++X)
        for (int Y = 0; Y < NPCLASS; ++Y)
            for (int f = 0; f < 2; ++f) {
                best[X][Y][f] = 1e300;
                bv[X][Y][f] = c->variant[X][Y][f];
                bw[X][Y][f] = c->wpb[X][Y][f];
            }
    const int wpbs[3] = {1, 2, 4};
    fsim_status st = FSIM_OK;
    // one warm-up build
    st = fock_build(c, D, c->F, nullptr, nullptr, nullptr, prec, s);
    for (int v = 0; v < ERI_NVARIANT && st == FSIM_OK; ++v)
        for (int w = 0; w < 3 && st == FSIM_OK; ++w) {
            if (v == ERI_NVARIANT - 1 && w > 0) break;   // the wave kernel ignores it
            // the wave kernel is only a candidate for the high angular-momentum
            // classes (L >= 5); elsewhere it is far slower, so those classes keep
            // a lane variant during that pass and are not scored in it
            const bool wave = v == ERI_NVARIANT - 1;
            auto Ltot = [](int X, int Y) {
                return pclass_l1(X) + pclass_l2(X) + pclass_l1(Y) + pclass_l2(Y);
            };
            for (int X = 0; X < NPCLASS; ++X)
                for (int Y = 0; Y < NPCLASS; ++Y)
                    for (int f = 0; f < 2; ++f) {
                        const bool cand = !wave || Ltot(X, Y) >= 5;
                        c->variant[X][Y][f] = cand ? v : ERI_DEFAULT_VARIANT;
                        c->wpb[X][Y][f] = wpbs[w];
                    }
            st = fock_build(c, D, c->F, nullptr, nullptr, nullptr, prec, s);
            if (st != FSIM_OK) break;
            for (const auto &r : c->prof)
                if ((!wave || Ltot(r.bra_class, r.ket_class) >= 5) &&
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
    c->profiling = was;
    return st;
}

extern "C" fsim_status fsim_core_guess(fsim_ctx *c, double *D, void *stream) {
    if (!c || !D) return fail(FSIM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    STCHK(density_from_fock(c, c->H, D, s));
    HIPCHK(hipStreamSynchronize(s));
    return FSIM_OK;
}

extern "C" fsim_status fsim_scf_reset(fsim_ctx *c) {
    if (!c) return fail(FSIM_EINVAL, "ctx is NULL");
    c->diis_count = 0;
    c->diis_next = 0;
    std::fill(c->Bm.begin(), c->Bm.end(), 0.0);
    c->iter = 0;
    c->have_prev = false;
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

extern "C" fsim_status fsim_scf_step(fsim_ctx *c, double *D, fsim_scf_info *info,
                                     fsim_precision prec, void *stream) {
    if (!c || !D || !info) return fail(FSIM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int N = c->nbf;
    const size_t N2 = (size_t)N * N;
    double Eel = 0.0;
    STCHK(fock_build(c, D, c->F, nullptr, nullptr, &Eel, prec, s));
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
    info->converged = info->rms_dD < c->opt.conv_rms_dD &&
                      (c->opt.conv_dE <= 0 || (c->have_prev && std::fabs(info->dE) < c->opt.conv_dE));
    c->have_prev = true;
    c->E_prev = Etot;
    return FSIM_OK;
}
