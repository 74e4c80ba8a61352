/*
 * fsim.h -- C ABI of libfsim.so: the direct-SCF restricted Hartree-Fock Fock
 * build (McMurchie-Davidson electron-repulsion integrals over Schwarz-screened
 * shell quartets, digested on the fly into J and K) for AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns fsim_status: FSIM_OK (0) or a negative error.
 *    fsim_last_error() returns a thread-local message for the last error.
 *    No C++ exception crosses this boundary.
 *  - "device" pointers are HIP device memory owned by the caller (the library
 *    never frees them); "host" pointers are ordinary memory, read during the
 *    call and not retained.
 *  - Matrices are N x N FP64, row-major, N = number of Cartesian basis
 *    functions.  Basis functions are ordered shell by shell in input order;
 *    within a shell the Cartesian components run lx descending, then ly
 *    descending (p: x, y, z; d: xx, xy, xz, yy, yz, zz).  Each primitive is
 *    normalised to unit self-overlap and each contracted Cartesian function
 *    is rescaled to unit self-overlap, so diag(S) = 1.
 *  - Spherical basis (fsim_options.spherical = 1, one-molecule contexts):
 *    every Cartesian d shell is replaced by the 5 Racah-normalised real solid
 *    harmonics of Sec. 2.1.1, m = -2..2 (sqrt3 xy, sqrt3 yz, zz - (xx+yy)/2,
 *    sqrt3 xz, sqrt3/2 (xx - yy)), each contracted function rescaled to unit
 *    self-overlap; s and p shells are unchanged.  Every N x N matrix of the
 *    ABI (S, Hcore, X, D, F, J, K) is then over these N functions; the
 *    integral kernels still work on the Cartesian ones (fsim_eri_quartets
 *    returns Cartesian blocks).  Not available with batches, incremental or
 *    allocation-free builds; Fock builds are not graph-replayed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is ordered on it; calls that return host values (energies,
 *    statistics, SCF info) synchronise the stream before returning.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef FSIM_H
#define FSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSIM_OK = 0,
    FSIM_EINVAL = -1, /* invalid argument: message names it */
    FSIM_ENOMEM = -2, /* device or host allocation failed */
    FSIM_EHIP = -3,   /* a HIP, rocBLAS or rocSOLVER call failed */
    FSIM_ESTATE = -4  /* call out of order (e.g. SCF step before a screen) */
} fsim_status;

typedef enum {
    FSIM_FP64 = 0, /* every integral in FP64 */
    FSIM_MIXED = 1 /* quartets with Schwarz bound below tau_fp32 in FP32,
                      the rest in FP64; J/K accumulate in FP64 */
} fsim_precision;

/* Molecule and contracted Cartesian basis (Sec. 2.1: contracted shells of
 * primitive Cartesian Gaussians sharing a centre and an exponent set).
 * All host pointers; copied by fsim_ctx_create. */
typedef struct {
    int32_t natom;
    const double *xyz;          /* [natom*3] nuclear positions, bohr */
    const double *Z;            /* [natom] nuclear charges */
    int32_t nshell;
    const int32_t *shell_atom;  /* [nshell] centre of each shell */
    const int32_t *shell_l;     /* [nshell] 0, 1 or 2 (Cartesian d) */
    const int32_t *shell_nprim; /* [nshell] 1..8 primitives */
    const int32_t *shell_prim0; /* [nshell] offset into exps / coefs */
    const double *exps;         /* primitive exponents, > 0 */
    const double *coefs;        /* raw contraction coefficients d_k */
    int32_t nelec;              /* even, 2 <= nelec <= 2N (closed shell) */
} fsim_basis;

typedef struct {
    double tau_screen;  /* Schwarz threshold: quartet kept iff Q_ab Q_cd >= tau */
    double tau_fp32;    /* mixed precision: FP32 iff Q_ab Q_cd < tau_fp32 */
    int32_t diis_m;     /* DIIS subspace size (1..16); 0 disables DIIS */
    double conv_rms_dD; /* converged when RMS(D_new - D) < conv_rms_dD ... */
    double conv_dE;     /* ... and |dE| < conv_dE (ignored if <= 0) */
    int32_t max_iter;   /* informational: fsim_scf_step never loops */
    int32_t spherical;  /* 1: d shells are the 5 real solid harmonics (see below) */
} fsim_options;

typedef struct fsim_ctx fsim_ctx;

typedef struct {
    int64_t shell_pairs;       /* a >= b */
    int64_t pairs_kept;        /* Q_ab * Q_max >= tau */
    int64_t quartets_total;    /* canonical shell quartets */
    int64_t quartets_kept;     /* Schwarz survivors */
    int64_t quartets_fp64;     /* of which evaluated in FP64 (mixed mode) */
    int64_t quartets_fp32;     /* of which evaluated in FP32 (mixed mode) */
    int64_t prim_quartets_kept;
    double flops_fp64;         /* reference flop model (see fsim_class_profile) of
                                  one FP64-mode build */
    double flops_mixed_fp64;   /* same, mixed mode, FP64 part */
    double flops_mixed_fp32;   /* same, mixed mode, FP32 part */
    int64_t prim_pairs_total;  /* primitive pairs of the kept shell pairs */
    int64_t prim_pairs_kept;   /* of which in use (fewer with fsim_set_prim_screen) */
} fsim_screen_stats;

typedef struct {
    double E_total;   /* E_elec + E_nuc of the density passed in */
    double E_elec;    /* 1/2 Tr[D (H + F(D))] */
    double dE;        /* E_total minus the previous step's (0 on the first) */
    double rms_dD;    /* ||D_new - D||_F / N */
    double comm_norm; /* ||F D S - S D F||_F */
    int32_t iter;     /* steps taken since create / reset */
    int32_t converged;
    int32_t diis_used;  /* 1 when the DIIS extrapolation was applied */
    int32_t full_build; /* 0 when the step's Fock build was incremental */
    int64_t quartets;   /* contracted shell quartets the step's build evaluated */
} fsim_scf_info;

/* Message of the last failed call on this thread ("" if none). */
const char *fsim_last_error(void);

/* Library version string. */
const char *fsim_version(void);

/* Build a context on the current HIP device: normalise the basis, build the
 * shell-pair tables (Sec. 2.4: product centres, exponents and the Hermite
 * tensors E^{ab}_{tuv} of Eq. E-tuv), the Boys-function tables, the
 * one-electron matrices S, T + V (Eqs. s-overall, Tab-final, Vab-final), the
 * symmetric orthogonaliser X = U s^-1/2 U^T, and E_nuc.  Runs on the null
 * stream and synchronises.  Errors: FSIM_EINVAL for l > 2, nprim outside
 * 1..8, exps <= 0, non-finite input, odd or out-of-range nelec, NULL
 * pointers, or an overlap matrix with an eigenvalue below 1e-10. */
fsim_status fsim_ctx_create(const fsim_basis *basis, const fsim_options *opt, fsim_ctx **out);

/* Free every device and host resource of the context.  NULL is accepted. */
fsim_status fsim_ctx_destroy(fsim_ctx *ctx);

/* Number of basis functions N (Cartesian, or spherical when the context
 * uses the spherical basis), and the shell count. */
fsim_status fsim_nbf(const fsim_ctx *ctx, int32_t *nbf, int32_t *nshell);

/* Nuclear repulsion sum_{A<B} Z_A Z_B / R_AB (host out). */
fsim_status fsim_nuclear_repulsion(const fsim_ctx *ctx, double *enuc);

/* Copy the one-electron matrices into caller device buffers (any may be
 * NULL): S, Hcore = T + V, X = U s^-1/2 U^T.  Each N x N. */
fsim_status fsim_one_electron(fsim_ctx *ctx, double *S, double *H, double *X, void *stream);

/* Schwarz screening.  Q_ab = sqrt(max over components (ab|ab)) for every
 * shell pair, from diagonal integrals evaluated by the same kernels as the
 * Fock build.  Pairs with Q_ab * Q_max < tau are dropped; the rest are sorted
 * by Q in each angular-momentum pair class and rebuilt; the quartet work
 * lists are then formed per quartet class (canonical (ab|cd), kept iff
 * Q_ab Q_cd >= tau; in mixed mode FP32 iff Q_ab Q_cd < tau_fp32).  Must be
 * called before fsim_fock_build; calling it again replaces the lists.
 * Q_out: device [nshell*nshell] (symmetric) or NULL.  stats: host or NULL.
 * Screening is not in the paper (it names it as future work, Sec. 5); the
 * bound is the Cauchy-Schwarz inequality of the ERI inner product. */
fsim_status fsim_schwarz_screen(fsim_ctx *ctx, double tau, double tau_fp32, double *Q_out,
                                fsim_screen_stats *stats);

/* Direct Fock build (Eq. fock): from the density D (device, N x N, symmetric)
 * form J_mn = sum_ls (mn|ls) D_ls, K_mn = sum_ls (ml|ns) D_ls and
 * F = Hcore + J - K/2, evaluating every kept canonical quartet once and
 * digesting it into J and K with its permutational-degeneracy factor.
 * F, J, K: device N x N or NULL.  E_elec: host or NULL; when given, the
 * stream is synchronised and E_elec = 1/2 Tr[D (Hcore + F)].
 * FSIM_ESTATE if no screen was run. */
fsim_status fsim_fock_build(fsim_ctx *ctx, const double *D, double *F, double *J, double *K,
                            double *E_elec, fsim_precision prec, void *stream);

/* fsim_fock_build for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same inputs, outputs, kernels and errors, but the
 * J' and K' half-sum accumulators live in a static device array of the
 * library (2 x 2,097,152 FP64, 32 MiB, one copy per GPU, held until the
 * process ends, its address resolved at fsim_ctx_create) instead of buffers
 * the library allocates; the call itself allocates nothing (no hipMalloc,
 * no allocating library routine) and uses one shared accumulator copy, not
 * per-XCD copies.  Limit: the packed matrix size (N^2, or sum of N_m^2 for a
 * batch) must be <= 2,097,152 (N <= 1448), else FSIM_EINVAL.  Every call on
 * one GPU shares the array and clears what it uses before the build: calls
 * that overlap on one GPU (other streams, other threads, other contexts)
 * race and must be serialised by the caller.  No per-launch profiling and
 * no graph replay on this path. */
fsim_status fsim_fock_build_noalloc(fsim_ctx *ctx, const double *D, double *F, double *J,
                                    double *K, double *E_elec, fsim_precision prec, void *stream);

/* Core-Hamiltonian guess (Sec. 3.2, step 1): diagonalise X^T Hcore X and
 * write D = 2 C_occ C_occ^T into D (device N x N). */
fsim_status fsim_core_guess(fsim_ctx *ctx, double *D, void *stream);

/* One SCF iteration (Sec. 3.2, with DIIS of Sec. 3.2.1) on the density D
 * (device, N x N, overwritten): F = F(D); E = 1/2 Tr[D(H+F)];
 * e = F D S - S D F joins the DIIS history (size diis_m); from two stored
 * pairs on, F is replaced by sum c_i F_i with the c_i of the bordered DIIS
 * system (falling back to F when that system is singular);
 * F' = X^T F X is diagonalised (rocSOLVER dsyevd) and D <- 2 C_occ C_occ^T
 * with C = X C'.  info (host, required) reports E, dE, RMS(dD), ||e|| and
 * convergence (see fsim_options).  Synchronises the stream. */
fsim_status fsim_scf_step(fsim_ctx *ctx, double *D, fsim_scf_info *info, fsim_precision prec,
                          void *stream);

/* Conventional (stored-integral) mode, the data path of the paper's own
 * implementation (Sec. 3.3.1-3.3.2: the unique integrals are computed once
 * and the G build of every SCF iteration runs over them).  enable != 0:
 * every kept canonical quartet of the current screen is evaluated once, in
 * FP64, by its class's tuned Fock-build kernel and its contracted block is
 * written to a device buffer the context owns (tile order, one coalesced
 * line per component and wave); from then on every full Fock build of the
 * context (fsim_fock_build, fsim_scf_step, graph replays) digests the stored
 * blocks with the density instead of recomputing them -- in both precisions,
 * since the store is FP64.  Incremental builds still recompute.  bytes
 * (host, may be NULL) receives the store size.  FSIM_ENOMEM if the store
 * would take more than 90% of the free device memory (it grows with the
 * kept quartets: about 1 GB for 210 basis functions); FSIM_ESTATE before a
 * screen.  enable = 0 frees the store; a new screen also drops it. */
fsim_status fsim_store_eris(fsim_ctx *ctx, int32_t enable, int64_t *bytes);

/* Forget the DIIS history, the step counter and the incremental-build
 * reference. */
fsim_status fsim_scf_reset(fsim_ctx *ctx);

/* Incremental Fock build (the difference-density refinement of direct SCF,
 * which the paper names as future work in Sec. 5; J and K are linear in the
 * density, Eq. fock): with dD = D - D_ref,
 *   J = J_ref + J[dD],  K = K_ref + K[dD],  F = Hcore + J - K/2,
 * where J[dD], K[dD] come from the kept quartets (ab|cd) whose
 * density-weighted bound Q_ab Q_cd max|dD| over the six shell-pair blocks
 * the digest reads (ab, cd, ac, ad, bc, bd) is >= tau_delta (<= 0: the
 * screen's tau): each bra's Q-sorted ket range is cut where that bound,
 * maximised over the rest of the range, falls below tau_delta, so no
 * skipped quartet changes any digest term by tau_delta or more.
 * One-molecule contexts only (FSIM_EINVAL for a batch).
 * D, D_ref, J_ref, K_ref: device N x N (symmetric); J, K: device N x N
 * outputs, required, and may alias J_ref, K_ref (updated in place); F:
 * device or NULL; E_elec: host or NULL (synchronises; 1/2 Tr[D (H + F)]);
 * quartets: host or NULL, receives the number of contracted quartets
 * evaluated.  The call synchronises the stream once to read the block
 * maxima of dD back to the host.  FSIM_ESTATE before a screen. */
fsim_status fsim_fock_build_delta(fsim_ctx *ctx, const double *D, const double *D_ref,
                                  const double *J_ref, const double *K_ref, double *F, double *J,
                                  double *K, double *E_elec, double tau_delta, int64_t *quartets,
                                  fsim_precision prec, void *stream);

/* rebuild_every > 0: fsim_scf_step builds F incrementally from the previous
 * step's density and J, K (fsim_fock_build_delta with threshold tau_delta,
 * <= 0 for the screen's tau), with a full build on the first step and then
 * every rebuild_every steps (info->full_build says which, info->quartets how
 * many quartets were evaluated).  0 (default): every step runs a full
 * build.  Allocates the reference D, J, K (3 N x N) on first use;
 * one-molecule contexts only. */
fsim_status fsim_set_incremental(fsim_ctx *ctx, int32_t rebuild_every, double tau_delta);

/* Per-launch record of the last profiled Fock build: one entry per quartet
 * class (bra pair class >= ket pair class; 0..5 = ss ps pp ds dp dd) and
 * precision that had work.  ms is the kernel's duration measured with HIP
 * events recorded on the build's stream around that launch. */
typedef struct {
    int32_t bra_class, ket_class;
    int32_t fp32;             /* 1 for the FP32 part of a mixed build */
    int32_t tiles;            /* wave tiles (one bra pair x up to 64 kets) */
    int64_t quartets;         /* contracted quartets evaluated */
    int64_t prim_quartets;    /* primitive quartets */
    double flops;             /* reference flop model of the launch: per primitive
                                 quartet 25 + 30 + 3(L+1) + 2 C(L+4,4)
                                 + 2 C(Lab+3,3) C(Lcd+3,3) n_cart(cd), per bra
                                 primitive pair 2 C(Lab+3,3) n_cart(ab) n_cart(cd),
                                 per quartet 12 n_cart(abcd) (FMA = 2) */
    double ms;                /* measured kernel time */
    double flops_exec;        /* flops the kernels execute: nonzero Hermite box
                                 entries only, chunk recomputation not counted */
} fsim_class_profile;

/* Enable (1) or disable (0) per-launch timing of subsequent Fock builds. */
fsim_status fsim_set_profiling(fsim_ctx *ctx, int32_t enable);

/* Copy up to cap records of the last profiled build into out (host);
 * *count receives the number of records available. */
fsim_status fsim_get_class_profile(fsim_ctx *ctx, fsim_class_profile *out, int32_t cap,
                               int32_t *count);

/* Launch configuration of one quartet class and precision.  variant 0..2
 * selects the one-lane-per-quartet kernel with a per-lane register budget of
 * 96 / 128 / 160 live values (the block is then produced in chunks that fit;
 * a budget that cannot be met falls back to variant 3), variant 3 the
 * one-wave-per-quartet kernel, variant 4 the one-lane-per-quartet kernel with
 * the primitive loops in ket-outer order (ss, ps, pp and ds bra pairs; other
 * classes run variant 1), variant 5 the one-lane-per-quartet kernel at a
 * budget of 192 live values for classes whose chunks do not fit 160 or that
 * need fewer chunks at 192 ((ds|pp), (dp|pp), (dp|ds); others run
 * variant 2), variant 6 the one-wave-per-quartet kernel whose two
 * Hermite contraction steps run as dense products on the matrix cores
 * (16x16x4 FP64 / FP32 MFMA; classes with a d bra pair, others run variant
 * 3).  waves_per_block is 1, 2 or 4 for launches over tiles, every K'
 * term a global atomic (variants 3 and 6 use one block shape), or 8 for the
 * segment mode of the lane variants 0, 1, 2, 4 and 5 (see
 * fsim_set_krow_lds: blocks of 8 waves (12 for the ket-outer kernel of the
 * s/p classes of total angular momentum 2), or 4 for kernels held to one wave
 * per SIMD, over segments of one bra's tiles with the bra's K' rows in LDS;
 * launches whose rows do not fit run over tiles with 4 waves per block).
 * The default is variant 1 in segment mode with 64 tiles per segment;
 * seg_tiles sets the segment length per class and precision (fsim_autotune
 * times 32, 64, 128 and 256 for the classes that choose segment mode). */
typedef struct {
    int32_t bra_class, ket_class;   /* pair classes, bra >= ket */
    int32_t fp32;
    int32_t variant;
    int32_t waves_per_block;
    int32_t kbra, kket;             /* max primitive pairs of the classes (cache key) */
    int32_t seg_tiles;              /* segment mode: tiles per segment, a power of 2 in
                                       16..512; 0 in fsim_set_tuning: 64 */
    double ms;                      /* measured time of the chosen setting (autotune) */
} fsim_tuning;

/* Replace the settings of the listed classes (host array of n records). */
fsim_status fsim_set_tuning(fsim_ctx *ctx, const fsim_tuning *t, int32_t n);

/* All 42 class/precision settings currently in use (host out, cap >= 42). */
fsim_status fsim_get_tuning(fsim_ctx *ctx, fsim_tuning *out, int32_t cap, int32_t *n);

/* Autotuner: time every variant x waves-per-block setting of every class
 * with work, by per-launch HIP events over Fock builds at the density D
 * (device, N x N) in precision prec on stream, and keep the fastest per
 * class.  Needs a screen first.  Synchronises the stream.  With the
 * environment variable FSIM_AUTOTUNE_VERBOSE=1 each timed pass prints one
 * progress line (precision, variant, waves per block, summed kernel time)
 * on stderr. */
fsim_status fsim_autotune(fsim_ctx *ctx, const double *D, fsim_precision prec, void *stream);

/* Contracted ERI blocks (Eq. twoe-final summed over primitives) for n shell
 * quartets, evaluated by the Fock-build kernels but written out instead of
 * digested: each quartet class runs the kernel variant and waves per block
 * currently set for it (fsim_set_tuning), in FP32 for prec = FSIM_MIXED.  quartets: host [n*4] shell indices (a, b, c, d) in any order.
 * offsets: host [n] element offsets into out; block q is written as
 * out[offsets[q] + ((i*nb + j)*nc + k)*nd + l] over Cartesian components.
 * out: device FP64.  Unscreened; works before or after a screen. */
fsim_status fsim_eri_quartets(fsim_ctx *ctx, int64_t n, const int32_t *quartets,
                              const int64_t *offsets, double *out, fsim_precision prec,
                              void *stream);

/* ---- batches of molecules --------------------------------------------- */

/* Context over nmol independent molecules (host array of bases).  Shell
 * pairs and quartets never mix molecules; one class launch serves every
 * molecule's quartets (the kets of each pair class are ordered by molecule,
 * then Q, so every bra's ket range stays inside its molecule).  Every N x N
 * argument of the other entry points becomes a packed array: molecule m's
 * N_m x N_m row-major block at element offset offsets[m] (fsim_batch_layout).
 * fsim_scf_step runs the SCF step on all molecules at once (zero-padded
 * blocks, strided-batched rocBLAS / rocSOLVER dsyevd, DIIS per molecule);
 * its info aggregates (sum of energies, max RMS(dD), all converged) and
 * fsim_batch_scf_info gives the per-molecule records.  fsim_eri_quartets
 * accepts only quartets within one molecule. */
fsim_status fsim_batch_create(const fsim_basis *mols, int32_t nmol, const fsim_options *opt,
                              fsim_ctx **out);

/* Layout of a context (one molecule: nmol = 1, offset 0).  Any pointer may
 * be NULL; nbf/offsets/enuc are host arrays of nmol entries. */
fsim_status fsim_batch_layout(const fsim_ctx *ctx, int32_t *nmol, int32_t *nbf, int64_t *offsets,
                              double *enuc, int64_t *packed);

/* Per-molecule electronic energies of the last Fock build that computed an
 * energy (host array of nmol). */
fsim_status fsim_batch_energies(const fsim_ctx *ctx, double *E_elec);

/* Per-molecule records of the last batched fsim_scf_step (host array of nmol). */
fsim_status fsim_batch_scf_info(const fsim_ctx *ctx, fsim_scf_info *info);

/* Capture the Fock build (zeroing kernels, every class kernel, the Fock
 * assembly) once per precision as a hipGraph on an internal stream and
 * replay it for every later fsim_fock_build / fsim_scf_step that asks for F
 * without J and K.  The caller's stream is ordered before and after the
 * replay with events.  Rescreening drops the graphs.  enable = 0 returns to
 * direct launches. */
fsim_status fsim_set_graph(fsim_ctx *ctx, int32_t enable);

/* enable != 0: every s/p quartet class ((ss|ss) .. (pp|pp)) of a Fock build
 * runs in one resident launch per precision part instead of one launch per
 * class: a global queue of (class, tile) items, heaviest class first, served
 * by an atomic tile counter, each item evaluated by the class's ket-outer
 * tile code (d classes keep their own launches, so a C/H batch needs one
 * ERI launch per build and precision).  Per-launch profiling then reports
 * the persistent launch as one record with bra_class = ket_class = 6.  The
 * launch is captured in graphs like the others.  With fsim_set_krow_lds on
 * (default) and segments averaging at least 16 tiles, the queue items are
 * segments taken by whole blocks, which keep the bra's K' rows in LDS (if
 * they fit); otherwise tile items taken by single waves.  enable = 0 (default): per-class launches with the tuned
 * variants.  Drops captured graphs. */
fsim_status fsim_set_persistent(fsim_ctx *ctx, int32_t enable);

/* enable != 0 (default): lane-kernel launches tuned to segment mode
 * (waves_per_block = 8) take whole segments of up to seg_tiles (64 by
 * default, see fsim_tuning) tiles of one bra pair per workgroup and add the
 * quartets' K' terms, which all lie in the rows of the bra's functions
 * (Eq. fock: K'_ac, K'_ad, K'_bc, K'_bd), into an LDS copy of those rows;
 * the non-zero entries go to global K' once per segment (incremental
 * builds cut their segments again for every build).  A launch whose rows
 * (ncart(l_a) + ncart(l_b) rows of N doubles, N the largest molecule) do
 * not fit in LDS next to the kernel's own use adds every K' term with a
 * global atomic instead, as enable = 0 does everywhere.  The same holds for
 * the persistent s/p launch (segment items) and the stored-integral digest (segment-mode settings then run over tiles with 4 waves
 * per block).  Results differ only in summation order.  Drops captured
 * graphs. */
fsim_status fsim_set_krow_lds(fsim_ctx *ctx, int32_t enable);

/* Primitive-pair screening (an addition to the shell-quartet screen of
 * Sec. 5, which keeps every primitive of a kept shell pair).  For primitive
 * pair k of a kept shell pair, Q_k = sqrt(max over its component pairs of
 * (Omega_k|Omega_k)), the self-repulsion of its Hermite distribution (Eq.
 * twoe-final at zero separation), bounds its part of any integral (ab|cd) by
 * Q_k Q_cd.  The next fsim_schwarz_screen drops every primitive pair with
 * Q_k * Q_max < tau_prim (Q_max: the largest shell-pair factor of the
 * molecule) from the kept pair tables, so each evaluated integral differs
 * from the unscreened one by at most (primitive pairs dropped from its bra
 * and ket) * tau_prim.  tau_prim = 0 (default) keeps every primitive pair.
 * tau_prim must be finite and >= 0 (FSIM_EINVAL).  The call invalidates the
 * current screen: Fock builds return FSIM_ESTATE until fsim_schwarz_screen
 * runs again.  The Schwarz factors themselves and fsim_eri_quartets always
 * use every primitive. */
fsim_status fsim_set_prim_screen(fsim_ctx *ctx, double tau_prim);

/* Digest target of the Fock build (the J' and K' half-sums of Eq. fock).
 * enable != 0 (the default): every XCD of the GPU adds into its own private
 * copy of J' and K' (the XCD is read from the wave's XCC_ID register) and
 * the copies are summed after the class kernels, so that the FP64 atomics
 * of one cache line stay within one XCD's L2.  Costs 2 x 8 x (packed matrix
 * size) doubles of device memory, allocated on the next build.  enable = 0:
 * one shared copy.  Results agree to rounding either way; changing the
 * setting drops captured graphs. */
fsim_status fsim_set_xcd_private(fsim_ctx *ctx, int32_t enable);

/* McWeeny purification of a trial density of a one-molecule context: with
 * P = D/2, P <- 3 PSP - 2 PSPSP, at most iters times or until
 * ||PSP - P||_F / ||P||_F < 1e-12 (idempotency of the closed-shell density,
 * D = 2 C_occ C_occ^T, Sec. 2.2 Eq. density).  D: device N x N, overwritten.
 * err_in / err_out (host, may be NULL): the measure before and after. */
fsim_status fsim_purify(fsim_ctx *ctx, double *D, int32_t iters, double *err_in, double *err_out,
                        void *stream);

/* ---- learned initial guess: BF16 matrix-core kernels -------------------- */
/* BF16 values are raw uint16_t bit patterns (round-to-nearest-even from
 * FP32).  All pointers are device memory; calls are asynchronous on stream
 * and return FSIM_EINVAL for bad sizes / NULL pointers, FSIM_EHIP on a
 * launch failure. */

/* C[M x N] = op(A)[M x K] op(B)[K x N] with FP32 accumulation on
 * v_mfma_f32_16x16x16bf16_1k.  A, B: BF16 row-major with leading dimensions
 * lda, ldb; ta / tb = 1 reads them transposed.  Epilogue: C = act(acc + bias)
 * with act = ReLU when relu = 1 (bias: FP32 [N] or NULL); the result goes to
 * C (FP32, leading dimension ldc) and/or Cb (BF16, same layout).  ksplit > 1
 * splits K over that many blocks and adds the partial sums atomically into C
 * (the caller zeroes C first; no bias, ReLU or Cb then). */
fsim_status fsim_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda,
                           int32_t ta, const uint16_t *B, int32_t ldb, int32_t tb, float *C,
                           int32_t ldc, uint16_t *Cb, const float *bias, int32_t relu,
                           int32_t ksplit, void *stream);

/* y = bf16(x) for n values. */
fsim_status fsim_f32_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream);

/* dH <- dH * [H > 0] (FP32) and, if dHb is not NULL, its BF16 copy. */
fsim_status fsim_relu_backward(int64_t n, const float *H, float *dH, uint16_t *dHb, void *stream);

/* db[j] = sum_i dY[i*m + j] for an n x m FP32 matrix. */
fsim_status fsim_bias_grad(int32_t n, int32_t m, const float *dY, float *db, void *stream);

/* Masked mean-square error: *loss += sum mask (Y - T)^2 * inv_count and
 * dY = 2 mask (Y - T) inv_count (n values; loss is a device scalar). */
fsim_status fsim_mse(int64_t n, const float *Y, const float *T, const float *mask, float inv_count,
                     float *dY, float *loss, void *stream);

/* One Adam step (bias-corrected, step >= 1) on FP32 master weights w with
 * gradient g and moments m1, m2; wb (BF16 copy of w) is refreshed if given. */
fsim_status fsim_adam(int64_t n, float *w, const float *g, float *m1, float *m2, float lr,
                      float b1, float b2, float eps, int32_t step, uint16_t *wb, void *stream);

/* Fragment packing of a K x N BF16 weight matrix (row-major, ld = N; K a
 * multiple of 16) for fsim_mlp_forward.  Wp holds (K/16) * ceil(N/16) * 256
 * BF16 values, caller-allocated: for K step s and column tile t, lane l of
 * the 16x16x16 MFMA B operand holds rows 16s + 4(l/16) + j (j < 4) of
 * column 16t + l%16, zero past N, at Wp[((s*ceil(N/16) + t)*64 + l)*4 + j].
 * FSIM_EINVAL for K <= 0, K % 16 != 0, N <= 0, NULL pointers or Wp not
 * 8-byte aligned. */
fsim_status fsim_mlp_pack(int32_t K, int32_t N, const uint16_t *W, uint16_t *Wp, void *stream);

/* Fused inference of the guess network (the per-pair MLP of the learned
 * initial guess): Y = W3^T r(W2^T r(W1^T x + b1) + b2) + b3 per row, r =
 * ReLU with the hidden activations rounded to BF16, in one kernel that keeps
 * them in LDS.  The result equals the three fsim_gemm_bf16 calls with
 * bias/ReLU epilogues bit for bit (same MFMA steps in the same order).
 * X: n x 64 BF16 row-major (8-byte aligned); W1p, W2p, W3p: fsim_mlp_pack
 * of W1 (64 x 256), W2 (256 x 256), W3 (256 x 36); b1, b2: FP32 [256],
 * b3: FP32 [36]; Y: n x 36 FP32 row-major.  n = 0 does nothing; FSIM_EINVAL
 * for n < 0, NULL pointers, or X or a packed weight not 8-byte aligned. */
fsim_status fsim_mlp_forward(int32_t n, const uint16_t *X, const uint16_t *W1p, const float *b1,
                             const uint16_t *W2p, const float *b2, const uint16_t *W3p,
                             const float *b3, float *Y, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FSIM_H */
