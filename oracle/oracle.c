/*
 * oracle.c -- plain, slow FP64 reference for the McMurchie-Davidson RHF
 * Fock build.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every routine writes out the paper's formulas in the paper's order:
 *   Boys function             F_n(x) = int_0^1 exp(-x t^2) t^(2n) dt  (Sec. 2.3.3);
 *                             evaluated by the textbook series / asymptotic
 *                             form, since the paper gives no method.
 *   Hermite coefficients E    Eqs. recurrence-A / recurrence-B with the
 *                             initial and boundary conditions (Sec. 2.1.3).
 *   Hermite Coulomb R^n_tuv   Eq. Rn-definition source term, Eq. R-recursion.
 *   overlap                   Eq. s-overall;  kinetic  Eq. Tab-final;
 *   nuclear attraction        Eq. Vab-final with V = -sum_C Z_C V_ab(C).
 *   primitive ERI             Eq. twoe-final, reduced exponent pq/(p+q) and
 *                             R_PQ as the R arguments (Sec. 2.3.4).
 *   contraction               sum over primitives with d_k (Sec. 2.3.4).
 *   Fock / G                  Eq. fock with J_mn = sum (mn|ls) D_ls and
 *                             K_mn = sum (ml|ns) D_ls, G = J - K/2.
 * Parity status of each function is listed in the Python wrapper's header.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_LMAX 2                       /* s, p, Cartesian d */
#define OR_LTOT (4 * OR_LMAX)           /* highest total angular momentum of a quartet */
#define OR_EMAX (OR_LMAX + 2)           /* kinetic needs j + 2 */

/* ------------------------------------------------------------------ */
/* Boys function                                                        */
/* ------------------------------------------------------------------ */

/* F_0..F_nmax at T.  Below T = 30 the series
 *   F_N(T) = exp(-T) sum_i (2T)^i / ((2N+1)(2N+3)...(2N+2i+1))
 * at N = nmax, then the downward recursion F_{n-1} = (2T F_n + e^-T)/(2n-1).
 * From T = 30 on, F_0 = (1/2) sqrt(pi/T) erf(sqrt T) and the upward recursion
 * F_{n+1} = ((2n+1) F_n - e^-T) / (2T). */
void or_boys(int nmax, double T, double *F)
{
    double et = exp(-T);
    if (T < 30.0) {
        double term = 1.0 / (2 * nmax + 1), sum = term;
        for (int i = 1; i < 100000; i++) {
            term *= 2.0 * T / (2 * nmax + 2 * i + 1);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        F[nmax] = et * sum;
        for (int n = nmax; n > 0; n--) F[n - 1] = (2.0 * T * F[n] + et) / (2 * n - 1);
    } else {
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int n = 0; n < nmax; n++) F[n + 1] = ((2 * n + 1) * F[n] - et) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------ */
/* Hermite expansion coefficients (one Cartesian direction)             */
/* ------------------------------------------------------------------ */

/* E^{ij}_t for 0<=i<=imax, 0<=j<=jmax, 0<=t<=i+j, exponents a (centre A)
 * and b (centre B).  Layout E[(i*(jmax+1)+j)*(imax+jmax+1) + t]. */
void or_hermite_e(int imax, int jmax, double a, double b, double A, double B, double *E)
{
    int tm = imax + jmax + 1;
    double p = a + b, mu = a * b / p, P = (a * A + b * B) / p;
    double XPA = P - A, XPB = P - B, XAB = A - B;
    memset(E, 0, sizeof(double) * (imax + 1) * (jmax + 1) * tm);
#define EIX(i, j, t) E[((i) * (jmax + 1) + (j)) * tm + (t)]
    EIX(0, 0, 0) = exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; i++) {
        for (int j = 0; j <= jmax; j++) {
            if (i == 0 && j == 0) continue;
            /* grow i from (i-1, j) with recurrence-A, else j from (i, j-1)
             * with recurrence-B; E is zero outside 0 <= t <= i+j */
            int pi = i > 0 ? i - 1 : i, pj = i > 0 ? j : j - 1;
            double X = i > 0 ? XPA : XPB;
            int ptop = pi + pj;
            for (int t = 0; t <= i + j; t++) {
                double v = 0.0;
                if (t - 1 >= 0 && t - 1 <= ptop) v += EIX(pi, pj, t - 1) / (2.0 * p);
                if (t <= ptop) v += X * EIX(pi, pj, t);
                if (t + 1 <= ptop) v += (t + 1) * EIX(pi, pj, t + 1);
                EIX(i, j, t) = v;
            }
        }
    }
#undef EIX
}

/* ------------------------------------------------------------------ */
/* Hermite Coulomb integrals R^0_tuv                                     */
/* ------------------------------------------------------------------ */

/* R0[(t*(L+1)+u)*(L+1)+v] for t+u+v <= L, exponent a, vector (X, Y, Z):
 * source R^n_000 = (-2a)^n F_n(a |R|^2), then Eq. R-recursion from the
 * highest n down to n = 0. */
void or_hermite_r(int L, double a, double X, double Y, double Z, double *R0)
{
    int d = L + 1;
    double F[OR_LTOT + 3];
    /* every entry read below was written first: R^{n+1} at lower t+u+v */
    double Rn[(OR_LTOT + 1) * (OR_LTOT + 1) * (OR_LTOT + 1) * (OR_LTOT + 1)];
#define RIX(n, t, u, v) Rn[(((n) * d + (t)) * d + (u)) * d + (v)]
    or_boys(L, a * (X * X + Y * Y + Z * Z), F);
    for (int n = L; n >= 0; n--) {
        for (int t = 0; t <= L - n; t++)
            for (int u = 0; u <= L - n - t; u++)
                for (int v = 0; v <= L - n - t - u; v++) {
                    double r;
                    if (t == 0 && u == 0 && v == 0) {
                        r = pow(-2.0 * a, n) * F[n];
                    } else if (t > 0) {
                        r = X * RIX(n + 1, t - 1, u, v);
                        if (t > 1) r += (t - 1) * RIX(n + 1, t - 2, u, v);
                    } else if (u > 0) {
                        r = Y * RIX(n + 1, t, u - 1, v);
                        if (u > 1) r += (u - 1) * RIX(n + 1, t, u - 2, v);
                    } else {
                        r = Z * RIX(n + 1, t, u, v - 1);
                        if (v > 1) r += (v - 1) * RIX(n + 1, t, u, v - 2);
                    }
                    RIX(n, t, u, v) = r;
                }
    }
    memset(R0, 0, sizeof(double) * d * d * d);
    for (int t = 0; t <= L; t++)
        for (int u = 0; u <= L - t; u++)
            for (int v = 0; v <= L - t - u; v++) R0[(t * d + u) * d + v] = RIX(0, t, u, v);
#undef RIX
}

/* ------------------------------------------------------------------ */
/* Basis                                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    int natom;
    double *xyz, *Z;
    int nshell;
    int *sh_atom, *sh_l, *sh_nprim, *sh_prim0, *sh_bf0;
    double *exps;
    int nbf, maxprim;
    int *bf_shell, *bf_lx, *bf_ly, *bf_lz;
    double *bf_coef;            /* [nbf * maxprim]: normalised d_k per primitive */
} or_basis;

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian components in the order lx descending, then ly descending. */
static void cart_comp(int l, int c, int *lx, int *ly, int *lz)
{
    int k = 0;
    for (int x = l; x >= 0; x--)
        for (int y = l - x; y >= 0; y--) {
            if (k == c) { *lx = x; *ly = y; *lz = l - x - y; return; }
            k++;
        }
}

static double dfact(int n) /* n!! with (-1)!! = 1 */
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

/* primitive overlap of two Cartesian Gaussians on the same centre (Eq. s-overall) */
static double prim_overlap(int ix, int iy, int iz, double a, const double *A,
                           int jx, int jy, int jz, double b, const double *B)
{
    double Ex[(OR_EMAX + 1) * (OR_EMAX + 1) * (2 * OR_EMAX + 1)];
    double Ey[(OR_EMAX + 1) * (OR_EMAX + 1) * (2 * OR_EMAX + 1)];
    double Ez[(OR_EMAX + 1) * (OR_EMAX + 1) * (2 * OR_EMAX + 1)];
    int tm = ix + jx + 1;
    or_hermite_e(ix, jx, a, b, A[0], B[0], Ex);
    or_hermite_e(iy, jy, a, b, A[1], B[1], Ey);
    or_hermite_e(iz, jz, a, b, A[2], B[2], Ez);
    double p = a + b;
    return Ex[(ix * (jx + 1) + jx) * tm] * Ey[(iy * (jy + 1) + jy) * (iy + jy + 1)] *
           Ez[(iz * (jz + 1) + jz) * (iz + jz + 1)] * pow(M_PI / p, 1.5);
}

or_basis *or_basis_create(int natom, const double *xyz, const double *Z, int nshell,
                          const int *sh_atom, const int *sh_l, const int *sh_nprim,
                          const int *sh_prim0, const double *exps, const double *coefs)
{
    or_basis *b = (or_basis *)calloc(1, sizeof(or_basis));
    b->natom = natom;
    b->xyz = (double *)malloc(sizeof(double) * 3 * natom);
    b->Z = (double *)malloc(sizeof(double) * natom);
    memcpy(b->xyz, xyz, sizeof(double) * 3 * natom);
    memcpy(b->Z, Z, sizeof(double) * natom);
    b->nshell = nshell;
    b->sh_atom = (int *)malloc(sizeof(int) * nshell);
    b->sh_l = (int *)malloc(sizeof(int) * nshell);
    b->sh_nprim = (int *)malloc(sizeof(int) * nshell);
    b->sh_prim0 = (int *)malloc(sizeof(int) * nshell);
    b->sh_bf0 = (int *)malloc(sizeof(int) * nshell);
    memcpy(b->sh_atom, sh_atom, sizeof(int) * nshell);
    memcpy(b->sh_l, sh_l, sizeof(int) * nshell);
    memcpy(b->sh_nprim, sh_nprim, sizeof(int) * nshell);
    memcpy(b->sh_prim0, sh_prim0, sizeof(int) * nshell);
    int nprim = 0, nbf = 0, maxprim = 1;
    for (int s = 0; s < nshell; s++) {
        int e = sh_prim0[s] + sh_nprim[s];
        if (e > nprim) nprim = e;
        if (sh_nprim[s] > maxprim) maxprim = sh_nprim[s];
        b->sh_bf0[s] = nbf;
        nbf += ncart(sh_l[s]);
    }
    b->exps = (double *)malloc(sizeof(double) * (nprim > 0 ? nprim : 1));
    memcpy(b->exps, exps, sizeof(double) * nprim);
    b->nbf = nbf;
    b->maxprim = maxprim;
    b->bf_shell = (int *)malloc(sizeof(int) * nbf);
    b->bf_lx = (int *)malloc(sizeof(int) * nbf);
    b->bf_ly = (int *)malloc(sizeof(int) * nbf);
    b->bf_lz = (int *)malloc(sizeof(int) * nbf);
    b->bf_coef = (double *)calloc((size_t)nbf * maxprim, sizeof(double));
    for (int s = 0; s < nshell; s++) {
        const double *A = xyz + 3 * sh_atom[s];
        for (int c = 0; c < ncart(sh_l[s]); c++) {
            int mu = b->sh_bf0[s] + c, lx = 0, ly = 0, lz = 0;
            cart_comp(sh_l[s], c, &lx, &ly, &lz);
            b->bf_shell[mu] = s;
            b->bf_lx[mu] = lx;
            b->bf_ly[mu] = ly;
            b->bf_lz[mu] = lz;
            /* primitive normalisation so that <G|G> = 1 */
            double *d = b->bf_coef + (size_t)mu * maxprim;
            for (int k = 0; k < sh_nprim[s]; k++) {
                double a = exps[sh_prim0[s] + k];
                double N = pow(2.0 * a / M_PI, 0.75) * pow(4.0 * a, 0.5 * sh_l[s]) /
                           sqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
                d[k] = coefs[sh_prim0[s] + k] * N;
            }
            /* rescale the contracted Cartesian function to unit self-overlap */
            double ss = 0.0;
            for (int k = 0; k < sh_nprim[s]; k++)
                for (int m = 0; m < sh_nprim[s]; m++)
                    ss += d[k] * d[m] *
                          prim_overlap(lx, ly, lz, exps[sh_prim0[s] + k], A, lx, ly, lz,
                                       exps[sh_prim0[s] + m], A);
            for (int k = 0; k < sh_nprim[s]; k++) d[k] /= sqrt(ss);
        }
    }
    return b;
}

void or_basis_destroy(or_basis *b)
{
    if (!b) return;
    free(b->xyz); free(b->Z); free(b->sh_atom); free(b->sh_l); free(b->sh_nprim);
    free(b->sh_prim0); free(b->sh_bf0); free(b->exps); free(b->bf_shell);
    free(b->bf_lx); free(b->bf_ly); free(b->bf_lz); free(b->bf_coef);
    free(b);
}

int or_nbf(const or_basis *b) { return b->nbf; }

/* normalised contraction coefficient of primitive k of basis function mu */
double or_bf_coef(const or_basis *b, int mu, int k) { return b->bf_coef[(size_t)mu * b->maxprim + k]; }

double or_nuclear_repulsion(const or_basis *b)
{
    double e = 0.0;
    for (int A = 0; A < b->natom; A++)
        for (int B = 0; B < A; B++) {
            double dx = b->xyz[3 * A] - b->xyz[3 * B], dy = b->xyz[3 * A + 1] - b->xyz[3 * B + 1],
                   dz = b->xyz[3 * A + 2] - b->xyz[3 * B + 2];
            e += b->Z[A] * b->Z[B] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return e;
}

/* ------------------------------------------------------------------ */
/* One-electron integrals                                               */
/* ------------------------------------------------------------------ */

#define E1D(E, jmax, tm, i, j, t) (E)[((i) * ((jmax) + 1) + (j)) * (tm) + (t)]

/* S, T and V (N x N, row-major) for the contracted Cartesian functions. */
void or_one_electron(const or_basis *b, double *S, double *T, double *V)
{
    int N = b->nbf;
    const int jm = OR_EMAX, tm = 2 * OR_EMAX + 1;
    for (int mu = 0; mu < N; mu++) {
        for (int nu = 0; nu < N; nu++) {
            int sa = b->bf_shell[mu], sb = b->bf_shell[nu];
            const double *A = b->xyz + 3 * b->sh_atom[sa], *B = b->xyz + 3 * b->sh_atom[sb];
            int i[3] = {b->bf_lx[mu], b->bf_ly[mu], b->bf_lz[mu]};
            int j[3] = {b->bf_lx[nu], b->bf_ly[nu], b->bf_lz[nu]};
            double s = 0.0, t = 0.0, v = 0.0;
            for (int ka = 0; ka < b->sh_nprim[sa]; ka++)
                for (int kb = 0; kb < b->sh_nprim[sb]; kb++) {
                    double a = b->exps[b->sh_prim0[sa] + ka], be = b->exps[b->sh_prim0[sb] + kb];
                    double p = a + be;
                    double dd = or_bf_coef(b, mu, ka) * or_bf_coef(b, nu, kb);
                    double E[3][(OR_EMAX + 1) * (OR_EMAX + 1) * (2 * OR_EMAX + 1)];
                    for (int x = 0; x < 3; x++) or_hermite_e(jm, jm, a, be, A[x], B[x], E[x]);
                    /* overlap, Eq. s-overall */
                    double e0[3];
                    for (int x = 0; x < 3; x++) e0[x] = E1D(E[x], jm, tm, i[x], j[x], 0);
                    double sp = e0[0] * e0[1] * e0[2] * pow(M_PI / p, 1.5);
                    /* kinetic, Eq. Tab-final */
                    double tp = 0.0;
                    for (int x = 0; x < 3; x++) {
                        double bracket = -2.0 * be * be * E1D(E[x], jm, tm, i[x], j[x] + 2, 0) +
                                         be * (2 * j[x] + 1) * E1D(E[x], jm, tm, i[x], j[x], 0);
                        if (j[x] >= 2)
                            bracket -= 0.5 * j[x] * (j[x] - 1) * E1D(E[x], jm, tm, i[x], j[x] - 2, 0);
                        tp += bracket * e0[(x + 1) % 3] * e0[(x + 2) % 3];
                    }
                    tp *= pow(M_PI / p, 1.5);
                    /* nuclear attraction, Eq. Vab-final for every nucleus */
                    double P[3];
                    for (int x = 0; x < 3; x++) P[x] = (a * A[x] + be * B[x]) / p;
                    int L = i[0] + i[1] + i[2] + j[0] + j[1] + j[2], d = L + 1;
                    double R0[(OR_LTOT + 1) * (OR_LTOT + 1) * (OR_LTOT + 1)];
                    double vp = 0.0;
                    for (int C = 0; C < b->natom; C++) {
                        const double *Cc = b->xyz + 3 * C;
                        or_hermite_r(L, p, P[0] - Cc[0], P[1] - Cc[1], P[2] - Cc[2], R0);
                        double acc = 0.0;
                        for (int tt = 0; tt <= i[0] + j[0]; tt++)
                            for (int uu = 0; uu <= i[1] + j[1]; uu++)
                                for (int vv = 0; vv <= i[2] + j[2]; vv++)
                                    acc += E1D(E[0], jm, tm, i[0], j[0], tt) *
                                           E1D(E[1], jm, tm, i[1], j[1], uu) *
                                           E1D(E[2], jm, tm, i[2], j[2], vv) *
                                           R0[(tt * d + uu) * d + vv];
                        vp -= b->Z[C] * (2.0 * M_PI / p) * acc;
                    }
                    s += dd * sp;
                    t += dd * tp;
                    v += dd * vp;
                }
            if (S) S[mu * N + nu] = s;
            if (T) T[mu * N + nu] = t;
            if (V) V[mu * N + nu] = v;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Two-electron integrals                                               */
/* ------------------------------------------------------------------ */

/* Contracted ERI block (ab|cd) for shells sa, sb, sc, sd, written as
 * out[((a*nb + b)*nc + c)*nd + d] over Cartesian components, by the final
 * McMurchie-Davidson formula (Eq. twoe-final) summed over primitives with
 * the normalised contraction coefficients. */
void or_eri_block(const or_basis *b, int sa, int sb, int sc, int sd, double *out)
{
    int sh[4] = {sa, sb, sc, sd};
    int l[4], nc[4], bf0[4];
    const double *X[4];
    for (int k = 0; k < 4; k++) {
        l[k] = b->sh_l[sh[k]];
        nc[k] = ncart(l[k]);
        bf0[k] = b->sh_bf0[sh[k]];
        X[k] = b->xyz + 3 * b->sh_atom[sh[k]];
    }
    int nout = nc[0] * nc[1] * nc[2] * nc[3];
    memset(out, 0, sizeof(double) * nout);
    int L = l[0] + l[1] + l[2] + l[3], d = L + 1;
    int tab = l[0] + l[1] + 1, tcd = l[2] + l[3] + 1;
    double Eab[3][(OR_LMAX + 1) * (OR_LMAX + 1) * (2 * OR_LMAX + 1)];
    double Ecd[3][(OR_LMAX + 1) * (OR_LMAX + 1) * (2 * OR_LMAX + 1)];
    double R0[(OR_LTOT + 1) * (OR_LTOT + 1) * (OR_LTOT + 1)];
    for (int ka = 0; ka < b->sh_nprim[sa]; ka++)
        for (int kb = 0; kb < b->sh_nprim[sb]; kb++) {
            double a = b->exps[b->sh_prim0[sa] + ka], be = b->exps[b->sh_prim0[sb] + kb];
            double p = a + be, P[3];
            for (int x = 0; x < 3; x++) {
                P[x] = (a * X[0][x] + be * X[1][x]) / p;
                or_hermite_e(l[0], l[1], a, be, X[0][x], X[1][x], Eab[x]);
            }
            for (int kc = 0; kc < b->sh_nprim[sc]; kc++)
                for (int kd = 0; kd < b->sh_nprim[sd]; kd++) {
                    double g = b->exps[b->sh_prim0[sc] + kc], de = b->exps[b->sh_prim0[sd] + kd];
                    double q = g + de, Q[3];
                    for (int x = 0; x < 3; x++) {
                        Q[x] = (g * X[2][x] + de * X[3][x]) / q;
                        or_hermite_e(l[2], l[3], g, de, X[2][x], X[3][x], Ecd[x]);
                    }
                    double alpha = p * q / (p + q);
                    or_hermite_r(L, alpha, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], R0);
                    double pref = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q));
                    for (int ia = 0; ia < nc[0]; ia++)
                        for (int ib = 0; ib < nc[1]; ib++)
                            for (int ic = 0; ic < nc[2]; ic++)
                                for (int id = 0; id < nc[3]; id++) {
                                    int mu = bf0[0] + ia, nu = bf0[1] + ib, la = bf0[2] + ic,
                                        si = bf0[3] + id;
                                    int i[3] = {b->bf_lx[mu], b->bf_ly[mu], b->bf_lz[mu]};
                                    int j[3] = {b->bf_lx[nu], b->bf_ly[nu], b->bf_lz[nu]};
                                    int k[3] = {b->bf_lx[la], b->bf_ly[la], b->bf_lz[la]};
                                    int m[3] = {b->bf_lx[si], b->bf_ly[si], b->bf_lz[si]};
                                    double acc = 0.0;
                                    for (int t = 0; t <= i[0] + j[0]; t++)
                                    for (int u = 0; u <= i[1] + j[1]; u++)
                                    for (int v = 0; v <= i[2] + j[2]; v++) {
                                        double eab = E1D(Eab[0], l[1], tab, i[0], j[0], t) *
                                                     E1D(Eab[1], l[1], tab, i[1], j[1], u) *
                                                     E1D(Eab[2], l[1], tab, i[2], j[2], v);
                                        for (int ta = 0; ta <= k[0] + m[0]; ta++)
                                        for (int nn = 0; nn <= k[1] + m[1]; nn++)
                                        for (int ph = 0; ph <= k[2] + m[2]; ph++) {
                                            double ecd = E1D(Ecd[0], l[3], tcd, k[0], m[0], ta) *
                                                         E1D(Ecd[1], l[3], tcd, k[1], m[1], nn) *
                                                         E1D(Ecd[2], l[3], tcd, k[2], m[2], ph);
                                            double sgn = ((ta + nn + ph) & 1) ? -1.0 : 1.0;
                                            acc += sgn * eab * ecd *
                                                   R0[((t + ta) * d + (u + nn)) * d + (v + ph)];
                                        }
                                    }
                                    double dd = or_bf_coef(b, mu, ka) * or_bf_coef(b, nu, kb) *
                                                or_bf_coef(b, la, kc) * or_bf_coef(b, si, kd);
                                    out[((ia * nc[1] + ib) * nc[2] + ic) * nc[3] + id] +=
                                        dd * pref * acc;
                                }
                }
        }
}

/* The full ERI tensor g[((m*N+n)*N+l)*N+s] = (mn|ls), every ordered shell
 * quartet evaluated on its own (no permutational symmetry used). */
void or_eri_tensor(const or_basis *b, double *g)
{
    int N = b->nbf, ns = b->nshell;
#pragma omp parallel for schedule(dynamic, 1)
    for (int sa = 0; sa < ns; sa++) {
        double blk[6 * 6 * 6 * 6];
        for (int sb = 0; sb < ns; sb++)
            for (int sc = 0; sc < ns; sc++)
                for (int sd = 0; sd < ns; sd++) {
                    or_eri_block(b, sa, sb, sc, sd, blk);
                    int n[4] = {ncart(b->sh_l[sa]), ncart(b->sh_l[sb]), ncart(b->sh_l[sc]),
                                ncart(b->sh_l[sd])};
                    for (int i = 0; i < n[0]; i++)
                        for (int j = 0; j < n[1]; j++)
                            for (int k = 0; k < n[2]; k++)
                                for (int m = 0; m < n[3]; m++) {
                                    size_t mu = b->sh_bf0[sa] + i, nu = b->sh_bf0[sb] + j,
                                           la = b->sh_bf0[sc] + k, si = b->sh_bf0[sd] + m;
                                    g[((mu * N + nu) * N + la) * N + si] =
                                        blk[((i * n[1] + j) * n[2] + k) * n[3] + m];
                                }
                }
    }
}

/* Schwarz factors Q[sa*nshell+sb] = sqrt(max over components of (ab|ab)). */
void or_schwarz(const or_basis *b, double *Q)
{
    int ns = b->nshell;
#pragma omp parallel for schedule(dynamic, 1)
    for (int sa = 0; sa < ns; sa++) {
        double blk[6 * 6 * 6 * 6];
        for (int sb = 0; sb < ns; sb++) {
            int na = ncart(b->sh_l[sa]), nb = ncart(b->sh_l[sb]);
            or_eri_block(b, sa, sb, sa, sb, blk);
            double mx = 0.0;
            for (int i = 0; i < na; i++)
                for (int j = 0; j < nb; j++) {
                    double v = blk[((i * nb + j) * na + i) * nb + j];
                    if (v > mx) mx = v;
                }
            Q[sa * ns + sb] = sqrt(mx);
        }
    }
}

/* Direct J and K over canonical shell quartets (sa>=sb, sc>=sd,
 * pair(sa,sb) >= pair(sc,sd)) kept by the Schwarz test Q_ab Q_cd >= tau.
 * Each canonical quartet stands for its orbit under the 8-fold
 * permutational symmetry; the factor f = (1/2)^[a=b] (1/2)^[c=d]
 * (1/2)^[ab=cd] makes every ordered index quartet count once.  Half-sums
 * J', K' are symmetrised at the end: J = J' + J'^T, K = K' + K'^T.
 * counts[0] = quartets kept, counts[1] = canonical quartets in total. */
void or_fock_jk(const or_basis *b, const double *D, double tau, const double *Q, double *J,
                double *K, int64_t *counts)
{
    int N = b->nbf, ns = b->nshell;
    double *Jh = (double *)calloc((size_t)N * N, sizeof(double));
    double *Kh = (double *)calloc((size_t)N * N, sizeof(double));
    int64_t kept = 0, total = 0;
#pragma omp parallel
    {
        double *Jt = (double *)calloc((size_t)N * N, sizeof(double));
        double *Kt = (double *)calloc((size_t)N * N, sizeof(double));
        double blk[6 * 6 * 6 * 6];
        int64_t kt = 0, tt = 0;
#pragma omp for schedule(dynamic, 1)
        for (int sa = ns - 1; sa >= 0; sa--) {
            for (int sb = 0; sb <= sa; sb++)
                for (int sc = 0; sc <= sa; sc++)
                    for (int sd = 0; sd <= (sc == sa ? sb : sc); sd++) {
                        tt++;
                        if (Q[sa * ns + sb] * Q[sc * ns + sd] < tau) continue;
                        kt++;
                        or_eri_block(b, sa, sb, sc, sd, blk);
                        double f = 1.0;
                        if (sa == sb) f *= 0.5;
                        if (sc == sd) f *= 0.5;
                        if (sa == sc && sb == sd) f *= 0.5;
                        int n[4] = {ncart(b->sh_l[sa]), ncart(b->sh_l[sb]), ncart(b->sh_l[sc]),
                                    ncart(b->sh_l[sd])};
                        for (int i = 0; i < n[0]; i++)
                            for (int j = 0; j < n[1]; j++)
                                for (int k = 0; k < n[2]; k++)
                                    for (int m = 0; m < n[3]; m++) {
                                        size_t I = b->sh_bf0[sa] + i, Jx = b->sh_bf0[sb] + j,
                                               Kx = b->sh_bf0[sc] + k, Lx = b->sh_bf0[sd] + m;
                                        double v = f * blk[((i * n[1] + j) * n[2] + k) * n[3] + m];
                                        Jt[I * N + Jx] += 2.0 * v * D[Kx * N + Lx];
                                        Jt[Kx * N + Lx] += 2.0 * v * D[I * N + Jx];
                                        Kt[I * N + Kx] += v * D[Jx * N + Lx];
                                        Kt[Jx * N + Kx] += v * D[I * N + Lx];
                                        Kt[I * N + Lx] += v * D[Jx * N + Kx];
                                        Kt[Jx * N + Lx] += v * D[I * N + Kx];
                                    }
                    }
        }
#pragma omp critical
        {
            for (size_t x = 0; x < (size_t)N * N; x++) {
                Jh[x] += Jt[x];
                Kh[x] += Kt[x];
            }
            kept += kt;
            total += tt;
        }
        free(Jt);
        free(Kt);
    }
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            J[i * N + j] = Jh[i * N + j] + Jh[j * N + i];
            K[i * N + j] = Kh[i * N + j] + Kh[j * N + i];
        }
    if (counts) {
        counts[0] = kept;
        counts[1] = total;
    }
    free(Jh);
    free(Kh);
}

/* J and K contributions (already symmetrised) of an explicit list of
 * canonical shell quartets q[4*i..4*i+3] = (sa, sb, sc, sd) with sa >= sb,
 * sc >= sd and pair(sa,sb) >= pair(sc,sd), digested exactly as in
 * or_fock_jk.  Used to time the oracle on a bounded sample of a workload. */
void or_fock_jk_list(const or_basis *b, const double *D, int64_t n, const int *q, double *J,
                     double *K)
{
    int N = b->nbf;
    double *Jh = (double *)calloc((size_t)N * N, sizeof(double));
    double *Kh = (double *)calloc((size_t)N * N, sizeof(double));
#pragma omp parallel
    {
        double *Jt = (double *)calloc((size_t)N * N, sizeof(double));
        double *Kt = (double *)calloc((size_t)N * N, sizeof(double));
        double blk[6 * 6 * 6 * 6];
#pragma omp for schedule(dynamic, 16)
        for (int64_t e = 0; e < n; e++) {
            int sa = q[4 * e], sb = q[4 * e + 1], sc = q[4 * e + 2], sd = q[4 * e + 3];
            or_eri_block(b, sa, sb, sc, sd, blk);
            double f = 1.0;
            if (sa == sb) f *= 0.5;
            if (sc == sd) f *= 0.5;
            if (sa == sc && sb == sd) f *= 0.5;
            int nn[4] = {ncart(b->sh_l[sa]), ncart(b->sh_l[sb]), ncart(b->sh_l[sc]),
                         ncart(b->sh_l[sd])};
            for (int i = 0; i < nn[0]; i++)
                for (int j = 0; j < nn[1]; j++)
                    for (int k = 0; k < nn[2]; k++)
                        for (int m = 0; m < nn[3]; m++) {
                            size_t I = b->sh_bf0[sa] + i, Jx = b->sh_bf0[sb] + j,
                                   Kx = b->sh_bf0[sc] + k, Lx = b->sh_bf0[sd] + m;
                            double v = f * blk[((i * nn[1] + j) * nn[2] + k) * nn[3] + m];
                            Jt[I * N + Jx] += 2.0 * v * D[Kx * N + Lx];
                            Jt[Kx * N + Lx] += 2.0 * v * D[I * N + Jx];
                            Kt[I * N + Kx] += v * D[Jx * N + Lx];
                            Kt[Jx * N + Kx] += v * D[I * N + Lx];
                            Kt[I * N + Lx] += v * D[Jx * N + Kx];
                            Kt[Jx * N + Lx] += v * D[I * N + Kx];
                        }
        }
#pragma omp critical
        {
            for (size_t x = 0; x < (size_t)N * N; x++) {
                Jh[x] += Jt[x];
                Kh[x] += Kt[x];
            }
        }
        free(Jt);
        free(Kt);
    }
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            J[i * N + j] = Jh[i * N + j] + Jh[j * N + i];
            K[i * N + j] = Kh[i * N + j] + Kh[j * N + i];
        }
    free(Jh);
    free(Kh);
}

/* Single elements J_mn = sum_ls (mn|ls) D_ls and K_mn = sum_ls (ml|ns) D_ls
 * straight from their definition (every ordered shell pair on the summed
 * side), keeping a quartet when its Schwarz bound is >= tau.  For sampled
 * checks on systems too large for the full build. */
void or_jk_elements(const or_basis *b, const double *D, double tau, const double *Q, int nel,
                    const int *mus, const int *nus, double *Jout, double *Kout)
{
    int N = b->nbf, ns = b->nshell;
#pragma omp parallel for schedule(dynamic, 1)
    for (int e = 0; e < nel; e++) {
        double blk[6 * 6 * 6 * 6];
        int mu = mus[e], nu = nus[e];
        int sm = b->bf_shell[mu], sn = b->bf_shell[nu];
        int im = mu - b->sh_bf0[sm], in = nu - b->sh_bf0[sn];
        int nn = ncart(b->sh_l[sn]);
        double j = 0.0, k = 0.0;
        for (int sc = 0; sc < ns; sc++)
            for (int sd = 0; sd < ns; sd++) {
                int nc = ncart(b->sh_l[sc]), nd = ncart(b->sh_l[sd]);
                /* J: (sm sn | sc sd) */
                if (Q[sm * ns + sn] * Q[sc * ns + sd] >= tau) {
                    or_eri_block(b, sm, sn, sc, sd, blk);
                    for (int c = 0; c < nc; c++)
                        for (int d = 0; d < nd; d++)
                            j += blk[((im * nn + in) * nc + c) * nd + d] *
                                 D[(b->sh_bf0[sc] + c) * N + b->sh_bf0[sd] + d];
                }
                /* K: (sm sc | sn sd) */
                if (Q[sm * ns + sc] * Q[sn * ns + sd] >= tau) {
                    or_eri_block(b, sm, sc, sn, sd, blk);
                    for (int c = 0; c < nc; c++)
                        for (int d = 0; d < nd; d++)
                            k += blk[((im * nc + c) * nn + in) * nd + d] *
                                 D[(b->sh_bf0[sc] + c) * N + b->sh_bf0[sd] + d];
                }
            }
        Jout[e] = j;
        Kout[e] = k;
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
