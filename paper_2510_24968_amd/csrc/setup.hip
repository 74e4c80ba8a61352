// Once-per-geometry kernels: the Boys grid, shell normalisation, the
// shell-pair tables (Sec. 2.1.2 Gaussian product, Sec. 2.1.3 Hermite
// coefficients, Eq. E-tuv) and the one-electron matrices S, T, V
// (Eqs. s-overall, Tab-final, Vab-final).
#include "boys.h"
#include "fsim_internal.h"

namespace fsim {

// ---------------------------------------------------------------------------
// Boys grid: F_n(T_k) for n < BOYS_NORD by the power series of the highest
// order, F_N(T) = exp(-T) sum_i (2T)^i / ((2N+1)(2N+3)...(2N+2i+1)), followed
// by the (stable) downward recursion.
// ---------------------------------------------------------------------------
__global__ void k_boys_table(double *tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= BOYS_NT) return;
    const double T = k * BOYS_DT;
    const int N = BOYS_NORD - 1;
    double term = 1.0 / (2 * N + 1), sum = term;
    for (int i = 1; i < 2000; ++i) {
        term *= 2.0 * T / (2 * N + 2 * i + 1);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    const double e = exp(-T);
    double f = e * sum;
    tab[k * BOYS_NORD + N] = f;
    for (int n = N; n > 0; --n) {
        f = (2.0 * T * f + e) / (2 * n - 1);
        tab[k * BOYS_NORD + n - 1] = f;
    }
}

hipError_t launch_boys_table(double *tab, hipStream_t s) {
    hipLaunchKernelGGL(k_boys_table, dim3((BOYS_NT + 127) / 128), dim3(128), 0, s, tab);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shell normalisation.  Primitive radial factor (2a/pi)^(3/4) (4a)^(l/2);
// the component factor prod (2 l_i - 1)!!^(-1/2) is applied per component in
// the pair tables.  The contracted function is then rescaled to unit norm:
// with c_k = d_k N(a_k), <phi|phi> = sum_kl c_k c_l (pi/p)^(3/2) / (2p)^l,
// p = a_k + a_l (the same for every Cartesian component of the shell).
// ---------------------------------------------------------------------------
__global__ void k_shell_norm(ShellsDev sh) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= sh.nshell) return;
    const int l = sh.l[s], np = sh.nprim[s], p0 = sh.prim0[s];
    double c[MAXPRIM];
    for (int k = 0; k < np; ++k) {
        const double a = sh.exps[p0 + k];
        c[k] = sh.coef[p0 + k] * pow(2.0 * a / M_PI, 0.75) * pow(4.0 * a, 0.5 * l);
    }
    double ss = 0.0;
    for (int k = 0; k < np; ++k)
        for (int m = 0; m < np; ++m) {
            const double p = sh.exps[p0 + k] + sh.exps[p0 + m];
            ss += c[k] * c[m] * pow(M_PI / p, 1.5) / pow(2.0 * p, (double)l);
        }
    const double r = 1.0 / sqrt(ss);
    for (int k = 0; k < np; ++k) sh.coef[p0 + k] = c[k] * r;
}

hipError_t launch_shell_norm(const ShellsDev &sh, hipStream_t s) {
    hipLaunchKernelGGL(k_shell_norm, dim3((sh.nshell + 127) / 128), dim3(128), 0, s, sh);
    return hipGetLastError();
}

// 1 / sqrt((2lx-1)!! (2ly-1)!! (2lz-1)!!) for component c of shell l.
__host__ __device__ constexpr double comp_norm(int l, int c) {
    double d = 1.0;
    for (int dir = 0; dir < 3; ++dir)
        for (int k = 2 * cart_exp(l, c, dir) - 1; k > 1; k -= 2) d *= k;
    return d == 1.0 ? 1.0 : (d == 3.0 ? 0.57735026918962576451 : 1.0 / __builtin_sqrt(d));
}

// One-direction Hermite coefficients E^{ij}_t, i <= IM, j <= JM (Sec. 2.1.3:
// E^{00}_0 = exp(-mu X_AB^2); recurrence-A raises i with X_PA, recurrence-B
// raises j with X_PB; zero outside 0 <= t <= i + j).
template <int IM, int JM>
struct Herm1D {
    double e[IM + 1][JM + 1][IM + JM + 1];
    __device__ __forceinline__ void build(double a, double b, double A, double B) {
        const double p = a + b, P = (a * A + b * B) / p;
        const double xpa = P - A, xpb = P - B, xab = A - B, h = 0.5 / p;
#pragma unroll
        for (int i = 0; i <= IM; ++i)
#pragma unroll
            for (int j = 0; j <= JM; ++j)
#pragma unroll
                for (int t = 0; t <= IM + JM; ++t) e[i][j][t] = 0.0;
        e[0][0][0] = exp(-a * b / p * xab * xab);
#pragma unroll
        for (int i = 0; i <= IM; ++i) {
#pragma unroll
            for (int j = 0; j <= JM; ++j) {
                if (i == 0 && j == 0) continue;
                const int pi = i > 0 ? i - 1 : 0, pj = i > 0 ? j : j - 1;
                const double x = i > 0 ? xpa : xpb;
#pragma unroll
                for (int t = 0; t <= i + j; ++t) {
                    double v = (t <= pi + pj) ? x * e[pi][pj][t] : 0.0;
                    if (t >= 1) v += h * e[pi][pj][t - 1];
                    if (t + 1 <= pi + pj) v += (t + 1) * e[pi][pj][t + 1];
                    e[i][j][t] = v;
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Pair tables, one thread per (pair, primitive-pair slot).
// ---------------------------------------------------------------------------
template <int L1, int L2>
__global__ void k_build_pairs(ShellsDev sh, PairTable t, const int *__restrict__ ps1,
                              const int *__restrict__ ps2) {
    constexpr int N1 = ncart(L1), N2 = ncart(L2), NE = n_entries(L1, L2);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= t.n * t.kmax) return;
    const int pr = idx % t.n, k = idx / t.n;
    const int s1 = ps1[pr], s2 = ps2[pr];
    const int np1 = sh.nprim[s1], np2 = sh.nprim[s2];
    if (k == 0) {
        t.sh1[pr] = s1;
        t.sh2[pr] = s2;
        t.bf1[pr] = sh.bf0[s1];
        t.bf2[pr] = sh.bf0[s2];
        t.mol[pr] = sh.mol[s1];
        t.nprim[pr] = np1 * np2;
    }
    const size_t n = t.n;
    if (k >= np1 * np2) {   // padding slot: contributes exactly zero
        t.p[k * n + pr] = 1.0;
        for (int d = 0; d < 3; ++d) t.P[(k * 3 + d) * n + pr] = 0.0;
        for (int e = 0; e < NE; ++e) {
            t.E[((size_t)k * NE + e) * n + pr] = 0.0;
            t.Ef[((size_t)k * NE + e) * n + pr] = 0.0f;
        }
        return;
    }
    const int k1 = k / np2, k2 = k - k1 * np2;
    const double a = sh.exps[sh.prim0[s1] + k1], b = sh.exps[sh.prim0[s2] + k2];
    const double p = a + b;
    const double *A = sh.xyz + 3 * s1, *B = sh.xyz + 3 * s2;
    t.p[k * n + pr] = p;
    Herm1D<L1, L2> h[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t.P[(k * 3 + d) * n + pr] = (a * A[d] + b * B[d]) / p;
        h[d].build(a, b, A[d], B[d]);
    }
    // each pair carries the square root of the 2 pi^(5/2) of Eq. twoe-final
    const double scale = sh.coef[sh.prim0[s1] + k1] * sh.coef[sh.prim0[s2] + k2] *
                         sqrt(2.0 * M_PI * M_PI * sqrt(M_PI)) / p;
#pragma unroll
    for (int cp = 0; cp < N1 * N2; ++cp) {
        const int c1 = cp / N2, c2 = cp % N2;
        const int ix = cart_exp(L1, c1, 0), iy = cart_exp(L1, c1, 1), iz = cart_exp(L1, c1, 2);
        const int jx = cart_exp(L2, c2, 0), jy = cart_exp(L2, c2, 1), jz = cart_exp(L2, c2, 2);
        const double cs = scale * comp_norm(L1, c1) * comp_norm(L2, c2);
        int e = box_off(L1, L2, cp);
#pragma unroll
        for (int tt = 0; tt <= ix + jx; ++tt)
#pragma unroll
            for (int uu = 0; uu <= iy + jy; ++uu)
#pragma unroll
                for (int vv = 0; vv <= iz + jz; ++vv) {
                    const double v = cs * h[0].e[ix][jx][tt] * h[1].e[iy][jy][uu] *
                                     h[2].e[iz][jz][vv];
                    t.E[((size_t)k * NE + e) * n + pr] = v;
                    t.Ef[((size_t)k * NE + e) * n + pr] = (float)v;
                    ++e;
                }
    }
}

hipError_t launch_build_pairs(const ShellsDev &sh, PairTable &t, const int *ps1, const int *ps2,
                              hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    const int total = t.n * t.kmax;
    dim3 g((total + 127) / 128), b(128);
    switch (pclass(t.l1, t.l2)) {
        case 0: hipLaunchKernelGGL((k_build_pairs<0, 0>), g, b, 0, s, sh, t, ps1, ps2); break;
        case 1: hipLaunchKernelGGL((k_build_pairs<1, 0>), g, b, 0, s, sh, t, ps1, ps2); break;
        case 2: hipLaunchKernelGGL((k_build_pairs<1, 1>), g, b, 0, s, sh, t, ps1, ps2); break;
        case 3: hipLaunchKernelGGL((k_build_pairs<2, 0>), g, b, 0, s, sh, t, ps1, ps2); break;
        case 4: hipLaunchKernelGGL((k_build_pairs<2, 1>), g, b, 0, s, sh, t, ps1, ps2); break;
        case 5: hipLaunchKernelGGL((k_build_pairs<2, 2>), g, b, 0, s, sh, t, ps1, ps2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Primitive-pair screening, one thread per pair.  The Hermite distribution
// Omega_k of primitive pair k and component pair cp is the sum of the slot's
// box entries E_tuv times Hermite Gaussians of exponent p at P; by the
// Cauchy-Schwarz inequality of the Coulomb inner product its part of any
// integral (ab|cd) is at most sqrt((Omega_k|Omega_k)) Q_cd.  The
// self-repulsion is Eq. twoe-final with both pairs equal (q = p, R_PQ = 0,
// alpha = p/2), where R^0_tuv vanishes unless t, u, v are all even and is
// otherwise (-p)^s (t-1)!! (u-1)!! (v-1)!! / (2s + 1), s = (t + u + v) / 2
// (the Taylor coefficients of F_0 at zero).  The table's entries carry
// sqrt(2 pi^(5/2)) / p each, so the sum is scaled by 1 / sqrt(2p) only.
// Slots whose bound times the molecule's largest shell-pair factor falls
// below tau_prim are dropped; the kept ones move to the front in their
// original order and the freed slots become zero padding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double odd_dfact(int n) {   // (n - 1)!! for even n >= 0
    double r = 1.0;
    for (int k = n - 1; k > 1; k -= 2) r *= k;
    return r;
}

template <int L1, int L2>
__global__ void k_prim_screen(PairTable t, const double *__restrict__ qmax_mol, double tau_prim) {
    constexpr int NCP = ncart(L1) * ncart(L2), NE = n_entries(L1, L2);
    const int pr = blockIdx.x * blockDim.x + threadIdx.x;
    if (pr >= t.n) return;
    const size_t n = t.n;
    const int np = t.nprim[pr];
    const double qm = qmax_mol[t.mol[pr]];
    int kept = 0;
    for (int k = 0; k < np; ++k) {
        const double p = t.p[k * n + pr];
        const double *E = t.E + (size_t)k * NE * n + pr;
        double q2 = 0.0;
        for (int cp = 0; cp < NCP; ++cp) {
            const int bx = box_dim(L1, L2, cp, 0), by = box_dim(L1, L2, cp, 1),
                      bz = box_dim(L1, L2, cp, 2), eo = box_off(L1, L2, cp);
            double s = 0.0;
            for (int t1 = 0; t1 <= bx; ++t1)
                for (int u1 = 0; u1 <= by; ++u1)
                    for (int v1 = 0; v1 <= bz; ++v1) {
                        const double e1 = E[(size_t)(eo + (t1 * (by + 1) + u1) * (bz + 1) + v1) * n];
                        for (int t2 = t1 & 1; t2 <= bx; t2 += 2)
                            for (int u2 = u1 & 1; u2 <= by; u2 += 2)
                                for (int v2 = v1 & 1; v2 <= bz; v2 += 2) {
                                    const double e2 =
                                        E[(size_t)(eo + (t2 * (by + 1) + u2) * (bz + 1) + v2) * n];
                                    const int tt = t1 + t2, uu = u1 + u2, vv = v1 + v2;
                                    const int sh = (tt + uu + vv) / 2;
                                    double r = odd_dfact(tt) * odd_dfact(uu) * odd_dfact(vv) /
                                               (2 * sh + 1);
                                    for (int m = 0; m < sh; ++m) r *= -p;
                                    if ((t2 + u2 + v2) & 1) r = -r;
                                    s += e1 * e2 * r;
                                }
                    }
            q2 = fmax(q2, s);
        }
        const double bound = sqrt(fmax(q2, 0.0) * rsqrt(2.0 * p));
        if (bound * qm >= tau_prim) {
            if (kept != k) {
                t.p[kept * n + pr] = p;
                for (int d = 0; d < 3; ++d) t.P[(kept * 3 + d) * n + pr] = t.P[(k * 3 + d) * n + pr];
                for (int e = 0; e < NE; ++e) {
                    t.E[((size_t)kept * NE + e) * n + pr] = t.E[((size_t)k * NE + e) * n + pr];
                    t.Ef[((size_t)kept * NE + e) * n + pr] = t.Ef[((size_t)k * NE + e) * n + pr];
                }
            }
            ++kept;
        }
    }
    for (int k = kept; k < np; ++k) {
        t.p[k * n + pr] = 1.0;
        for (int d = 0; d < 3; ++d) t.P[(k * 3 + d) * n + pr] = 0.0;
        for (int e = 0; e < NE; ++e) {
            t.E[((size_t)k * NE + e) * n + pr] = 0.0;
            t.Ef[((size_t)k * NE + e) * n + pr] = 0.0f;
        }
    }
    t.nprim[pr] = kept;
}

hipError_t launch_prim_screen(PairTable &t, const double *qmax_mol, double tau_prim,
                              hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    dim3 g((t.n + 127) / 128), b(128);
    switch (pclass(t.l1, t.l2)) {
        case 0: hipLaunchKernelGGL((k_prim_screen<0, 0>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        case 1: hipLaunchKernelGGL((k_prim_screen<1, 0>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        case 2: hipLaunchKernelGGL((k_prim_screen<1, 1>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        case 3: hipLaunchKernelGGL((k_prim_screen<2, 0>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        case 4: hipLaunchKernelGGL((k_prim_screen<2, 1>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        case 5: hipLaunchKernelGGL((k_prim_screen<2, 2>), g, b, 0, s, t, qmax_mol, tau_prim); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-electron matrices, one thread per (mu, nu).
//   S_ab = E^{ij}_0 E^{kl}_0 E^{mn}_0 (pi/p)^(3/2)                 (Eq. s-overall)
//   T_ab = sum over directions of
//          [-2 b^2 E^{i,j+2}_0 + b(2j+1) E^{ij}_0 - j(j-1)/2 E^{i,j-2}_0]
//          x (other two E_0) (pi/p)^(3/2)                          (Eq. Tab-final)
//   V_ab = -sum_C Z_C (2 pi / p) sum_tuv E_t E_u E_v R^0_tuv(p, P - C)
//                                                                   (Eq. Vab-final)
// ---------------------------------------------------------------------------
struct BfInfo {
    int shell, lx, ly, lz;
};

__device__ inline void r_table_rt(int L, const double *src, double X, double Y, double Z,
                                  double *r) {
    // in-place Hermite Coulomb recursion (Eq. R-recursion), graded storage
    r[0] = src[L];
    for (int n = L - 1; n >= 0; --n) {
        for (int s = L - n; s >= 1; --s) {
            for (int a = s; a >= 0; --a)      // a = u + v, t = s - a
                for (int v = a; v >= 0; --v) {
                    const int t = s - a, u = a - v;
                    double val;
                    if (t > 0) {
                        val = X * r[hidx(t - 1, u, v)];
                        if (t > 1) val += (t - 1) * r[hidx(t - 2, u, v)];
                    } else if (u > 0) {
                        val = Y * r[hidx(t, u - 1, v)];
                        if (u > 1) val += (u - 1) * r[hidx(t, u - 2, v)];
                    } else {
                        val = Z * r[hidx(t, u, v - 1)];
                        if (v > 1) val += (v - 1) * r[hidx(t, u, v - 2)];
                    }
                    r[hidx(t, u, v)] = val;
                }
        }
        r[0] = src[n];
    }
}

__global__ void k_one_electron(ShellsDev sh, const double *__restrict__ boys,
                               const int *__restrict__ bf_shell, const int *__restrict__ bf_comp,
                               double *S, double *T, double *V) {
    // one molecule per grid z, element (mu, nu) of its packed block
    const int m = blockIdx.z, nm = sh.mol_n[m];
    const int mu = blockIdx.y, nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (mu >= nm || nu >= nm) return;
    const int g0 = sh.mol_bf0[m];
    const int s1 = bf_shell[g0 + mu], s2 = bf_shell[g0 + nu];
    const int l1 = sh.l[s1], l2 = sh.l[s2];
    const int c1 = bf_comp[g0 + mu], c2 = bf_comp[g0 + nu];
    int i[3], j[3];
    for (int d = 0; d < 3; ++d) {
        i[d] = cart_exp(l1, c1, d);
        j[d] = cart_exp(l2, c2, d);
    }
    const double n12 = comp_norm(l1, c1) * comp_norm(l2, c2);
    const double *A = sh.xyz + 3 * s1, *B = sh.xyz + 3 * s2;
    double sacc = 0.0, tacc = 0.0, vacc = 0.0;
    for (int k1 = 0; k1 < sh.nprim[s1]; ++k1)
        for (int k2 = 0; k2 < sh.nprim[s2]; ++k2) {
            const double a = sh.exps[sh.prim0[s1] + k1], b = sh.exps[sh.prim0[s2] + k2];
            const double p = a + b;
            const double cc = sh.coef[sh.prim0[s1] + k1] * sh.coef[sh.prim0[s2] + k2] * n12;
            Herm1D<2, 4> h[3];
            double P[3];
            for (int d = 0; d < 3; ++d) {
                h[d].build(a, b, A[d], B[d]);
                P[d] = (a * A[d] + b * B[d]) / p;
            }
            const double pp = M_PI / p, f3 = pp * sqrt(pp);
            double e0[3], tk[3];
            for (int d = 0; d < 3; ++d) {
                e0[d] = h[d].e[i[d]][j[d]][0];
                double v = -2.0 * b * b * h[d].e[i[d]][j[d] + 2][0] +
                           b * (2 * j[d] + 1) * h[d].e[i[d]][j[d]][0];
                if (j[d] >= 2) v -= 0.5 * j[d] * (j[d] - 1) * h[d].e[i[d]][j[d] - 2][0];
                tk[d] = v;
            }
            sacc += cc * e0[0] * e0[1] * e0[2] * f3;
            tacc += cc * f3 * (tk[0] * e0[1] * e0[2] + e0[0] * tk[1] * e0[2] + e0[0] * e0[1] * tk[2]);
            const int L = l1 + l2;
            double vsum = 0.0;
            const int a0 = sh.mol_atom0[m];
            for (int C = a0; C < a0 + sh.mol_natom[m]; ++C) {
                const double X = P[0] - sh.atom_xyz[3 * C], Y = P[1] - sh.atom_xyz[3 * C + 1],
                             Zc = P[2] - sh.atom_xyz[3 * C + 2];
                double F[2 * LMAX + 1], src[2 * LMAX + 1], r[nherm(2 * LMAX)];
                boys_eval_rt(L, p * (X * X + Y * Y + Zc * Zc), boys, F);
                double m = 1.0;
                for (int n = 0; n <= L; ++n) {
                    src[n] = m * F[n];
                    m *= -2.0 * p;
                }
                r_table_rt(L, src, X, Y, Zc, r);
                double acc = 0.0;
                for (int tt = 0; tt <= i[0] + j[0]; ++tt)
                    for (int uu = 0; uu <= i[1] + j[1]; ++uu)
                        for (int vv = 0; vv <= i[2] + j[2]; ++vv)
                            acc += h[0].e[i[0]][j[0]][tt] * h[1].e[i[1]][j[1]][uu] *
                                   h[2].e[i[2]][j[2]][vv] * r[hidx(tt, uu, vv)];
                vsum -= sh.atom_Z[C] * acc;
            }
            vacc += cc * 2.0 * M_PI / p * vsum;
        }
    const size_t o = (size_t)sh.mol_off[m] + (size_t)mu * nm + nu;
    S[o] = sacc;
    T[o] = tacc;
    V[o] = vacc;
}

hipError_t launch_one_electron_impl(const ShellsDev &sh, const double *boys, int nmax,
                                    const int *bf_shell, const int *bf_comp, double *S,
                                    double *T, double *V, hipStream_t s) {
    dim3 g((nmax + 63) / 64, nmax, sh.nmol), b(64);
    hipLaunchKernelGGL(k_one_electron, g, b, 0, s, sh, boys, bf_shell, bf_comp, S, T, V);
    return hipGetLastError();
}

}  // namespace fsim
