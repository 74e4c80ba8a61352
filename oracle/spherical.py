"""Real solid harmonics and the spherical (pure) basis: the oracle's side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): tests and the benchmark's
CPU baseline may use it; the GPU library never does.

Sec. 2.1.1 writes each primitive real solid harmonic Gaussian as a sum over
Cartesian Gaussians of degree l with coefficients S^{lm}_i, taken from the
textbook it cites.  The coefficients here are that textbook's closed form for
the Racah-normalised real solid harmonics S_lm = r^l C_lm, for any l:

  S_lm = N_lm sum_{t=0}^{floor((l-|m|)/2)} sum_{u=0}^{t} sum_{v}
         C^{lm}_{tuv} x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|)
  C^{lm}_{tuv} = (-1)^(t+v-v_m) (1/4)^t binom(l,t) binom(l-t,|m|+t)
                 binom(t,u) binom(|m|,2v)
  N_lm = sqrt(2 (l+|m|)! (l-|m|)! / 2^[m=0]) / (2^|m| l!)

with v_m = 0 for m >= 0 and 1/2 for m < 0, and v running over v_m, v_m + 1,
..., floor(|m|/2 - v_m) + v_m.

Parity status: pinned (tests/test_oracle_spherical.py) by harmonicity
(the Laplacian of every S_lm vanishes), the Racah normalisation and
orthogonality on the unit sphere (int S_lm S_lm' dOmega =
4 pi / (2l + 1) delta_mm'), S_l0 = 1 at the pole, closure of each l-span
under rotations, and, for whole molecules, the variational bound (the
spherical d space lies inside the Cartesian one, so E_sph >= E_cart) and
rotation invariance of the spherical SCF energy.

The spherical basis keeps s and p shells as they are (p in the Cartesian
order x, y, z, i.e. S_11, S_1-1, S_10) and replaces each Cartesian d shell
(6 functions) by the 5 functions m = -2..2.  Every contracted spherical
function is rescaled to unit self-overlap, as the Cartesian ones are.
"""

from fractions import Fraction
from math import comb, factorial, sqrt

import numpy as np

from . import NCART, cart_components


def solid_harmonic(l, m):
    """{(ix, iy, iz): coefficient} of S_lm (Racah normalisation)."""
    am = abs(m)
    vm = Fraction(0) if m >= 0 else Fraction(1, 2)
    N = sqrt(2.0 * factorial(l + am) * factorial(l - am) / (2.0 if m == 0 else 1.0)) / (
        2 ** am * factorial(l))
    out = {}
    for t in range((l - am) // 2 + 1):
        for u in range(t + 1):
            v = vm
            vmax = Fraction((am - 2 * vm) // 2) + vm     # floor(|m|/2 - v_m) + v_m
            while v <= vmax:
                two_v = int(2 * v)
                sign = -1.0 if int(t + v - vm) % 2 else 1.0
                c = sign * 0.25 ** t * comb(l, t) * comb(l - t, am + t) * comb(t, u) * comb(am, two_v)
                ex = (2 * t + am - 2 * u - two_v, 2 * u + two_v, l - 2 * t - am)
                out[ex] = out.get(ex, 0.0) + N * c
                v += 1
    return {k: v for k, v in out.items() if v != 0.0}


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def nsph(l):
    return 2 * l + 1 if l >= 2 else NCART[l]


def transform(shell_l, S):
    """T (N_cart x N_sph): spherical function nu = sum_mu T[mu, nu] phi_mu over
    the Cartesian contracted functions (each of unit self-overlap, in the
    order x^lx y^ly z^lz, lx then ly descending).  S is the Cartesian overlap
    matrix; each column is scaled to unit self-overlap."""
    ncart = sum(NCART[l] for l in shell_l)
    ns = sum(nsph(l) for l in shell_l)
    T = np.zeros((ncart, ns))
    c0 = s0 = 0
    for l in shell_l:
        comps = cart_components(l)
        if l < 2:
            T[c0:c0 + len(comps), s0:s0 + len(comps)] = np.eye(len(comps))
        else:
            for k, m in enumerate(range(-l, l + 1)):
                coef = solid_harmonic(l, m)
                for c, ex in enumerate(comps):
                    # x^i e^{-a r^2} = sqrt(prod (2i-1)!!) phi_c up to a factor
                    # common to the shell
                    scale = sqrt(_dfact(2 * ex[0] - 1) * _dfact(2 * ex[1] - 1) * _dfact(2 * ex[2] - 1))
                    T[c0 + c, s0 + k] = coef.get(ex, 0.0) * scale
        blk = slice(c0, c0 + len(comps))
        for k in range(nsph(l)):
            col = T[blk, s0 + k]
            T[blk, s0 + k] = col / np.sqrt(col @ S[blk, blk] @ col)
        c0 += len(comps)
        s0 += nsph(l)
    return T


def scf(basis, conv_rms_dD=1e-10, conv_dE=0.0, max_iter=100, diis_m=8, tau=0.0, verbose=False):
    """RHF (Sec. 3.2 with DIIS, Sec. 3.2.1) in the spherical basis: the
    one-electron matrices and J, K over spherical functions are the Cartesian
    ones contracted with T on every index (integrals are linear in each
    function), i.e. S' = T^T S T, H' = T^T H T, J'(D') = T^T J(T D' T^T) T and
    likewise K'."""
    from . import Basis, density_from_fock, diis_extrapolate, orthogonalizer
    B = basis if isinstance(basis, Basis) else Basis(basis)
    Sc, Tc, Vc = B.one_electron()
    T = transform(list(B.shell_l), Sc)
    S = T.T @ Sc @ T
    H = T.T @ (Tc + Vc) @ T
    X = orthogonalizer(S)
    nocc = B.nelec // 2
    Q = B.schwarz()
    D, _, _ = density_from_fock(H, X, nocc)
    Enuc = B.nuclear_repulsion()
    Fs, es = [], []
    E_prev = None
    N = T.shape[1]
    converged = False
    for it in range(1, max_iter + 1):
        Jc, Kc = B.fock_jk(T @ D @ T.T, tau, Q)
        F = H + T.T @ (Jc - 0.5 * Kc) @ T
        E = 0.5 * np.sum(D * (H + F))
        err = F @ D @ S - S @ D @ F
        Fuse = F
        Fs.append(F)
        es.append(err)
        if len(Fs) > diis_m:
            Fs.pop(0)
            es.pop(0)
        if len(Fs) >= 2:
            Fx = diis_extrapolate(Fs, es)
            if Fx is not None:
                Fuse = Fx
        Dn, eps, C = density_from_fock(Fuse, X, nocc)
        rms = np.linalg.norm(Dn - D) / N
        dE = 0.0 if E_prev is None else E - E_prev
        if verbose:
            print(f"oracle sph scf {it:3d} E={E + Enuc:.12f} dE={dE:.2e} rmsD={rms:.2e}", flush=True)
        ok = rms < conv_rms_dD and (conv_dE <= 0 or (E_prev is not None and abs(dE) < conv_dE))
        E_prev = E
        if ok:
            converged = True
            break
        D = Dn
    return dict(E_total=E + Enuc, E_elec=E, D=D, F=F, S=S, H=H, T=T, iterations=it,
                converged=converged, nbf=N)
