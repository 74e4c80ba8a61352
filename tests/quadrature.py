"""Independent numerical integrators for pinning the oracle.

Nothing here uses Hermite expansions, Hermite Coulomb integrals or the Boys
function: overlaps and kinetic integrals come from Gauss-Hermite quadrature of
the Cartesian Gaussians themselves, and the Coulomb operators from the
Gaussian transform 1/r = (2/sqrt(pi)) int_0^inf exp(-s^2 r^2) ds, with the
inner Gaussian integrals done exactly by Gauss-Hermite and the outer s
integral by adaptive quadrature.
"""

import math

import numpy as np
from numpy.polynomial import polynomial as P
from scipy import integrate

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(12)


def _poly_shift(i, A):
    """Coefficients (ascending) of (x - A)^i."""
    c = np.array([1.0])
    for _ in range(i):
        c = P.polymul(c, [-A, 1.0])
    return c


def overlap_1d(i, a, A, j, b, B):
    """int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) dx by Gauss-Hermite."""
    p = a + b
    Px = (a * A + b * B) / p
    K = math.exp(-a * b / p * (A - B) ** 2)
    x = Px + _GH_X / math.sqrt(p)
    f = (x - A) ** i * (x - B) ** j
    return K * np.sum(_GH_W * f) / math.sqrt(p)


def kinetic_1d(i, a, A, j, b, B):
    """-1/2 int G_i(a, x_A) d^2/dx^2 G_j(b, x_B) dx, the derivative taken on the
    polynomial-times-Gaussian directly (numpy polynomial algebra)."""
    # g(x) = poly(x) * exp(-b (x-B)^2); g'' = (poly'' - 4b(x-B) poly' + (4b^2 (x-B)^2 - 2b) poly) e
    pj = _poly_shift(j, B)
    xb = np.array([-B, 1.0])
    d1 = P.polyder(pj)
    d2 = P.polyder(pj, 2)
    second = P.polyadd(P.polyadd(d2, P.polymul([-4 * b], P.polymul(xb, d1))),
                       P.polymul(P.polyadd(P.polymul([4 * b * b], P.polymul(xb, xb)), [-2 * b]), pj))
    p = a + b
    Px = (a * A + b * B) / p
    K = math.exp(-a * b / p * (A - B) ** 2)
    x = Px + _GH_X / math.sqrt(p)
    f = (x - A) ** i * P.polyval(x, second)
    return -0.5 * K * np.sum(_GH_W * f) / math.sqrt(p)


def overlap_3d(la, a, A, lb, b, B):
    return np.prod([overlap_1d(la[k], a, A[k], lb[k], b, B[k]) for k in range(3)])


def kinetic_3d(la, a, A, lb, b, B):
    s = [overlap_1d(la[k], a, A[k], lb[k], b, B[k]) for k in range(3)]
    t = [kinetic_1d(la[k], a, A[k], lb[k], b, B[k]) for k in range(3)]
    return t[0] * s[1] * s[2] + s[0] * t[1] * s[2] + s[0] * s[1] * t[2]


def nuclear_3d(la, a, A, lb, b, B, C):
    """int G_a G_b / |r - C| dr (the positive operator 1/r_C)."""
    p = a + b

    def inner(s):
        out = 1.0
        for k in range(3):
            # exponent a(x-A)^2 + b(x-B)^2 + s^2 (x-C)^2
            e = p + s * s
            cx = (a * A[k] + b * B[k] + s * s * C[k]) / e
            c0 = a * A[k] ** 2 + b * B[k] ** 2 + s * s * C[k] ** 2 - e * cx * cx
            x = cx + _GH_X / math.sqrt(e)
            f = (x - A[k]) ** la[k] * (x - B[k]) ** lb[k]
            out *= math.exp(-c0) * np.sum(_GH_W * f) / math.sqrt(e)
        return out

    val, _ = integrate.quad(inner, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
    return 2.0 / math.sqrt(math.pi) * val


_GH2_X, _GH2_W = np.polynomial.hermite.hermgauss(10)


def _coulomb_1d(i, a, A, j, b, B, k, c, C, l, d, D, s2):
    """int int (x1-A)^i (x1-B)^j (x2-C)^k (x2-D)^l
    exp(-a(x1-A)^2 - b(x1-B)^2 - c(x2-C)^2 - d(x2-D)^2 - s2 (x1-x2)^2) dx1 dx2."""
    M = np.array([[a + b + s2, -s2], [-s2, c + d + s2]])
    rhs = np.array([a * A + b * B, c * C + d * D])
    m = np.linalg.solve(M, rhs)
    const = a * A * A + b * B * B + c * C * C + d * D * D - m @ M @ m
    Lc = np.linalg.cholesky(M)            # M = Lc Lc^T
    Linv_T = np.linalg.inv(Lc.T)
    y1, y2 = np.meshgrid(_GH2_X, _GH2_X, indexing="ij")
    w = np.outer(_GH2_W, _GH2_W)
    Y = np.stack([y1.ravel(), y2.ravel()])
    Xp = m[:, None] + Linv_T @ Y
    x1, x2 = Xp
    f = (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k * (x2 - D) ** l
    return math.exp(-const) * np.sum(w.ravel() * f) / np.prod(np.diag(Lc))


def eri_primitive(la, a, A, lb, b, B, lc, c, C, ld, d, D):
    """[ab|cd] over unnormalised primitive Cartesian Gaussians by the Gaussian
    transform of 1/r12."""

    def inner(s):
        s2 = s * s
        out = 1.0
        for k in range(3):
            out *= _coulomb_1d(la[k], a, A[k], lb[k], b, B[k], lc[k], c, C[k], ld[k], d, D[k], s2)
        return out

    val, _ = integrate.quad(inner, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
    return 2.0 / math.sqrt(math.pi) * val
