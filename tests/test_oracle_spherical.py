"""Pins of the oracle's real solid harmonics and spherical basis (Sec. 2.1.1)
against closed forms and invariants that do not use its own formula."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import spherical as sp
from helpers import random_rotation, transformed


def _laplacian(poly):
    out = {}
    for (a, b, c), v in poly.items():
        for d, e in ((0, a), (1, b), (2, c)):
            if e >= 2:
                k = [a, b, c]
                k[d] -= 2
                out[tuple(k)] = out.get(tuple(k), 0.0) + v * e * (e - 1)
    return out


def _sphere_moment(a, b, c):
    """Integral of x^a y^b z^c over the unit sphere (closed form)."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    return 2.0 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)


def _inner(p, q):
    return sum(v * w * _sphere_moment(a[0] + b[0], a[1] + b[1], a[2] + b[2])
               for a, v in p.items() for b, w in q.items())


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_solid_harmonics_are_harmonic_and_racah_normalised(l):
    hs = {m: sp.solid_harmonic(l, m) for m in range(-l, l + 1)}
    for m, p in hs.items():
        assert all(sum(k) == l for k in p)
        lap = _laplacian(p)
        assert max((abs(v) for v in lap.values()), default=0.0) < 1e-12, (l, m)
        for m2, q in hs.items():
            ref = 4 * math.pi / (2 * l + 1) if m == m2 else 0.0
            assert abs(_inner(p, q) - ref) < 1e-12, (l, m, m2)
    # S_l0 at the pole is the Legendre value P_l(1) = 1
    assert abs(hs[0].get((0, 0, l), 0.0) - 1.0) < 1e-14


def test_explicit_d_harmonics():
    """The five d functions of the textbook table: sqrt3 xy, sqrt3 yz,
    z^2 - (x^2 + y^2)/2, sqrt3 xz, sqrt3/2 (x^2 - y^2)."""
    r3 = math.sqrt(3.0)
    ref = {-2: {(1, 1, 0): r3}, -1: {(0, 1, 1): r3},
           0: {(0, 0, 2): 1.0, (2, 0, 0): -0.5, (0, 2, 0): -0.5},
           1: {(1, 0, 1): r3}, 2: {(2, 0, 0): r3 / 2, (0, 2, 0): -r3 / 2}}
    for m, p in ref.items():
        got = sp.solid_harmonic(2, m)
        assert set(got) == set(p) and all(abs(got[k] - v) < 1e-14 for k, v in p.items())


@pytest.mark.parametrize("l", [2, 3])
def test_span_is_closed_under_rotation(l):
    """S_lm(R r) is a combination of the S_lm'(r): sampled at random points,
    the rotated values lie in the span of the unrotated ones."""
    rng = np.random.default_rng(l)
    R = random_rotation(rng)
    pts = rng.standard_normal((60, 3))

    def ev(p, x):
        return sum(v * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for (a, b, c), v in p.items())
    A = np.stack([ev(sp.solid_harmonic(l, m), pts) for m in range(-l, l + 1)], axis=1)
    Bm = np.stack([ev(sp.solid_harmonic(l, m), pts @ R.T) for m in range(-l, l + 1)], axis=1)
    coef, *_ = np.linalg.lstsq(A, Bm, rcond=None)
    assert np.max(np.abs(A @ coef - Bm)) < 1e-11
    assert np.allclose(coef.T @ coef, np.eye(2 * l + 1), atol=1e-11)   # orthogonal


def test_transform_gives_orthonormal_d_shell_without_s_part():
    """On one d shell the spherical functions are orthonormal, and the
    Cartesian d space splits into them plus r^2 (the s-type combination),
    which is orthogonal to all five."""
    b = synth.water_cluster(1, 0)
    B = oracle.Basis(b)
    S, _, _ = B.one_electron()
    T = sp.transform(list(B.shell_l), S)
    assert T.shape == (21, 20)
    Ss = T.T @ S @ T
    d0 = int(np.flatnonzero(np.asarray(B.shell_l) == 2)[0])
    c0 = int(B.shell_bf0[d0])
    s0 = c0                                   # shells before the d shell are s, s, p
    blk = Ss[s0:s0 + 5, s0:s0 + 5]
    assert np.allclose(blk, np.eye(5), atol=1e-13)
    # r^2 = x^2 + y^2 + z^2 in the unit-norm Cartesian functions: xx, yy, zz
    # each carry sqrt(3!!) = sqrt3 relative to the mixed ones
    r2 = np.zeros(21)
    for k, ex in enumerate(oracle.cart_components(2)):
        if max(ex) == 2:
            r2[c0 + k] = math.sqrt(3.0)
    assert np.max(np.abs(r2 @ S @ T[:, s0:s0 + 5])) < 1e-13
    assert np.allclose(np.diag(Ss), 1.0, atol=1e-13)


def test_spherical_scf_variational_and_rotation_invariant():
    b = synth.water_cluster(1, 3)
    rc = oracle.scf(b, conv_rms_dD=1e-10)
    rs = sp.scf(b, conv_rms_dD=1e-10)
    assert rs["converged"] and rs["nbf"] == 20
    # the spherical space is a subspace of the Cartesian one: E_sph >= E_cart
    assert rs["E_total"] > rc["E_total"] + 1e-6
    R = random_rotation(np.random.default_rng(5))
    rr = sp.scf(transformed(b, R, [0.3, -1.0, 2.0]), conv_rms_dD=1e-10)
    assert abs(rr["E_total"] - rs["E_total"]) < 1e-9
    D = rs["D"]
    P = D / 2
    assert np.allclose(P @ rs["S"] @ P, P, atol=1e-9)
    assert abs(np.trace(D @ rs["S"]) - b["nelec"]) < 1e-9
