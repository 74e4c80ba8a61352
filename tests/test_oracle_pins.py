"""Pins for the FP64 oracle: closed forms, independent quadrature, symmetries
and SCF invariants.  Nothing here compares the oracle with itself only."""

import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
import quadrature as qd
import synth
from helpers import custom_basis, random_rotation, spd_molecule, transformed

# ---------------------------------------------------------------------------
# Boys function (Sec. 2.3.3 definition; the paper gives no evaluation method)
# ---------------------------------------------------------------------------


def test_boys_at_zero():
    F = oracle.boys(12, 0.0)
    for n in range(13):
        assert F[n] == pytest.approx(1.0 / (2 * n + 1), rel=1e-15)


@pytest.mark.parametrize("T", [1e-9, 1e-4, 0.1, 1.0, 5.0, 17.3, 29.999, 30.0, 30.001, 45.0, 120.0])
def test_boys_f0_is_erf(T):
    ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    assert oracle.boys(0, T)[0] == pytest.approx(ref, rel=2e-15)


def test_boys_incomplete_gamma_closed_form():
    # F_n(T) = gamma(n + 1/2, T) / (2 T^(n + 1/2)), lower incomplete gamma
    Ts = np.concatenate([np.logspace(-6, 0, 13), np.linspace(1.3, 29.9, 23), [30.0, 30.2],
                         np.linspace(31, 200, 9)])
    for T in Ts:
        F = oracle.boys(10, T)
        for n in range(11):
            ref = special.gammainc(n + 0.5, T) * special.gamma(n + 0.5) / (2.0 * T ** (n + 0.5))
            assert F[n] == pytest.approx(ref, rel=5e-13, abs=1e-300), (n, T)


@pytest.mark.parametrize("T,n", [(0.3, 0), (0.3, 8), (7.7, 3), (29.9, 8), (30.1, 8), (55.0, 5)])
def test_boys_quadrature(T, n):
    mpmath.mp.dps = 30
    ref = mpmath.quad(lambda t: mpmath.e ** (-T * t * t) * t ** (2 * n), [0, 1])
    assert oracle.boys(n, T)[n] == pytest.approx(float(ref), rel=1e-13)


def test_boys_recursions_hold_across_branches():
    # the downward identity checked in the upward branch and vice versa
    for T in (3.0, 12.0, 29.0, 31.0, 60.0):
        F = oracle.boys(9, T)
        et = math.exp(-T)
        for n in range(1, 10):
            assert F[n - 1] == pytest.approx((2 * T * F[n] + et) / (2 * n - 1), rel=1e-13)


# ---------------------------------------------------------------------------
# Hermite expansion coefficients (Sec. 2.1.3)
# ---------------------------------------------------------------------------


def test_hermite_e00_is_kappa():
    a, b, A, B = 0.7, 1.9, 0.3, -1.1
    E = oracle.hermite_e(0, 0, a, b, A, B)
    assert E[0, 0, 0] == pytest.approx(math.exp(-a * b / (a + b) * (A - B) ** 2), rel=1e-15)


@pytest.mark.parametrize("a,b,A,B", [(0.7, 1.9, 0.3, -1.1), (0.15, 2.4, 0.0, 1.4),
                                     (3.0, 0.2, -0.4, 0.9)])
def test_hermite_expansion_identity(a, b, A, B):
    # x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = sum_t E_t^ij Lambda_t(x_P),
    # Lambda_t(x_P) = p^(t/2) H_t(sqrt(p) x_P) exp(-p x_P^2)
    p = a + b
    Px = (a * A + b * B) / p
    E = oracle.hermite_e(4, 4, a, b, A, B)
    xs = np.random.default_rng(1).uniform(-2.5, 2.5, 9)
    for i in range(5):
        for j in range(5):
            for x in xs:
                lhs = (x - A) ** i * (x - B) ** j * math.exp(-a * (x - A) ** 2 - b * (x - B) ** 2)
                y = math.sqrt(p) * (x - Px)
                rhs = 0.0
                for t in range(i + j + 1):
                    c = np.zeros(t + 1)
                    c[t] = 1.0
                    rhs += E[i, j, t] * p ** (t / 2) * np.polynomial.hermite.hermval(y, c) * \
                        math.exp(-y * y)
                assert rhs == pytest.approx(lhs, rel=1e-11, abs=1e-14), (i, j, x)
            # zero outside 0 <= t <= i + j
            assert np.all(E[i, j, i + j + 1:] == 0.0)


# ---------------------------------------------------------------------------
# Hermite Coulomb integrals (Eq. Rn-definition, Eq. R-recursion)
# ---------------------------------------------------------------------------


def test_hermite_r_source():
    a, X, Y, Z = 0.8, 0.3, -0.7, 1.2
    R = oracle.hermite_r(0, a, X, Y, Z)
    assert R[0, 0, 0] == pytest.approx(oracle.boys(0, a * (X * X + Y * Y + Z * Z))[0], rel=1e-15)


@pytest.mark.parametrize("a,X,Y,Z", [(0.8, 0.3, -0.7, 1.2), (2.5, 1.9, 0.4, -2.2),
                                     (0.05, 3.0, -1.0, 0.5)])
def test_hermite_r_is_derivative_of_f0(a, X, Y, Z):
    # R^0_tuv = d^t/dX^t d^u/dY^u d^v/dZ^v F_0(a (X^2 + Y^2 + Z^2))
    mpmath.mp.dps = 40

    def f0(x, y, z):
        T = a * (x * x + y * y + z * z)
        return mpmath.sqrt(mpmath.pi / T) * mpmath.erf(mpmath.sqrt(T)) / 2

    L = 4
    R = oracle.hermite_r(L, a, X, Y, Z)
    for t in range(L + 1):
        for u in range(L + 1 - t):
            for v in range(L + 1 - t - u):
                ref = float(mpmath.diff(f0, (X, Y, Z), (t, u, v)))
                assert R[t, u, v] == pytest.approx(ref, rel=1e-10, abs=1e-13), (t, u, v)


# ---------------------------------------------------------------------------
# Normalisation and one-electron integrals (Sec. 2.3.1 - 2.3.3)
# ---------------------------------------------------------------------------


def _contracted(B, mu, shell):
    """(exponents, normalised coefficients) of basis function mu."""
    src = B.src
    p0, n = src["shell_prim0"][shell], src["shell_nprim"][shell]
    return src["exps"][p0:p0 + n], [B.bf_coef(mu, k) for k in range(n)]


def _bf_list(B):
    out = []
    src = B.src
    for s in range(B.nshell):
        A = src["xyz"][src["shell_atom"][s]]
        for comp in oracle.cart_components(src["shell_l"][s]):
            out.append((s, comp, A))
    return out


def test_normalisation_by_quadrature():
    B = oracle.Basis(spd_molecule())
    for mu, (s, comp, A) in enumerate(_bf_list(B)):
        ex, d = _contracted(B, mu, s)
        norm = sum(d[k] * d[m] * qd.overlap_3d(comp, ex[k], A, comp, ex[m], A)
                   for k in range(len(ex)) for m in range(len(ex)))
        assert norm == pytest.approx(1.0, rel=1e-13)
        # relative primitive weights follow the raw coefficients times the
        # primitive norms <G|G>^-1/2 (computed here by quadrature)
        src = B.src
        raw = src["coefs"][src["shell_prim0"][s]:src["shell_prim0"][s] + len(ex)]
        for k in range(1, len(ex)):
            nk = qd.overlap_3d(comp, ex[k], A, comp, ex[k], A) ** -0.5
            n0 = qd.overlap_3d(comp, ex[0], A, comp, ex[0], A) ** -0.5
            assert d[k] / d[0] == pytest.approx(raw[k] * nk / (raw[0] * n0), rel=1e-12)


def test_one_electron_by_quadrature():
    B = oracle.Basis(spd_molecule())
    S, T, V = B.one_electron()
    bfs = _bf_list(B)
    src = B.src
    rng = np.random.default_rng(5)
    N = B.nbf
    pairs = [(m, n) for m in range(N) for n in range(N)]
    for (mu, nu) in pairs:
        s1, c1, A = bfs[mu]
        s2, c2, Bc = bfs[nu]
        e1, d1 = _contracted(B, mu, s1)
        e2, d2 = _contracted(B, nu, s2)
        sref = sum(d1[k] * d2[m] * qd.overlap_3d(c1, e1[k], A, c2, e2[m], Bc)
                   for k in range(len(e1)) for m in range(len(e2)))
        tref = sum(d1[k] * d2[m] * qd.kinetic_3d(c1, e1[k], A, c2, e2[m], Bc)
                   for k in range(len(e1)) for m in range(len(e2)))
        assert S[mu, nu] == pytest.approx(sref, rel=1e-11, abs=1e-13)
        assert T[mu, nu] == pytest.approx(tref, rel=1e-11, abs=1e-13)
    # nuclear attraction on a random subset (adaptive quadrature is slow)
    for idx in rng.choice(len(pairs), 12, replace=False):
        mu, nu = pairs[idx]
        s1, c1, A = bfs[mu]
        s2, c2, Bc = bfs[nu]
        e1, d1 = _contracted(B, mu, s1)
        e2, d2 = _contracted(B, nu, s2)
        vref = 0.0
        for C in range(len(src["Z"])):
            vref -= src["Z"][C] * sum(
                d1[k] * d2[m] * qd.nuclear_3d(c1, e1[k], A, c2, e2[m], Bc, src["xyz"][C])
                for k in range(len(e1)) for m in range(len(e2)))
        assert V[mu, nu] == pytest.approx(vref, rel=1e-10, abs=1e-12), (mu, nu)
    assert np.allclose(S, S.T, atol=1e-15) and np.allclose(np.diag(S), 1.0, atol=1e-14)


def test_ss_one_electron_closed_forms():
    a, b = 0.9, 0.35
    A, Bc = np.array([0.0, 0.0, 0.0]), np.array([0.4, -1.0, 0.8])
    basis = custom_basis([(A, 2.0, [(0, [a], [1.0])]), (Bc, 1.0, [(0, [b], [1.0])])])
    B = oracle.Basis(basis)
    S, T, V = B.one_electron()
    p = a + b
    kap = math.exp(-a * b / p * np.sum((A - Bc) ** 2))
    n = B.bf_coef(0, 0) * B.bf_coef(1, 0)
    assert S[0, 1] == pytest.approx(n * (math.pi / p) ** 1.5 * kap, rel=1e-14)
    P = (a * A + b * Bc) / p
    vref = 0.0
    for Z, C in ((2.0, A), (1.0, Bc)):
        vref -= Z * 2 * math.pi / p * kap * oracle.boys(0, p * np.sum((P - C) ** 2))[0]
    assert V[0, 1] == pytest.approx(n * vref, rel=1e-13)


def test_nuclear_repulsion():
    b = synth.h_chain(4, 1.4)
    ref = sum(1.0 / (1.4 * abs(i - j)) for i in range(4) for j in range(i))
    assert oracle.Basis(b).nuclear_repulsion() == pytest.approx(ref, rel=1e-15)


# ---------------------------------------------------------------------------
# Electron-repulsion integrals (Sec. 2.3.4, 2.5)
# ---------------------------------------------------------------------------


def test_eri_ssss_closed_form():
    ex = [0.8, 0.3, 1.7, 0.55]
    cen = [np.array(c) for c in ([0, 0, 0], [0.6, 0.2, -0.4], [-1.0, 0.7, 0.5], [0.3, -0.9, 1.1])]
    basis = custom_basis([(cen[k], 1.0, [(0, [ex[k]], [1.0])]) for k in range(4)])
    B = oracle.Basis(basis)
    a, b, c, d = ex
    p, q = a + b, c + d
    P = (a * cen[0] + b * cen[1]) / p
    Q = (c * cen[2] + d * cen[3]) / q
    kab = math.exp(-a * b / p * np.sum((cen[0] - cen[1]) ** 2))
    kcd = math.exp(-c * d / q * np.sum((cen[2] - cen[3]) ** 2))
    al = p * q / (p + q)
    ref = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * kab * kcd * \
        0.5 * math.sqrt(math.pi / (al * np.sum((P - Q) ** 2))) * math.erf(
            math.sqrt(al * np.sum((P - Q) ** 2)))
    nrm = np.prod([B.bf_coef(k, 0) for k in range(4)])
    assert B.eri_block(0, 1, 2, 3)[0, 0, 0, 0] == pytest.approx(nrm * ref, rel=1e-14)


def _single_prim_molecule():
    return custom_basis([
        ([0.0, 0.0, 0.0], 1.0, [(2, [0.9], [1.0]), (1, [0.6], [1.0])]),
        ([0.7, -0.4, 0.5], 1.0, [(1, [1.3], [1.0]), (0, [0.45], [1.0])]),
        ([-0.6, 0.9, -0.3], 1.0, [(2, [0.5], [1.0]), (0, [1.6], [1.0])]),
    ])


@pytest.mark.parametrize("quartet", [(3, 2, 5, 3), (1, 2, 1, 2), (0, 3, 5, 2), (0, 4, 0, 1),
                                     (0, 2, 4, 1), (0, 0, 4, 4), (1, 0, 2, 4)])
def test_eri_by_brute_force_quadrature(quartet):
    """Primitive p/d integrals against the Gaussian transform of 1/r12 with
    exact Gauss-Hermite inner integrals: no E, R or Boys function inside."""
    basis = _single_prim_molecule()
    B = oracle.Basis(basis)
    blk = B.eri_block(*quartet)
    shells = [(basis["shell_l"][s], basis["exps"][basis["shell_prim0"][s]],
               basis["xyz"][basis["shell_atom"][s]], B.shell_bf0[s]) for s in quartet]
    comps = [oracle.cart_components(l) for (l, _, _, _) in shells]
    rng = np.random.default_rng(sum(quartet))
    idx = list(np.ndindex(*blk.shape))
    for k in rng.choice(len(idx), min(6, len(idx)), replace=False):
        ia, ib, ic, id_ = idx[k]
        ref = qd.eri_primitive(comps[0][ia], shells[0][1], shells[0][2],
                               comps[1][ib], shells[1][1], shells[1][2],
                               comps[2][ic], shells[2][1], shells[2][2],
                               comps[3][id_], shells[3][1], shells[3][2])
        nrm = (B.bf_coef(shells[0][3] + ia, 0) * B.bf_coef(shells[1][3] + ib, 0) *
               B.bf_coef(shells[2][3] + ic, 0) * B.bf_coef(shells[3][3] + id_, 0))
        assert blk[ia, ib, ic, id_] == pytest.approx(nrm * ref, rel=1e-10, abs=1e-13), \
            (quartet, ia, ib, ic, id_)


@pytest.fixture(scope="module")
def spd_tensor():
    B = oracle.Basis(spd_molecule())
    return B, B.eri_tensor()


def test_eri_eightfold_symmetry(spd_tensor):
    _, g = spd_tensor
    for perm in ("nmls", "mnsl", "nmsl", "lsmn", "slmn", "lsnm", "slnm"):
        assert np.allclose(np.einsum(f"mnls->{perm}", g), g, rtol=0, atol=1e-14), perm


def test_eri_schwarz_inequality(spd_tensor):
    _, g = spd_tensor
    N = g.shape[0]
    diag = np.einsum("mnmn->mn", g)
    assert np.all(diag >= -1e-15)
    bound = np.sqrt(np.maximum(diag, 0)).reshape(N, N, 1, 1) * \
        np.sqrt(np.maximum(diag, 0)).reshape(1, 1, N, N)
    assert np.all(np.abs(g) <= bound * (1 + 1e-12) + 1e-15)


def test_eri_translation_invariance(spd_tensor):
    _, g = spd_tensor
    g2 = oracle.Basis(transformed(spd_molecule(), shift=[3.1, -2.0, 0.7])).eri_tensor()
    assert np.allclose(g2, g, rtol=0, atol=1e-13)


def _cart_transform(l, R):
    """T with m_c(R^T y) = sum_c' T[c, c'] m_c'(y) for the Cartesian monomials
    of degree l, rescaled for unit-normalised components."""
    comps = oracle.cart_components(l)
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((40, 3))
    Yr = Y @ R          # rows: (R^T y)^T
    Mnew = np.array([[np.prod(y ** np.array(c)) for c in comps] for y in Y])
    Mold = np.array([[np.prod(y ** np.array(c)) for c in comps] for y in Yr])
    T = np.linalg.lstsq(Mnew, Mold, rcond=None)[0].T
    # normalised components: n_c proportional to prod (2 l_i - 1)!!^-1/2
    dfac = lambda k: np.prod(np.arange(2 * k - 1, 0, -2)) if k > 0 else 1.0
    n = np.array([1.0 / math.sqrt(np.prod([dfac(k) for k in c])) for c in comps])
    return (n[:, None] * T) / n[None, :]


def test_eri_rotation_covariance(spd_tensor):
    B, g = spd_tensor
    R = random_rotation(np.random.default_rng(11))
    g2 = oracle.Basis(transformed(spd_molecule(), R=R)).eri_tensor()
    N = B.nbf
    M = np.zeros((N, N))
    for s in range(B.nshell):
        l = B.shell_l[s]
        o = B.shell_bf0[s]
        n = oracle.NCART[l]
        M[o:o + n, o:o + n] = _cart_transform(l, R)
    g_rot = np.einsum("ai,bj,ck,dl,ijkl->abcd", M, M, M, M, g2, optimize=True)
    assert np.allclose(g_rot, g, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# J / K digest (Eq. fock) and Schwarz screening
# ---------------------------------------------------------------------------


def _random_density(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    return 0.5 * (A + A.T)


def test_digest_equals_full_tensor(spd_tensor):
    B, g = spd_tensor
    D = _random_density(B.nbf, 3)
    J, K = B.fock_jk(D, tau=0.0)
    Jr, Kr = oracle.jk_from_tensor(g, D)
    assert np.allclose(J, Jr, rtol=0, atol=1e-12)
    assert np.allclose(K, Kr, rtol=0, atol=1e-12)


def test_digest_equals_full_tensor_water():
    B = oracle.Basis(synth.water_cluster(2, 0))
    g = B.eri_tensor()
    D = _random_density(B.nbf, 4)
    J, K, (kept, total) = B.fock_jk(D, tau=0.0, with_counts=True)
    ns = B.nshell
    npair = ns * (ns + 1) // 2
    assert kept == total == npair * (npair + 1) // 2
    Jr, Kr = oracle.jk_from_tensor(g, D)
    assert np.allclose(J, Jr, rtol=0, atol=1e-12)
    assert np.allclose(K, Kr, rtol=0, atol=1e-12)


def test_jk_elements_match_digest(spd_tensor):
    B, _ = spd_tensor
    D = _random_density(B.nbf, 8)
    J, K = B.fock_jk(D)
    mus = np.arange(B.nbf)
    nus = (mus * 7 + 3) % B.nbf
    Je, Ke = B.jk_elements(D, mus, nus)
    assert np.allclose(Je, J[mus, nus], rtol=0, atol=1e-12)
    assert np.allclose(Ke, K[mus, nus], rtol=0, atol=1e-12)


def test_jk_positive_for_density():
    B = oracle.Basis(synth.water_cluster(2, 1))
    S, T, V = B.one_electron()
    X = oracle.orthogonalizer(S)
    D, _, _ = oracle.density_from_fock(T + V, X, B.nelec // 2)
    J, K = B.fock_jk(D)
    assert 0.5 * np.sum(D * J) > 0 and 0.5 * np.sum(D * K) > 0


def test_screening_error_is_bounded():
    B = oracle.Basis(synth.water_cluster(3, 2))
    S, T, V = B.one_electron()
    X = oracle.orthogonalizer(S)
    D, _, _ = oracle.density_from_fock(T + V, X, B.nelec // 2)
    Q = B.schwarz()
    tau = 1e-7
    J0, K0, (k0, t0) = B.fock_jk(D, 0.0, Q, with_counts=True)
    J1, K1, (k1, t1) = B.fock_jk(D, tau, Q, with_counts=True)
    assert t0 == t1 and k1 < k0
    # every skipped quartet contributes at most tau * |D| per element, at most
    # 8 orbit images x (dropped quartets) in total
    bound = 8 * (k0 - k1) * tau * np.max(np.abs(D)) * 6 ** 2
    assert np.max(np.abs(J1 - J0)) < bound and np.max(np.abs(K1 - K0)) < bound
    assert np.max(np.abs(J1 - J0)) > 0


@pytest.mark.parametrize("which", ["spd", "water_dimer"])
def test_schwarz_factor_is_diagonal_tensor_maximum(which):
    """Q_ab^2 is the largest diagonal integral (mn|mn) over the components
    m of shell a and n of shell b, read here from the full tensor (each
    element from its own quartet evaluation)."""
    basis = spd_molecule() if which == "spd" else synth.water_cluster(2, 1)
    B = oracle.Basis(basis)
    g = B.eri_tensor()
    Q = B.schwarz()
    N = B.nbf
    diag = g.reshape(N * N, N * N)[np.arange(N * N), np.arange(N * N)].reshape(N, N)
    shell_of = np.concatenate([[s] * oracle.NCART[l] for s, l in enumerate(B.shell_l)])
    for a in range(B.nshell):
        for b in range(B.nshell):
            mx = diag[np.ix_(shell_of == a, shell_of == b)].max()
            assert abs(Q[a, b] ** 2 - mx) <= 1e-14 * mx, (a, b)
    assert np.max(np.abs(Q - Q.T)) <= 1e-14 * Q.max()


def _canonical_quartets(B, Q, tau):
    """Every canonical shell quartet (a >= b, c >= d, pair (a,b) >= pair
    (c,d) in lexicographic order) with Q_ab Q_cd >= tau."""
    pairs = [(a, b) for a in range(B.nshell) for b in range(a + 1)]
    out = []
    for i, (a, b) in enumerate(pairs):
        for c, d in pairs[:i + 1]:
            if Q[a, b] * Q[c, d] >= tau:
                out.append((a, b, c, d))
    return np.array(out, dtype=np.int32)


def test_quartet_list_digest_equals_screened_build():
    """fock_jk_list over the whole kept canonical list of a water trimer is
    the screened fock_jk, and two disjoint halves of the list add up to it
    (J and K are linear in the quartet set)."""
    B = oracle.Basis(synth.water_cluster(3, 2))
    S, T, V = B.one_electron()
    X = oracle.orthogonalizer(S)
    D, _, _ = oracle.density_from_fock(T + V, X, B.nelec // 2)
    Q = B.schwarz()
    tau = 1e-9
    J, K, (kept, total) = B.fock_jk(D, tau, Q, with_counts=True)
    q = _canonical_quartets(B, Q, tau)
    npair = B.nshell * (B.nshell + 1) // 2
    assert len(q) == kept and total == npair * (npair + 1) // 2
    Jl, Kl = B.fock_jk_list(D, q)
    scale = max(np.abs(J).max(), np.abs(K).max())
    assert np.max(np.abs(Jl - J)) <= 1e-13 * scale
    assert np.max(np.abs(Kl - K)) <= 1e-13 * scale
    rng = np.random.default_rng(7)
    pick = rng.random(len(q)) < 0.5
    J1, K1 = B.fock_jk_list(D, q[pick])
    J2, K2 = B.fock_jk_list(D, q[~pick])
    assert np.max(np.abs(J1 + J2 - J)) <= 1e-13 * scale
    assert np.max(np.abs(K1 + K2 - K)) <= 1e-13 * scale
    # a quartet listed twice counts twice
    J3, _ = B.fock_jk_list(D, np.concatenate([q, q[:1]]))
    J4, _ = B.fock_jk_list(D, q[:1])
    assert np.max(np.abs(J3 - J - J4)) <= 1e-13 * scale


# ---------------------------------------------------------------------------
# SCF (Sec. 3.2, 3.2.1)
# ---------------------------------------------------------------------------


@pytest.fixture(scope="module")
def water_scf():
    b = synth.water_cluster(1, 0)
    return b, oracle.scf(b, conv_rms_dD=1e-10, conv_dE=1e-12)


def test_scf_converged_invariants(water_scf):
    b, r = water_scf
    assert r["converged"]
    D, S, F = r["D"], r["S"], r["F"]
    P = D / 2
    assert np.allclose(P @ S @ P, P, atol=1e-8)
    assert np.trace(D @ S) == pytest.approx(b["nelec"], abs=1e-9)
    assert np.linalg.norm(F @ D @ S - S @ D @ F) < 1e-7


def test_scf_two_centre_closed_form():
    """H2-like: one s function per centre, two electrons.  The occupied
    orbital is fixed by symmetry, g = (phi1 + phi2) / sqrt(2 + 2 S12), so
    E_elec = 2 h_gg + (gg|gg)."""
    basis = custom_basis([([0, 0, 0], 1.0, [(0, [1.2, 0.3], [0.5, 0.6])]),
                          ([0, 0, 1.4], 1.0, [(0, [1.2, 0.3], [0.5, 0.6])])])
    B = oracle.Basis(basis)
    S, T, V = B.one_electron()
    H = T + V
    g = B.eri_tensor()
    s = S[0, 1]
    hgg = (H[0, 0] + H[0, 1]) / (1 + s)
    gggg = (2 * g[0, 0, 0, 0] + 2 * g[0, 0, 1, 1] + 4 * g[0, 1, 0, 1] + 8 * g[0, 0, 0, 1]) / \
        (4 * (1 + s) ** 2)
    r = oracle.scf(basis, conv_rms_dD=1e-12)
    assert r["E_elec"] == pytest.approx(2 * hgg + gggg, abs=1e-12)
    assert r["iterations"] <= 2


def test_scf_rigid_motion_and_permutation_invariance():
    b = synth.water_cluster(2, 5)
    E0 = oracle.scf(b, conv_rms_dD=1e-9, conv_dE=1e-11)["E_total"]
    R = random_rotation(np.random.default_rng(2))
    E1 = oracle.scf(transformed(b, R=R, shift=[1.0, -2.0, 0.5]), conv_rms_dD=1e-9,
                    conv_dE=1e-11)["E_total"]
    assert E1 == pytest.approx(E0, abs=1e-9)
    # reverse the atom order
    order = list(range(len(b["Z"])))[::-1]
    b2 = synth.assemble([b["types"][i] for i in order], b["xyz"][order])
    E2 = oracle.scf(b2, conv_rms_dD=1e-9, conv_dE=1e-11)["E_total"]
    assert E2 == pytest.approx(E0, abs=1e-9)


def test_scf_energy_is_variational(water_scf):
    b, r = water_scf
    B = oracle.Basis(b)
    C = r["C"]
    nocc = b["nelec"] // 2
    S, H = r["S"], r["H"]
    E0 = r["E_elec"]
    rng = np.random.default_rng(0)
    for _ in range(3):
        kappa = np.zeros((B.nbf, B.nbf))
        kappa[:nocc, nocc:] = 1e-2 * rng.standard_normal((nocc, B.nbf - nocc))
        kappa = kappa - kappa.T
        w, U = np.linalg.eig(kappa)
        Uk = np.real(U @ np.diag(np.exp(w)) @ np.linalg.inv(U))
        C2 = C @ Uk
        D2 = 2 * C2[:, :nocc] @ C2[:, :nocc].T
        P2 = D2 / 2
        assert np.allclose(P2 @ S @ P2, P2, atol=1e-10)
        J, K = B.fock_jk(D2)
        E2 = 0.5 * np.sum(D2 * (2 * H + J - 0.5 * K))
        assert E2 > E0


def test_h8_density_has_inversion_symmetry():
    b = synth.h_chain(8, 1.4)
    r = oracle.scf(b, conv_rms_dD=1e-10)
    D = r["D"]
    rev = np.arange(8)[::-1]
    assert np.allclose(D[np.ix_(rev, rev)], D, atol=1e-9)
