"""Plain FP64 CPU oracle for the McMurchie-Davidson RHF Fock build.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the GPU library and its Python binding
never do, and the two share no code.

The integrals live in oracle.c (built into liboracle.so with gcc); the SCF
driver below is numpy.  Parity status of each function (what pins it,
besides itself; see tests/test_oracle_pins.py):

  boys            pinned: F_n(0) = 1/(2n+1), F_0 = erf closed form, the
                  incomplete-gamma closed form, mpmath quadrature of the
                  defining integral, both recursions.
  hermite_e       pinned: E^00_0 = kappa, the Hermite expansion identity
                  evaluated pointwise, the 1-D overlap by quadrature.
  hermite_r       pinned: R^0_000 = F_0, finite differences of F_0 in P.
  one_electron    pinned: s-s closed forms, Gauss-Hermite quadrature of S, T
                  and (via the Gaussian transform of 1/r) V for p and d.
  eri_block       pinned: (ss|ss) closed form, brute-force quadrature of
                  primitive p/d integrals (no E, R or Boys inside), 8-fold
                  symmetry, rotation covariance, translation invariance,
                  the Schwarz inequality.
  schwarz         pinned: Q_ab^2 equals the largest diagonal element
                  (mn|mn), m in a, n in b, of the full tensor.
  fock_jk         pinned: literal Eq. fock by einsum over the full tensor.
  fock_jk_list    pinned: over the whole kept canonical list it equals the
                  screened fock_jk; disjoint sublists add up to it.
  jk_elements     pinned: agrees with fock_jk element by element.
  scf             pinned: P S P = P, Tr(D S) = N_elec, FDS - SDF = 0 at
                  convergence, two-centre minimal-basis closed form,
                  invariance under rigid motions and atom permutations,
                  variational rise under idempotent perturbations.
  mcweeny         pinned: fixed points are the SCF densities; the
                  idempotency error falls quadratically on a perturbed one.
  mlp (module)    pinned: finite differences of the loss; the BF16 rounding
                  against torch's own float -> bfloat16 conversion.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(
            os.path.join(_HERE, "oracle.c")):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.or_boys.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    lib.or_hermite_e.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _dp]
    lib.or_hermite_r.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp]
    lib.or_basis_create.restype = ctypes.c_void_p
    lib.or_basis_create.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _ip, _ip, _ip, _ip,
                                    _dp, _dp]
    lib.or_basis_destroy.argtypes = [ctypes.c_void_p]
    lib.or_nbf.argtypes = [ctypes.c_void_p]
    lib.or_nbf.restype = ctypes.c_int
    lib.or_bf_coef.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.or_bf_coef.restype = ctypes.c_double
    lib.or_nuclear_repulsion.argtypes = [ctypes.c_void_p]
    lib.or_nuclear_repulsion.restype = ctypes.c_double
    lib.or_one_electron.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.or_eri_block.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, _dp]
    lib.or_eri_tensor.argtypes = [ctypes.c_void_p, _dp]
    lib.or_schwarz.argtypes = [ctypes.c_void_p, _dp]
    lib.or_fock_jk.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, _dp, _dp, _i64p]
    lib.or_jk_elements.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, ctypes.c_int,
                                   _ip, _ip, _dp, _dp]
    lib.or_fock_jk_list.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, _ip, _dp, _dp]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def set_threads(n):
    _load().or_set_threads(int(n))


def num_threads():
    return _load().or_num_threads()


NCART = (1, 3, 6)


def cart_components(l):
    """Cartesian exponents of a shell, lx descending then ly descending."""
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


# ---------------------------------------------------------------------------
# Boys function, Hermite E and R (one call each, for the pins)
# ---------------------------------------------------------------------------

def boys(nmax, T):
    """[F_0(T), ..., F_nmax(T)]; F_n(x) = int_0^1 exp(-x t^2) t^2n dt (Sec. 2.3.3)."""
    F = np.zeros(nmax + 1)
    _load().or_boys(int(nmax), float(T), _d(F))
    return F


def hermite_e(imax, jmax, a, b, A, B):
    """E[i, j, t] (Eqs. recurrence-A/B), zero for t > i + j."""
    E = np.zeros((imax + 1) * (jmax + 1) * (imax + jmax + 1))
    _load().or_hermite_e(int(imax), int(jmax), float(a), float(b), float(A), float(B), _d(E))
    return E.reshape(imax + 1, jmax + 1, imax + jmax + 1)


def hermite_r(L, a, X, Y, Z):
    """R^0[t, u, v] for t + u + v <= L (Eq. Rn-definition, Eq. R-recursion)."""
    R = np.zeros((L + 1) ** 3)
    _load().or_hermite_r(int(L), float(a), float(X), float(Y), float(Z), _d(R))
    return R.reshape(L + 1, L + 1, L + 1)


# ---------------------------------------------------------------------------
# Basis-level integrals
# ---------------------------------------------------------------------------

class Basis:
    """A contracted Cartesian basis: primitives normalised to <G|G> = 1, each
    contracted Cartesian function rescaled to unit self-overlap."""

    def __init__(self, basis):
        lib = _load()
        self.src = basis
        self._keep = [np.ascontiguousarray(basis["xyz"], dtype=np.float64).ravel(),
                      np.ascontiguousarray(basis["Z"], dtype=np.float64),
                      np.ascontiguousarray(basis["shell_atom"], dtype=np.int32),
                      np.ascontiguousarray(basis["shell_l"], dtype=np.int32),
                      np.ascontiguousarray(basis["shell_nprim"], dtype=np.int32),
                      np.ascontiguousarray(basis["shell_prim0"], dtype=np.int32),
                      np.ascontiguousarray(basis["exps"], dtype=np.float64),
                      np.ascontiguousarray(basis["coefs"], dtype=np.float64)]
        k = self._keep
        self.natom = len(k[1])
        self.nshell = len(k[2])
        self.h = lib.or_basis_create(self.natom, _d(k[0]), _d(k[1]), self.nshell, _i(k[2]),
                                     _i(k[3]), _i(k[4]), _i(k[5]), _d(k[6]), _d(k[7]))
        self.nbf = lib.or_nbf(self.h)
        self.nelec = int(basis["nelec"])
        self.shell_l = k[3]
        self.shell_nprim = k[4]
        self.shell_bf0 = np.concatenate([[0], np.cumsum([NCART[l] for l in k[3]])[:-1]]).astype(int)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_basis_destroy(self.h)
            self.h = None

    def bf_coef(self, mu, k):
        return _lib.or_bf_coef(self.h, int(mu), int(k))

    def nuclear_repulsion(self):
        """E_nuc = sum_{A<B} Z_A Z_B / R_AB."""
        return _lib.or_nuclear_repulsion(self.h)

    def one_electron(self):
        """(S, T, V): Eqs. s-overall, Tab-final and Vab-final, contracted."""
        N = self.nbf
        S, T, V = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
        _lib.or_one_electron(self.h, _d(S), _d(T), _d(V))
        return S, T, V

    def eri_block(self, sa, sb, sc, sd):
        """Contracted block (ab|cd) over Cartesian components (Eq. twoe-final)."""
        n = [NCART[self.shell_l[s]] for s in (sa, sb, sc, sd)]
        out = np.zeros(n[0] * n[1] * n[2] * n[3])
        _lib.or_eri_block(self.h, int(sa), int(sb), int(sc), int(sd), _d(out))
        return out.reshape(n)

    def eri_tensor(self):
        """Full (mn|ls) tensor, every ordered shell quartet on its own."""
        N = self.nbf
        if N > 64:
            raise ValueError("full ERI tensor only for N <= 64")
        g = np.zeros(N ** 4)
        _lib.or_eri_tensor(self.h, _d(g))
        return g.reshape(N, N, N, N)

    def schwarz(self):
        """Q[a, b] = sqrt(max over components (ab|ab))."""
        Q = np.zeros(self.nshell * self.nshell)
        _lib.or_schwarz(self.h, _d(Q))
        return Q.reshape(self.nshell, self.nshell)

    def fock_jk(self, D, tau=0.0, Q=None, with_counts=False):
        """Direct J, K over canonical Schwarz-kept shell quartets."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        if Q is None:
            Q = self.schwarz()
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        N = self.nbf
        J, K = np.zeros((N, N)), np.zeros((N, N))
        counts = np.zeros(2, dtype=np.int64)
        _lib.or_fock_jk(self.h, _d(D), float(tau), _d(Q), _d(J), _d(K),
                        counts.ctypes.data_as(_i64p))
        if with_counts:
            return J, K, (int(counts[0]), int(counts[1]))
        return J, K

    def jk_elements(self, D, mus, nus, tau=0.0, Q=None):
        """J_mn and K_mn for the listed (mu, nu) straight from their definition."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        if Q is None:
            Q = self.schwarz()
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        mus = np.ascontiguousarray(mus, dtype=np.int32)
        nus = np.ascontiguousarray(nus, dtype=np.int32)
        Jo, Ko = np.zeros(len(mus)), np.zeros(len(mus))
        _lib.or_jk_elements(self.h, _d(D), float(tau), _d(Q), len(mus), _i(mus), _i(nus),
                            _d(Jo), _d(Ko))
        return Jo, Ko


    def fock_jk_list(self, D, quartets):
        """J, K contributions of an explicit list of canonical shell quartets."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
        N = self.nbf
        J, K = np.zeros((N, N)), np.zeros((N, N))
        _lib.or_fock_jk_list(self.h, _d(D), len(q), _i(q), _d(J), _d(K))
        return J, K


def jk_from_tensor(g, D):
    """Eq. fock applied literally: J_mn = sum_ls (mn|ls) D_ls,
    K_mn = sum_ls (ml|ns) D_ls."""
    J = np.einsum("mnls,ls->mn", g, D)
    K = np.einsum("mlns,ls->mn", g, D)
    return J, K


# ---------------------------------------------------------------------------
# SCF (Sec. 3.2) with DIIS (Sec. 3.2.1)
# ---------------------------------------------------------------------------

def orthogonalizer(S):
    """Symmetric orthogonalisation X = U s^-1/2 U^T."""
    s, U = np.linalg.eigh(S)
    return (U / np.sqrt(s)) @ U.T


def density_from_fock(F, X, nocc):
    """F' = X^T F X, diagonalise, C = X C', D = 2 C_occ C_occ^T (aufbau on
    the lowest nocc eigenvalues)."""
    eps, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    Co = C[:, :nocc]
    return 2.0 * Co @ Co.T, eps, C


def mcweeny(D, S, iters):
    """McWeeny purification of a closed-shell density (an extension: not in
    the paper): with P = D / 2, P <- 3 P S P - 2 P S P S P, repeated.
    Returns the purified D and ||PSP - P||_F / ||P||_F before and after."""
    P = 0.5 * np.asarray(D, dtype=np.float64)

    def err(P):
        return np.linalg.norm(P @ S @ P - P) / max(np.linalg.norm(P), 1e-300)

    e0 = err(P)
    for _ in range(iters):
        PS = P @ S
        P = 3.0 * PS @ P - 2.0 * PS @ PS @ P
    return 2.0 * P, e0, err(P)


def diis_extrapolate(Fs, es):
    """Bordered DIIS system: B_ij = Tr(e_i^T e_j), sum c_i = 1; returns
    sum c_i F_i, or None when the system is singular."""
    m = len(Fs)
    B = -np.ones((m + 1, m + 1))
    B[m, m] = 0.0
    for i in range(m):
        for j in range(m):
            B[i, j] = np.sum(es[i] * es[j])
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    try:
        c = np.linalg.solve(B, rhs)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(c)):
        return None
    return sum(ci * Fi for ci, Fi in zip(c[:m], Fs))


def scf(basis, tau=0.0, conv_rms_dD=1e-10, conv_dE=0.0, max_iter=100, diis_m=8, D0=None,
        use_diis=True, verbose=False):
    """Restricted Hartree-Fock by the SCF of Sec. 3.2.

    Each iteration n: F(D_n) = H + J - K/2;  E_n = 1/2 Tr[D_n (H + F(D_n))];
    DIIS on e = F D S - S D F (m most recent pairs, from two pairs on);
    F' = X^T F X, diagonalise, D_{n+1} = 2 C_occ C_occ^T.  Converged when
    RMS(D_{n+1} - D_n) < conv_rms_dD and (if conv_dE > 0) |E_n - E_{n-1}| < conv_dE.
    """
    B = basis if isinstance(basis, Basis) else Basis(basis)
    S, T, V = B.one_electron()
    H = T + V
    X = orthogonalizer(S)
    nocc = B.nelec // 2
    Q = B.schwarz()
    if D0 is None:
        D, _, _ = density_from_fock(H, X, nocc)
    else:
        D = np.array(D0, dtype=np.float64)
    Enuc = B.nuclear_repulsion()
    Fs, es = [], []
    E_prev = None
    hist = []
    converged = False
    N = B.nbf
    for it in range(1, max_iter + 1):
        J, K = B.fock_jk(D, tau, Q)
        F = H + J - 0.5 * K
        E = 0.5 * np.sum(D * (H + F))
        err = F @ D @ S - S @ D @ F
        Fuse = F
        if use_diis:
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
        hist.append(dict(iter=it, E=E + Enuc, dE=dE, rms_dD=rms, comm=np.linalg.norm(err)))
        if verbose:
            print(f"oracle scf {it:3d}  E={E + Enuc:.12f}  dE={dE:.2e}  rmsD={rms:.2e}", flush=True)
        ok = rms < conv_rms_dD and (conv_dE <= 0 or (E_prev is not None and abs(dE) < conv_dE))
        E_prev = E
        if ok:
            converged = True
            break
        D = Dn
    return dict(E_total=E + Enuc, E_elec=E, E_nuc=Enuc, D=D, D_next=Dn, F=F, C=C, eps=eps,
                S=S, H=H, X=X, iterations=it, converged=converged, history=hist)
