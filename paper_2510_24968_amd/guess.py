"""Learned initial guess for the SCF (an extension; the paper starts from the
core-Hamiltonian guess, Sec. 2 "initial guess").

A 3-layer network (64 -> 256 -> 256 -> 36, ReLU, BF16 weights, FP32
accumulation on the matrix cores through the library's fsim_gemm_bf16) maps
the features of a shell pair (A, a), (B, b) to that pair's density block:

* features: 32 Gaussian radial functions of R_AB (centres k * 12/31 bohr,
  width 12/31), one-hot element types of A and B, one-hot shell slots of a
  and b on their atoms (slot, not l: two s shells on one atom are different
  functions);
* output: the block in a bond-aligned frame (z' along A -> B), at most 6 x 6
  Cartesian components, masked to the shells' sizes.  It is projected onto
  the blocks that the bond's own symmetry group (rotations about z' and
  mirror planes through it) leaves unchanged, then rotated to the molecular
  frame with the Cartesian transformation of each shell.  On-site blocks
  (A = B) use R = 0 and are projected onto the O(3)-invariant blocks.  With
  invariant features, the assembled density is then exactly covariant under
  rigid rotations and reflections of the molecule;
* pairs farther apart than 12 bohr are set to zero.

The assembled density is symmetrised and McWeeny-purified (fsim_purify); if
it still departs from idempotency by more than 1e-2 (||PSP - P||_F / ||P||_F,
P = D/2) the core-Hamiltonian guess is used instead.

Training targets are converged densities produced by this library's own
FP64 SCF on seeded H chains and water-like clusters.
"""

import ctypes
import math
import time

import numpy as np
import torch
from numpy.polynomial.legendre import leggauss

from . import fsim

TYPES = ("Hc", "O", "Hw", "C", "Hr")
NSLOT = 4
NRBF = 32
RCUT = 12.0
RBF_MU = np.arange(NRBF) * RCUT / (NRBF - 1)
RBF_SIGMA = RCUT / (NRBF - 1)
NIN, NHID, NOUT = 64, 256, 36
NCART = (1, 3, 6)


def _lib():
    L = fsim.lib()
    if not getattr(L, "_guess_sigs", False):
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        for name, args in {
            "fsim_gemm_bf16": [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, vp, vp, i32,
                               i32, vp],
            "fsim_f32_to_bf16": [i64, vp, vp, vp],
            "fsim_relu_backward": [i64, vp, vp, vp, vp],
            "fsim_bias_grad": [i32, i32, vp, vp, vp],
            "fsim_mse": [i64, vp, vp, vp, f32, vp, vp, vp],
            "fsim_adam": [i64, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp, vp],
            "fsim_mlp_pack": [i32, i32, vp, vp, vp],
            "fsim_mlp_forward": [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "fsim_purify": [vp, vp, i32, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), vp],
        }.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L._guess_sigs = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _chk(st):
    if st != 0:
        raise fsim.FsimError(f"fsim error {st}: {fsim.lib().fsim_last_error().decode()}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# Cartesian transformations of shells under orthogonal maps
# ---------------------------------------------------------------------------

def cart_components(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


# generic probe points: monomials of degree <= 2 are linearly independent on them
_PROBE = np.random.default_rng(12345).standard_normal((40, 3))
_EXPS = [np.array(cart_components(l)) for l in range(3)]
_NORM = [np.array([1.0 / math.sqrt(np.prod([_dfact(2 * k - 1) for k in c])) for c in cart_components(l)])
         for l in range(3)]
_PINV = [np.linalg.pinv(np.prod(_PROBE[:, None, :] ** _EXPS[l][None], axis=2)) for l in range(3)]


def cart_rotation(l, R):
    """T (..., nc, nc) with phi'_c = sum_c' T[c, c'] phi_c' for unit-normalised
    Cartesian components, phi' being the shell written in the coordinates
    y' = R y (R orthogonal, batched over leading axes)."""
    R = np.asarray(R, dtype=np.float64)
    Yr = np.einsum("ij,...kj->...ik", _PROBE, R)                  # (..., 40, 3) = R y_i
    Mrot = np.prod(Yr[..., None, :] ** _EXPS[l], axis=-1)         # (..., 40, nc)
    C = np.swapaxes(_PINV[l] @ Mrot, -1, -2)                      # m_c(Ry) = sum C[c,c'] m_c'(y)
    return _NORM[l][:, None] * C / _NORM[l][None, :]


def bond_frames(d):
    """Rotations (P, 3, 3) whose last row is the unit vector along each d."""
    z = d / np.linalg.norm(d, axis=1, keepdims=True)
    e = np.eye(3)[np.argmin(np.abs(z), axis=1)]
    x = np.cross(e, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def _group_bond():
    """Rotations about z by multiples of 2 pi / 8, with and without the mirror
    y -> -y: averaging over them is exact for blocks of l <= 2 shells (angular
    frequencies up to 4 about the axis)."""
    out = []
    for k in range(8):
        c, s = math.cos(2 * math.pi * k / 8), math.sin(2 * math.pi * k / 8)
        R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
        out += [R, R @ np.diag([1.0, -1.0, 1.0])]
    return np.array(out), np.full(len(out), 1.0 / len(out))


def _group_site():
    """Quadrature over O(3): Euler angles with 5 equal steps in the two
    azimuths and 3-point Gauss-Legendre in cos(beta), times inversion.  Exact
    for polynomials of degree <= 4 in the entries of R (blocks of l <= 2
    shells are at most that)."""
    x, w = leggauss(3)
    rz = lambda a: np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0],
                             [0.0, 0.0, 1.0]])
    Rs, Ws = [], []
    for i in range(5):
        for j in range(3):
            cb, sb = x[j], math.sqrt(1.0 - x[j] ** 2)
            Ry = np.array([[cb, 0.0, sb], [0.0, 1.0, 0.0], [-sb, 0.0, cb]])
            for k in range(5):
                R = rz(2 * math.pi * i / 5) @ Ry @ rz(2 * math.pi * k / 5)
                for sgn in (1.0, -1.0):
                    Rs.append(sgn * R)
                    Ws.append(w[j] / 2.0 / 25.0 / 2.0)
    return np.array(Rs), np.array(Ws)


def _projectors(group):
    """36 x 36 projector per (la, lb) on the flattened 6 x 6 block: the group
    average of D' -> T_g^T D' T_g (embedded in the top-left na x nb corner)."""
    Rs, Ws = group
    P = {}
    for la in range(3):
        Ta = cart_rotation(la, Rs)
        for lb in range(3):
            Tb = cart_rotation(lb, Rs)
            na, nb = NCART[la], NCART[lb]
            M = np.zeros((36, 36))
            for i in range(na):
                for j in range(nb):
                    E = np.zeros((na, nb))
                    E[i, j] = 1.0
                    avg = np.einsum("g,gki,gkl->il", Ws, Ta, np.einsum("kl,glm->gkm", E, Tb))
                    out = np.zeros((6, 6))
                    out[:na, :nb] = avg
                    M[:, 6 * i + j] = out.ravel()
            P[(la, lb)] = M
    return P


PROJ_BOND = _projectors(_group_bond())
PROJ_SITE = _projectors(_group_site())


# ---------------------------------------------------------------------------
# pair features, targets and assembly
# ---------------------------------------------------------------------------

def shell_slots(basis):
    """Index of every shell among the shells of its atom."""
    slot = np.zeros(len(basis["shell_l"]), dtype=int)
    seen = {}
    for s, a in enumerate(basis["shell_atom"]):
        slot[s] = seen.get(a, 0)
        seen[a] = slot[s] + 1
    return slot


def _pad_T(T, n):
    """Embed (P, n, n) in (P, 6, 6) with identity on the padding."""
    out = np.tile(np.eye(6), (T.shape[0], 1, 1))
    out[:, :n, :n] = T
    return out


def pair_samples(basis, D=None):
    """Every shell pair a >= b within the cutoff: features (P x 64 float32),
    the transformations that place its block, and (given the converged
    density D) the projected bond-frame target with its mask (P x 36)."""
    xyz = np.asarray(basis["xyz"], dtype=np.float64)
    sl = np.asarray(basis["shell_l"])
    sa = np.asarray(basis["shell_atom"])
    tix = np.array([TYPES.index(t) for t in basis["types"]])
    slot = shell_slots(basis)
    nc = np.array(NCART)[sl]
    bf0 = np.concatenate([[0], np.cumsum(nc)[:-1]]).astype(np.int64)
    ia, ib = np.tril_indices(len(sl))
    dvec = xyz[sa[ib]] - xyz[sa[ia]]
    r = np.linalg.norm(dvec, axis=1)
    keep = r <= RCUT
    ia, ib, dvec, r = ia[keep], ib[keep], dvec[keep], r[keep]
    P = len(ia)
    f = np.zeros((P, NIN), dtype=np.float32)
    f[:, :NRBF] = np.exp(-((r[:, None] - RBF_MU[None]) / RBF_SIGMA) ** 2)
    rows = np.arange(P)
    f[rows, NRBF + tix[sa[ia]]] = 1.0
    f[rows, NRBF + len(TYPES) + tix[sa[ib]]] = 1.0
    f[rows, NRBF + 2 * len(TYPES) + slot[ia]] = 1.0
    f[rows, NRBF + 2 * len(TYPES) + NSLOT + slot[ib]] = 1.0
    site = sa[ia] == sa[ib]
    R = np.tile(np.eye(3), (P, 1, 1))
    if (~site).any():
        R[~site] = bond_frames(dvec[~site])
    Ta = np.tile(np.eye(6), (P, 1, 1))
    Tb = np.tile(np.eye(6), (P, 1, 1))
    for l in range(3):
        for T, idx in ((Ta, ia), (Tb, ib)):
            m = sl[idx] == l
            if m.any():
                T[m] = _pad_T(cart_rotation(l, R[m]), NCART[l])
    mask = np.zeros((P, 6, 6), dtype=np.float32)
    k6 = np.arange(6)
    mask[(k6[None, :, None] < nc[ia][:, None, None]) & (k6[None, None, :] < nc[ib][:, None, None])] = 1
    out = {"feats": f, "ia": ia, "ib": ib, "la": sl[ia], "lb": sl[ib], "site": site,
           "Ta": Ta, "Tb": Tb, "bf_a": bf0[ia], "bf_b": bf0[ib], "mask": mask.reshape(P, 36),
           "nbf": int(nc.sum())}
    if D is not None:
        D = np.asarray(D, dtype=np.float64)
        Dp = np.pad(D, ((0, 6), (0, 6)))
        blk = Dp[bf0[ia][:, None, None] + k6[None, :, None], bf0[ib][:, None, None] + k6[None, None, :]]
        blk = blk * mask
        # bond-frame density D' = Ta^-T D Tb^-1
        loc = np.linalg.solve(np.swapaxes(Ta, 1, 2), blk) @ np.linalg.inv(Tb)
        out["target"] = project(out, (loc * mask).reshape(P, 36)).astype(np.float32)
    return out


def project(smp, Y):
    """Symmetry projection of bond-frame blocks (P x 36)."""
    Y = np.asarray(Y, dtype=np.float64)
    out = np.zeros_like(Y)
    for la in range(3):
        for lb in range(3):
            for site, PR in ((False, PROJ_BOND), (True, PROJ_SITE)):
                m = (smp["la"] == la) & (smp["lb"] == lb) & (smp["site"] == site)
                if m.any():
                    out[m] = Y[m] @ PR[(la, lb)].T
    return out


def assemble(smp, pred):
    """Molecular-frame density from predicted bond-frame blocks: projected,
    masked, D_ab = Ta^T D' Tb, mirrored and symmetrised."""
    P = len(smp["ia"])
    loc = (project(smp, pred) * smp["mask"]).reshape(P, 6, 6)
    blk = np.swapaxes(smp["Ta"], 1, 2) @ loc @ smp["Tb"]
    blk *= smp["mask"].reshape(P, 6, 6)
    N = smp["nbf"]
    k6 = np.arange(6)
    rows = np.broadcast_to(smp["bf_a"][:, None, None] + k6[None, :, None], (P, 6, 6))
    cols = np.broadcast_to(smp["bf_b"][:, None, None] + k6[None, None, :], (P, 6, 6))
    m = smp["mask"].reshape(P, 6, 6) > 0
    D = np.zeros((N, N))
    D[cols[m], rows[m]] = blk[m]
    D[rows[m], cols[m]] = blk[m]
    return 0.5 * (D + D.T)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

class GuessNet:
    """3 x Linear (64 -> 256 -> 256 -> 36), ReLU after the first two; BF16
    weights refreshed from FP32 master copies by Adam.  Every matrix product
    of the forward and backward passes is fsim_gemm_bf16."""

    dims = ((NIN, NHID), (NHID, NHID), (NHID, NOUT))

    def __init__(self, seed=0, device="cuda"):
        g = torch.Generator().manual_seed(seed)
        self.dev = torch.device(device)
        self.W = [(torch.randn(i, o, generator=g, dtype=torch.float32) * math.sqrt(2.0 / i)).to(self.dev)
                  for i, o in self.dims]
        self.b = [torch.zeros(o, dtype=torch.float32, device=self.dev) for _, o in self.dims]
        self.Wb = [torch.empty(i, o, dtype=torch.int16, device=self.dev) for i, o in self.dims]
        self.m1 = [torch.zeros_like(t) for t in self.W + self.b]
        self.m2 = [torch.zeros_like(t) for t in self.W + self.b]
        self.step = 0
        self.refresh()

    def refresh(self):
        """BF16 copies of the FP32 master weights."""
        for W, Wb in zip(self.W, self.Wb):
            _chk(_lib().fsim_f32_to_bf16(W.numel(), _p(W), _p(Wb), _stream()))

    @staticmethod
    def to_bf16(x):
        x = x.contiguous().float()
        y = torch.empty(x.shape, dtype=torch.int16, device=x.device)
        _chk(_lib().fsim_f32_to_bf16(x.numel(), _p(x), _p(y), _stream()))
        return y

    @staticmethod
    def gemm(M, N, K, A, lda, ta, B, ldb, tb, C=None, Cb=None, bias=None, relu=False, ksplit=1):
        _chk(_lib().fsim_gemm_bf16(M, N, K, _p(A), lda, ta, _p(B), ldb, tb, _p(C), N, _p(Cb),
                                   _p(bias), 1 if relu else 0, ksplit, _stream()))

    def forward(self, Xb):
        """Xb: (n, 64) BF16 bits.  Returns Y (n, 36) FP32 and the saved
        activations (BF16 inputs of each layer, FP32 outputs)."""
        n = Xb.shape[0]
        acts, outs = [Xb], []
        h = Xb
        for k, (i, o) in enumerate(self.dims):
            C = torch.empty(n, o, dtype=torch.float32, device=self.dev)
            Cb = torch.empty(n, o, dtype=torch.int16, device=self.dev) if k < 2 else None
            self.gemm(n, o, i, h, i, 0, self.Wb[k], o, 0, C=C, Cb=Cb, bias=self.b[k], relu=k < 2)
            outs.append(C)
            if k < 2:
                acts.append(Cb)
                h = Cb
        return outs[-1], (acts, outs)

    def gradients(self, Xb, T, mask):
        """Masked mean-square loss (device scalar) and FP32 gradients."""
        n = Xb.shape[0]
        Y, (acts, outs) = self.forward(Xb)
        loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        g = torch.empty_like(Y)
        cnt = max(float(mask.sum().item()), 1.0)
        _chk(_lib().fsim_mse(Y.numel(), _p(Y), _p(T), _p(mask), 1.0 / cnt, _p(g), _p(loss),
                             _stream()))
        gb = self.to_bf16(g)
        ks = max(1, min(64, n // 256))
        dW, db = [None] * 3, [None] * 3
        for k in (2, 1, 0):
            i, o = self.dims[k]
            dW[k] = torch.zeros(i, o, dtype=torch.float32, device=self.dev)
            self.gemm(i, o, n, acts[k], i, 1, gb, o, 0, C=dW[k], ksplit=ks)        # act^T g
            db[k] = torch.empty(o, dtype=torch.float32, device=self.dev)
            _chk(_lib().fsim_bias_grad(n, o, _p(g), _p(db[k]), _stream()))
            if k > 0:
                gp = torch.empty(n, i, dtype=torch.float32, device=self.dev)
                self.gemm(n, i, o, gb, o, 0, self.Wb[k], o, 1, C=gp)               # g W^T
                gpb = torch.empty(n, i, dtype=torch.int16, device=self.dev)
                _chk(_lib().fsim_relu_backward(gp.numel(), _p(outs[k - 1]), _p(gp), _p(gpb),
                                               _stream()))
                g, gb = gp, gpb
        return loss, dW, db

    def adam(self, dW, db, lr=1e-3):
        self.step += 1
        for k, (w, gr) in enumerate(zip(self.W + self.b, dW + db)):
            wb = self.Wb[k] if k < 3 else None
            _chk(_lib().fsim_adam(w.numel(), _p(w), _p(gr), _p(self.m1[k]), _p(self.m2[k]), lr,
                                  0.9, 0.999, 1e-8, self.step, _p(wb), _stream()))

    def train(self, feats, target, mask, epochs=4, batch=8192, lr=1e-3, seed=0, log=None):
        X = self.to_bf16(torch.as_tensor(feats, device=self.dev))
        T = torch.as_tensor(target, dtype=torch.float32, device=self.dev)
        M = torch.as_tensor(mask, dtype=torch.float32, device=self.dev)
        n = X.shape[0]
        batch = min(batch, n)
        g = torch.Generator().manual_seed(seed)
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(self.dev)
            tot = torch.zeros((), dtype=torch.float32, device=self.dev)
            nb = 0
            for s0 in range(0, n - batch + 1, batch):
                idx = perm[s0:s0 + batch]
                loss, dW, db = self.gradients(X[idx].contiguous(), T[idx].contiguous(),
                                              M[idx].contiguous())
                self.adam(dW, db, lr)
                tot += loss[0]
                nb += 1
            hist.append(float(tot.item()) / max(nb, 1))
            if log:
                log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.3e}")
        return hist

    def packed(self):
        """The BF16 weights in MFMA fragment order (fsim_mlp_pack), for the
        fused forward pass.  Packed afresh on each call: training updates the
        BF16 copies in place."""
        out = []
        for (i, o), Wb in zip(self.dims, self.Wb):
            Wp = torch.empty((i // 16) * ((o + 15) // 16) * 256, dtype=torch.int16, device=self.dev)
            _chk(_lib().fsim_mlp_pack(i, o, _p(Wb), _p(Wp), _stream()))
            out.append(Wp)
        return out

    def infer(self, Xb, Wp=None):
        """Y (n, 36) FP32 from the fused three-layer kernel (equal to
        forward(Xb)[0] bit for bit, without the saved activations)."""
        Xb = Xb.contiguous()
        Wp = Wp if Wp is not None else self.packed()
        n = Xb.shape[0]
        Y = torch.empty(n, NOUT, dtype=torch.float32, device=self.dev)
        _chk(_lib().fsim_mlp_forward(n, _p(Xb), _p(Wp[0]), _p(self.b[0]), _p(Wp[1]),
                                     _p(self.b[1]), _p(Wp[2]), _p(self.b[2]), _p(Y), _stream()))
        return Y

    def predict(self, feats):
        X = self.to_bf16(torch.as_tensor(feats, dtype=torch.float32, device=self.dev))
        return self.infer(X).cpu().numpy()

    def state(self, full=False):
        """Weights and biases; with full, also the Adam moments and step, so
        that training can continue in another process."""
        st = {f"W{k}": self.W[k].cpu().numpy() for k in range(3)}
        st.update({f"b{k}": self.b[k].cpu().numpy() for k in range(3)})
        if full:
            st.update({f"m1_{k}": t.cpu().numpy() for k, t in enumerate(self.m1)})
            st.update({f"m2_{k}": t.cpu().numpy() for k, t in enumerate(self.m2)})
            st["step"] = np.array(self.step)
        return st

    def load(self, st):
        for k in range(3):
            self.W[k].copy_(torch.as_tensor(st[f"W{k}"]))
            self.b[k].copy_(torch.as_tensor(st[f"b{k}"]))
        if "step" in st:
            for k in range(len(self.m1)):
                self.m1[k].copy_(torch.as_tensor(st[f"m1_{k}"]))
                self.m2[k].copy_(torch.as_tensor(st[f"m2_{k}"]))
            self.step = int(st["step"])
        self.refresh()


# ---------------------------------------------------------------------------
# training data, the guess, evaluation
# ---------------------------------------------------------------------------

def training_molecules(n_chain, n_water, seed0=5_000_000):
    """Seeded H chains (even 4..32 atoms, spacing U[1.2, 2.0] bohr) and water
    clusters (2..16 molecules)."""
    import synth
    mols = []
    for i in range(n_chain):
        rng = np.random.default_rng(seed0 + i)
        natom = 2 * int(rng.integers(2, 17))
        mols.append(synth.h_chain(natom, float(rng.uniform(1.2, 2.0))))
    for i in range(n_water):
        s = seed0 + n_chain + i
        mols.append(synth.water_cluster(int(np.random.default_rng(s).integers(2, 17)), s))
    return mols


def training_set(n, seed0=5_000_000):
    """The configured training population as one interleaved list: molecule
    i (seed seed0 + i) is an H chain (even 4..32 atoms, spacing U[1.2, 2.0]
    bohr) for even i and a water-like cluster of 2..16 molecules for odd i,
    so that any contiguous slice holds both kinds half and half."""
    import synth
    mols = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        if i % 2 == 0:
            mols.append(synth.h_chain(2 * int(rng.integers(2, 17)), float(rng.uniform(1.2, 2.0))))
        else:
            mols.append(synth.water_cluster(int(rng.integers(2, 17)), seed0 + i))
    return mols


def converged_densities(mols, chunk=128, tau=1e-10, max_iter=60, conv_rms_dD=1e-7,
                        conv_dE=1e-9, stop_fraction=None, log=None):
    """FP64 batched SCF (this library) of every molecule, in size-sorted
    chunks (a chunk may end once stop_fraction of it has converged); returns
    the densities of those that meet the convergence test at the chunk's
    last step, and their indices."""
    import synth
    order = sorted(range(len(mols)), key=lambda i: synth.nbf_of(mols[i]))
    out, idx = {}, []
    for c0 in range(0, len(order), chunk):
        ids = order[c0:c0 + chunk]
        part = [mols[i] for i in ids]
        bt = fsim.Batch(part, tau=tau, conv_rms_dD=conv_rms_dD, conv_dE=conv_dE)
        bt.set_graph(True)
        t0 = time.time()
        r = bt.scf(max_iter=max_iter, stop_fraction=stop_fraction, verbose=log is not None)
        blocks = bt.unpack(r["D"])
        ok = [m for m, rec in enumerate(r["per_molecule"]) if rec["converged"]]
        for m in ok:
            out[ids[m]] = blocks[m].cpu().numpy()
            idx.append(ids[m])
        if log:
            log(f"SCF chunk {c0 // chunk + 1}: {len(ok)}/{len(part)} converged after "
                f"{r['iterations']} iterations, {time.time() - t0:.1f} s")
        bt.close()
    idx.sort()
    return [out[i] for i in idx], idx


def _samples_of(args):
    b, D = args
    s = pair_samples(b, D)
    return s["feats"], s["target"], s["mask"]


def dataset(mols, dens, workers=1):
    """Shell-pair samples (features, targets, masks) of every molecule; the
    numpy work can run in a process pool."""
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_samples_of, list(zip(mols, dens)), chunksize=16)
    else:
        parts = [_samples_of(a) for a in zip(mols, dens)]
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
            np.concatenate([p[2] for p in parts]))


def predicted_density(net, basis):
    """Assembled (unpurified) density of one molecule, FP64 numpy."""
    smp = pair_samples(basis)
    return assemble(smp, net.predict(smp["feats"]))


def purify(ctx, D, iters=8):
    """McWeeny purification in place on the GPU; (error before, error after)."""
    e0, e1 = ctypes.c_double(), ctypes.c_double()
    _chk(_lib().fsim_purify(ctx.h, _p(D), iters, ctypes.byref(e0), ctypes.byref(e1), _stream()))
    return e0.value, e1.value


def learned_guess(net, ctx, basis, iters=24, tol=1e-2):
    """Guess density for a one-molecule context: predicted, purified, and
    replaced by the core-Hamiltonian guess if it stays non-idempotent beyond
    tol.  Returns (D, info).  McWeeny iterations are cheap (three N^3
    products each); a predicted eigenvalue near 1/2 needs up to about 24 of
    them to leave the slow region around it."""
    D = torch.tensor(predicted_density(net, basis), dtype=torch.float64, device=ctx.device)
    e0, e1 = purify(ctx, D, iters)
    info = {"idempotency_raw": e0, "idempotency_purified": e1, "fallback": not (e1 <= tol)}
    if info["fallback"]:
        D = ctx.core_guess()
    return D, info


def evaluate(net, mols, tau=1e-11, max_iter=60, log=None):
    """SCF of held-out molecules from the core-Hamiltonian guess and from the
    learned guess (one batch each); per-molecule iterations to convergence,
    wall time and the converged energies of both runs."""
    guesses, infos = [], []
    torch.cuda.synchronize()
    tg = time.time()
    for b in mols:
        ctx = fsim.Context(b, tau=tau)
        D, info = learned_guess(net, ctx, b)
        guesses.append(D)
        infos.append(info)
        ctx.close()
    torch.cuda.synchronize()
    # features, inference, assembly, purification and fallbacks, with the
    # one-molecule contexts they need
    guess_seconds = time.time() - tg
    res = {"guess_seconds": guess_seconds}
    for name in ("core", "learned"):
        bt = fsim.Batch(mols, tau=tau, conv_rms_dD=1e-8, conv_dE=1e-10)
        bt.set_graph(True)
        bt.schwarz_screen()
        D0 = bt.pack(guesses) if name == "learned" else None
        torch.cuda.synchronize()
        t0 = time.time()
        r = bt.scf(max_iter=max_iter, D0=D0, verbose=log is not None)
        torch.cuda.synchronize()
        fc = r["first_converged"]
        res[name] = {"seconds": time.time() - t0, "first_converged": fc.tolist(),
                     "E": r["E_total"].tolist(), "iterations": r["iterations"]}
        if log:
            med = float(np.median(fc[fc >= 0])) if (fc >= 0).any() else -1.0
            log(f"{name} guess: {r['iterations']} batch iterations, {res[name]['seconds']:.2f} s, "
                f"per-molecule median {med}, unconverged {int((fc < 0).sum())}")
        bt.close()
    res["guess_info"] = infos
    res["learned"]["seconds_with_guess"] = res["learned"]["seconds"] + guess_seconds
    if log:
        log(f"learned guess construction {guess_seconds:.1f} s; learned total "
            f"{res['learned']['seconds_with_guess']:.1f} s vs core {res['core']['seconds']:.1f} s")
    return res


def stream_part(a, log):
    """One part of the training set: converged densities from batched SCFs,
    their shell-pair samples, and a.epochs epochs of Adam continuing from the
    saved state; the full state and a record of the part are written to
    a.out."""
    import json
    import os
    t0 = time.time()
    full = training_set(a.total)
    per = (a.total + a.stream_parts - 1) // a.stream_parts
    lo, hi = a.stream_part * per, min(a.total, (a.stream_part + 1) * per)
    mols = full[lo:hi]
    log(f"part {a.stream_part + 1}/{a.stream_parts}: molecules {lo}..{hi - 1}")
    dens, idx = converged_densities(mols, chunk=512, max_iter=40, conv_rms_dD=a.conv, conv_dE=0.0,
                                    stop_fraction=0.98, log=log)
    t_scf = time.time() - t0
    mols = [mols[i] for i in idx]
    log(f"{len(mols)} converged densities in {t_scf:.1f} s")
    t1 = time.time()
    X, T, M = dataset(mols, dens, workers=a.workers)
    t_feat = time.time() - t1
    log(f"{X.shape[0]} shell-pair samples in {t_feat:.1f} s")
    net = GuessNet(seed=0)
    if a.state_in:
        with np.load(a.state_in) as st:
            net.load({k: st[k] for k in st.files})
    t2 = time.time()
    hist = net.train(X, T, M, epochs=a.epochs, seed=a.stream_part, log=log)
    torch.cuda.synchronize()
    np.savez(os.path.join(a.out, "guess_state.npz"), **net.state(full=True))
    rec = {"part": a.stream_part, "parts": a.stream_parts, "molecules": [lo, hi],
           "converged": len(mols), "samples": int(X.shape[0]), "scf_seconds": t_scf,
           "feature_seconds": t_feat, "train_seconds": time.time() - t2, "loss": hist,
           "adam_step": net.step, "conv_rms_dD": a.conv}
    with open(os.path.join(a.out, f"guess_part{a.stream_part}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    log(f"part done: {json.dumps({k: v for k, v in rec.items() if k != 'loss'})}")


def main():
    import argparse
    import json
    import os
    import synth
    ap = argparse.ArgumentParser(description="train and evaluate the learned SCF guess")
    ap.add_argument("--chains", type=int, default=256)
    ap.add_argument("--waters", type=int, default=512)
    ap.add_argument("--eval", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--out", default="guess_out")
    ap.add_argument("--weights", default=None,
                    help="evaluate saved weights (guess_weights.npz) instead of training")
    ap.add_argument("--eval-offset", type=int, default=0,
                    help="first held-out cluster index (seed 6_000_000 + index)")
    ap.add_argument("--stream-part", type=int, default=None,
                    help="train on part K of the --total training set (continuing from "
                         "--state-in) and save the full training state")
    ap.add_argument("--stream-parts", type=int, default=4)
    ap.add_argument("--total", type=int, default=20000)
    ap.add_argument("--state-in", default=None)
    ap.add_argument("--conv", type=float, default=1e-5,
                    help="RMS density change that ends a training SCF (streaming)")
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    log = lambda s: print(f"[guess] {s}", flush=True)
    if a.stream_part is not None:
        return stream_part(a, log)
    if a.weights:
        net = GuessNet(seed=0)
        with np.load(a.weights) as st:
            net.load({k: st[k] for k in st.files})
        idx = range(a.eval_offset, a.eval_offset + a.eval)
        log(f"weights {a.weights}; held-out clusters {idx.start}..{idx.stop - 1}")
        ev = [synth.water_cluster(32, 6_000_000 + i) for i in idx]
        res = evaluate(net, ev, log=log)
        res["eval_indices"] = [idx.start, idx.stop]
        with open(os.path.join(a.out, "guess_eval.json"), "w") as f:
            json.dump(res, f, indent=1)
        return
    t0 = time.time()
    mols = training_molecules(a.chains, a.waters)
    dens, idx = converged_densities(mols, log=log)
    mols = [mols[i] for i in idx]
    log(f"{len(mols)} converged training densities, {time.time() - t0:.1f} s")
    X, T, M = dataset(mols, dens)
    log(f"{X.shape[0]} shell-pair samples")
    net = GuessNet(seed=0)
    t1 = time.time()
    hist = net.train(X, T, M, epochs=a.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    log(f"training {t_train:.1f} s")
    np.savez(os.path.join(a.out, "guess_weights.npz"), **net.state())
    # inference throughput of the three BF16 GEMMs over the training samples
    Xd = net.to_bf16(torch.as_tensor(X, device=net.dev))
    nrow = (Xd.shape[0] // 65536) * 65536 or Xd.shape[0]
    chunks = [Xd[i:i + 65536] for i in range(0, nrow, 65536)]
    reps = -(-(1 << 21) // nrow)          # at least 2M rows timed, cycling the samples
    chunks, nrow = chunks * reps, nrow * reps
    net.forward(chunks[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for c in chunks:
        net.forward(c)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    flops = 2.0 * nrow * sum(i * o for i, o in GuessNet.dims)
    # the same rows through the fused kernel (weights packed once)
    Wp = net.packed()
    net.infer(chunks[0], Wp)
    e0.record()
    for c in chunks:
        net.infer(c, Wp)
    e1.record()
    torch.cuda.synchronize()
    sec_f = e0.elapsed_time(e1) / 1e3
    fwd = {"rows": nrow, "seconds": sec, "TFLOP/s": flops / sec / 1e12,
           "fused_seconds": sec_f, "fused_TFLOP/s": flops / sec_f / 1e12}
    log(f"forward over {nrow} pairs: layered {sec * 1e3:.2f} ms, {fwd['TFLOP/s']:.1f} TFLOP/s; "
        f"fused {sec_f * 1e3:.2f} ms, {fwd['fused_TFLOP/s']:.1f} TFLOP/s (BF16)")
    ev = [synth.water_cluster(32, 6_000_000 + i)
          for i in range(a.eval_offset, a.eval_offset + a.eval)]
    res = evaluate(net, ev, log=log)
    res["loss"] = hist
    res["train_molecules"] = len(mols)
    res["train_samples"] = int(X.shape[0])
    res["forward"] = fwd
    res["train_seconds"] = t_train
    with open(os.path.join(a.out, "guess_eval.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
