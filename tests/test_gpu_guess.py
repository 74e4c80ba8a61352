"""Learned initial guess on the GPU, through the C ABI: the BF16 matrix-core
GEMM against a CPU FP32 product of the same BF16 inputs, the training
kernels against numpy, forward/backward against the FP64 network oracle,
the fused three-layer inference kernel against the layered GEMMs (bit for
bit) and the oracle,
McWeeny purification against the oracle's, and a small train -> guess ->
SCF run.

Tolerances: the GEMM's FP32 accumulation differs from the CPU's only in
summation order, so |C - C_ref| <= K 2^-23 (|A| |B|) elementwise; BF16
outputs are bit-exact (both sides round the same FP32 value to nearest
even).  Forward output and gradients against the oracle that rounds at the
same points as the GPU, element by element: each element within 2^-6 of its
magnitude scale (the same product over absolute values, |A|^T |G| for a
weight gradient), since FP32 accumulation order can flip single BF16
roundings (2^-8 relative each) that then propagate; and almost every element
(all but 0.5%) within 2^-12 of it."""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _g():
    from paper_2510_24968_amd import guess
    return guess


def _bf16_pair(shape, gen, scale=1.0):
    """(int16 bits on the GPU, FP64 values on the CPU) of random BF16 numbers."""
    x = (torch.randn(shape, generator=gen) * scale).to(torch.bfloat16)
    return x.view(torch.int16).cuda(), x.double().numpy()


@pytest.mark.parametrize("M,N,K", [(70, 37, 40), (128, 256, 64), (5, 3, 17), (256, 36, 1000)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_bf16_matches_cpu(M, N, K, ta, tb):
    g = _g()
    print(f"[gpu] gemm {M}x{N}x{K} ta={ta} tb={tb}", flush=True)
    gen = torch.Generator().manual_seed(M * 1000 + N + K + 7 * ta + 13 * tb)
    Ad, A = _bf16_pair((K, M) if ta else (M, K), gen)
    Bd, B = _bf16_pair((N, K) if tb else (K, N), gen)
    bias = torch.randn(N, generator=gen).float()
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = opA @ opB
    bound = K * 2.0 ** -23 * (np.abs(opA) @ np.abs(opB)) + 1e-30
    lda = M if ta else K
    ldb = K if tb else N
    # plain product
    C = torch.empty(M, N, dtype=torch.float32, device="cuda")
    g.GuessNet.gemm(M, N, K, Ad, lda, ta, Bd, ldb, tb, C=C)
    assert np.all(np.abs(C.cpu().double().numpy() - ref) <= bound)
    # bias + ReLU epilogue with the BF16 copy
    C2 = torch.empty(M, N, dtype=torch.float32, device="cuda")
    Cb = torch.empty(M, N, dtype=torch.int16, device="cuda")
    g.GuessNet.gemm(M, N, K, Ad, lda, ta, Bd, ldb, tb, C=C2, Cb=Cb, bias=bias.cuda(), relu=True)
    ref2 = np.maximum(ref + bias.double().numpy()[None, :], 0.0)
    c2 = C2.cpu()
    assert np.all(np.abs(c2.double().numpy() - ref2) <= bound + 1e-6 * np.abs(ref2))
    assert torch.equal(Cb.cpu(), c2.to(torch.bfloat16).view(torch.int16))
    # split-K into a zeroed accumulator
    for ks in (2, 7):
        C3 = torch.zeros(M, N, dtype=torch.float32, device="cuda")
        g.GuessNet.gemm(M, N, K, Ad, lda, ta, Bd, ldb, tb, C=C3, ksplit=ks)
        assert np.all(np.abs(C3.cpu().double().numpy() - ref) <= bound)


def test_gemm_rejects_bad_arguments():
    g = _g()
    L = g._lib()
    x = torch.zeros(16, dtype=torch.int16, device="cuda")
    c = torch.zeros(16, dtype=torch.float32, device="cuda")
    s = g._stream()
    assert L.fsim_gemm_bf16(0, 4, 4, g._p(x), 4, 0, g._p(x), 4, 0, g._p(c), 4, None, None, 0, 1, s) != 0
    # split-K cannot take an epilogue
    assert L.fsim_gemm_bf16(4, 4, 4, g._p(x), 4, 0, g._p(x), 4, 0, g._p(c), 4, None, None, 1, 2, s) != 0


def test_f32_to_bf16_matches_torch_rounding():
    g = _g()
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(100000) * 10.0 ** rng.integers(-30, 30, 100000),
                        [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 3.0e38, 1e-40, np.inf,
                         -np.inf]]).astype(np.float32)
    xt = torch.from_numpy(x)
    got = g.GuessNet.to_bf16(xt.cuda()).cpu()
    assert torch.equal(got, xt.to(torch.bfloat16).view(torch.int16))


def test_training_kernels_against_numpy():
    g = _g()
    L = g._lib()
    s = g._stream()
    rng = np.random.default_rng(2)
    n, m = 3001, 37
    H = rng.standard_normal((n, m)).astype(np.float32)
    dH = rng.standard_normal((n, m)).astype(np.float32)
    Ht, dHt = torch.from_numpy(H).cuda(), torch.from_numpy(dH).cuda()
    dHb = torch.empty(n, m, dtype=torch.int16, device="cuda")
    assert L.fsim_relu_backward(n * m, g._p(Ht), g._p(dHt), g._p(dHb), s) == 0
    ref = np.where(H > 0, dH, 0.0).astype(np.float32)
    assert np.array_equal(dHt.cpu().numpy(), ref)
    assert torch.equal(dHb.cpu(), torch.from_numpy(ref).to(torch.bfloat16).view(torch.int16))
    db = torch.empty(m, dtype=torch.float32, device="cuda")
    assert L.fsim_bias_grad(n, m, g._p(Ht), g._p(db), s) == 0
    assert np.allclose(db.cpu().numpy(), H.astype(np.float64).sum(0), rtol=0,
                       atol=n * 2.0 ** -23 * np.abs(H).sum(0).max())
    T = rng.standard_normal((n, m)).astype(np.float32)
    mask = (rng.random((n, m)) < 0.6).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dY = torch.empty(n, m, dtype=torch.float32, device="cuda")
    Tt, Mt = torch.from_numpy(T).cuda(), torch.from_numpy(mask).cuda()
    inv = 1.0 / mask.sum()
    assert L.fsim_mse(n * m, g._p(Ht), g._p(Tt), g._p(Mt), inv, g._p(dY), g._p(loss), s) == 0
    d = (H.astype(np.float64) - T) * mask
    assert abs(loss.item() - (d * d).sum() * inv) < 1e-5 * (d * d).sum() * inv
    assert np.allclose(dY.cpu().numpy(), 2 * d * inv, rtol=1e-6, atol=1e-12)
    # Adam, three steps, against torch.optim.Adam (an independent
    # implementation of the same bias-corrected update) in FP64 on the CPU
    w = rng.standard_normal(1000).astype(np.float32)
    wt = torch.from_numpy(w.copy()).cuda()
    m1 = torch.zeros(1000, device="cuda")
    m2 = torch.zeros(1000, device="cuda")
    wb = torch.empty(1000, dtype=torch.int16, device="cuda")
    wref = torch.nn.Parameter(torch.from_numpy(w.astype(np.float64)))
    opt = torch.optim.Adam([wref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 4):
        gr = rng.standard_normal(1000).astype(np.float32)
        assert L.fsim_adam(1000, g._p(wt), g._p(torch.from_numpy(gr).cuda()), g._p(m1), g._p(m2),
                           1e-2, 0.9, 0.999, 1e-8, step, g._p(wb), s) == 0
        wref.grad = torch.from_numpy(gr.astype(np.float64))
        opt.step()
    wr = wref.detach().numpy()
    assert np.allclose(wt.cpu().numpy(), wr, rtol=0, atol=1e-5)
    assert torch.equal(wb.cpu(), wt.cpu().to(torch.bfloat16).view(torch.int16))


def _net_and_batch(n=700, seed=3):
    g = _g()
    net = g.GuessNet(seed=seed)
    rng = np.random.default_rng(seed)
    X = rng.random((n, g.NIN)).astype(np.float32)
    T = (rng.standard_normal((n, g.NOUT)) * 0.3).astype(np.float32)
    M = (rng.random((n, g.NOUT)) < 0.5).astype(np.float32)
    return net, X, T, M


def _magnitude_scales(X, T, M, W, b):
    """Element-wise magnitude scales of the oracle's forward output and
    gradients: the same products taken over absolute values (|X||W| + |b|
    through the layers; |A_k|^T |G_k| for the weight gradients with |G|
    back-propagated through |W| under the oracle's ReLU masks)."""
    rd = omlp.round_bf16
    pre, acts, Y = omlp.forward(X, W, b, bf16=True)
    h = np.abs(acts[0])
    for k in range(3):
        h = h @ np.abs(rd(W[k])) + np.abs(b[k])
        if k < 2:
            h = h * (pre[k] > 0)
    y_scale = h
    count = float(np.sum(M))
    g = np.abs(2.0 * (Y - T) * M / count)
    sW, sb = [None] * 3, [None] * 3
    for k in (2, 1, 0):
        sW[k] = np.abs(acts[k]).T @ g
        sb[k] = g.sum(axis=0)
        if k > 0:
            g = (g @ np.abs(rd(W[k])).T) * (pre[k - 1] > 0)
    return y_scale, sW, sb


def _elementwise(name, got, ref, scale):
    err = np.abs(got - ref)
    worst = float(np.max(err / (scale + 1e-30)))
    loose = float(np.mean(err > 2.0 ** -12 * scale + 1e-30))
    print(f"{name}: max |err|/scale {worst:.2e}, share above 2^-12 {loose:.2e}", flush=True)
    assert np.all(err <= 2.0 ** -6 * scale + 1e-30), name
    assert loose <= 5e-3, name


def test_forward_backward_against_oracle():
    g = _g()
    net, X, T, M = _net_and_batch()
    W = [w.cpu().double().numpy() for w in net.W]
    b = [v.cpu().double().numpy() for v in net.b]
    Xb = net.to_bf16(torch.from_numpy(X).cuda())
    loss, dW, db = net.gradients(Xb, torch.from_numpy(T).cuda(), torch.from_numpy(M).cuda())
    Y = net.forward(Xb)[0].cpu().double().numpy()
    # the oracle rounding at the same points, compared element by element
    l16, gW16, gb16 = omlp.loss_and_grads(X, T, M, W, b, bf16=True)
    y16 = omlp.forward(X, W, b, bf16=True)[2]
    y_scale, sW, sb = _magnitude_scales(X, T, M, W, b)
    _elementwise("forward Y", Y, y16, y_scale)
    assert abs(loss.item() - l16) < 1e-3 * l16
    for k in range(3):
        _elementwise(f"layer {k} dW", dW[k].cpu().double().numpy(), gW16[k], sW[k])
        _elementwise(f"layer {k} db", db[k].cpu().double().numpy(), gb16[k], sb[k])
    # and against exact FP64 arithmetic: BF16 costs well under a percent
    l64, gW64, _ = omlp.loss_and_grads(X, T, M, W, b)
    assert abs(loss.item() - l64) < 2e-2 * l64
    for k in range(3):
        a = dW[k].cpu().double().numpy().ravel()
        r = gW64[k].ravel()
        assert a @ r / (np.linalg.norm(a) * np.linalg.norm(r)) > 0.999


def _pack_reference(W, K, N):
    """The fragment order restated in numpy: for K step s, column tile t and
    lane l, rows 16 s + 4 (l // 16) + j of column 16 t + l % 16 (zero past N)."""
    nt = (N + 15) // 16
    out = np.zeros(((K // 16) * nt * 64, 4), dtype=W.dtype)
    for s_ in range(K // 16):
        for t in range(nt):
            for l in range(64):
                col = 16 * t + l % 16
                if col < N:
                    out[(s_ * nt + t) * 64 + l] = W[16 * s_ + 4 * (l // 16) + np.arange(4), col]
    return out.ravel()


@pytest.mark.parametrize("K,N", [(64, 256), (256, 36), (32, 20)])
def test_mlp_pack_layout(K, N):
    g = _g()
    gen = torch.Generator().manual_seed(K + N)
    Wd, _ = _bf16_pair((K, N), gen)
    Wp = torch.empty((K // 16) * ((N + 15) // 16) * 256, dtype=torch.int16, device="cuda")
    g._chk(g._lib().fsim_mlp_pack(K, N, g._p(Wd), g._p(Wp), g._stream()))
    assert np.array_equal(Wp.cpu().numpy(), _pack_reference(Wd.cpu().numpy(), K, N))


@pytest.mark.parametrize("n", [1, 31, 32, 1000, 4099])
def test_fused_forward_equals_layered_and_oracle(n):
    """The fused kernel against the three layered GEMMs (bit for bit: same
    MFMA steps, same rounding points) and against the FP64 network oracle
    that rounds at the same points; ragged row counts around the 32-row
    block."""
    g = _g()
    print(f"[gpu] fused forward n={n}", flush=True)
    net, X, _, _ = _net_and_batch(n=n, seed=11)
    net.b = [torch.randn(b.shape, generator=torch.Generator().manual_seed(k)).cuda() * 0.1
             for k, b in enumerate(net.b)]          # non-zero biases exercise the epilogues
    Xb = net.to_bf16(torch.from_numpy(X).cuda())
    Y_fused = net.infer(Xb)
    Y_layer = net.forward(Xb)[0]
    torch.cuda.synchronize()
    assert torch.equal(Y_fused, Y_layer)
    W = [w.cpu().double().numpy() for w in net.W]
    b = [v.cpu().double().numpy() for v in net.b]
    y16 = omlp.forward(X, W, b, bf16=True)[2]
    err = np.linalg.norm(Y_fused.cpu().double().numpy() - y16) / np.linalg.norm(y16)
    assert err < 1e-3


def test_fused_forward_rejects_bad_arguments():
    g = _g()
    L = g._lib()
    Y = torch.empty(4, g.NOUT, dtype=torch.float32, device="cuda")
    assert L.fsim_mlp_forward(-1, None, None, None, None, None, None, None, None, None) != 0
    assert L.fsim_mlp_forward(0, None, None, None, None, None, None, None, None, None) == 0
    assert L.fsim_mlp_forward(4, None, None, None, None, None, None, None, g._p(Y), None) != 0
    W = torch.zeros(20, 8, dtype=torch.int16, device="cuda")
    assert L.fsim_mlp_pack(20, 8, g._p(W), g._p(W), None) != 0      # K not a multiple of 16
    assert L.fsim_mlp_pack(16, 0, g._p(W), g._p(W), None) != 0
    # misaligned input rows or fragments are refused before any launch
    net = g.GuessNet(seed=0)
    Wp = net.packed()
    X = torch.zeros(4 * g.NIN + 1, dtype=torch.int16, device="cuda")
    odd = ctypes.c_void_p(X.data_ptr() + 2)
    args = [g._p(Wp[0]), g._p(net.b[0]), g._p(Wp[1]), g._p(net.b[1]), g._p(Wp[2]), g._p(net.b[2]),
            g._p(Y), None]
    assert L.fsim_mlp_forward(4, odd, *args) != 0
    args[2] = ctypes.c_void_p(Wp[1].data_ptr() + 2)
    assert L.fsim_mlp_forward(4, g._p(X), *args) != 0


def test_training_reduces_loss():
    g = _g()
    net, X, T, M = _net_and_batch(n=4096, seed=4)
    # a learnable target: a fixed smooth function of the features
    T = np.tanh(X @ np.random.default_rng(5).standard_normal((g.NIN, g.NOUT)) * 0.2).astype(np.float32)
    hist = net.train(X, T, M, epochs=30, batch=1024, lr=3e-3)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.1 * hist[0]


def test_purify_against_oracle():
    g = _g()
    from paper_2510_24968_amd import fsim
    b = synth.water_cluster(2, 21)
    ctx = fsim.Context(b)
    r = ctx.scf()
    S = ctx.one_electron()[0].cpu().numpy()
    D = r["D"].cpu().numpy()
    rng = np.random.default_rng(7)
    E = rng.standard_normal(D.shape)
    Dp = D + 3e-3 * (E + E.T)
    Dt = torch.tensor(Dp, dtype=torch.float64, device="cuda")
    e0, e1 = g.purify(ctx, Dt, 8)
    Dref, r0, r1 = oracle.mcweeny(Dp, S, 8)
    print("idempotency", e0, "->", e1, "oracle", r0, "->", r1)
    assert abs(e0 - r0) < 1e-10 * max(r0, 1.0)
    assert e1 < 1e-10 and r1 < 1e-10
    assert np.abs(Dt.cpu().numpy() - Dref).max() < 1e-9
    # a converged density is (nearly) a fixed point
    Dc = r["D"].clone()
    f0, f1 = g.purify(ctx, Dc, 2)
    assert f0 < 1e-6 and f1 < 1e-12
    assert (Dc - r["D"]).abs().max().item() < 1e-6
    ctx.close()


def test_learned_guess_small_end_to_end():
    """Train on a few small molecules, guess a held-out water trimer, and
    converge the SCF from it, in fewer iterations than from the core guess,
    to the energy reached from the core guess."""
    g = _g()
    from paper_2510_24968_amd import fsim
    mols = g.training_molecules(6, 10, seed0=7_000_000)
    dens, idx = g.converged_densities(mols, chunk=16, log=print)
    assert len(idx) >= 12
    X, T, M = g.dataset([mols[i] for i in idx], dens)
    net = g.GuessNet(seed=1)
    hist = net.train(X, T, M, epochs=40, batch=2048, lr=2e-3)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.2 * hist[0]
    b = synth.water_cluster(3, 7_500_000)
    ctx = fsim.Context(b, conv_rms_dD=1e-8, conv_dE=1e-10)
    D0, info = g.learned_guess(net, ctx, b)
    print("guess", info)
    assert not info["fallback"]
    r_core = ctx.scf()
    r_learn = ctx.scf(D0=D0)
    print("iterations core", r_core["iterations"], "learned", r_learn["iterations"])
    assert r_core["converged"] and r_learn["converged"]
    assert abs(r_core["E_total"] - r_learn["E_total"]) < 1e-7
    # what the trained network gains: fewer SCF iterations than the core guess
    assert r_learn["iterations"] < r_core["iterations"]
    ctx.close()
