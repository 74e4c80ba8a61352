"""fsim_fock_build_noalloc (accumulators in the library's static device
array) against fsim_fock_build and the oracle, through the C ABI: two calls
in a row on two contexts, the second with a smaller molecule, in FP64 and
mixed precision; and the size limit."""

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fsim():
    from paper_2510_24968_amd import fsim
    return fsim


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _density(B):
    S, T, V = B.one_electron()
    D, _, _ = oracle.density_from_fock(T + V, oracle.orthogonalizer(S), B.nelec // 2)
    return D


def test_noalloc_matches_fock_build_two_calls():
    fsim = _fsim()
    tau = 1e-10
    for step, b in enumerate((synth.water_cluster(3, 2), synth.water_cluster(1, 4))):
        print(f"[gpu] noalloc call {step}: {b['name']}", flush=True)
        ctx = fsim.Context(b, tau=tau, tau_fp32=1e-6)
        ctx.schwarz_screen()
        B = oracle.Basis(b)
        D = _density(B)
        Jo, Ko = B.fock_jk(D, tau=tau)
        Dd = _dev(D)
        for prec, tol in (("fp64", 1e-11), ("mixed", 1e-9)):
            ref = ctx.fock_build(Dd, prec, want_jk=True)
            N = ctx.nbf
            F = torch.full((N, N), np.nan, dtype=torch.float64, device="cuda")
            J = torch.full_like(F, np.nan)
            K = torch.full_like(F, np.nan)
            E = ctx.fock_build_noalloc(Dd, F, J, K, prec)
            torch.cuda.synchronize()
            dJ = torch.max(torch.abs(J - ref["J"])).item()
            dK = torch.max(torch.abs(K - ref["K"])).item()
            dF = torch.max(torch.abs(F - ref["F"])).item()
            print(f"  {prec}: |dJ| {dJ:.2e} |dK| {dK:.2e} |dF| {dF:.2e} "
                  f"dE {E - ref['E_elec']:.2e}", flush=True)
            assert dJ < tol and dK < tol and dF < tol
            assert abs(E - ref["E_elec"]) < 1e-9
            assert np.max(np.abs(J.cpu().numpy() - Jo)) < tol
            assert np.max(np.abs(K.cpu().numpy() - Ko)) < tol
        ctx.close()


def test_noalloc_rejects_sizes_beyond_its_limit():
    fsim = _fsim()
    b = synth.h_chain(1500, 1.4)                 # N = 1500: N^2 > 2,097,152
    ctx = fsim.Context(b)
    D = torch.zeros((ctx.nbf, ctx.nbf), dtype=torch.float64, device="cuda")
    F = torch.empty_like(D)
    with pytest.raises(fsim.FsimError, match="exceeds the maximum"):
        ctx.fock_build_noalloc(D, F)
    ctx.close()
