"""Spherical (real solid harmonic) basis through the C ABI against the
oracle's spherical layer (Sec. 2.1.1): one-electron matrices, J and K at a
spherical density, and the SCF energy; the Cartesian kernels underneath."""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import spherical as osph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fsim():
    from paper_2510_24968_amd import fsim
    return fsim


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _oracle_sph(b):
    B = oracle.Basis(b)
    S, T, V = B.one_electron()
    Tm = osph.transform(list(B.shell_l), S)
    return B, Tm, Tm.T @ S @ Tm, Tm.T @ (T + V) @ Tm


def test_spherical_one_electron_and_jk():
    b = synth.water_cluster(2, 3)
    print("[gpu] spherical water dimer", flush=True)
    ctx = _fsim().Context(b, tau=0.0, spherical=True)
    B, Tm, So, Ho = _oracle_sph(b)
    assert ctx.nbf == Tm.shape[1] == 40
    S, H, X = (t.cpu().numpy() for t in ctx.one_electron())
    assert np.max(np.abs(S - So)) < 1e-13 and np.max(np.abs(H - Ho)) < 1e-11
    assert np.max(np.abs(X @ So @ X - np.eye(40))) < 1e-10
    ctx.schwarz_screen()
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40))
    D = 0.5 * (A + A.T)
    Jc, Kc = B.fock_jk(Tm @ D @ Tm.T, tau=0.0)
    Jo, Ko = Tm.T @ Jc @ Tm, Tm.T @ Kc @ Tm
    r = ctx.fock_build(_dev(D), want_jk=True)
    dJ = np.max(np.abs(r["J"].cpu().numpy() - Jo))
    dK = np.max(np.abs(r["K"].cpu().numpy() - Ko))
    print(f"  |dJ| {dJ:.2e} |dK| {dK:.2e}", flush=True)
    assert dJ < 1e-11 and dK < 1e-11
    F = r["F"].cpu().numpy()
    assert np.max(np.abs(F - (Ho + Jo - 0.5 * Ko))) < 1e-11
    assert r["E_elec"] == pytest.approx(0.5 * np.sum(D * (Ho + F)), abs=1e-10)


@pytest.mark.parametrize("nmol,seed", [(1, 3), (3, 2)])
def test_spherical_scf_against_oracle(nmol, seed):
    """SCF in the spherical basis equals the oracle's spherical SCF within
    1e-8 Ha, lies above the Cartesian SCF (variational), and the stored-
    integral mode gives the same energy."""
    b = synth.water_cluster(nmol, seed)
    ro = osph.scf(b, conv_rms_dD=1e-9, conv_dE=1e-11, tau=1e-12)
    ctx = _fsim().Context(b, tau=1e-12, conv_rms_dD=1e-9, conv_dE=1e-11, spherical=True)
    r = ctx.scf()
    rc = _fsim().Context(b, tau=1e-12, conv_rms_dD=1e-9, conv_dE=1e-11).scf()
    print(f"spherical (H2O){nmol}: E - oracle = {r['E_total'] - ro['E_total']:.2e}, "
          f"E_sph - E_cart = {r['E_total'] - rc['E_total']:.3e}", flush=True)
    assert r["converged"] and abs(r["E_total"] - ro["E_total"]) < 1e-8
    assert r["E_total"] > rc["E_total"]
    ctx.store_eris()
    r2 = ctx.scf()
    assert abs(r2["E_total"] - ro["E_total"]) < 1e-8


def test_spherical_limits():
    fsim = _fsim()
    ctx = fsim.Context(synth.water_cluster(1, 0), spherical=True)
    with pytest.raises(fsim.FsimError, match="Cartesian"):
        ctx.set_incremental(4)
    ctx.schwarz_screen()
    D = torch.zeros((ctx.nbf, ctx.nbf), dtype=torch.float64, device="cuda")
    with pytest.raises(fsim.FsimError, match="Cartesian"):
        fsim._check(fsim.lib().fsim_fock_build_noalloc(ctx.h, fsim._ptr(D), fsim._ptr(D), None,
                                                       None, None, 0, fsim._stream()))
    # batches stay Cartesian
    mols = [synth.h_chain(2, 1.4), synth.water_cluster(1, 1)]
    structs = [fsim.basis_struct(m) for m in mols]
    arr = (fsim._Basis * 2)(*[st for st, _ in structs])
    opt = fsim._Options(0.0, 0.0, 8, 1e-8, 1e-10, 100, 1)
    h = ctypes.c_void_p()
    st = fsim.lib().fsim_batch_create(arr, 2, ctypes.byref(opt), ctypes.byref(h))
    assert st == -1 and b"one-molecule" in fsim.lib().fsim_last_error()
