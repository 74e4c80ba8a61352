"""Primitive-pair screening (fsim_set_prim_screen) against the FP64 oracle,
which keeps every primitive pair.

A dropped primitive pair k changes an integral (ab|cd) by at most
Q_k Q_cd <= tau_prim (Cauchy-Schwarz for the Coulomb inner product, with
Q_k Q_max < tau_prim), so each integral moves by at most
(dropped primitive pairs of its bra and ket) * tau_prim: the one-pair-density
test reads single integrals out of J and K and checks that bound; the others
check J, K and energies at the screening thresholds the benchmark uses
against the oracle's unscreened values."""

import json
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fsim():
    from paper_2510_24968_amd import fsim
    return fsim


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _random_density(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    return 0.5 * (A + A.T)


def test_single_integrals_within_the_bound():
    """A water trimer without shell screening and a loose tau_prim = 1e-7
    (so that many primitive pairs go): with D = e_ls + e_sl, J_mn =
    2 (mn|ls) and K_mn = (ml|ns) + (ms|nl), so every integral of the
    chosen (l, s) columns is compared with the oracle's; the largest
    contracted pair here holds 9 primitive pairs."""
    b = synth.water_cluster(3, 2)
    B = oracle.Basis(b)
    g = B.eri_tensor()
    tau_prim = 1e-7
    print(f"[gpu] water trimer, tau_prim {tau_prim}", flush=True)
    ctx = _fsim().Context(b)
    ctx.set_prim_screen(tau_prim)
    _, st = ctx.schwarz_screen(tau=0.0)
    print("primitive pairs kept", st["prim_pairs_kept"], "of", st["prim_pairs_total"], flush=True)
    assert st["prim_pairs_kept"] < 0.9 * st["prim_pairs_total"]
    bound = 2 * 9 * tau_prim * 1.01
    N = B.nbf
    rng = np.random.default_rng(3)
    worst = 0.0
    for l, s in [(0, 0), (5, 30), (N - 1, 2), (11, 12)] + \
            [tuple(rng.integers(0, N, 2)) for _ in range(4)]:
        D = np.zeros((N, N))
        D[l, s] += 1.0
        D[s, l] += 1.0
        r = ctx.fock_build(_dev(D), want_jk=True)
        J, K = r["J"].cpu().numpy(), r["K"].cpu().numpy()
        Jo = g[:, :, l, s] + g[:, :, s, l]
        Ko = g[:, l, :, s] + g[:, s, :, l]
        dJ, dK = np.max(np.abs(J - Jo)), np.max(np.abs(K - Ko))
        worst = max(worst, dJ, dK)
        # two integrals per element (one, doubled, on the diagonal)
        assert dJ < 2 * bound + 1e-12, (l, s, dJ)
        assert dK < 2 * bound + 1e-12, (l, s, dK)
    print(f"largest integral change {worst:.3e} (bound {bound:.2e})", flush=True)


def test_water10_scf_energy_and_stored_mode():
    """The 10-water workload with tau_prim = 1e-4 tau: J and K at a random
    density against the oracle's unscreened build (1e-10), the SCF energy
    against the stored oracle SCF (1e-8 Ha), and the conventional mode built
    over the same compacted tables agreeing with the direct build."""
    b, w = synth.workload("water10")
    with open(os.path.join(GOLDEN, "water10_oracle.json")) as f:
        gold = json.load(f)
    fs = _fsim()
    ctx = fs.Context(b, tau=w["tau"], conv_rms_dD=w["conv_rms_dD"], conv_dE=w["conv_dE"])
    _, st0 = ctx.schwarz_screen()
    ctx.set_prim_screen(1e-4 * w["tau"])
    with pytest.raises(fs.FsimError):
        ctx.fock_build(_dev(np.zeros((ctx.nbf, ctx.nbf))))
    _, st = ctx.schwarz_screen()
    print("water10 primitive quartets", st["prim_quartets_kept"], "of", st0["prim_quartets_kept"],
          flush=True)
    assert st["quartets_kept"] == st0["quartets_kept"]
    assert st["prim_quartets_kept"] < 0.9 * st0["prim_quartets_kept"]
    D = _random_density(ctx.nbf, 77)
    Jo, Ko = oracle.Basis(b).fock_jk(D, tau=w["tau"])
    r = ctx.fock_build(_dev(D), want_jk=True)
    dJ = np.max(np.abs(r["J"].cpu().numpy() - Jo))
    dK = np.max(np.abs(r["K"].cpu().numpy() - Ko))
    print(f"water10 random density: max |dJ| {dJ:.3e}, max |dK| {dK:.3e}", flush=True)
    assert dJ < 1e-10 and dK < 1e-10
    res = ctx.scf()
    assert res["converged"]
    print("water10 dE vs oracle =", res["E_total"] - gold["E_total"], flush=True)
    assert abs(res["E_total"] - gold["E_total"]) < 1e-8
    Dd = _dev(D)
    direct = ctx.fock_build(Dd, want_jk=True)
    assert ctx.store_eris() > 0
    stored = ctx.fock_build(Dd, want_jk=True)
    assert torch.max(torch.abs(stored["J"] - direct["J"])).item() < 1e-12
    assert torch.max(torch.abs(stored["K"] - direct["K"])).item() < 1e-12


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_with_prim_screen(persistent):
    """Batched contexts (per-molecule Q_max in the rule), with the persistent
    s/p launch and without: J and K per molecule against the oracle."""
    mols = [synth.ch_molecule(5_000_000 + i, nmin=4, nmax=12) for i in range(5)]
    mols.append(synth.water_cluster(2, 9))
    bt = _fsim().Batch(mols)
    bt.set_persistent(persistent)
    bt.set_prim_screen(1e-15)
    _, st = bt.schwarz_screen(tau=1e-11)
    assert st["prim_pairs_kept"] < st["prim_pairs_total"]
    blocks = [_random_density(synth.nbf_of(b), 60 + k) for k, b in enumerate(mols)]
    r = bt.fock_build(bt.pack([_dev(x) for x in blocks]), want_jk=True)
    Js, Ks = bt.unpack(r["J"]), bt.unpack(r["K"])
    for k, b in enumerate(mols):
        Jo, Ko = oracle.Basis(b).fock_jk(blocks[k], tau=1e-11)
        assert np.max(np.abs(Js[k].cpu().numpy() - Jo)) < 1e-10, k
        assert np.max(np.abs(Ks[k].cpu().numpy() - Ko)) < 1e-10, k


def test_invalid_threshold():
    fs = _fsim()
    ctx = fs.Context(synth.h_chain(4, 1.4))
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(fs.FsimError):
            ctx.set_prim_screen(bad)
    ctx.set_prim_screen(0.0)
    _, st = ctx.schwarz_screen()
    assert st["prim_pairs_kept"] == st["prim_pairs_total"]


def test_incremental_and_noalloc_builds_with_prim_screen():
    """The compacted tables under the other build paths of the 10-water
    workload: the incremental SCF (segments cut again every build) reaches
    the stored oracle SCF energy within 1e-8 Ha, and the allocation-free
    entry point equals fsim_fock_build up to summation order."""
    b, w = synth.workload("water10")
    with open(os.path.join(GOLDEN, "water10_oracle.json")) as f:
        gold = json.load(f)
    ctx = _fsim().Context(b, tau=w["tau"], conv_rms_dD=w["conv_rms_dD"], conv_dE=w["conv_dE"])
    ctx.set_prim_screen(1e-4 * w["tau"])
    ctx.schwarz_screen()
    ctx.set_incremental(8)
    inc = ctx.scf(refine=False)
    ctx.set_incremental(0)
    print("water10 incremental, primitive screen: dE vs oracle =",
          inc["E_total"] - gold["E_total"], flush=True)
    assert inc["converged"] and abs(inc["E_total"] - gold["E_total"]) < 1e-8
    assert any(not h["full_build"] for h in inc["history"])
    D = _dev(_random_density(ctx.nbf, 91))
    ref = ctx.fock_build(D, want_jk=True)
    F = torch.empty_like(ref["F"])
    J, K = torch.empty_like(ref["J"]), torch.empty_like(ref["K"])
    e = ctx.fock_build_noalloc(D, F, J, K)
    assert torch.max(torch.abs(J - ref["J"])).item() < 1e-11
    assert torch.max(torch.abs(K - ref["K"])).item() < 1e-11
    assert abs(e - ref["E_elec"]) < 1e-9
