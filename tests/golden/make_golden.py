"""Write the stored oracle results the GPU parity tests compare with.

Calls only the oracle and the seeded input generators.  Run from the repo
root:  python tests/golden/make_golden.py [--threads N] [name ...]

  h8_chain, water10   full oracle SCF -> tests/golden/<name>_oracle.json
  water64_fock        one oracle Fock build of the 64-water cluster (Schwarz
                      tau = 1e-11) at the oracle's own core-Hamiltonian density
                      of the whole cluster: E_elec = 1/2 Tr[D (H + F(D))]
                      (Sec. 2.2 Eq. fock, the energy of Sec. 3.2), Tr(DJ),
                      Tr(DK) and sampled J/K elements ->
                      tests/golden/water64_fock_oracle.json, and that density
                      (upper triangle, compressed) ->
                      tests/golden/water64_core_density.npz.  About an hour
                      of CPU on 8 threads.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(name, threads):
    if threads:
        oracle.set_threads(threads)
    basis, w = synth.workload(name)
    t0 = time.time()
    B = oracle.Basis(basis)
    r = oracle.scf(B, tau=w["tau"], conv_rms_dD=w["conv_rms_dD"], conv_dE=w["conv_dE"],
                   max_iter=60, verbose=True)
    Q = B.schwarz()
    _, _, (kept, total) = B.fock_jk(r["D"], w["tau"], Q, with_counts=True)
    out = {
        "workload": name,
        "generator": "synth.workload('%s')" % name,
        "method": "oracle.scf: RHF, core-Hamiltonian guess, DIIS m=8, "
                  "Schwarz tau=%g" % w["tau"],
        "nbf": B.nbf,
        "nelec": B.nelec,
        "E_total": r["E_total"],
        "E_elec": r["E_elec"],
        "E_nuc": r["E_nuc"],
        "iterations": r["iterations"],
        "converged": r["converged"],
        "screened_quartets": kept,
        "canonical_quartets": total,
        "history": r["history"],
        "oracle_threads": oracle.num_threads(),
        "wall_s": time.time() - t0,
    }
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "history"}), flush=True)


def _sample_elements(basis, nbf, rng):
    """(mu, nu, kind) pairs spread over the cluster: every diagonal element,
    pairs inside one molecule, pairs between nearest-neighbour molecules and
    uniformly random pairs (mostly between distant molecules)."""
    nmol = len(basis["Z"]) // 3
    per = nbf // nmol                      # basis functions per molecule
    oxy = np.asarray(basis["xyz"])[0::3]
    d = np.linalg.norm(oxy[:, None, :] - oxy[None, :, :], axis=-1)
    np.fill_diagonal(d, np.inf)
    nn = np.argmin(d, axis=1)
    mus, nus, kinds = list(range(nbf)), list(range(nbf)), ["diag"] * nbf
    for _ in range(600):
        m = int(rng.integers(nmol))
        a, b = rng.integers(per, size=2)
        mus.append(m * per + int(a)); nus.append(m * per + int(b)); kinds.append("intra")
    for _ in range(600):
        m = int(rng.integers(nmol))
        a, b = rng.integers(per, size=2)
        mus.append(m * per + int(a)); nus.append(int(nn[m]) * per + int(b)); kinds.append("neighbour")
    for _ in range(600):
        a, b = rng.integers(nbf, size=2)
        mus.append(int(a)); nus.append(int(b)); kinds.append("random")
    return np.array(mus, dtype=np.int32), np.array(nus, dtype=np.int32), kinds


def run_water64_fock(threads):
    if threads:
        oracle.set_threads(threads)
    basis, w = synth.workload("water64")
    tau = w["tau"]
    t0 = time.time()
    B = oracle.Basis(basis)
    S, T, V = B.one_electron()
    H = T + V
    X = oracle.orthogonalizer(S)
    D, _, _ = oracle.density_from_fock(H, X, B.nelec // 2)
    D = 0.5 * (D + D.T)
    N = B.nbf
    iu = np.triu_indices(N)
    np.savez_compressed(os.path.join(HERE, "water64_core_density.npz"), D_upper=D[iu], nbf=N)
    print(f"core density done at {time.time() - t0:.0f}s", flush=True)
    Q = B.schwarz()
    J, K, (kept, total) = B.fock_jk(D, tau, Q, with_counts=True)
    print(f"Fock build done at {time.time() - t0:.0f}s", flush=True)
    F = H + J - 0.5 * K
    E = 0.5 * float(np.sum(D * (H + F)))
    mus, nus, kinds = _sample_elements(basis, N, np.random.default_rng(64))
    out = {
        "workload": "water64",
        "generator": "synth.workload('water64')",
        "method": "oracle core-Hamiltonian density of the whole cluster (D = 2 C_occ C_occ^T "
                  "of X^T H X), then one oracle Fock build over canonical quartets with "
                  "Q_ab Q_cd >= tau",
        "tau": tau,
        "nbf": N,
        "nelec": B.nelec,
        "density_file": "water64_core_density.npz",
        "density_sum": float(D.sum()),
        "density_fro": float(np.linalg.norm(D)),
        "trace_DS": float(np.sum(D * S)),
        "E_elec": E,
        "E_one": float(np.sum(D * H)),
        "trace_DJ": float(np.sum(D * J)),
        "trace_DK": float(np.sum(D * K)),
        "E_nuc": B.nuclear_repulsion(),
        "screened_quartets": kept,
        "canonical_quartets": total,
        "elements": {"mu": mus.tolist(), "nu": nus.tolist(), "kind": kinds,
                     "J": [float(J[a, b]) for a, b in zip(mus, nus)],
                     "K": [float(K[a, b]) for a, b in zip(mus, nus)]},
        "max_abs_J": float(np.abs(J).max()),
        "max_abs_K": float(np.abs(K).max()),
        "oracle_threads": oracle.num_threads(),
        "wall_s": time.time() - t0,
    }
    assert math.isfinite(E)
    with open(os.path.join(HERE, "water64_fock_oracle.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(json.dumps({k: v for k, v in out.items() if k != "elements"}), flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("names", nargs="*", default=["h8_chain", "water10"])
    a = ap.parse_args()
    for n in a.names:
        if n == "water64_fock":
            run_water64_fock(a.threads)
        else:
            run(n, a.threads)
