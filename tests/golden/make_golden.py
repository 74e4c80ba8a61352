"""Write the stored oracle results the GPU parity tests compare with.

Calls only the oracle and the seeded input generators.  Run from the repo
root:  python tests/golden/make_golden.py [--threads N] [name ...]
Each result goes to tests/golden/<name>_oracle.json.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

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


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("names", nargs="*", default=["h8_chain", "water10"])
    a = ap.parse_args()
    for n in a.names:
        run(n, a.threads)
