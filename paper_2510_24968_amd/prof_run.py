"""Short driver for hardware-counter runs under rocprofv3.

One FP64 (or mixed) Fock build of a named workload with its committed
autotuner settings, preceded by a plain device copy of a known size whose
FETCH_SIZE / WRITE_SIZE readings calibrate the HBM byte counters:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -- \\
        python3 -m paper_2510_24968_amd.prof_run --workload water64
"""

import argparse
import os
import time

COPY_BYTES = 1 << 30


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="water64")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--builds", type=int, default=1)
    ap.add_argument("--density", default="diag", choices=("diag", "core"),
                    help="diag: 0.01 I (the build evaluates every kept quartet whatever the "
                         "density, so the kernels' work is the same and no eigensolver "
                         "dispatches run under the counters); core: the core-Hamiltonian guess")
    ap.add_argument("--stored", action="store_true",
                    help="compute the kept quartets once into the store (fsim_store_eris) and "
                         "time builds that digest it")
    ap.add_argument("--tau-prim", type=float, default=None,
                    help="primitive-pair screening threshold (default 1e-4 x the Schwarz tau, "
                         "as the benchmark runs; 0: every primitive pair)")
    a = ap.parse_args()
    import torch
    import synth
    from paper_2510_24968_amd import autotune, fsim
    log = lambda s: print(f"[prof_run] {s}", flush=True)
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)                       # the calibration copy: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    log(f"calibration copy of {COPY_BYTES} bytes done")
    del src, dst
    basis, w = synth.workload(a.workload)
    log("context (pair tables, one-electron matrices, orthogonaliser)")
    ctx = fsim.Context(basis, tau=w["tau"], tau_fp32=w["tau_fp32"] if w["tau_fp32"] > 0 else 1e-5)
    tau_prim = 1e-4 * w["tau"] if a.tau_prim is None else a.tau_prim
    if tau_prim > 0:
        ctx.set_prim_screen(tau_prim)
    log(f"Schwarz screen (primitive-pair threshold {tau_prim:g})")
    ctx.schwarz_screen()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                        f"{a.workload}_mi355x.json")
    if os.path.exists(path):
        log(f"applied {autotune.apply(ctx, autotune.load(path))} tuned class settings")
    if a.density == "core":
        log("core-Hamiltonian guess (rocSOLVER dsyevd)")
        D = ctx.core_guess()
    else:
        D = 0.01 * torch.eye(ctx.nbf, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    if a.stored:
        log(f"stored integrals: {ctx.store_eris() / 1e9:.2f} GB")
    log(f"density ready ({a.density}); Fock builds follow")
    for k in range(a.builds):
        t0 = time.time()
        ctx.fock_build(D, a.precision, energy=False)
        torch.cuda.synchronize()
        log(f"{a.precision} Fock build {k + 1}/{a.builds}: {time.time() - t0:.2f} s")
    ctx.close()


if __name__ == "__main__":
    main()
