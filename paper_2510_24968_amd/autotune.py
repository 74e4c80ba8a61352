"""Autotuner front end: runs the library's per-class variant search
(fsim_autotune: every kernel variant x waves-per-block, timed per launch with
HIP events on the workload itself) and keeps the result in a JSON cache keyed
by quartet class, precision and primitive-pair counts, so that later contexts
with the same shapes start from the tuned settings.

    python -m paper_2510_24968_amd.autotune --workload water64 --out tuning.json
"""

import argparse
import json
import os
import sys
import time


def cache_key(rec):
    prec = "fp32" if rec["fp32"] else "fp64"
    return f"{rec['cls']}|{prec}|K{rec['kbra']}x{rec['kket']}"


def tune(ctx, D, precisions=("mixed", "fp64"), progress=True):
    """Run the search for each precision; returns {key: record}.  FP32
    settings come from the mixed build and FP64 settings from the FP64
    build (whose FP64 lists hold every kept quartet, not only the mixed
    build's FP64 part); the context ends with the combined settings."""
    table = {}
    if progress:
        # one line per timed pass from the library (see fsim_autotune)
        os.environ["FSIM_AUTOTUNE_VERBOSE"] = "1"
    for prec in precisions:
        print(f"[autotune] {prec}: searching variants x waves-per-block", file=sys.stderr,
              flush=True)
        t0 = time.time()
        recs = ctx.autotune(D, prec)
        print(f"[autotune] {prec}: done in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        for rec in recs:
            if rec["ms"] > 0 and bool(rec["fp32"]) == (prec == "mixed"):
                table[cache_key(rec)] = {k: rec[k] for k in
                                         ("cls", "bra_class", "ket_class", "fp32", "variant",
                                          "waves_per_block", "seg_tiles", "kbra", "kket", "ms")}
    apply(ctx, table)
    return table


def save(table, path, meta=None):
    data = {"meta": meta or {}, "entries": table}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(path):
    with open(path) as f:
        return json.load(f)["entries"]


def apply(ctx, table):
    """Apply cached settings whose key matches this context's classes."""
    cur = ctx.get_tuning()
    recs = []
    for r in cur:
        hit = table.get(cache_key(r))
        if hit is not None:
            recs.append(dict(bra_class=r["bra_class"], ket_class=r["ket_class"], fp32=r["fp32"],
                             variant=hit["variant"], waves_per_block=hit["waves_per_block"],
                             seg_tiles=hit.get("seg_tiles", 0), ms=hit.get("ms", 0.0)))
    if recs:
        ctx.set_tuning(recs)
    return len(recs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="water10")
    ap.add_argument("--out", default=None)
    ap.add_argument("--tau-prim", type=float, default=None,
                    help="primitive-pair screening threshold to tune under (default 1e-4 x "
                         "the Schwarz tau, as the benchmark runs; 0: every primitive pair)")
    a = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth
    from paper_2510_24968_amd import fsim
    basis, w = synth.workload(a.workload)
    if isinstance(basis, list):     # a batch of molecules in one context
        ctx = fsim.Batch(basis, tau=w["tau"], tau_fp32=w["tau_fp32"] or 1e-5)
    else:
        ctx = fsim.Context(basis, tau=w["tau"], tau_fp32=w["tau_fp32"] or 1e-5)
    tau_prim = 1e-4 * w["tau"] if a.tau_prim is None else a.tau_prim
    if tau_prim > 0:
        ctx.set_prim_screen(tau_prim)
    ctx.schwarz_screen()
    D = ctx.core_guess()
    t0 = time.time()
    table = tune(ctx, D)
    print(f"tuned {len(table)} class settings in {time.time() - t0:.1f}s", file=sys.stderr)
    out = a.out or os.path.join(os.getcwd(), f"tuning_{a.workload}.json")
    save(table, out, {"workload": a.workload, "device": "MI355X (gfx950)", "tau_prim": tau_prim})
    print(json.dumps({k: (v["variant"], v["waves_per_block"], v.get("seg_tiles", 0), round(v["ms"], 3))
                      for k, v in sorted(table.items())}))


if __name__ == "__main__":
    main()
