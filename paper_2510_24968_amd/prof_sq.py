"""SQ counter summary per ERI kernel from two rocprofv3 counter runs.

    rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_LDS \\
        SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_INSTS_LDS SQ_INSTS_VALU \\
        --output-format csv -d S -o w64 -- python3 -m paper_2510_24968_amd.prof_run
    rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 \\
        SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_ADD_F32 \\
        SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 \\
        --output-format csv -d M -o w64 -- python3 -m paper_2510_24968_amd.prof_run
    python -m paper_2510_24968_amd.prof_sq S/w64_counter_collection.csv \\
        M/w64_counter_collection.csv --workload water64 --command "..."

The instruction counters count wave instructions, so the FP64 VALU work a
kernel issued is 64 (ADD + MUL + TRANS + 2 FMA) flops per counted
instruction (every lane, active or not), plus 512 flops per FP64 MFMA MOPS
unit; divided by the dispatch's duration under the counters it gives the
issued FP64 rate against the 78.6 TFLOP/s vector peak.  The wait and busy
ratios are per wave cycle.  Like the traffic summary, the file records the
kernel-source digest it was taken on.
"""

import argparse
import json
import os

from paper_2510_24968_amd.prof_traffic import ROOT, _class_of, _per_dispatch_counters, source_digest

FP64_PEAK_TFLOPS = 78.6


def summarise(sq_csv, mix_csv):
    sq, mix = _per_dispatch_counters(sq_csv), _per_dispatch_counters(mix_csv)
    out = {}
    for rows, tag in ((sq, "sq"), (mix, "mix")):
        for r in rows:
            cls = _class_of(r["name"])
            if cls is None:
                continue
            rec = out.setdefault(cls, {"kernel": r["name"].replace("void fsim::", "")
                                       .replace("(fsim::EriArgs)", ""), "launches": {}})
            # keep the longest launch of the class (the FP64 build's full list)
            best = rec["launches"].get(tag)
            if best is None or r["ns"] > best["ns"]:
                rec["launches"][tag] = {"ns": r["ns"], "c": dict(r["c"])}
    res = {}
    for cls, rec in out.items():
        if "sq" not in rec["launches"] or "mix" not in rec["launches"]:
            continue
        c, m = rec["launches"]["sq"]["c"], rec["launches"]["mix"]["c"]
        cyc = max(c.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        fl64 = 64.0 * (m.get("SQ_INSTS_VALU_ADD_F64", 0) + m.get("SQ_INSTS_VALU_MUL_F64", 0) +
                       m.get("SQ_INSTS_VALU_TRANS_F64", 0) +
                       2.0 * m.get("SQ_INSTS_VALU_FMA_F64", 0)) + \
            512.0 * m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0)
        fl32 = 64.0 * (m.get("SQ_INSTS_VALU_ADD_F32", 0) + m.get("SQ_INSTS_VALU_MUL_F32", 0) +
                       2.0 * m.get("SQ_INSTS_VALU_FMA_F32", 0))
        ms = rec["launches"]["mix"]["ns"] / 1e6
        res[cls] = {"kernel": rec["kernel"], "ms_under_counters": ms,
                    "wave_cycles": c.get("SQ_WAVE_CYCLES", 0.0),
                    "wait": c.get("SQ_WAIT_ANY", 0.0) / cyc,
                    "valu_busy": c.get("SQ_ACTIVE_INST_VALU", 0.0) / cyc,
                    "lds_busy": c.get("SQ_ACTIVE_INST_LDS", 0.0) / cyc,
                    "valu_insts": c.get("SQ_INSTS_VALU", 0.0),
                    "lds_insts": c.get("SQ_INSTS_LDS", 0.0),
                    "fp64_flops_issued": fl64, "fp32_flops_issued": fl32,
                    "fp64_tflops_issued": fl64 / (ms * 1e-3) / 1e12,
                    "fp64_frac_of_peak": fl64 / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sq_csv")
    ap.add_argument("mix_csv")
    ap.add_argument("--workload", default="water64")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    res = summarise(a.sq_csv, a.mix_csv)
    keep = ("kernel", "ms_under_counters", "wait", "valu_busy", "fp64_tflops_issued",
            "fp64_frac_of_peak")
    blob = {"source_digest": source_digest(), "workload": a.workload,
            "kernels": {c: {k: r[k] for k in keep} for c, r in res.items()}}
    lines = [f"# SQ counters per ERI launch: {a.workload}, FP64 Fock build", "",
             "Commands (from the repository root on the GPU host):", "", "```", a.command, "```", "",
             "One FP64 Fock build with the committed tuning cache and the benchmark's primitive "
             "screen (`prof_run`), two counter passes. Per class the longest launch (the FP64 "
             "build's full list). `wait`, `VALU`, `LDS`: SQ_WAIT_ANY, SQ_ACTIVE_INST_VALU, "
             "SQ_ACTIVE_INST_LDS per SQ_WAVE_CYCLES. `FP64 issued`: 64 x (ADD + MUL + TRANS + "
             "2 FMA) FP64 wave instructions (+ 512 per FP64 MFMA MOPS) per launch second, every "
             "lane counted; `of peak`: against 78.6 TFLOP/s.", "",
             "| class | kernel | ms | wait | VALU | LDS | FP64 issued TFLOP/s | of peak |",
             "|---|---|---|---|---|---|---|---|"]
    for cls, r in sorted(res.items(), key=lambda kv: -kv[1]["ms_under_counters"]):
        lines.append(f"| {cls} | `{r['kernel']}` | {r['ms_under_counters']:.1f} | {r['wait']:.2f} | "
                     f"{r['valu_busy']:.2f} | {r['lds_busy']:.2f} | {r['fp64_tflops_issued']:.1f} | "
                     f"{r['fp64_frac_of_peak']:.3f} |")
    lines += ["", "```json", json.dumps(blob, indent=1), "```", ""]
    out = os.path.join(ROOT, "profiles", f"k_eri_{a.workload}_fp64_sq_counters.md")
    with open(out, "w") as f:
        f.write("\n".join(lines))
    print(out)


if __name__ == "__main__":
    main()
