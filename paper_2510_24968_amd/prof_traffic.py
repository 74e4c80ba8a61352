"""HBM traffic per ERI kernel launch from two rocprofv3 counter runs.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o w64 -- \\
        python3 -m paper_2510_24968_amd.prof_run --workload water64
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o w64 -- \\
        python3 -m paper_2510_24968_amd.prof_run --workload water64
    python -m paper_2510_24968_amd.prof_traffic F/w64_counter_collection.csv \\
        W/w64_counter_collection.csv --workload water64 --command "..."

Both counters are in KiB per dispatch.  Each is scaled by what it reads for
the counter run's plain 1 GiB device copy (read 1 GiB, write 1 GiB), so the
result is bytes.  The summary records a digest of the kernel sources:
readings from other sources do not describe the kernels any more.
"""

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PAIR = {(0, 0): "ss", (1, 0): "ps", (1, 1): "pp", (2, 0): "ds", (2, 1): "dp", (2, 2): "dd"}
COPY_BYTES = 1 << 30


def source_digest():
    """Hash of the ERI kernel sources (class files, kernel header, Boys,
    shared definitions)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("eri_") or f in ("boys.h", "fsim_internal.h"):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _per_dispatch(path):
    agg = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        k = int(r["Dispatch_Id"])
        if k not in agg:
            agg[k] = {"name": r["Kernel_Name"], "kib": 0.0,
                      "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])}
        agg[k]["kib"] += float(r["Counter_Value"])
    return list(agg.values())


def _per_dispatch_counters(path):
    """Per dispatch: kernel name, duration and every counter summed over its
    instances."""
    agg = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        k = int(r["Dispatch_Id"])
        if k not in agg:
            agg[k] = {"name": r["Kernel_Name"], "c": collections.Counter(),
                      "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])}
        agg[k]["c"][r["Counter_Name"]] += float(r["Counter_Value"])
    return list(agg.values())


def _class_of(name):
    m = re.search(r"k_eri_(?:lane_ko|lane|wave|mfma)<(\d), (\d), (\d), (\d), (double|float)(, true)?",
                  name)
    if not m or m.group(6):      # stored-block (screening) launches are not Fock-build work
        return None
    la, lb, lc, ld = (int(m.group(i)) for i in range(1, 5))
    return f"({PAIR[(la, lb)]}|{PAIR[(lc, ld)]})" + ("" if m.group(5) == "double" else " f32")


def summarise(fetch_csv, write_csv):
    fetch, write = _per_dispatch(fetch_csv), _per_dispatch(write_csv)
    cal_f = max((d for d in fetch if "copyBuffer" in d["name"]), key=lambda d: d["kib"])
    cal_w = max((d for d in write if "copyBuffer" in d["name"]), key=lambda d: d["kib"])
    f_fac = COPY_BYTES / (cal_f["kib"] * 1024.0)
    w_fac = COPY_BYTES / (cal_w["kib"] * 1024.0)
    kern = {}
    for df, dw in zip(fetch, write):
        cls = _class_of(df["name"])
        if cls is None or df["name"] != dw["name"]:
            continue
        b = df["kib"] * 1024.0 * f_fac + dw["kib"] * 1024.0 * w_fac
        kern[cls] = {"kernel": df["name"].replace("void fsim::", "").split("(")[0],
                     "fetch_kib": df["kib"], "write_kib": dw["kib"], "bytes_per_launch": b,
                     "ms_under_counters": df["ns"] / 1e6}
    return {"fetch_factor": f_fac, "write_factor": w_fac,
            "copy_fetch_kib": cal_f["kib"], "copy_write_kib": cal_w["kib"], "kernels": kern}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--workload", default="water64")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    s = summarise(a.fetch_csv, a.write_csv)
    s["source_digest"] = source_digest()
    s["workload"] = a.workload
    lines = [f"# HBM traffic per ERI launch: {a.workload}, FP64 Fock build", "",
             "Commands (from the repository root on the GPU host):", "", "```", a.command, "```",
             "", f"Calibration: a 1 GiB device copy reads FETCH_SIZE = {s['copy_fetch_kib']:.0f} KiB "
             f"and WRITE_SIZE = {s['copy_write_kib']:.0f} KiB, so the factors are "
             f"{s['fetch_factor']:.3f} (fetch) and {s['write_factor']:.3f} (write).", "",
             "| class | kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes/launch (scaled) |",
             "|---|---|---|---|---|"]
    for cls, r in sorted(s["kernels"].items(), key=lambda kv: -kv[1]["bytes_per_launch"]):
        lines.append(f"| {cls} | `{r['kernel']}` | {r['fetch_kib']:.0f} | {r['write_kib']:.0f} | "
                     f"{r['bytes_per_launch']:.3e} |")
    lines += ["", "```json", json.dumps(s, indent=1), "```", ""]
    out = os.path.join(ROOT, "profiles", f"k_eri_{a.workload}_fp64_traffic.md")
    with open(out, "w") as f:
        f.write("\n".join(lines))
    print(out)


if __name__ == "__main__":
    main()
