"""Build libfsim.so in-tree: every HIP source compiled for gfx950 with hipcc,
linked against rocBLAS / rocSOLVER.

    python -m paper_2510_24968_amd.build [-j N] [--verbose]
"""

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfsim.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

_PC = ("ss", "ps", "pp", "ds", "dp", "dd")
# eri_class.hip once per (bra pair class, ket pair class, precision): object
# name -> defines; slowest (highest angular momentum) first so the pool stays busy
ERI_UNITS = [(f"eri_{_PC[b]}{_PC[k]}_{'f32' if p else 'f64'}",
              [f"-DFSIM_BRA={b}", f"-DFSIM_KET={k}", f"-DFSIM_FP32={p}"])
             for b in range(6) for k in range(b + 1) for p in (0, 1)][::-1]
SOURCES = [("eri_class.hip", name, defs) for name, defs in ERI_UNITS] + [
    (src, os.path.splitext(src)[0], []) for src in
    ("persistent.hip", "stored.hip", "eri_dispatch.hip", "setup.hip", "linalg.hip", "mlp.hip", "noalloc.hip",
     "api.cpp")]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP64 atomic add on (coarse-grained) device memory
    "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# headers the ERI kernel units include (the other sources may include any)
ERI_HEADERS = ("eri_kernels.h", "boys.h", "fsim_internal.h")
ERI_SOURCES = ("eri_class.hip", "stored.hip", "persistent.hip")


def _newest_header(src):
    names = ERI_HEADERS if src in ERI_SOURCES else [
        f for f in os.listdir(CSRC) if f.endswith(".h")]
    return max(os.path.getmtime(os.path.join(CSRC, f)) for f in names)


def _compile(unit, verbose, incremental=False):
    src, name, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        deps = max(os.path.getmtime(os.path.join(CSRC, src)), _newest_header(src))
        if src not in ERI_SOURCES:
            deps = max(deps, os.path.getmtime(os.path.join(ROOT, "include", "fsim.h")))
        if t > deps:
            return obj
    cmd = [HIPCC] + FLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + defs + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"  {name}: {time.time() - t0:.1f}s", flush=True)
    return obj


def build(jobs=None, verbose=False, incremental=False):
    """Compile every source (or, with incremental=True, only those older than
    their source or a header) and link libfsim.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    t0 = time.time()
    build(a.j, a.verbose, a.incremental)
    print(f"built {LIB} in {time.time() - t0:.1f}s")
    sys.exit(0)
