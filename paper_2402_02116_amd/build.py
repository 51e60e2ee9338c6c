"""Build libfwils.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage:  python -m paper_2402_02116_amd.build [--jobs N] [--verbose]

Sources are compiled in parallel into _build/ next to this file and linked
into paper_2402_02116_amd/libfwils.so.  Every build recompiles all sources.
"""

import argparse
import concurrent.futures
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfwils.so")
# The core (kernels and capi.cpp) is compiled once per precision: complex64
# and, with -DFW_C128, complex128; abi.cpp (the public entry points) once.
CORE = ["kernels_rows.hip", "kernels_cols.hip", "kernels_fft.hip", "kernels_vec.hip", "kernels_maps.hip",
        "kernels_gmres.hip", "kernels_srows.hip", "kernels_3d.hip", "capi.cpp"]
UNITS = [(s, "c64") for s in CORE] + [(s, "c128") for s in CORE] + [("abi.cpp", None)]
SOURCES = CORE + ["abi.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(unit, verbose):
    src, prec = unit
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + (f"_{prec}" if prec else "") + ".o")
    cmd = [HIPCC] + FLAGS
    if prec == "c128":
        cmd += ["-DFW_C128"]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    t = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
    if verbose:
        print(f"  {src} ({prec or 'abi'}): {time.time() - t:.1f}s", flush=True)
        if res.stderr.strip():
            print(res.stderr)
    return obj


def build(jobs=None, verbose=False):
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    # longest units first
    order = sorted(UNITS, key=lambda u: (u[0] not in ("kernels_rows.hip", "kernels_cols.hip", "kernels_3d.hip",
                                                     "kernels_srows.hip", "kernels_vec.hip"), u[1] != "c64"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), order))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    t = time.time()
    lib = build(a.jobs, a.verbose)
    print(f"built {lib} in {time.time() - t:.1f}s")


if __name__ == "__main__":
    sys.exit(main())
