"""Build libstag.so in-tree with hipcc for gfx950.

Usage: python paper_1111_0125_amd/build.py [-j JOBS] [-v]
(run as a script: importing the package needs the library this script builds)
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "libstag")
LIB = os.path.join(HERE, "libstag.so")

ARCH = os.environ.get("STAG_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: keep the compiler from forming packed fp32 instructions.
CXXFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
]

# (source, object name, extra flags)
UNITS = [
    ("hop.hip", "hop_f64.o", ["-DHOP_PREC=0", "-DHOP_NP=4"]),
    ("hop.hip", "hop_f32.o", ["-DHOP_PREC=1", "-DHOP_NP=4"]),
    ("hop.hip", "hop_f16s.o", ["-DHOP_PREC=2", "-DHOP_NP=4"]),
    ("hop.hip", "hop_f64_improved.o", ["-DHOP_PREC=0", "-DHOP_NP=8"]),
    ("hop.hip", "hop_f32_improved.o", ["-DHOP_PREC=1", "-DHOP_NP=8"]),
    ("hop.hip", "hop_f16s_improved.o", ["-DHOP_PREC=2", "-DHOP_NP=8"]),
    ("blas.hip", "blas.o", []),
    ("layout.hip", "layout.o", []),
    ("tiny.hip", "tiny.o", []),
    ("scratch.hip", "scratch.o", []),
    ("capi.cpp", "capi.o", []),
    ("solver.cpp", "solver.o", []),
    ("serve.cpp", "serve.o", []),
    ("tune.cpp", "tune.o", []),
]


def _compile(unit, verbose):
    src, obj, extra = unit
    if not os.path.exists(os.path.join(CSRC, src)):
        return None
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC, *CXXFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return out


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = [o for o in ex.map(lambda u: _compile(u, verbose), UNITS) if o]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=0)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.j, a.v))
    sys.exit(0)
