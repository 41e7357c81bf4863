"""Build the HIP/C++ library libdd4dvar.so in-tree for gfx950.

Usage: python -m paper_2205_06649_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdd4dvar.so")
ARCH = os.environ.get("DD4DVAR_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

# (source, object, extra flags): the sweep kernels are compiled once per state
# type; FP64 without floating-point contraction (separately rounded multiply
# and add, as in the FP64 reference), FP32 with the default FMA contraction.
HIP_UNITS = [
    ("sweep.hip", "sweep_f32.o", ["-DDD4DVAR_SWEEP_T=float", "-DDD4DVAR_SWEEP_PRIMARY=1"]),
    ("sweep.hip", "sweep_f64.o", ["-DDD4DVAR_SWEEP_T=double", "-DDD4DVAR_SWEEP_PRIMARY=0",
                                  "-ffp-contract=off"]),
    ("tlm.hip", "tlm_f32.o", ["-DDD4DVAR_TLM_T=float"]),
    ("tlm.hip", "tlm_f64.o", ["-DDD4DVAR_TLM_T=double", "-ffp-contract=off"]),
    ("tz.hip", "tz_f32.o", ["-DDD4DVAR_TZ_T=float"]),
    ("tz.hip", "tz_f64.o", ["-DDD4DVAR_TZ_T=double", "-ffp-contract=off"]),
    ("tzbox.hip", "tzbox.o", []),
    ("gn.hip", "gn.o", []),
    ("exchange.hip", "exchange.o", []),
    ("box.hip", "box.o", []),
    ("solve.hip", "solve.o", []),
    ("engine.hip", "engine.o", []),
]
CXX_SOURCES = ["plan.cpp"]

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return res


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src, oname, extra in HIP_UNITS:
        obj = os.path.join(BUILD, oname)
        objs.append(obj)
        jobs.append([HIPCC, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        objs.append(obj)
        jobs.append([CXX, *CXX_FLAGS, "-I/opt/rocm/include", "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                sys.stderr.write(r.stdout + r.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
