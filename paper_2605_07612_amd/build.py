"""Builds libfoap4.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled to an object under _build/ (stage.hip once per
scheme) and the objects are linked into paper_2605_07612_amd/libfoap4.so.  Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfoap4.so")
BUILD = os.path.join(ROOT, "_build", "foap4")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["topology.cpp", "capi.cpp", "pattern.hip", "ghost.hip", "reduce.hip", "regrid.hip", "mlp.hip", "weno.hip", "advect.hip"]
# the stage kernels, one compile per scheme bit mask (limiter, flux, gravity)
N_SCHEMES = 8
UNITS = [(s, [], s) for s in SOURCES] + [("stage.hip", [f"-DF4_SCHEME={k}"], f"stage_s{k}.hip")
                                         for k in range(N_SCHEMES)]

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=on", f"--offload-arch={ARCH}", "-I" + os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _compile(unit) -> str:
    src, defines, name = unit
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, name + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + FLAGS + defines + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(CSRC, u[0]))]
    jobs = min(len(units), max(1, min(8, os.cpu_count() or 1)))
    # longest compiles first
    units.sort(key=lambda u: u[0] != "stage.hip" and u[0] != "mlp.hip")
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build()
