"""Build the gfx950 shared library ``libttcconv.so`` in-tree with hipcc.

Usage: ``python -m paper_1612_08825_amd.build`` (or ``build()`` from Python).
Objects go to ``_build/`` at the repository root; the library is written next
to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libttcconv.so")

SOURCES = ["conv.hip", "fft.hip", "pyramid.hip", "ttc.hip", "ttc_variant.hip", "noalloc.hip", "ttcconv.cpp"]
# the fused pass is built once per frame type (0 = u8, 1 = f16) and level count
FUSED = [("ttc_fused.hip", f"ttc_fused_dt{dt}_l{lv}", [f"-DTC_FUSED_DT={dt}", f"-DTC_FUSED_LV={lv}"])
         for dt in (1, 0) for lv in (4, 3, 2, 1)]
# the row-streaming convolution is built once per input type (0 f32, 1 f16, 2 u8)
ROWS = [("conv_rows.hip", f"conv_rows_dt{dt}", [f"-DTC_ROWS_DT={dt}"]) for dt in (0, 1, 2)]

ARCH = "gfx950"
COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=on",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(job, verbose: bool) -> str:
    src, name, defs = job if isinstance(job, tuple) else (job, os.path.basename(job), [])
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *COMMON, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source for gfx950 and link libttcconv.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        # the slowest objects (the fused pass) first
        objs = list(ex.map(lambda s: _compile(s, verbose), FUSED + ROWS + SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
