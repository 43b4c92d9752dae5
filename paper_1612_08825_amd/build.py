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


# ----------------------------------------------------------------------------- host sanitizers
SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libttcconv_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def sanitizer_runtimes() -> list:
    """Paths of g++'s ASan and UBSan runtimes (to preload into an uninstrumented
    Python), or [] when they are not installed."""
    out = []
    for name in ("libasan.so", "libubsan.so"):
        r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
        path = r.stdout.strip()
        if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
            return []
        out.append(path)
    return out


def build_sanitized(verbose: bool = False) -> str:
    """The library with its host code -- argument validation, shape rules,
    planning, the tuning table, the dispatcher -- built by g++ with AddressSanitizer
    and UndefinedBehaviorSanitizer (the device objects are the regular build's,
    which is built first if missing).  Host code only: no device code is
    instrumented.  Load it with TC_LIBRARY=<path> and the runtimes of
    `sanitizer_runtimes()` preloaded; returns its path."""
    objs = [os.path.join(BUILD, n + ".o") for _, n, _ in FUSED + ROWS] + \
           [os.path.join(BUILD, s + ".o") for s in SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in objs):
        build(verbose)
    os.makedirs(SAN_DIR, exist_ok=True)
    host_obj = os.path.join(SAN_DIR, "ttcconv.o")
    cmd = ["g++", "-std=c++17", "-fPIC", "-O1", "-g", *SAN_FLAGS, "-D__HIP_PLATFORM_AMD__",
           "-I", "/opt/rocm/include", "-I", INCLUDE, "-c", os.path.join(CSRC, "ttcconv.cpp"), "-o", host_obj]
    link = ["g++", "-shared", *SAN_FLAGS, host_obj, *objs, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
            "-lamdhip64", "-o", SAN_LIB]
    for c in (cmd, link):
        if verbose:
            print(" ".join(c), flush=True)
        r = subprocess.run(c, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitizer build failed:\n{r.stdout}\n{r.stderr}")
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
