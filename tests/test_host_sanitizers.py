"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): argument validation, shape rules, planning, the tuning table and
the convolution dispatcher's host side, exercised by the CPU ABI tests, the
serving scheduler's tests and the host rank-one test, run in a child Python
that loads the sanitizer build (`build.build_sanitized`) with the sanitizer
runtimes preloaded.  Any report fails the run (errors are not recoverable in
that build)."""
import os
import re
import subprocess
import sys

import pytest

from paper_1612_08825_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITES = ["tests/test_abi.py", "tests/test_serving_host.py", "tests/test_separable_host.py"]


def test_host_code_under_asan_ubsan():
    runtimes = B.sanitizer_runtimes()
    if not runtimes:
        pytest.skip("g++'s ASan/UBSan runtimes are not installed")
    if not os.path.exists(B.LIB):
        pytest.skip("the library is not built (python -m paper_1612_08825_amd.build)")
    lib = B.build_sanitized()
    env = dict(os.environ)
    env.update({
        "TC_LIBRARY": lib,
        "LD_PRELOAD": ":".join(runtimes),
        # Python's own allocations are never freed at exit: leak reports would be noise
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "print_stacktrace=1",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *SUITES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert re.search(r"\d+ passed", out), out[-2000:]
    # and the library such a child loads is the instrumented one
    probe = ("from paper_1612_08825_amd import _lib as L; L.load(); "
             "print(any(l.rstrip().endswith('libttcconv_san.so') for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "True", r.stdout + r.stderr
