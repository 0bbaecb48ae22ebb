"""The host-side C and C++ code (the oracle, the host builds of the
library's walk, coded rows and segment records) built with AddressSanitizer
and UndefinedBehaviorSanitizer, and the CPU tests that exercise it run
against those builds in a child process with the ASan runtime preloaded:
any out-of-bounds access, use after free or undefined behaviour ends the
child with a report."""
import os
import subprocess
import sys

import pytest

from oracle.oracle import build_oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")

TESTS = ["test_lib_walk_cpu.py", "test_lib_segments_cpu.py", "test_oracle_trace.py", "test_oracle_mart.py",
         "test_oracle_grid.py", "test_oracle_remap.py", "test_oracle_rebin.py"]
# the slowest cases (tens of seconds unsanitized) are left to the plain run
SKIP = "not near_tangent and not dense_sampling and not full_size"


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")
def test_host_code_under_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    lib = build_oracle(out=os.path.join(BUILD, "liboracle_asan.so"), sanitize=True)
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": _runtime("libasan.so"),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "USPG_ORACLE_LIB": lib,
        "USPG_HOST_SANITIZE": "1",
        "OMP_NUM_THREADS": "4",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-k", SKIP,
           *[os.path.join(HERE, t) for t in TESTS]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")
def test_harness_reports_a_planted_overflow():
    # the same build flags and child set-up report a heap overflow planted in
    # a throw-away C file (so a clean run above means the checks were live)
    from oracle.oracle import SANITIZE
    os.makedirs(BUILD, exist_ok=True)
    src = os.path.join(BUILD, "planted.c")
    so = os.path.join(BUILD, "planted_asan.so")
    with open(src, "w") as f:
        f.write("#include <stdlib.h>\nunsigned planted(int n) { unsigned *a = calloc(n, sizeof(unsigned));"
                " unsigned s = 0; for (int i = 0; i <= n; ++i) s += a[i]; free(a); return s; }\n")
    subprocess.run(["gcc", *SANITIZE, "-fPIC", "-shared", src, "-o", so], check=True)
    env = dict(os.environ, LD_PRELOAD=_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=86")
    code = f"import ctypes; ctypes.CDLL({so!r}).planted(8)"
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 86 and "heap-buffer-overflow" in r.stderr
