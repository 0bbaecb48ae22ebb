"""The C-ABI library loads and exports every function include/uspg.h declares
(no compute calls: runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uspg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("uspg_build_grid", "uspg_build_coeffs", "mart_run", "uspg_to_cartesian"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2208_12964_amd import LIB_PATH, EXPORTED
    if not os.path.exists(LIB_PATH):
        pytest.fail("libuspg.so is not built")
    L = C.CDLL(LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(EXPORTED) == set(declared_functions())


def test_error_path_without_device_work():
    # argument validation happens on the host before any device call
    from paper_2208_12964_amd import lib
    L = lib()
    h = C.c_void_p()
    assert L.uspg_build_grid(None, C.byref(h)) == -1
    assert b"null" in L.uspg_last_error()


def test_bench_refuses_more_than_one_gpu():
    # the one-GPU refusal happens before torch or the library is touched
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout
