"""CPU checks of the boundary: host plan (g++ build) and the exported C ABI."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_2240_amd", "csrc")
HEADER = os.path.join(ROOT, "include", "mg.h")


def header_functions():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", text)))


def test_host_plan_program(tmp_path):
    exe = tmp_path / "test_plan"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", f"-I{CSRC}", os.path.join(ROOT, "tests", "host", "test_plan.cpp"),
                    os.path.join(CSRC, "mg_plan.cpp"), os.path.join(CSRC, "sym_pinv.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr


def test_library_exports_every_declared_symbol():
    from paper_1410_2240_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the Python binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == names


def test_workspace_size_is_host_arithmetic():
    from paper_1410_2240_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    s64 = lib.mg_workspace_size(_lib.dims3(256), 0)
    s32 = lib.mg_workspace_size(_lib.dims3(256), 1)
    n = 256 ** 3
    assert n * (3 * 8 + 1 + 8 + 8) < s64 < n * 49
    assert s32 - s64 > n * 6 * 4
    assert lib.mg_workspace_size(_lib.dims3(48), 0) == 0
    assert lib.mg_workspace_size((ctypes.c_int * 3)(64, 64, 32), 0) == 0
    assert lib.mg_workspace_size(_lib.dims3(64), 8) == 0
    assert lib.mg_workspace_size(_lib.dims3(64), 4) == lib.mg_workspace_size(_lib.dims3(64), 0)
