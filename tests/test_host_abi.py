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
    assert lib.mg_workspace_size(_lib.dims3(64), 16) == 0
    assert lib.mg_workspace_size(_lib.dims3(64), 4) == lib.mg_workspace_size(_lib.dims3(64), 0)
    # a mixed setup from the density leaves out the FP32 face arrays of the finest grid
    assert s32 - lib.mg_workspace_size(_lib.dims3(256), 1 | _lib.MG_FROM_RHO) >= 3 * n * 4
    # flexible CG from the density: a third direction (128^3 and up) and, in FP64 (256^3
    # and up), a second residual; the mixed workspace still drops its FP32 finest faces
    ws = lambda N, fl: lib.mg_workspace_size(_lib.dims3(N), fl)
    K, R, M = _lib.MG_KRYLOV, _lib.MG_FROM_RHO, _lib.MG_MIXED
    assert ws(256, K | R) - ws(256, K) == 2 * n * 8
    assert ws(256, K | M) - ws(256, K | M | R) == 3 * n * 4 - n * 8
    assert ws(128, K | R) - ws(128, K) == 128 ** 3 * 8
    assert ws(64, K | R) == ws(64, K)
    # one concurrent right-hand side's scratch: every grid's f, e and second buffer
    # (the finest grid's f and e are the caller's), without the coefficients
    lane = lib.mg_lane_workspace_size(_lib.dims3(256), 0)
    assert n * 8 < lane < n * 8 * (1 + 3 / 7 + 0.01) + (1 << 20)
    assert lib.mg_lane_workspace_size(_lib.dims3(256), 2) - lane >= 4 * n * 8
    assert lib.mg_lane_workspace_size(_lib.dims3(48), 0) == 0
    assert lib.mg_lane_workspace_size(_lib.dims3(64), 16) == 0


def test_invalid_arguments_rejected_on_the_host():
    """Argument checks run on the host before any device work: bad dims, null arrays and
    unsupported sample counts return MG_EINVAL with a message (no GPU needed)."""
    from paper_1410_2240_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    fake = ctypes.c_void_p(256)   # never dereferenced: every call below fails validation first
    good, bad = _lib.dims3(32), _lib.dims3(48)
    assert lib.mg_cut_cells(fake, bad, 8, fake, fake, fake, fake, fake, None) == _lib.MG_EINVAL
    assert lib.mg_cut_cells(fake, good, 3, fake, fake, fake, fake, fake, None) == _lib.MG_EINVAL
    assert "samples" in _lib.last_error()
    assert lib.mg_cut_cells(None, good, 8, fake, fake, fake, fake, fake, None) == _lib.MG_EINVAL
    assert lib.mg_cut_coeffs(fake, fake, fake, fake, fake, None, good, fake, fake, fake, fake, None) == _lib.MG_EINVAL
    assert lib.mg_merge_rhs(fake, fake, fake, good, None) == _lib.MG_EINVAL   # f_merged aliases f
    assert "alias" in _lib.last_error()
    assert lib.mg_merge_fill(None, fake, good, None) == _lib.MG_EINVAL
    assert lib.mg_coeffs_from_rho(fake, fake, bad, fake, fake, fake, None) == _lib.MG_EINVAL
    ctx = ctypes.c_void_p()
    assert lib.mg_setup_from_rho(ctypes.byref(ctx), fake, 1 << 20, fake, fake, good, 1.0 / 32, 16, None) == _lib.MG_EINVAL
    # the layout flag of a setup from the density is no flag of a setup from face arrays
    assert lib.mg_setup(ctypes.byref(ctx), fake, 1 << 20, fake, fake, fake, fake, good, 1.0 / 32, _lib.MG_FROM_RHO,
                        None) == _lib.MG_EINVAL
    assert "MG_FROM_RHO" in _lib.last_error()
    assert lib.mg_setup_from_rho(ctypes.byref(ctx), fake, 16, fake, fake, good, 1.0 / 32, 0, None) == _lib.MG_EWORKSPACE
    assert not ctx.value
    assert lib.mg_add_lanes(None, fake, 1 << 20, 1) == _lib.MG_EINVAL
