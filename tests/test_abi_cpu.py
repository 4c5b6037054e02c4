"""CPU checks of the C-ABI library: it loads (no GPU needed to dlopen) and
exports every function that include/xrl.h declares.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xrl.h")
LIB = os.path.join(ROOT, "paper_2409_12375_amd", "libxrl.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xrl_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2409_12375_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("xrl_tree_build", "xrl_fmm_plan", "xrl_nearfield_assemble", "xrl_fmm_matvec", "xrl_gmres_solve"):
        assert need in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string(lib):
    lib.xrl_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.xrl_version()


def test_argument_errors_need_no_gpu(lib):
    # validation happens before any HIP call
    lib.xrl_tree_build.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.xrl_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    assert lib.xrl_tree_build(None, 64, 21, None, ctypes.byref(out)) == -1
    assert b"null" in lib.xrl_last_error()
    lib.xrl_fmm_matvec.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                           ctypes.c_void_p]
    assert lib.xrl_fmm_matvec(None, None, 1, 1, 1, None, 1, None, None) == -1
