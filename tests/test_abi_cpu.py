"""CPU checks of the C-ABI library: it loads (no GPU needed to dlopen) and
exports every function that include/xrl.h declares.  No compute calls."""
import ctypes
import os
import re

import numpy as np
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
    # the allocator hand-off: both hooks or none
    alloc_t = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    free_t = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

    class Allocator(ctypes.Structure):
        _fields_ = [("alloc", alloc_t), ("free", free_t), ("ctx", ctypes.c_void_p)]

    lib.xrl_set_allocator.argtypes = [ctypes.POINTER(Allocator)]
    half = Allocator(alloc_t(lambda n, s, c: None), free_t(), None)
    assert lib.xrl_set_allocator(ctypes.byref(half)) == -1
    assert b"hooks" in lib.xrl_last_error()
    assert lib.xrl_set_allocator(None) == 0


def _reflection_signs(p):
    """Sign of each real coefficient (index n^2 for m = 0, n^2 + 2m - 1 real
    part, n^2 + 2m imaginary part) under x -> -x, y -> -y, z -> -z, from
    R_n^m ~ P_n^m(cos theta) e^{i m phi}: phi -> pi - phi gives (-1)^m and a
    conjugate, phi -> -phi a conjugate, cos theta -> -cos theta (-1)^(n+m)."""
    K = (p + 1) ** 2
    s = np.ones((3, K))
    for n in range(p + 1):
        for m in range(n + 1):
            for part in ((0,) if m == 0 else (0, 1)):
                k = n * n if m == 0 else n * n + 2 * m - 1 + part
                conj = -1.0 if part == 1 else 1.0
                s[0, k] = (-1.0) ** m * conj
                s[1, k] = conj
                s[2, k] = (-1.0) ** (n + m)
    return s


def test_m2l_operator_reflections(lib):
    """The target-stationary M2L streams only the operators of non-negative
    offsets and applies T_o = S T_|o| S for the reflected ones."""
    p = 8
    K = (p + 1) ** 2
    lib.xrl_m2l_operator.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_void_p]

    def op(o):
        out = np.zeros((K, K))
        assert lib.xrl_m2l_operator(p, o[0], o[1], o[2], out.ctypes.data) == 0
        return out

    S = _reflection_signs(p)
    for base in [(2, 0, 0), (3, 1, 2), (2, 2, 3), (0, 3, 1), (1, 0, 2)]:
        T0 = op(base)
        for r in range(1, 8):
            o = tuple(-c if r >> a & 1 else c for a, c in enumerate(base))
            s = np.prod([S[a] for a in range(3) if r >> a & 1], axis=0)
            assert np.allclose(op(o), s[:, None] * T0 * s[None, :], rtol=1e-12, atol=1e-12 * np.abs(T0).max())
    # the reflection really changes the operator (the test is not vacuous)
    assert not np.allclose(op((3, 1, 2)), op((-3, 1, 2)))
    assert lib.xrl_m2l_operator(p, 1, 1, 0, np.zeros((K, K)).ctypes.data) != 0
