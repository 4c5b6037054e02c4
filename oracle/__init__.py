"""ctypes wrapper of the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may load this module.  The GPU library never does.

The oracle evaluates the Galerkin 1/R panel operator of the XRL method
(arXiv 2409.12375, Sec. II-A eq. (6) second term, without j*omega*mu0/4pi,
which the paper extracts from the integral, Sec. II-D) by direct O(N^2)
summation in FP64.  See the header of ``oracle.c`` for the per-class rules.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)


def build(force=True):
    """Compile oracle.c with gcc (-O2, OpenMP).  Plain C, no GPU."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_gauss_legendre01.argtypes = [ctypes.c_int, _d, _d]
        L.orc_panel_geometry.argtypes = [_d, _i32, ctypes.c_int64, _d, _d, _d, _d]
        L.orc_self.argtypes = [_d]
        L.orc_self.restype = ctypes.c_double
        L.orc_point_potential.argtypes = [_d, _d]
        L.orc_point_potential.restype = ctypes.c_double
        L.orc_semianalytic_sigmoid.argtypes = [_d, _d, ctypes.c_int, ctypes.c_int]
        L.orc_semianalytic_sigmoid.restype = ctypes.c_double
        L.orc_semianalytic_subdiv.argtypes = [_d, _d, ctypes.c_int, ctypes.c_int]
        L.orc_semianalytic_subdiv.restype = ctypes.c_double
        L.orc_init.argtypes = []
        L.orc_init()
        L.orc_conical_monomial.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_conical_monomial.restype = ctypes.c_double
        L.orc_far_pair.argtypes = [_d, _d, ctypes.c_int]
        L.orc_far_pair.restype = ctypes.c_double
        L.orc_entry_idx.argtypes = [_d, _i32, ctypes.c_int64, ctypes.c_int64]
        L.orc_entry_idx.restype = ctypes.c_double
        L.orc_matvec_rows.argtypes = [_d, _i32, ctypes.c_int64, _d, ctypes.c_int64, _i64,
                                      ctypes.c_int64, _d, ctypes.c_int]
        L.orc_matvec_rows.restype = ctypes.c_int
        L.orc_dense.argtypes = [_d, _i32, _i64, ctypes.c_int64, _i64, ctypes.c_int64, _d, ctypes.c_int]
        L.orc_pairs.argtypes = [_d, _i32, _i64, _i64, ctypes.c_int64, _d, ctypes.c_int]
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(_d)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def gauss_legendre01(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre01(n, _pd(x), _pd(w))
    return x, w


def panel_geometry(V, T):
    V = _f64(V)
    T = np.ascontiguousarray(T, dtype=np.int32)
    N = T.shape[0]
    area = np.zeros(N)
    cen = np.zeros((N, 3))
    nrm = np.zeros((N, 3))
    diam = np.zeros(N)
    lib().orc_panel_geometry(_pd(V), T.ctypes.data_as(_i32), N, _pd(area), _pd(cen), _pd(nrm), _pd(diam))
    return area, cen, nrm, diam


def self_term(tri):
    """Closed-form int_T int_T 1/|r-r'| for a triangle given as [3][3]."""
    return lib().orc_self(_pd(_f64(tri, (9,))))


def point_potential(tri, r):
    """int_T 1/|r - r'| dS' (exact, Wilton et al. 1984)."""
    return lib().orc_point_potential(_pd(_f64(tri, (9,))), _pd(_f64(r, (3,))))


def semianalytic_sigmoid(tgt, src, collapse=0, n=40):
    return lib().orc_semianalytic_sigmoid(_pd(_f64(tgt, (9,))), _pd(_f64(src, (9,))), collapse, n)


def semianalytic_subdiv(tgt, src, n=10, levels=0):
    """int_tgt phi_src with an n x n conical rule on 4^levels sub-triangles."""
    return lib().orc_semianalytic_subdiv(_pd(_f64(tgt, (9,))), _pd(_f64(src, (9,))), n, levels)


def conical_monomial(n, a, b):
    """n x n conical rule on the reference triangle applied to x^a y^b."""
    return lib().orc_conical_monomial(n, a, b)


def far_pair(tk, tl, n):
    return lib().orc_far_pair(_pd(_f64(tk, (9,))), _pd(_f64(tl, (9,))), n)


def entry(V, T, k, l):
    V = _f64(V)
    T = np.ascontiguousarray(T, dtype=np.int32)
    return lib().orc_entry_idx(_pd(V), T.ctypes.data_as(_i32), k, l)


def dense(V, T, rows=None, cols=None, nthreads=0):
    """Dense block P[rows][cols] (small meshes only)."""
    V = _f64(V)
    T = np.ascontiguousarray(T, dtype=np.int32)
    N = T.shape[0]
    rows = np.arange(N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.arange(N, dtype=np.int64) if cols is None else np.ascontiguousarray(cols, dtype=np.int64)
    P = np.zeros((len(rows), len(cols)))
    lib().orc_dense(_pd(V), T.ctypes.data_as(_i32), rows.ctypes.data_as(_i64), len(rows),
                    cols.ctypes.data_as(_i64), len(cols), _pd(P), nthreads)
    return P


def pairs(V, T, ks, ls, nthreads=0):
    """P_kl for explicit index pairs (k, l)."""
    V = _f64(V)
    T = np.ascontiguousarray(T, dtype=np.int32)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    ls = np.ascontiguousarray(ls, dtype=np.int64)
    out = np.zeros(len(ks))
    lib().orc_pairs(_pd(V), T.ctypes.data_as(_i32), ks.ctypes.data_as(_i64), ls.ctypes.data_as(_i64), len(ks),
                    _pd(out), nthreads)
    return out


def matvec(V, T, x, rows=None, nthreads=0):
    """y[rows] = P[rows, :] @ x for real x of shape [N] or [N][C] (FP64).

    Complex x is split into real and imaginary columns (P is real).
    Returns (y, threads_used)."""
    V = _f64(V)
    T = np.ascontiguousarray(T, dtype=np.int32)
    N = T.shape[0]
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    squeeze = x.ndim == 1
    X = x.reshape(N, -1)
    if cplx:
        Xr = np.empty((N, 2 * X.shape[1]))
        Xr[:, 0::2] = X.real
        Xr[:, 1::2] = X.imag
    else:
        Xr = X.astype(np.float64)
    Xr = np.ascontiguousarray(Xr)
    C = Xr.shape[1]
    rows = np.arange(N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    Y = np.zeros((len(rows), C))
    used = lib().orc_matvec_rows(_pd(V), T.ctypes.data_as(_i32), N, _pd(Xr), C,
                                 rows.ctypes.data_as(_i64), len(rows), _pd(Y), nthreads)
    if cplx:
        Y = Y[:, 0::2] + 1j * Y[:, 1::2]
    if squeeze:
        Y = Y[:, 0]
    return Y, used
