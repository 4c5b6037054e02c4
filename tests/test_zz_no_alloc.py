"""GPU test of xrl_fmm_matvec_noalloc (the matvec whose work arrays live in
the library's fixed device scratch): called through the C ABI, it gives the
product of xrl_fmm_matvec on two calls in a row, the second smaller, in
mixed and FP64 precision, with and without the epilogue."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, plan, x, y, ep=None):
    X = x.reshape(x.shape[0], -1)
    Y = y.reshape(y.shape[0], -1)
    dt = xrl.C64 if X.dtype == torch.complex64 else xrl.C128
    code = fn(plan.h, ctypes.c_void_p(X.data_ptr()), X.stride(0), X.shape[1], dt, ctypes.c_void_p(Y.data_ptr()),
              Y.stride(0), ctypes.byref(ep) if ep is not None else None, xrl._stream(None))
    assert code == 0, xrl.lib().xrl_last_error()


def _epilogue(nc, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(2 * nc)
    b = rng.standard_normal(2 * nc)
    ep = xrl.Epilogue()
    ep.alpha = a.ctypes.data
    ep.beta = b.ctypes.data
    return ep, (a, b)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matvec_matches_matvec_twice(precision):
    L = xrl.lib()
    dt = np.complex128 if precision == "fp64" else np.complex64
    V, T = I.bar()
    N = len(T)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision=precision, max_cols=18)
    plan.assemble()
    # first call: 18 columns (target-stationary in both entry points: the
    # same kernels, so the same bits); second call: 5 columns with an
    # epilogue (the allocating entry point takes the offset-stationary form)
    for nc, seed, use_ep in ((18, 1, False), (5, 2, True)):
        say("case: noalloc %s, bar 4096, %d columns, epilogue %s" % (precision, nc, use_ep))
        x = torch.from_numpy(I.densities(N, nc, dt, seed=seed)).cuda()
        ep, keep = _epilogue(nc, seed) if use_ep else (None, None)
        y_ref = torch.empty_like(x)
        y = torch.full_like(x, float("nan"))
        _call(L.xrl_fmm_matvec, plan, x, y_ref, ep)
        _call(L.xrl_fmm_matvec_noalloc, plan, x, y, ep)
        torch.cuda.synchronize()
        d = (torch.linalg.norm(y - y_ref, dim=0) / torch.linalg.norm(y_ref, dim=0)).max().item()
        say("  max relative L2 difference per column %.3e" % d)
        assert torch.isfinite(y).all()
        if nc == 18:
            assert torch.equal(y, y_ref)
        else:
            assert d < (1e-12 if precision == "fp64" else 1e-6)


def test_noalloc_rejects_requests_beyond_the_scratch():
    say("case: noalloc size limit")
    V, T = I.bar()
    N = len(T)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=1024)
    plan.assemble()
    x = torch.from_numpy(I.densities(N, 1024, np.complex128, seed=3)).cuda()
    y = torch.empty_like(x)
    code = xrl.lib().xrl_fmm_matvec_noalloc(plan.h, ctypes.c_void_p(x.data_ptr()), 1024, 1024, xrl.C128,
                                            ctypes.c_void_p(y.data_ptr()), 1024, None, xrl._stream(None))
    msg = xrl.lib().xrl_last_error().decode()
    say("  status %d: %s" % (code, msg))
    assert code == -1 and "scratch" in msg
