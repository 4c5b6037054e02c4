"""Thin ctypes binding of libxrl.so (include/xrl.h).

Argument marshalling only: every step of the operator runs in the HIP
library.  PyTorch provides device memory and the stream.  There is no CPU
fallback: if the library is missing, `lib()` raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxrl.so")
_lib = None

C64, C128 = 1, 2
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
ENGINE = {"auto": 0, "mfma": 1, "valu": 2, "mfma_os": 3, "mfma_ts": 4}
N_PHASES = 8
PHASES = ["gather", "p2p", "p2m", "m2m", "m2l", "l2l", "l2p", "scatter"]

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class XrlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("xrl error %d: %s" % (code, msg))
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_vertices", _i64), ("n_panels", _i64), ("vertices", _vp), ("tris", _vp), ("on_device", _i32),
                ("verts_per_panel", _i32)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_panels", _i64), ("n_boxes", _i64), ("n_leaves", _i64), ("depth", _i32),
                ("n_overfull_leaves", _i32), ("root_center", ctypes.c_double * 3), ("root_size", ctypes.c_double),
                ("n_elements", _i64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("n_tried", _i32), ("engine", _i32 * 8), ("ts_kernel", _i32 * 8), ("ms", ctypes.c_double * 8),
                ("best_engine", _i32), ("best_ts_kernel", _i32), ("best_ms", ctypes.c_double),
                ("n_p2p_tried", _i32), ("p2p_ms", ctypes.c_double * 3), ("best_p2p_form", _i32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("order", _i32), ("precision", _i32), ("m2l_engine", _i32), ("max_cols", _i32),
                ("theta", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_panels", _i64), ("n_boxes", _i64), ("n_leaves", _i64), ("n_m2l_pairs", _i64),
                ("n_near_rows", _i64), ("n_near_entries", _i64), ("n_near_pairs", _i64), ("order", _i32),
                ("precision", _i32), ("max_sep_ratio", ctypes.c_double), ("n_demoted_pairs", _i64),
                ("theta", ctypes.c_double), ("n_elements", _i64)]


class Mlp(ctypes.Structure):
    _fields_ = [("hidden", _i32), ("w1", _vp), ("b1", _vp), ("w2", _vp), ("b2", _vp), ("w3", _vp), ("b3", _vp),
                ("feat_lo", _vp), ("feat_hi", _vp), ("log10_err_bound", ctypes.c_float)]


class NfOpts(ctypes.Structure):
    _fields_ = [("r_near", ctypes.c_double), ("r_mid", ctypes.c_double), ("surrogate", ctypes.POINTER(Mlp)),
                ("audit_every", _i32)]


class NfStats(ctypes.Structure):
    _fields_ = [("n_entries", _i64), ("n_self", _i64), ("n_touching", _i64), ("n_near_singular", _i64),
                ("n_regular", _i64), ("n_mlp_accepted", _i64), ("n_mlp_fallback", _i64),
                ("audit_max_rel_err", ctypes.c_double), ("audit_rms_rel_err", ctypes.c_double),
                ("ms", ctypes.c_double), ("n_regular_fine", _i64)]


class Epilogue(ctypes.Structure):
    _fields_ = [("alpha", _vp), ("beta", _vp)]


class MlpTrainOpts(ctypes.Structure):
    _fields_ = [("hidden", _i32), ("batch", _i32), ("epochs", _i32), ("lr", ctypes.c_float),
                ("lr_decay", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("calib_weight", ctypes.c_float), ("log_mu", ctypes.c_float),
                ("log_sigma", ctypes.c_float), ("target_scale", ctypes.c_float), ("seed", ctypes.c_uint64)]


class LoopsInfo(ctypes.Structure):
    _fields_ = [("n_panels", _i64), ("n_edges", _i64), ("n_loops", _i64), ("n_vertex_loops", _i64),
                ("n_global_loops", _i64), ("n_components", _i64), ("nnz_loop_matrix", _i64)]


_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
_FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", _vp)]


class GmresStats(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("restarts", _i32), ("converged", _i32),
                ("max_rel_residual", ctypes.c_double)]


def lib():
    """Load libxrl.so (built in-tree by paper_2409_12375_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libxrl.so is not built (run paper_2409_12375_amd/build.py or "
                               "__graft_entry__.build()); there is no CPU fallback")
        # Device pointers and streams pass between torch and the library, so
        # both must use one HIP runtime.  torch ships its own libamdhip64.so.7
        # (same soname as the system one): loading torch first makes the
        # library bind to that copy instead of a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.xrl_last_error.restype = ctypes.c_char_p
        L.xrl_version.restype = ctypes.c_char_p
        L.xrl_tree_build.argtypes = [ctypes.POINTER(MeshDesc), _i32, _i32, _vp, ctypes.POINTER(_vp)]
        L.xrl_tree_destroy.argtypes = [_vp]
        L.xrl_tree_destroy.restype = None
        L.xrl_tree_get_info.argtypes = [_vp, ctypes.POINTER(TreeInfo)]
        L.xrl_fmm_plan.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(PlanOpts), _vp, ctypes.POINTER(_vp)]
        L.xrl_plan_destroy.argtypes = [_vp]
        L.xrl_plan_destroy.restype = None
        L.xrl_plan_get_info.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
        L.xrl_nearfield_assemble.argtypes = [_vp, ctypes.POINTER(NfOpts), _vp, ctypes.POINTER(NfStats)]
        L.xrl_fmm_matvec.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _i64, ctypes.POINTER(Epilogue), _vp]
        L.xrl_fmm_matvec_noalloc.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _i64, ctypes.POINTER(Epilogue), _vp]
        L.xrl_set_allocator.argtypes = [ctypes.POINTER(Allocator)]
        L.xrl_plan_set_profiling.argtypes = [_vp, _i32]
        L.xrl_plan_get_phase_ms.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.xrl_plan_set_tuning.argtypes = [_vp, _i32, _i32]
        L.xrl_plan_set_graph.argtypes = [_vp, _i32]
        L.xrl_plan_autotune.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _i64, _i32, _vp, ctypes.POINTER(TuneResult)]
        L.xrl_plan_export.argtypes = [_vp, _i32, _vp, ctypes.POINTER(_i64)]
        L.xrl_surrogate_features.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp]
        L.xrl_mlp_train.argtypes = [_vp, _vp, _i64, ctypes.POINTER(MlpTrainOpts), _vp, _vp, _vp]
        L.xrl_mlp_loss_grad.argtypes = [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp]
        L.xrl_mlp_forward.argtypes = [_vp, _i32, _vp, _i64, _i32, _vp, _vp]
        L.xrl_selftest_mfma.argtypes = [_i32, _vp, _vp, _vp]
        L.xrl_selftest_mfma_bf16.argtypes = [_vp, _vp, _vp]
        L.xrl_gmres_solve.argtypes = [_vp, ctypes.POINTER(Epilogue), _vp, _vp, _i32, _i32, _i32, ctypes.c_double,
                                      _i32, _vp, ctypes.POINTER(GmresStats)]
        L.xrl_loops_build.argtypes = [ctypes.POINTER(MeshDesc), _vp, ctypes.POINTER(_vp)]
        L.xrl_loops_destroy.argtypes = [_vp]
        L.xrl_loops_destroy.restype = None
        L.xrl_loops_get_info.argtypes = [_vp, ctypes.POINTER(LoopsInfo)]
        L.xrl_loops_export.argtypes = [_vp, _i32, _vp, ctypes.POINTER(_i64)]
        L.xrl_surface_impedance.argtypes = [ctypes.c_double, ctypes.c_double, _vp, _i32, _vp]
        L.xrl_edge_matvec.argtypes = [_vp, _vp, ctypes.POINTER(Epilogue), _vp, _vp, _i32, _vp]
        L.xrl_loop_gmres_solve.argtypes = [_vp, _vp, ctypes.POINTER(Epilogue), _vp, _vp, _i32, _i32, _i32,
                                           ctypes.c_double, _i32, _vp, ctypes.POINTER(GmresStats)]
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise XrlError(code, lib().xrl_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


_allocator = None  # the installed hooks (kept alive while installed)


def use_torch_allocator(on=True):
    """Route every device allocation of the library through torch's caching
    allocator (xrl_set_allocator), on the stream of the library call that
    allocates; on=False restores hipMalloc/hipFree for later allocations.
    Buffers made while torch's hooks were installed are still released
    through them, so the hooks stay referenced here for the process."""
    global _allocator
    if not on:
        _check(lib().xrl_set_allocator(None))
        return
    if _allocator is None:
        import torch

        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            except Exception:  # reported by the library as XRL_E_OOM
                return None

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:  # interpreter shutdown: the caching allocator is gone
                pass

        _allocator = Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)
    _check(lib().xrl_set_allocator(ctypes.byref(_allocator)))


class Tree:
    """Octree over one mesh (xrl_tree_build)."""

    def __init__(self, V, T, max_leaf=64, max_depth=21, stream=None):
        """T: [N][3] triangles, or [N][4] panels of a hybrid mesh (-1 as the
        fourth index of a triangle)."""
        self._V = np.ascontiguousarray(V, dtype=np.float64)
        self._T = np.ascontiguousarray(T, dtype=np.int32)
        d = MeshDesc(self._V.shape[0], self._T.shape[0], self._V.ctypes.data, self._T.ctypes.data, 0,
                     self._T.shape[1])
        h = _vp()
        _check(lib().xrl_tree_build(ctypes.byref(d), max_leaf, max_depth, _stream(stream), ctypes.byref(h)))
        self.h = h
        self.n_panels = self._T.shape[0]

    def info(self):
        i = TreeInfo()
        _check(lib().xrl_tree_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) if f not in ("root_center",) else list(i.root_center) for f, _ in TreeInfo._fields_}

    def close(self):
        if self.h:
            lib().xrl_tree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """FMM plan over one or more trees (xrl_fmm_plan)."""

    def __init__(self, trees, order=8, precision="mixed", engine="auto", max_cols=3, theta=0.0, stream=None):
        if isinstance(trees, Tree):
            trees = [trees]
        self.trees = list(trees)  # keep the trees alive
        arr = (_vp * len(trees))(*[t.h for t in trees])
        o = PlanOpts(order, PREC[precision], ENGINE[engine], max_cols, theta)
        h = _vp()
        _check(lib().xrl_fmm_plan(arr, len(trees), ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.precision = precision
        self.n_panels = sum(t.n_panels for t in trees)

    def info(self):
        i = PlanInfo()
        _check(lib().xrl_plan_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}

    def assemble(self, r_near=2.0, r_mid=4.0, surrogate=None, audit_every=0, stream=None):
        o = NfOpts(r_near, r_mid, None, audit_every)
        keep = None
        if surrogate is not None:
            keep = surrogate.as_struct()
            o.surrogate = ctypes.pointer(keep[0])
        st = NfStats()
        _check(lib().xrl_nearfield_assemble(self.h, ctypes.byref(o), _stream(stream), ctypes.byref(st)))
        del keep
        return {f: getattr(st, f) for f, _ in NfStats._fields_}

    def matvec(self, x, y=None, alpha=None, beta=None, stream=None):
        """y = alpha_c * (P x)_c + beta_c * area * x_c for a complex CUDA tensor x
        of shape [N] or [N][C] (user panel order)."""
        import torch
        if x.dtype not in (torch.complex64, torch.complex128) or not x.is_cuda:
            raise ValueError("x must be a complex64/complex128 CUDA tensor")
        squeeze = x.dim() == 1
        X = x.reshape(x.shape[0], -1)
        if X.stride(1) != 1:
            X = X.contiguous()
        ncols = X.shape[1]
        if y is None:
            y = torch.empty_like(X)
        Y = y.reshape(y.shape[0], -1)
        if Y.stride(1) != 1 or Y.dtype != X.dtype or Y.shape != X.shape:
            raise ValueError("y must match x in shape and dtype with unit column stride")
        ep = None
        keep = []
        if alpha is not None or beta is not None:
            ep = Epilogue()
            for name in ("alpha", "beta"):
                v = alpha if name == "alpha" else beta
                if v is not None:
                    a = np.empty(2 * ncols)
                    vv = np.broadcast_to(np.asarray(v, dtype=np.complex128), (ncols,))
                    a[0::2] = vv.real
                    a[1::2] = vv.imag
                    keep.append(a)
                    setattr(ep, name, a.ctypes.data)
        dt = C64 if X.dtype == torch.complex64 else C128
        _check(lib().xrl_fmm_matvec(self.h, _vp(X.data_ptr()), X.stride(0), ncols, dt, _vp(Y.data_ptr()), Y.stride(0),
                                    ctypes.byref(ep) if ep is not None else None, _stream(stream)))
        return Y[:, 0] if squeeze else Y

    def set_profiling(self, on=True):
        _check(lib().xrl_plan_set_profiling(self.h, 1 if on else 0))

    TUNE = {"ts_kernel": 0, "ts_min_cols": 1, "p2p_form": 2, "ts_narrow_cols": 3, "ts_order": 4, "l2l_form": 5, "m2m_form": 6, "leaf_form": 7,
            "valu_form": 8, "leaf_l2l": 9}

    def set_tuning(self, key, value):
        """Kernel-shape knob (see xrl_plan_set_tuning); results agree to rounding."""
        _check(lib().xrl_plan_set_tuning(self.h, self.TUNE[key], int(value)))

    def set_graph(self, on=True):
        """Replay each distinct matvec argument set from a captured HIP graph."""
        _check(lib().xrl_plan_set_graph(self.h, 1 if on else 0))

    def autotune(self, x, y=None, reps=3, stream=None):
        """Time the translation forms on (x, y) and keep the fastest; returns
        {"tried": [(engine, ts_kernel, ms), ...], "best": (engine, ts_kernel, ms)}."""
        import torch
        X = x if x.dim() == 2 else x.unsqueeze(1)
        Y = torch.empty_like(X) if y is None else y
        dt = C64 if X.dtype == torch.complex64 else C128
        r = TuneResult()
        _check(lib().xrl_plan_autotune(self.h, _vp(X.data_ptr()), X.stride(0), X.shape[1], dt, _vp(Y.data_ptr()),
                                       Y.stride(0), reps, _stream(stream), ctypes.byref(r)))
        names = {v: k for k, v in ENGINE.items()}
        tried = [(names[r.engine[i]], r.ts_kernel[i], r.ms[i]) for i in range(r.n_tried)]
        return {"tried": tried, "best": (names[r.best_engine], r.best_ts_kernel, r.best_ms),
                "p2p_tried": [(f, r.p2p_ms[f]) for f in range(r.n_p2p_tried)], "best_p2p_form": r.best_p2p_form}

    def phase_ms(self):
        a = (ctypes.c_double * N_PHASES)()
        _check(lib().xrl_plan_get_phase_ms(self.h, a))
        return dict(zip(PHASES, list(a)))

    def export(self, item):
        """Plan internals (xrl_plan_export); items 8 and 10 are float64."""
        n = _i64(0)
        _check(lib().xrl_plan_export(self.h, item, None, ctypes.byref(n)))
        out = np.zeros(n.value // 8, dtype=np.float64) if item in (8, 10) else np.zeros(n.value // 4, dtype=np.int32)
        _check(lib().xrl_plan_export(self.h, item, _vp(out.ctypes.data), ctypes.byref(n)))
        return out

    def gmres(self, b, x0=None, alpha=1.0, beta=0.0, restart=50, rtol=1e-6, max_iter=500, stream=None):
        """Solve (beta_c A + alpha_c P) x_c = b_c; b is a complex64 or
        complex128 CUDA tensor [N] or [N][R].  Returns (x, stats), x of b's dtype."""
        import torch
        squeeze = b.dim() == 1
        if b.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("b must be complex64 or complex128")
        Bm = b.reshape(b.shape[0], -1).contiguous()
        R = Bm.shape[1]
        X = torch.zeros_like(Bm) if x0 is None else x0.reshape(Bm.shape).to(Bm.dtype).contiguous().clone()
        dt = C64 if Bm.dtype == torch.complex64 else C128
        ep = Epilogue()
        keep = []
        for name, v in (("alpha", alpha), ("beta", beta)):
            a = np.empty(2 * R)
            vv = np.broadcast_to(np.asarray(v, dtype=np.complex128), (R,))
            a[0::2] = vv.real
            a[1::2] = vv.imag
            keep.append(a)
            setattr(ep, name, a.ctypes.data)
        st = GmresStats()
        code = lib().xrl_gmres_solve(self.h, ctypes.byref(ep), _vp(Bm.data_ptr()), _vp(X.data_ptr()), R, dt,
                                     restart, rtol, max_iter, _stream(stream), ctypes.byref(st))
        stats = {f: getattr(st, f) for f, _ in GmresStats._fields_}
        if code not in (0, -5):
            _check(code)
        stats["status"] = code
        return (X[:, 0] if squeeze else X), stats

    def close(self):
        if self.h:
            lib().xrl_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Surrogate of near-singular pairs
# ---------------------------------------------------------------------------
def mlp_size(H):
    return H * H + 22 * H + 2


def surrogate_features(tri_k, tri_l, stream=None):
    """Features [n][18] and cheap 3x3 values [n] of explicit triangle pairs
    (CUDA float64 tensors [n][9]), computed by the library."""
    import torch
    n = tri_k.shape[0]
    feat = torch.empty((n, 18), dtype=torch.float32, device=tri_k.device)
    cheap = torch.empty(n, dtype=torch.float64, device=tri_k.device)
    _check(lib().xrl_surrogate_features(_vp(tri_k.data_ptr()), _vp(tri_l.data_ptr()), n, _vp(feat.data_ptr()),
                                        _vp(cheap.data_ptr()), _stream(stream)))
    return feat, cheap


def mlp_loss_grad(w, H, X, t, lam, mu, sig, scale, stream=None):
    import torch
    g = torch.empty_like(w)
    la = np.array([lam, mu, sig, scale], dtype=np.float32)
    loss = np.zeros(2, dtype=np.float32)
    _check(lib().xrl_mlp_loss_grad(_vp(w.data_ptr()), H, _vp(X.data_ptr()), _vp(t.data_ptr()), X.shape[0],
                                   _vp(la.ctypes.data), _vp(loss.ctypes.data), _vp(g.data_ptr()), _stream(stream)))
    return loss, g


def mlp_forward(w, H, X, bf16=False, stream=None):
    import torch
    out = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    _check(lib().xrl_mlp_forward(_vp(w.data_ptr()), H, _vp(X.data_ptr()), X.shape[0], 1 if bf16 else 0,
                                 _vp(out.data_ptr()), _stream(stream)))
    return out


def mlp_train(w, X, t, hidden=128, batch=4096, epochs=10, lr=2e-3, lr_decay=0.85, calib_weight=0.2, log_mu=-5.0,
              log_sigma=2.0, target_scale=1.0, seed=12375, stream=None):
    """Train in place on the device; returns the per-epoch loss history."""
    o = MlpTrainOpts(hidden, batch, epochs, lr, lr_decay, 0.9, 0.999, 1e-8, calib_weight, log_mu, log_sigma,
                     target_scale, seed)
    hist = np.zeros(epochs, dtype=np.float32)
    _check(lib().xrl_mlp_train(_vp(X.data_ptr()), _vp(t.data_ptr()), X.shape[0], ctypes.byref(o), _vp(w.data_ptr()),
                               _vp(hist.ctypes.data), _stream(stream)))
    return hist


class Surrogate:
    """Trained weights (packed FP32, output scaling folded in), feature range
    and the log10 error bound used for the fall-back decision."""

    def __init__(self, w, hidden, feat_lo, feat_hi, bound):
        self.w = np.ascontiguousarray(w, dtype=np.float32)
        self.hidden = int(hidden)
        self.feat_lo = np.ascontiguousarray(feat_lo, dtype=np.float32)
        self.feat_hi = np.ascontiguousarray(feat_hi, dtype=np.float32)
        self.bound = float(bound)

    @classmethod
    def load(cls, path):
        d = np.load(path, allow_pickle=False)
        return cls(d["w"], int(d["hidden"]), d["feat_lo"], d["feat_hi"], float(d["bound"]))

    def save(self, path, **extra):
        np.savez(path, w=self.w, hidden=self.hidden, feat_lo=self.feat_lo, feat_hi=self.feat_hi, bound=self.bound,
                 **extra)

    def as_struct(self):
        H = self.hidden
        o = 0
        ptrs = []
        for size in (18 * H, H, H * H, H, 2 * H, 2):
            ptrs.append(self.w.ctypes.data + 4 * o)
            o += size
        s = Mlp(H, *ptrs, self.feat_lo.ctypes.data, self.feat_hi.ctypes.data, self.bound)
        return (s, self)  # keep the arrays alive with the struct


# ---------------------------------------------------------------------------
# Loop analysis (PEEC graph, Algorithm 1 maps, loop basis, eq. (8) solve)
# ---------------------------------------------------------------------------
PRECOND = {"none": 0, "diag_p": 1, "diag_l": 2}


def _epilogue_arrays(alpha, beta, R):
    ep = Epilogue()
    keep = []
    for name, v in (("alpha", alpha), ("beta", beta)):
        if v is None:
            continue
        a = np.empty(2 * R)
        vv = np.broadcast_to(np.asarray(v, dtype=np.complex128), (R,))
        a[0::2] = vv.real
        a[1::2] = vv.imag
        keep.append(a)
        setattr(ep, name, a.ctypes.data)
    return ep, keep


def surface_impedance(freq, sigma, thickness):
    """Z_s of eq. (3) at the given frequencies (host)."""
    f = np.ascontiguousarray(np.atleast_1d(freq), dtype=np.float64)
    out = np.zeros(2 * len(f))
    _check(lib().xrl_surface_impedance(sigma, thickness, _vp(f.ctypes.data), len(f), _vp(out.ctypes.data)))
    return out[0::2] + 1j * out[1::2]


class Loops:
    """Loop analysis of a closed mesh (xrl_loops_build)."""

    def __init__(self, V, T, stream=None):
        self._V = np.ascontiguousarray(V, dtype=np.float64)
        self._T = np.ascontiguousarray(T, dtype=np.int32)
        d = MeshDesc(self._V.shape[0], self._T.shape[0], self._V.ctypes.data, self._T.ctypes.data, 0,
                     self._T.shape[1])
        h = _vp()
        _check(lib().xrl_loops_build(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        self.h = h

    def info(self):
        i = LoopsInfo()
        _check(lib().xrl_loops_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in LoopsInfo._fields_}

    def export(self, item):
        n = _i64(0)
        _check(lib().xrl_loops_export(self.h, item, None, ctypes.byref(n)))
        out = np.zeros(n.value // 4, dtype=np.int32)
        _check(lib().xrl_loops_export(self.h, item, _vp(out.ctypes.data), ctypes.byref(n)))
        return out

    def edge_matvec(self, plan, i_edge, alpha=None, beta=None, stream=None):
        """V_edge = sum_t A_t (beta area + alpha P) A_t^T I_edge, complex128 [N_e][R]."""
        import torch
        X = i_edge.reshape(i_edge.shape[0], -1).to(torch.complex128).contiguous()
        R = X.shape[1]
        Y = torch.empty_like(X)
        ep, keep = _epilogue_arrays(alpha, beta, R)
        _check(lib().xrl_edge_matvec(self.h, plan.h, ctypes.byref(ep), _vp(X.data_ptr()), _vp(Y.data_ptr()), R,
                                     _stream(stream)))
        return Y

    def solve(self, plan, v_edge, alpha=None, beta=None, precond="none", restart=50, rtol=1e-6, max_iter=500,
              stream=None):
        """Branch currents of eq. (8) for branch voltages v_edge (complex128
        [N_e][R]); returns (i_edge, stats)."""
        import torch
        B = v_edge.reshape(v_edge.shape[0], -1).to(torch.complex128).contiguous()
        R = B.shape[1]
        X = torch.empty_like(B)
        ep, keep = _epilogue_arrays(alpha, beta, R)
        st = GmresStats()
        code = lib().xrl_loop_gmres_solve(self.h, plan.h, ctypes.byref(ep), _vp(B.data_ptr()), _vp(X.data_ptr()), R,
                                          PRECOND[precond], restart, rtol, max_iter, _stream(stream), ctypes.byref(st))
        stats = {f: getattr(st, f) for f, _ in GmresStats._fields_}
        if code not in (0, -5):
            _check(code)
        stats["status"] = code
        return X, stats

    def close(self):
        if self.h:
            lib().xrl_loops_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
