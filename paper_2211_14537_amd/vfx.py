"""Python binding of the vfx C-ABI library (argument marshalling only).

Every step of the extension and the volume FMM runs in the HIP library
``lib/libvfx.so``; this module converts arguments and raises on errors.  If
the library has not been built the import of the binding fails loudly.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VFX_LIBRARY selects another build of the same library (the host-sanitized
# one the CPU tests load); the default is the in-tree build
LIB_PATH = os.environ.get("VFX_LIBRARY") or os.path.join(_HERE, "lib", "libvfx.so")

VFX_OK = 0
VFX_EINVAL = -1
VFX_ETREE = -2
VFX_EHIP = -4
VFX_ENOMEM = -5


class VfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Kbar", ctypes.c_int32), ("deg", ctypes.c_int32),
                ("p", ctypes.c_int32), ("root_cx", ctypes.c_double), ("root_cy", ctypes.c_double),
                ("root_size", ctypes.c_double)]


class _Tree(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32),
                ("level", ctypes.POINTER(ctypes.c_int32)),
                ("ix", ctypes.POINTER(ctypes.c_int32)),
                ("iy", ctypes.POINTER(ctypes.c_int32)),
                ("kind", ctypes.POINTER(ctypes.c_int8)),
                ("cut_mask", ctypes.POINTER(ctypes.c_uint8))]


class _Stats(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32), ("n_boxes", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_cut", ctypes.c_int32), ("n_ext_targets", ctypes.c_int32),
                ("n_list1", ctypes.c_int64), ("n_list2", ctypes.c_int64), ("n_list3", ctypes.c_int64),
                ("n_list4", ctypes.c_int64), ("pinv_doubles", ctypes.c_int64),
                ("plan_seconds", ctypes.c_double)]


_lib = None

EXPORTED = ("vfx_create", "vfx_destroy", "vfx_stencil_size", "vfx_stencil_points", "vfx_leaf_nodes",
            "vfx_plan_create", "vfx_plan_destroy", "vfx_plan_stats_get", "vfx_plan_ext_owner",
            "vfx_execute", "vfx_plan_set_timing", "vfx_plan_timings", "vfx_plan_set_precision", "vfx_plan_set_near_mode", "vfx_interp", "vfx_net_charge", "vfx_net_charge_noalloc",
            "vfx_net_charge_noalloc_max_rhs", "vfx_execute_batch", "vfx_plan_create_ex",
            "vfx_plan_factor_gpu",
            "vfx_plan_autotune", "vfx_plan_set_launch", "vfx_graph_begin", "vfx_graph_end", "vfx_graph_launch", "vfx_graph_destroy",
            "vfx_mlp_param_count", "vfx_mlp_forward", "vfx_mlp_grad", "vfx_mlp_adam", "vfx_f32_to_f16",
            "vfx_mlp_infer_f16",
            "vfx_last_error", "vfx_status_string",
            "vfx_debug_table", "vfx_plan_lists", "vfx_plan_boxes")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"vfx: HIP library not built ({LIB_PATH}); run __graft_entry__.build()")
        # PyTorch bundles a HIP runtime with the same soname as the system
        # one the library links against; whichever is loaded first serves the
        # whole process.  Load PyTorch first so that its device memory and
        # streams and this library share one runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        L.vfx_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        L.vfx_destroy.argtypes = [vp]
        L.vfx_stencil_size.argtypes = [vp, i32p, i32p]
        L.vfx_stencil_points.argtypes = [vp, dp]
        L.vfx_leaf_nodes.argtypes = [vp, dp]
        L.vfx_plan_create.argtypes = [vp, ctypes.POINTER(_Tree), ctypes.POINTER(vp)]
        L.vfx_plan_destroy.argtypes = [vp]
        L.vfx_plan_stats_get.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.vfx_plan_ext_owner.argtypes = [vp, i32p]
        L.vfx_execute.argtypes = [vp, vp, vp, vp, vp, vp]
        L.vfx_plan_set_timing.argtypes = [vp, ctypes.c_int]
        L.vfx_plan_set_precision.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.vfx_plan_set_near_mode.argtypes = [vp, ctypes.c_int]
        L.vfx_interp.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, vp]
        L.vfx_net_charge.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        L.vfx_net_charge_noalloc.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        L.vfx_net_charge_noalloc_max_rhs.argtypes = []
        L.vfx_execute_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.vfx_plan_create_ex.argtypes = [vp, ctypes.POINTER(_Tree), ctypes.c_int, ctypes.POINTER(vp)]
        L.vfx_plan_factor_gpu.argtypes = [vp, vp]
        L.vfx_plan_autotune.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int, i32p]
        L.vfx_plan_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.vfx_graph_begin.argtypes = [vp]
        L.vfx_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
        L.vfx_graph_launch.argtypes = [vp, vp]
        L.vfx_graph_destroy.argtypes = [vp]
        L.vfx_mlp_param_count.argtypes = []
        L.vfx_mlp_grad_work.argtypes = [ctypes.c_int64]
        L.vfx_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
        L.vfx_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int64, vp]
        L.vfx_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, vp]
        L.vfx_f32_to_f16.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.vfx_mlp_infer_f16.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
        L.vfx_plan_timings.argtypes = [vp, dp, ctypes.c_int]
        L.vfx_last_error.restype = ctypes.c_char_p
        L.vfx_status_string.restype = ctypes.c_char_p
        L.vfx_status_string.argtypes = [ctypes.c_int]
        L.vfx_debug_table.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int64]
        L.vfx_plan_lists.argtypes = [vp, ctypes.c_int, i32p, i32p, i32p]
        L.vfx_plan_boxes.argtypes = [vp, i32p, i32p, i32p, i32p]
        for name in EXPORTED:
            if name not in ("vfx_last_error", "vfx_status_string"):
                getattr(L, name).restype = ctypes.c_int
        L.vfx_mlp_grad_work.restype = ctypes.c_int64
        _lib = L
    return _lib


def _check(rc):
    if rc != VFX_OK:
        raise VfxError(rc, f"{lib().vfx_status_string(rc).decode()}: {lib().vfx_last_error().decode()}")


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class Context:
    """Universal tables for (K, Kbar, deg, p) over one root box."""

    def __init__(self, K, p, Kbar=12, deg=10, root=(0.0, 0.0, 2.0)):
        prm = _Params(K, Kbar, deg, p, float(root[0]), float(root[1]), float(root[2]))
        h = ctypes.c_void_p()
        _check(lib().vfx_create(ctypes.byref(prm), ctypes.byref(h)))
        self._h = h
        self.K, self.p, self.Kbar, self.deg, self.root = K, p, Kbar, deg, tuple(root)
        nx = ctypes.c_int32()
        ng = ctypes.c_int32()
        _check(lib().vfx_stencil_size(self._h, ctypes.byref(nx), ctypes.byref(ng)))
        self.n_stencil, self.n_support = nx.value, ng.value

    def stencil_points(self):
        xy = np.zeros(2 * self.n_stencil)
        _check(lib().vfx_stencil_points(self._h, _ptr(xy, ctypes.c_double)))
        return xy.reshape(-1, 2)

    def leaf_nodes(self):
        t = np.zeros(self.K)
        _check(lib().vfx_leaf_nodes(self._h, _ptr(t, ctypes.c_double)))
        return t

    def debug_table(self, which, index, count):
        out = np.zeros(count)
        _check(lib().vfx_debug_table(self._h, which, index, _ptr(out, ctypes.c_double), count))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().vfx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A tree prepared for repeated execution (lists, extension operators)."""

    def __init__(self, ctx, level, ix, iy, kind, cut_mask=None, defer_factor=False):
        self.ctx = ctx
        self._level = np.ascontiguousarray(level, dtype=np.int32)
        self._ix = np.ascontiguousarray(ix, dtype=np.int32)
        self._iy = np.ascontiguousarray(iy, dtype=np.int32)
        self._kind = np.ascontiguousarray(kind, dtype=np.int8)
        ncut = int((self._kind == 2).sum())
        if cut_mask is None:
            cut_mask = np.zeros((ncut, ctx.n_stencil), dtype=np.uint8)
        self._mask = np.ascontiguousarray(cut_mask, dtype=np.uint8).reshape(ncut, ctx.n_stencil)
        tr = _Tree(self._level.size, _ptr(self._level, ctypes.c_int32), _ptr(self._ix, ctypes.c_int32),
                   _ptr(self._iy, ctypes.c_int32), _ptr(self._kind, ctypes.c_int8),
                   _ptr(self._mask, ctypes.c_uint8))
        h = ctypes.c_void_p()
        _check(lib().vfx_plan_create_ex(ctx._h, ctypes.byref(tr), 1 if defer_factor else 0, ctypes.byref(h)))
        self._h = h
        self.n_leaves = self._level.size
        self.n_cut = ncut

    def factor_gpu(self, stream=None):
        """Compute the cut leaves' least-squares operators on the GPU (plans
        created with defer_factor=True)."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().vfx_plan_factor_gpu(self._h, ctypes.c_void_p(st.cuda_stream)))

    def stats(self):
        s = _Stats()
        _check(lib().vfx_plan_stats_get(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def ext_owner(self):
        o = np.zeros(self.n_leaves, dtype=np.int32)
        _check(lib().vfx_plan_ext_owner(self._h, _ptr(o, ctypes.c_int32)))
        return o

    def lists(self, which):
        """Interaction list `which` (1..4) as (ptr, src, cfg) arrays."""
        st = self.stats()
        nb = st["n_leaves"] if which in (1, 3) else st["n_boxes"]
        cnt = st[f"n_list{which}"]
        ptr = np.zeros(nb + 1, dtype=np.int32)
        src = np.zeros(max(cnt, 1), dtype=np.int32)
        cfg = np.zeros(max(cnt, 1), dtype=np.int32)
        _check(lib().vfx_plan_lists(self._h, which, _ptr(ptr, ctypes.c_int32), _ptr(src, ctypes.c_int32),
                                    _ptr(cfg, ctypes.c_int32)))
        return ptr, src[:cnt], cfg[:cnt]

    def boxes(self):
        nb = self.stats()["n_boxes"]
        a = [np.zeros(nb, dtype=np.int32) for _ in range(4)]
        _check(lib().vfx_plan_boxes(self._h, *[_ptr(x, ctypes.c_int32) for x in a]))
        return dict(zip(("level", "ix", "iy", "leaf"), a))

    def execute(self, f_leaf, f_cut, fe_out, V_out, stream=None):
        """Enqueue the extension + FMM on `stream` (torch CUDA tensors, float64)."""
        import torch
        n = self.ctx.K * self.ctx.K
        for name, t, shape in (("f_leaf", f_leaf, (self.n_leaves, n)), ("fe_out", fe_out, (self.n_leaves, n)),
                               ("V_out", V_out, (self.n_leaves, n))):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
                raise ValueError(f"{name}: expected contiguous float64 CUDA tensor of shape {shape}")
        fc = 0
        if self.n_cut:
            if not (f_cut.is_cuda and f_cut.dtype == torch.float64 and f_cut.is_contiguous()
                    and tuple(f_cut.shape) == (self.n_cut, self.ctx.n_stencil)):
                raise ValueError("f_cut: expected contiguous float64 CUDA tensor (n_cut, |X|)")
            fc = f_cut.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().vfx_execute(self._h, f_leaf.data_ptr(), fc, fe_out.data_ptr(), V_out.data_ptr(),
                                 ctypes.c_void_p(stream.cuda_stream)))

    def _batch_args(self, nrhs, f_leaf, f_cut, fe_out, V_out):
        import torch
        n = self.ctx.K * self.ctx.K
        for name, t in (("f_leaf", f_leaf), ("fe_out", fe_out), ("V_out", V_out)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                    and t.numel() == nrhs * self.n_leaves * n):
                raise ValueError(f"{name}: expected contiguous float64 CUDA tensor of {nrhs} x {self.n_leaves} x {n}")
        fc = 0
        if self.n_cut:
            if not (f_cut.is_cuda and f_cut.dtype == torch.float64 and f_cut.is_contiguous()
                    and f_cut.numel() == nrhs * self.n_cut * self.ctx.n_stencil):
                raise ValueError("f_cut: expected contiguous float64 CUDA tensor (nrhs, n_cut, |X|)")
            fc = f_cut.data_ptr()
        return f_leaf.data_ptr(), fc, fe_out.data_ptr(), V_out.data_ptr()

    def execute_batch(self, nrhs, f_leaf, f_cut, fe_out, V_out, stream=None):
        """nrhs right-hand sides at once (stacked tensors)."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        a = self._batch_args(nrhs, f_leaf, f_cut, fe_out, V_out)
        _check(lib().vfx_execute_batch(self._h, int(nrhs), *a, ctypes.c_void_p(st.cuda_stream)))

    def autotune(self, nrhs, f_leaf, f_cut, fe_out, V_out, reps=3, stream=None):
        """Pick the near-field launch parameters by timing; returns them."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        a = self._batch_args(nrhs, f_leaf, f_cut, fe_out, V_out)
        ch = np.zeros(2, dtype=np.int32)
        _check(lib().vfx_plan_autotune(self._h, int(nrhs), *a, ctypes.c_void_p(st.cuda_stream), int(reps),
                                       _ptr(ch, ctypes.c_int32)))
        return {"near_wgs": int(ch[0]), "dense_mtb": int(ch[1])}

    def set_launch(self, near_wgs, dense_mtb):
        """Set the near-field launch parameters directly."""
        _check(lib().vfx_plan_set_launch(self._h, int(near_wgs), int(dense_mtb)))

    def interp(self, V, px, py, out, stream=None):
        """Interpolate leaf-grid data V (n_leaves x K^2) to the points
        (px, py) into out (all float64 CUDA tensors)."""
        import torch
        n = self.ctx.K * self.ctx.K
        if not (V.is_cuda and V.dtype == torch.float64 and V.is_contiguous() and tuple(V.shape) == (self.n_leaves, n)):
            raise ValueError(f"V: expected contiguous float64 CUDA tensor of shape {(self.n_leaves, n)}")
        m = px.numel()
        for name, t in (("px", px), ("py", py), ("out", out)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == m):
                raise ValueError(f"{name}: expected contiguous float64 CUDA tensor with {m} entries")
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().vfx_interp(self._h, V.data_ptr(), m, px.data_ptr(), py.data_ptr(), out.data_ptr(),
                                ctypes.c_void_p(st.cuda_stream)))

    def net_charge(self, fe, out, stream=None):
        """Integral of leaf-grid data fe ((nrhs x) n_leaves x K^2) over the
        tree into out (nrhs entries); float64 CUDA tensors."""
        import torch
        n = self.ctx.K * self.ctx.K
        if not (fe.is_cuda and fe.dtype == torch.float64 and fe.is_contiguous() and fe.numel() > 0
                and fe.numel() % (self.n_leaves * n) == 0):
            raise ValueError(f"fe: expected contiguous float64 CUDA tensor of nrhs x {(self.n_leaves, n)}")
        nrhs = fe.numel() // (self.n_leaves * n)
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == nrhs):
            raise ValueError(f"out: expected contiguous float64 CUDA tensor with {nrhs} entries")
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().vfx_net_charge(self._h, fe.data_ptr(), nrhs, out.data_ptr(), ctypes.c_void_p(st.cuda_stream)))

    def net_charge_noalloc(self, fe, out, stream=None):
        """net_charge through the allocation-free entry point (the plan's
        device data must already be resident; at most
        net_charge_noalloc_max_rhs() right-hand sides)."""
        import torch
        n = self.ctx.K * self.ctx.K
        if not (fe.is_cuda and fe.dtype == torch.float64 and fe.is_contiguous() and fe.numel() > 0
                and fe.numel() % (self.n_leaves * n) == 0):
            raise ValueError(f"fe: expected contiguous float64 CUDA tensor of nrhs x {(self.n_leaves, n)}")
        nrhs = fe.numel() // (self.n_leaves * n)
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == nrhs):
            raise ValueError(f"out: expected contiguous float64 CUDA tensor with {nrhs} entries")
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().vfx_net_charge_noalloc(self._h, fe.data_ptr(), nrhs, out.data_ptr(),
                                            ctypes.c_void_p(st.cuda_stream)))

    def set_near_mode(self, mode):
        """Near-field strategy (FP64, K = 16): 0 pair-based (default),
        1 target-stationary."""
        _check(lib().vfx_plan_set_near_mode(self._h, int(mode)))

    def set_precision(self, mode, min_level=0):
        """Near-field precision for sources at level >= min_level (K = 16):
        0 = FP64; 1 = four fixed-point bf16 slices per operand row on the
        bf16 matrix cores (exact FP32 block sums, FP64 results); 2 = five
        fixed-point int8 slices on the int8 matrix cores (exact int32 sums,
        FP64 results)."""
        _check(lib().vfx_plan_set_precision(self._h, int(mode), int(min_level)))

    def set_timing(self, on=True):
        _check(lib().vfx_plan_set_timing(self._h, 1 if on else 0))

    PHASES = ("extension", "p2m_up", "m2l", "down", "near_lowrank", "near_dense", "far", "total", "p2l", "m2p",
              "fe_init")

    def timings(self):
        """Per-phase milliseconds averaged over the executes recorded since
        set_timing(True), plus their count."""
        ms = np.zeros(len(self.PHASES) + 1)
        _check(lib().vfx_plan_timings(self._h, _ptr(ms, ctypes.c_double), ms.size))
        out = dict(zip(self.PHASES, ms[:-1].tolist()))
        out["count"] = int(ms[-1])
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().vfx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- refinement classifier (device tensors; argument marshalling only) ----

def _dev_f32(t, n=None, name="tensor"):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and (n is None or t.numel() == n)):
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor" + (f" with {n} entries" if n else ""))
    return t.data_ptr()


def _stream(stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def mlp_param_count():
    return int(lib().vfx_mlp_param_count())


def mlp_forward(theta, x, logits, stream=None):
    B = x.shape[0]
    _check(lib().vfx_mlp_forward(_dev_f32(theta, mlp_param_count(), "theta"), _dev_f32(x, B * 64, "x"), B,
                                 _dev_f32(logits, B, "logits"), _stream(stream)))


def mlp_grad_work(batch):
    return int(lib().vfx_mlp_grad_work(batch))


def mlp_grad(theta, x, y, grad, work, stream=None):
    B = x.shape[0]
    _check(lib().vfx_mlp_grad(_dev_f32(theta, mlp_param_count(), "theta"), _dev_f32(x, B * 64, "x"),
                              _dev_f32(y, B, "y"), B, _dev_f32(grad, mlp_param_count(), "grad"),
                              _dev_f32(work, None, "work"), work.numel(), _stream(stream)))


def mlp_adam(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = mlp_param_count()
    _check(lib().vfx_mlp_adam(_dev_f32(theta, n, "theta"), _dev_f32(grad, n, "grad"), _dev_f32(m, n, "m"),
                              _dev_f32(v, n, "v"), int(step), lr, beta1, beta2, eps, _stream(stream)))


def f32_to_f16(a, h, stream=None):
    import torch
    if not (h.is_cuda and h.dtype == torch.float16 and h.is_contiguous() and h.numel() == a.numel()):
        raise ValueError("h: expected a contiguous float16 CUDA tensor of the same size")
    _check(lib().vfx_f32_to_f16(_dev_f32(a, None, "a"), h.data_ptr(), a.numel(), _stream(stream)))


def mlp_infer_f16(theta_h, x_h, logits, stream=None):
    import torch
    B = x_h.shape[0]
    for name, t, n in (("theta_h", theta_h, mlp_param_count()), ("x_h", x_h, B * 64)):
        if not (t.is_cuda and t.dtype == torch.float16 and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name}: expected a contiguous float16 CUDA tensor with {n} entries")
    _check(lib().vfx_mlp_infer_f16(theta_h.data_ptr(), x_h.data_ptr(), B, _dev_f32(logits, B, "logits"),
                                   _stream(stream)))


class Graph:
    """Executes captured on a stream and replayed with one launch."""

    def __init__(self):
        self._h = None

    def begin(self, stream):
        _check(lib().vfx_graph_begin(ctypes.c_void_p(stream.cuda_stream)))

    def end(self, stream):
        h = ctypes.c_void_p()
        _check(lib().vfx_graph_end(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream):
        _check(lib().vfx_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if self._h is not None:
            lib().vfx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def net_charge_noalloc_max_rhs():
    """Right-hand sides vfx_net_charge_noalloc accepts per call."""
    return int(lib().vfx_net_charge_noalloc_max_rhs())
