"""Thin ctypes binding of libqpgf (include/qpgf.h): argument marshalling only.

Every step of the method runs in the HIP library; this module only turns torch
CUDA tensors into device pointers and the current torch stream into the
plan's HIP stream.  Loading fails loudly if ``libqpgf.so`` is missing: there is
no CPU fallback.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpgf.so")

C128, C64 = 0, 1
KIND_G2D, KIND_GD3D, KIND_MAXWELL3D, KIND_G2D_GRAD, KIND_G2D_HESS_DIFF = 0, 1, 2, 3, 4
STATUS = {0: "OK", 1: "E_ARG", 2: "E_WOOD", 3: "E_SPECIAL", 4: "E_SIZE", 5: "E_HIP", 6: "E_NOMEM",
          7: "E_UNSUPPORTED", 8: "E_IO"}


class QpgfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qpgf {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("prec", ctypes.c_int), ("m1", ctypes.c_int), ("m2", ctypes.c_int),
                ("m3", ctypes.c_int), ("c", ctypes.c_double), ("c_tilde", ctypes.c_double),
                ("eps", ctypes.c_double), ("quad_q", ctypes.c_int), ("far_h", ctypes.c_double),
                ("far_zmax", ctypes.c_double), ("wood_tol", ctypes.c_double), ("special_tol", ctypes.c_double),
                ("lattice_rmin", ctypes.c_double), ("sing_order", ctypes.c_int),
                ("ring_interp", ctypes.c_int), ("far_m", ctypes.c_int), ("maxwell_trace", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("prec", ctypes.c_int), ("m1", ctypes.c_int), ("m2", ctypes.c_int),
                ("m3", ctypes.c_int), ("far_slices", ctypes.c_int), ("far_h", ctypes.c_double),
                ("c", ctypes.c_double), ("c_tilde", ctypes.c_double), ("eps", ctypes.c_double),
                ("n_fields", ctypes.c_int), ("grid_bytes", ctypes.c_size_t), ("far_grid_bytes", ctypes.c_size_t),
                ("far_m1", ctypes.c_int), ("far_m2", ctypes.c_int), ("far_fields", ctypes.c_int),
                ("far_points", ctypes.c_int), ("far_points_t", ctypes.c_int)]


class TrainCfg(ctypes.Structure):
    """qpgf_train_cfg."""
    _fields_ = [("batch", ctypes.c_int64), ("steps", ctypes.c_int64), ("lr_max", ctypes.c_float),
                ("lr_min", ctypes.c_float), ("member", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


EXPORTS = ["qpgf_params_default", "qpgf_plan_create", "qpgf_plan_destroy", "qpgf_plan_set_stream",
           "qpgf_plan_get_info", "qpgf_prepare", "qpgf_evaluate", "qpgf_g2d", "qpgf_gd3d", "qpgf_maxwell3d",
           "qpgf_g2d_grad", "qpgf_g2d_hess_diff", "qpgf_prepare_hess_diff", "qpgf_prepare_stage", "qpgf_copy_field", "qpgf_plan_enable_timing", "qpgf_plan_get_timing",
           "qpgf_g2d_batched", "qpgf_plan_autotune", "qpgf_last_error", "qpgf_version", "qpgf_evaluate_smooth",
           "qpgf_mlp_param_count", "qpgf_mlp_create", "qpgf_mlp_destroy", "qpgf_mlp_set_stream",
           "qpgf_mlp_get_params", "qpgf_mlp_set_params", "qpgf_mlp_forward", "qpgf_mlp_gradient",
           "qpgf_mlp_train_step", "qpgf_mlp_last_error", "qpgf_surrogate_eval", "qpgf_mlp_set_calibration",
           "qpgf_mlp_get_calibration", "qpgf_surrogate_make_data", "qpgf_surrogate_train", "qpgf_surrogate_calibrate",
           "qpgf_mlp_save", "qpgf_mlp_load", "qpgf_plan_workspace_bytes", "qpgf_plan_set_workspace",
           "qpgf_evaluate_noalloc"]
TIMERS = ["htable", "fill", "fft_t", "fft_2", "fft_1", "far", "far_fft", "gather", "bin", "batch", "bin_place",
          "overflow", "layout", "ring", "gather_far"]

_lib = None


def lib():
    """Load libqpgf.so (once); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1801_05977_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I64, VP, U8P = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    L.qpgf_params_default.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int]
    L.qpgf_params_default.restype = None
    L.qpgf_plan_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(P)]
    L.qpgf_plan_destroy.argtypes = [P]
    L.qpgf_plan_destroy.restype = None
    L.qpgf_plan_set_stream.argtypes = [P, VP]
    L.qpgf_plan_get_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    L.qpgf_prepare.argtypes = [P, D, D, D]
    L.qpgf_prepare_stage.argtypes = [P, D, D, D, ctypes.c_int]
    L.qpgf_evaluate.argtypes = [P, VP, I64, VP, U8P]
    L.qpgf_g2d.argtypes = [P, D, D, VP, I64, VP, U8P]
    L.qpgf_g2d_grad.argtypes = [P, D, D, VP, I64, VP, U8P]
    L.qpgf_g2d_hess_diff.argtypes = [P, D, D, D, VP, I64, VP, U8P]
    L.qpgf_prepare_hess_diff.argtypes = [P, D, D, D, ctypes.c_int]
    L.qpgf_gd3d.argtypes = [P, D, D, D, VP, I64, VP, U8P]
    L.qpgf_maxwell3d.argtypes = [P, D, D, D, VP, I64, VP, U8P]
    L.qpgf_copy_field.argtypes = [P, ctypes.c_int, ctypes.c_int, VP]
    L.qpgf_plan_enable_timing.argtypes = [P, ctypes.c_int]
    L.qpgf_plan_get_timing.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    L.qpgf_g2d_batched.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64), VP, VP, U8P]
    L.qpgf_plan_autotune.argtypes = [P, ctypes.c_char_p]
    L.qpgf_last_error.restype = ctypes.c_char_p
    L.qpgf_version.restype = ctypes.c_char_p
    L.qpgf_evaluate_smooth.argtypes = [P, VP, I64, VP]
    L.qpgf_mlp_param_count.argtypes = []
    L.qpgf_mlp_param_count.restype = ctypes.c_long
    L.qpgf_mlp_create.argtypes = [ctypes.c_int, I64, ctypes.c_uint64, ctypes.POINTER(P)]
    L.qpgf_mlp_destroy.argtypes = [P]
    L.qpgf_mlp_destroy.restype = None
    L.qpgf_mlp_set_stream.argtypes = [P, VP]
    L.qpgf_mlp_get_params.argtypes = [P, ctypes.c_int, VP]
    L.qpgf_mlp_set_params.argtypes = [P, ctypes.c_int, VP]
    L.qpgf_mlp_forward.argtypes = [P, ctypes.c_int, VP, I64, VP]
    L.qpgf_mlp_gradient.argtypes = [P, ctypes.c_int, VP, VP, I64, VP, VP]
    L.qpgf_mlp_train_step.argtypes = [P, ctypes.c_int, VP, VP, I64, ctypes.c_float, VP]
    L.qpgf_mlp_last_error.restype = ctypes.c_char_p
    DP = ctypes.POINTER(ctypes.c_double)
    L.qpgf_surrogate_eval.argtypes = [P, P, D, D, D, ctypes.c_int, DP, DP, DP, ctypes.POINTER(ctypes.c_int64), VP,
                                      VP, U8P, ctypes.POINTER(ctypes.c_int64)]
    L.qpgf_mlp_set_calibration.argtypes = [P, D]
    L.qpgf_mlp_get_calibration.argtypes = [P, DP]
    L.qpgf_surrogate_make_data.argtypes = [P, P, ctypes.c_int, DP, DP, DP, ctypes.POINTER(ctypes.c_int64), VP, VP, VP]
    L.qpgf_surrogate_train.argtypes = [P, VP, VP, I64, ctypes.POINTER(TrainCfg), VP]
    L.qpgf_surrogate_calibrate.argtypes = [P, P, ctypes.c_int, DP, DP, DP, ctypes.POINTER(ctypes.c_int64), VP, D, D,
                                           DP]
    L.qpgf_plan_workspace_bytes.argtypes = [P, D, I64, ctypes.POINTER(ctypes.c_size_t)]
    L.qpgf_plan_set_workspace.argtypes = [P, VP, ctypes.c_size_t, D, I64]
    L.qpgf_evaluate_noalloc.argtypes = [P, VP, I64, VP, U8P]
    L.qpgf_mlp_save.argtypes = [P, ctypes.c_char_p]
    L.qpgf_mlp_load.argtypes = [P, ctypes.c_char_p]
    for name in ("qpgf_plan_create", "qpgf_plan_set_stream", "qpgf_plan_get_info", "qpgf_prepare",
                 "qpgf_prepare_stage", "qpgf_evaluate", "qpgf_g2d", "qpgf_gd3d", "qpgf_maxwell3d",
                 "qpgf_copy_field", "qpgf_plan_enable_timing", "qpgf_plan_get_timing", "qpgf_g2d_batched",
                 "qpgf_plan_autotune", "qpgf_evaluate_smooth", "qpgf_mlp_create", "qpgf_mlp_set_stream",
                 "qpgf_mlp_get_params", "qpgf_mlp_set_params", "qpgf_mlp_forward", "qpgf_mlp_gradient",
                 "qpgf_mlp_train_step", "qpgf_surrogate_eval", "qpgf_mlp_set_calibration", "qpgf_mlp_get_calibration",
                 "qpgf_surrogate_make_data", "qpgf_surrogate_train", "qpgf_surrogate_calibrate", "qpgf_mlp_save",
                 "qpgf_mlp_load", "qpgf_plan_workspace_bytes", "qpgf_plan_set_workspace",
                 "qpgf_evaluate_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise QpgfError(status, lib().qpgf_last_error().decode())


def _check_mlp(status):
    if status != 0:
        raise QpgfError(status, lib().qpgf_mlp_last_error().decode())


def default_params(kind, prec, m1, m2, m3=0, **overrides):
    p = Params()
    lib().qpgf_params_default(ctypes.byref(p), kind, prec, m1, m2, m3)
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _ptr(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A qpgf plan bound to torch's current CUDA stream at each call."""

    def __init__(self, kind, prec, m1, m2, m3=0, **overrides):
        self.params = default_params(kind, prec, m1, m2, m3, **overrides)
        self._h = ctypes.c_void_p()
        torch.cuda.init()
        _check(lib().qpgf_plan_create(ctypes.byref(self.params), ctypes.byref(self._h)))
        self.kind, self.prec = kind, prec
        self.dim = 2 if kind in (KIND_G2D, KIND_G2D_GRAD, KIND_G2D_HESS_DIFF) else 3
        self.cdtype = torch.complex128 if prec == C128 else torch.complex64

    @property
    def info(self):
        """qpgf_plan_get_info now (the far slab's geometry follows the last prepared instance)."""
        info = PlanInfo()
        _check(lib().qpgf_plan_get_info(self._h, ctypes.byref(info)))
        return info

    def close(self):
        if self._h:
            lib().qpgf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check(lib().qpgf_plan_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def workspace_bytes(self, kmax, max_targets):
        n = ctypes.c_size_t()
        _check(lib().qpgf_plan_workspace_bytes(self._h, float(kmax), int(max_targets), ctypes.byref(n)))
        return n.value

    def use_workspace(self, kmax, max_targets, buf=None):
        """qpgf_plan_set_workspace on a torch uint8 buffer (allocated here when not given); the plan keeps a
        reference to it.  use_workspace(None, None) returns the plan to its own arrays."""
        self._stream()
        if kmax is None:
            _check(lib().qpgf_plan_set_workspace(self._h, None, 0, 0.0, 0))
            self._ws = None
            return None
        if buf is None:
            buf = torch.empty(self.workspace_bytes(kmax, max_targets), dtype=torch.uint8, device="cuda")
        _check(lib().qpgf_plan_set_workspace(self._h, _ptr(buf, torch.uint8, "workspace"), buf.numel(),
                                             float(kmax), int(max_targets)))
        self._ws = buf
        return buf

    def out_tensor(self, T):
        shape = {KIND_MAXWELL3D: (T, 6), KIND_G2D_GRAD: (T, 2), KIND_G2D_HESS_DIFF: (T, 3)}.get(self.kind, (T,))
        return torch.empty(shape, dtype=self.cdtype, device="cuda")

    def prepare(self, k, a1, a2=0.0, stage=2):
        self._stream()
        _check(lib().qpgf_prepare_stage(self._h, k, a1, a2, stage))

    def evaluate(self, x, out=None, flags=None):
        T = x.shape[0]
        if out is None:
            out = self.out_tensor(T)
        self._stream()
        _check(lib().qpgf_evaluate(self._h, _ptr(x, torch.float64, "x"), T, _ptr(out, self.cdtype, "out"),
                                   _ptr(flags, torch.uint8, "flags")))
        return out

    def __call__(self, k, a1, a2=0.0, x=None, out=None, flags=None):
        """prepare + evaluate through the kind's own entry point (qpgf_g2d / qpgf_gd3d / qpgf_maxwell3d /
        qpgf_g2d_grad)."""
        T = x.shape[0]
        if out is None:
            out = self.out_tensor(T)
        self._stream()
        px, po, pf = _ptr(x, torch.float64, "x"), _ptr(out, self.cdtype, "out"), _ptr(flags, torch.uint8, "flags")
        if self.kind == KIND_G2D_HESS_DIFF:
            raise ValueError("a KIND_G2D_HESS_DIFF plan takes two wavenumbers: use Plan.hess_diff")
        if self.kind == KIND_G2D:
            _check(lib().qpgf_g2d(self._h, k, a1, px, T, po, pf))
        elif self.kind == KIND_G2D_GRAD:
            _check(lib().qpgf_g2d_grad(self._h, k, a1, px, T, po, pf))
        elif self.kind == KIND_GD3D:
            _check(lib().qpgf_gd3d(self._h, k, a1, a2, px, T, po, pf))
        else:
            _check(lib().qpgf_maxwell3d(self._h, k, a1, a2, px, T, po, pf))
        return out

    def prepare_hess_diff(self, k1, k2, alpha, stage=2):
        """qpgf_prepare_hess_diff (plans of kind KIND_G2D_HESS_DIFF)."""
        self._stream()
        _check(lib().qpgf_prepare_hess_diff(self._h, k1, k2, alpha, stage))

    def hess_diff(self, k1, k2, alpha, x, out=None, flags=None):
        """qpgf_g2d_hess_diff: [T, 3] = d11, d12, d22 of G_k1 - G_k2 at x [T, 2]."""
        T = x.shape[0]
        if out is None:
            out = self.out_tensor(T)
        self._stream()
        _check(lib().qpgf_g2d_hess_diff(self._h, k1, k2, alpha, _ptr(x, torch.float64, "x"), T,
                                        _ptr(out, self.cdtype, "out"), _ptr(flags, torch.uint8, "flags")))
        return out

    def batched(self, k, alpha, m1, t_off, x, out=None, flags=None):
        """qpgf_g2d_batched: instances (k[i], alpha[i], m1[i]) own targets x[t_off[i]:t_off[i+1]]."""
        n = len(k)
        T = int(t_off[-1])
        if out is None:
            out = self.out_tensor(T)
        arr = lambda ct, v: (ct * len(v))(*v)
        self._stream()
        _check(lib().qpgf_g2d_batched(self._h, n, arr(ctypes.c_double, [float(v) for v in k]),
                                      arr(ctypes.c_double, [float(v) for v in alpha]),
                                      arr(ctypes.c_int, [int(v) for v in m1]),
                                      arr(ctypes.c_int64, [int(v) for v in t_off]),
                                      _ptr(x, torch.float64, "x"), _ptr(out, self.cdtype, "out"),
                                      _ptr(flags, torch.uint8, "flags")))
        return out

    def smooth(self, x, out=None):
        """qpgf_evaluate_smooth: the interpolated smooth part L_N at x (GD3D, after prepare)."""
        T = x.shape[0]
        if out is None:
            out = torch.empty((T,), dtype=self.cdtype, device="cuda")
        self._stream()
        _check(lib().qpgf_evaluate_smooth(self._h, _ptr(x, torch.float64, "x"), T, _ptr(out, self.cdtype, "out")))
        return out

    def autotune(self, cache_path=None):
        self._stream()
        _check(lib().qpgf_plan_autotune(self._h, cache_path.encode() if cache_path else None))

    def enable_timing(self, on=True):
        _check(lib().qpgf_plan_enable_timing(self._h, int(on)))

    def timing(self):
        """{kernel class: (total ms, launches)} since timing was enabled."""
        res = {}
        for i, name in enumerate(TIMERS):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(lib().qpgf_plan_get_timing(self._h, i, ctypes.byref(ms), ctypes.byref(n)))
            res[name] = (ms.value, n.value)
        return res

    def field(self, which=0, field=0):
        """Copy of a near-grid (which=0) or far-slab (which=1) field as a flat complex tensor."""
        n = (self.info.grid_bytes if which == 0 else self.info.far_grid_bytes) // (16 if self.prec == C128 else 8)
        dst = torch.empty(n, dtype=self.cdtype, device="cuda")
        self._stream()
        _check(lib().qpgf_copy_field(self._h, which, field, ctypes.c_void_p(dst.data_ptr())))
        return dst


def g2d(k, alpha, x, m1, m2, prec=C128, **kw):
    return Plan(KIND_G2D, prec, m1, m2, **kw)(k, alpha, 0.0, x)


def gd3d(k, a1, a2, x, m1, m2, m3, prec=C128, **kw):
    return Plan(KIND_GD3D, prec, m1, m2, m3, **kw)(k, a1, a2, x)


def maxwell3d(k, a1, a2, x, m1, m2, m3, prec=C128, **kw):
    return Plan(KIND_MAXWELL3D, prec, m1, m2, m3, **kw)(k, a1, a2, x)


class Mlp:
    """Ensemble MLP surrogate of the smooth part L_d (qpgf_mlp_*), on torch's current stream."""

    def __init__(self, members=1, max_batch=65536, seed=0):
        torch.cuda.init()
        self._h = ctypes.c_void_p()
        _check_mlp(lib().qpgf_mlp_create(members, max_batch, seed, ctypes.byref(self._h)))
        self.members, self.max_batch = members, max_batch
        self.n_params = lib().qpgf_mlp_param_count()

    def close(self):
        if self._h:
            lib().qpgf_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check_mlp(lib().qpgf_mlp_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def params(self, member=0):
        dst = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._stream()
        _check_mlp(lib().qpgf_mlp_get_params(self._h, member, _ptr(dst, torch.float32, "dst")))
        return dst

    def set_params(self, p, member=0):
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self._stream()
        _check_mlp(lib().qpgf_mlp_set_params(self._h, member, _ptr(p, torch.float32, "src")))

    def forward(self, q, member=0):
        y = torch.empty((q.shape[0], 2), dtype=torch.float32, device="cuda")
        self._stream()
        _check_mlp(lib().qpgf_mlp_forward(self._h, member, _ptr(q, torch.float64, "q"), q.shape[0],
                                          _ptr(y, torch.float32, "y")))
        return y

    def gradient(self, q, y, member=0):
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        self._stream()
        _check_mlp(lib().qpgf_mlp_gradient(self._h, member, _ptr(q, torch.float64, "q"), _ptr(y, torch.float32, "y"),
                                           q.shape[0], _ptr(g, torch.float32, "grad"),
                                           _ptr(loss, torch.float32, "loss")))
        return g, loss

    def train_step(self, q, y, lr, member=0, loss=None):
        self._stream()
        _check_mlp(lib().qpgf_mlp_train_step(self._h, member, _ptr(q, torch.float64, "q"),
                                             _ptr(y, torch.float32, "y"), q.shape[0], float(lr),
                                             _ptr(loss, torch.float32, "loss")))

    def evaluate(self, plan, k, a1, a2, t_off, x, tol, wood_tol=1e-3, rmin=1e-3, out=None, fell_back=None):
        """qpgf_surrogate_eval: G_d for instances (k[i], a1[i], a2[i]) on x[t_off[i]:t_off[i+1]], falling
        back to the plain method of `plan` where flagged.  Returns (out, fell_back, n_fallback)."""
        n = len(k)
        T = int(t_off[-1])
        if out is None:
            out = plan.out_tensor(T)
        if fell_back is None:
            fell_back = torch.empty(T, dtype=torch.uint8, device="cuda")
        arr = lambda ct, v: (ct * len(v))(*v)
        nf = ctypes.c_int64()
        self._stream()
        _check_mlp(lib().qpgf_surrogate_eval(self._h, plan._h, float(tol), float(wood_tol), float(rmin), n,
                                             arr(ctypes.c_double, [float(v) for v in k]),
                                             arr(ctypes.c_double, [float(v) for v in a1]),
                                             arr(ctypes.c_double, [float(v) for v in a2]),
                                             arr(ctypes.c_int64, [int(v) for v in t_off]),
                                             _ptr(x, torch.float64, "x"), _ptr(out, plan.cdtype, "out"),
                                             _ptr(fell_back, torch.uint8, "fell_back"), ctypes.byref(nf)))
        return out, fell_back, nf.value

    @staticmethod
    def _inst(k, a1, a2, t_off):
        arr = lambda ct, v: (ct * len(v))(*v)
        return (len(k), arr(ctypes.c_double, [float(v) for v in k]), arr(ctypes.c_double, [float(v) for v in a1]),
                arr(ctypes.c_double, [float(v) for v in a2]), arr(ctypes.c_int64, [int(v) for v in t_off]))

    @property
    def kappa(self):
        """Calibration factor of the error estimate (+inf: uncalibrated, accepts nothing)."""
        v = ctypes.c_double()
        _check_mlp(lib().qpgf_mlp_get_calibration(self._h, ctypes.byref(v)))
        return v.value

    @kappa.setter
    def kappa(self, v):
        _check_mlp(lib().qpgf_mlp_set_calibration(self._h, float(v)))

    def make_data(self, plan, k, a1, a2, t_off, x):
        """qpgf_surrogate_make_data: training rows (q [T][6] float64, y [T][2] float32) from the plain method."""
        T = int(t_off[-1])
        q = torch.empty((T, 6), dtype=torch.float64, device="cuda")
        y = torch.empty((T, 2), dtype=torch.float32, device="cuda")
        self._stream()
        _check_mlp(lib().qpgf_surrogate_make_data(self._h, plan._h, *self._inst(k, a1, a2, t_off),
                                                  _ptr(x, torch.float64, "x"), _ptr(q, torch.float64, "q"),
                                                  _ptr(y, torch.float32, "y")))
        return q, y

    def train(self, q, y, batch, steps, lr_max, lr_min, seed=0, member=-1):
        """qpgf_surrogate_train; returns the last minibatch loss of each member (device float32 [members])."""
        cfg = TrainCfg(batch=batch, steps=steps, lr_max=lr_max, lr_min=lr_min, member=member, reserved=0, seed=seed)
        loss = torch.full((self.members,), float("nan"), dtype=torch.float32, device="cuda")
        self._stream()
        _check_mlp(lib().qpgf_surrogate_train(self._h, _ptr(q, torch.float64, "q"), _ptr(y, torch.float32, "y"),
                                              q.shape[0], ctypes.byref(cfg), _ptr(loss, torch.float32, "loss")))
        return loss

    def calibrate(self, plan, k, a1, a2, t_off, x, quantile=1.0, safety=2.0):
        """qpgf_surrogate_calibrate; returns the fitted kappa."""
        v = ctypes.c_double()
        self._stream()
        _check_mlp(lib().qpgf_surrogate_calibrate(self._h, plan._h, *self._inst(k, a1, a2, t_off),
                                                  _ptr(x, torch.float64, "x"), float(quantile), float(safety),
                                                  ctypes.byref(v)))
        return v.value

    def save(self, path):
        self._stream()
        _check_mlp(lib().qpgf_mlp_save(self._h, os.fsencode(path)))

    def load(self, path):
        self._stream()
        _check_mlp(lib().qpgf_mlp_load(self._h, os.fsencode(path)))
