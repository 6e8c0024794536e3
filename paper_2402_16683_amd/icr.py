"""Python binding of the ICR C ABI (include/icr.h): argument marshalling only.

Every computation runs in libicr.so's HIP kernels. PyTorch supplies device
memory (tensors) and streams. The functions carry the C names:

    plan = icr_build_matrices(cfg)                 # FP64 build on the device
    s    = icr_forward(plan, xi)                   # s = L xi
    xib  = icr_adjoint(plan, s_bar)                # xi_bar = L^T s_bar
    out  = icr_metric_apply(plan, w, v)            # L^T (w * L v) + v
    icr_plan_destroy(plan)

Tensors are CUDA (HIP) tensors, contiguous, batch outermost, of the plan's
storage dtype (float64 / float32 / bfloat16). A missing library raises: there is
no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicr.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "icr.h")

ICR_MAX_DEPTH = 15

STATUS = {0: "ICR_OK", 1: "ICR_ERR_INVALID_ARG", 2: "ICR_ERR_NOT_PD", 3: "ICR_ERR_HIP",
          4: "ICR_ERR_OUT_OF_MEMORY", 5: "ICR_ERR_UNSUPPORTED"}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2}
KERNELS = {"matern12": 0, "matern32": 1, "matern52": 2, "sqexp": 3}
CHARTS = {"regular": 0, "logradial2d": 1, "logradial_cyl3d": 2}
FLAG_NO_CLAMP = 1
FLAG_HYPERGRAD = 2


class IcrConfig(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape0", ctypes.c_int32 * 3), ("depth", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("chart", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("distances0", ctypes.c_double * 3), ("scale", ctypes.c_double),
                ("length", ctypes.c_double), ("chart_params", ctypes.c_double * 4)]


class IcrPlanInfo(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("depth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("chart", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("clamped_pivots", ctypes.c_int32 * (ICR_MAX_DEPTH + 1)),
                ("level_shapes", (ctypes.c_int32 * 3) * (ICR_MAX_DEPTH + 1)),
                ("level_offsets", ctypes.c_int64 * (ICR_MAX_DEPTH + 2)),
                ("n_xi", ctypes.c_int64), ("n_out", ctypes.c_int64),
                ("workspace_elems", ctypes.c_int64), ("metric_workspace_elems", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64),
                ("level_sets", ctypes.c_int64 * ICR_MAX_DEPTH),
                ("hypergrad_workspace_elems", ctypes.c_int64)]


class ICRError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libicr.so (built in-tree by build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2402_16683_amd.build`")
    # A process must hold one HIP runtime. PyTorch ships its own libamdhip64 with
    # the same SONAME as ROCm's; loading torch first makes libicr.so bind to it
    # instead of pulling in a second runtime that would not see torch's device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    sigs = {
        "icr_build_matrices": [ctypes.POINTER(IcrConfig), vp, ctypes.POINTER(vp)],
        "icr_plan_get_info": [vp, ctypes.POINTER(IcrPlanInfo)],
        "icr_plan_copy_level0": [vp, vp],
        "icr_plan_copy_refinement": [vp, i32, vp, vp],
        "icr_plan_set_level0": [vp, vp, vp],
        "icr_plan_set_refinement": [vp, i32, vp, vp, vp],
        "icr_forward": [vp, i64, vp, vp, vp, vp],
        "icr_adjoint": [vp, i64, vp, vp, vp, vp],
        "icr_metric_apply": [vp, i64, vp, i64, vp, vp, vp, vp],
        "icr_metric_apply_static": [vp, i64, vp, i64, vp, vp, vp],
        "icr_forward_level": [vp, i32, i64, vp, i64, vp, i64, vp, i64, vp],
        "icr_cg_workspace_bytes": [vp, i64, ctypes.POINTER(i64)],
        "icr_cg_metric": [vp, i64, vp, i64, vp, vp, i32, vp, vp, vp],
        "icr_cg_metric_sl": [vp, i64, vp, i64, vp, vp, ctypes.c_double, i32, vp, vp, vp, vp],
        "icr_adjoint_level": [vp, i32, i64, vp, i64, vp, i64, vp, i64, vp],
        "icr_hyper_grad": [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp],
        "icr_weighted_adjoint": [vp, i64, vp, i64, i32, vp, vp, vp, vp, vp],
        "icr_mgvi_workspace_bytes": [vp, i64, ctypes.POINTER(i64)],
        "icr_mgvi_newton_step": [vp, i64, vp, i64, vp, vp, i32, vp, vp, vp],
        "icr_plan_destroy": [vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.icr_last_error.argtypes = []
    lib.icr_last_error.restype = ctypes.c_char_p
    lib.icr_version.argtypes = []
    lib.icr_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def declared_functions(headers=None) -> list[str]:
    """Names of the functions the headers under include/ declare."""
    import glob
    headers = headers or sorted(glob.glob(os.path.join(os.path.dirname(HEADER), "*.h")))
    names = set()
    for h in headers:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(icr_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def icr_last_error() -> str:
    return load_library().icr_last_error().decode()


def _check(status: int):
    if status != 0:
        raise ICRError(status, icr_last_error())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_config(ndim, shape0, depth, distances0, kernel="matern32", scale=1.0, length=0.1,
                chart="regular", chart_params=(0.1, math.log(10.0), 0.5 * math.pi),
                precision="f32", clamp=True, hypergrad=False) -> IcrConfig:
    c = IcrConfig()
    c.ndim = ndim
    for a in range(3):
        c.shape0[a] = int(shape0[a]) if a < ndim else 1
        c.distances0[a] = float(distances0[a]) if a < ndim else 1.0
    c.depth = depth
    c.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    c.chart = CHARTS[chart] if isinstance(chart, str) else int(chart)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.flags = (0 if clamp else FLAG_NO_CLAMP) | (FLAG_HYPERGRAD if hypergrad else 0)
    c.reserved = 0
    c.scale = scale
    c.length = length
    for k in range(4):
        c.chart_params[k] = float(chart_params[k]) if k < len(chart_params) else 0.0
    return c


class Plan:
    """Owns an icr_plan*; freed by icr_plan_destroy (or when garbage collected)."""

    def __init__(self, handle: ctypes.c_void_p, cfg: IcrConfig):
        self.handle = handle
        self.cfg = cfg
        self.info = icr_plan_get_info(self)

    @property
    def dtype(self):
        import torch
        return {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}[self.cfg.precision]

    @property
    def acc_dtype(self):
        import torch
        return torch.float64 if self.cfg.precision == 0 else torch.float32

    def __del__(self):
        try:
            if self.handle:
                icr_plan_destroy(self)
        except Exception:
            pass


def icr_build_matrices(cfg: IcrConfig, stream=None) -> Plan:
    lib = load_library()
    out = ctypes.c_void_p()
    _check(lib.icr_build_matrices(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(out)))
    return Plan(out, cfg)


def icr_plan_get_info(plan: Plan) -> dict:
    info = IcrPlanInfo()
    _check(load_library().icr_plan_get_info(plan.handle, ctypes.byref(info)))
    depth = info.depth
    return dict(
        ndim=info.ndim, depth=depth, precision=info.precision, chart=info.chart,
        elem_bytes=info.elem_bytes,
        clamped_pivots=[info.clamped_pivots[l] for l in range(depth + 1)],
        level_shapes=[tuple(info.level_shapes[l][a] for a in range(info.ndim)) for l in range(depth + 1)],
        level_offsets=[info.level_offsets[l] for l in range(depth + 2)],
        n_xi=info.n_xi, n_out=info.n_out, workspace_elems=info.workspace_elems,
        metric_workspace_elems=info.metric_workspace_elems, device_bytes=info.device_bytes,
        level_sets=[info.level_sets[l] for l in range(depth)],
        hypergrad_workspace_elems=info.hypergrad_workspace_elems)


def icr_plan_copy_level0(plan: Plan) -> np.ndarray:
    n0 = plan.info["level_offsets"][1]
    out = np.empty((n0, n0), dtype=np.float64)
    _check(load_library().icr_plan_copy_level0(plan.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def icr_plan_copy_refinement(plan: Plan, level: int):
    """R_l and sqrtD_l in FP64: one pair on a regular grid, else (level_sets[l], ...)."""
    d = plan.info["ndim"]
    nsets = plan.info["level_sets"][level]
    r = np.empty((nsets, 2 ** d, 3 ** d), dtype=np.float64)
    s = np.empty((nsets, 2 ** d, 2 ** d), dtype=np.float64)
    _check(load_library().icr_plan_copy_refinement(plan.handle, level, r.ctypes.data_as(ctypes.c_void_p),
                                                   s.ctypes.data_as(ctypes.c_void_p)))
    if plan.info["chart"] == 0:
        return r[0], s[0]
    return r, s


def icr_plan_set_level0(plan: Plan, l00: np.ndarray, stream=None):
    n0 = plan.info["level_offsets"][1]
    a = np.ascontiguousarray(l00, dtype=np.float64)
    if a.shape != (n0, n0):
        raise ValueError(f"l00 must be ({n0}, {n0})")
    _check(load_library().icr_plan_set_level0(plan.handle, a.ctypes.data_as(ctypes.c_void_p),
                                              _stream_handle(stream)))


def icr_plan_set_refinement(plan: Plan, level: int, r: np.ndarray, sqrtd: np.ndarray, stream=None):
    d = plan.info["ndim"]
    nsets = plan.info["level_sets"][level]
    ra = np.ascontiguousarray(np.reshape(r, (nsets, 2 ** d, 3 ** d)), dtype=np.float64)
    sa = np.ascontiguousarray(np.reshape(sqrtd, (nsets, 2 ** d, 2 ** d)), dtype=np.float64)
    _check(load_library().icr_plan_set_refinement(plan.handle, level, ra.ctypes.data_as(ctypes.c_void_p),
                                                  sa.ctypes.data_as(ctypes.c_void_p),
                                                  _stream_handle(stream)))


def _batch_of(t, n):
    if t.dim() == 1:
        if t.numel() != n:
            raise ValueError(f"expected {n} elements, got {t.numel()}")
        return 1
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError(f"expected shape (batch, {n}), got {tuple(t.shape)}")
    return t.shape[0]


def _check_tensor(t, plan, name, shape=None, dtype=None):
    """Shape (when given), device, dtype and contiguity of a tensor the library reads or
    writes. The C ABI sees only pointers, so this is where sizes are enforced."""
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    dtype = dtype or plan.dtype
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _lead(t):
    """Leading shape of a batched (batch, n) or single (n,) tensor."""
    return tuple(t.shape[:-1])


def _check_numel(t, plan, name, need, dtype=None):
    """A flat buffer (workspace, level stack) of at least `need` elements."""
    if t.numel() < need:
        raise ValueError(f"{name} needs at least {need} elements, got {t.numel()}")
    _check_tensor(t, plan, name, dtype=dtype)


def _check_bytes(t, name, need):
    if t.numel() * t.element_size() < need:
        raise ValueError(f"{name} needs at least {need} bytes, got {t.numel() * t.element_size()}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")


def _empty(shape, plan, dtype=None):
    import torch
    return torch.empty(shape, dtype=dtype or plan.dtype, device="cuda")


def workspace_for(plan: Plan, batch: int, metric: bool = False):
    n = plan.info["metric_workspace_elems" if metric else "workspace_elems"]
    return _empty((batch, max(n, 1)), plan)


def icr_forward(plan: Plan, xi, s=None, workspace=None, stream=None):
    batch = _batch_of(xi, plan.info["n_xi"])
    _check_tensor(xi, plan, "xi")
    if s is None:
        s = _empty(xi.shape[:-1] + (plan.info["n_out"],), plan)
    _check_tensor(s, plan, "s", shape=_lead(xi) + (plan.info["n_out"],))
    if workspace is None:
        workspace = workspace_for(plan, batch)
    _check_numel(workspace, plan, "workspace", batch * plan.info["workspace_elems"])
    _check(load_library().icr_forward(plan.handle, batch, xi.data_ptr(), s.data_ptr(),
                                      workspace.data_ptr(), _stream_handle(stream)))
    return s


def icr_adjoint(plan: Plan, s_bar, xi_bar=None, workspace=None, stream=None):
    batch = _batch_of(s_bar, plan.info["n_out"])
    _check_tensor(s_bar, plan, "s_bar")
    if xi_bar is None:
        xi_bar = _empty(s_bar.shape[:-1] + (plan.info["n_xi"],), plan)
    _check_tensor(xi_bar, plan, "xi_bar", shape=_lead(s_bar) + (plan.info["n_xi"],))
    if workspace is None:
        workspace = workspace_for(plan, batch)
    _check_numel(workspace, plan, "workspace", batch * plan.info["workspace_elems"])
    _check(load_library().icr_adjoint(plan.handle, batch, s_bar.data_ptr(), xi_bar.data_ptr(),
                                      workspace.data_ptr(), _stream_handle(stream)))
    return xi_bar


def icr_metric_apply(plan: Plan, w, v, out=None, workspace=None, stream=None):
    batch = _batch_of(v, plan.info["n_xi"])
    _check_tensor(v, plan, "v")
    w_stride = _weights(plan, w, batch)
    if out is None:
        out = _empty(v.shape, plan)
    _check_tensor(out, plan, "out", shape=tuple(v.shape))
    if workspace is None:
        workspace = workspace_for(plan, batch, metric=True)
    _check_numel(workspace, plan, "workspace", batch * plan.info["metric_workspace_elems"])
    _check(load_library().icr_metric_apply(plan.handle, batch, w.data_ptr(), w_stride, v.data_ptr(),
                                           out.data_ptr(), workspace.data_ptr(), _stream_handle(stream)))
    return out


def icr_metric_apply_static(plan: Plan, w, v, out=None, stream=None):
    """icr_metric_apply with the library's static device scratch as its workspace (no
    allocation in the library; at most 64 MiB of workspace: batch * n_xi elements)."""
    batch = _batch_of(v, plan.info["n_xi"])
    _check_tensor(v, plan, "v")
    w_stride = _weights(plan, w, batch)
    if out is None:
        out = _empty(v.shape, plan)
    _check_tensor(out, plan, "out", shape=tuple(v.shape))
    _check(load_library().icr_metric_apply_static(plan.handle, batch, w.data_ptr(), w_stride, v.data_ptr(),
                                                  out.data_ptr(), _stream_handle(stream)))
    return out


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stride(t):
    return 0 if t is None else (t.stride(0) if t.dim() > 1 else t.numel())


def icr_hyper_grad(plan: Plan, xi, s, s_levels, s_bar, sbar_levels, grad=None, workspace=None, stream=None):
    """(dE/dsigma, dE/dlength) of E = <s_bar, L xi> per sample, float64 (batch, 2), from a
    forward (xi -> s, workspace s_levels) and an adjoint (s_bar, workspace sbar_levels)."""
    import torch
    batch = _batch_of(xi, plan.info["n_xi"])
    _check_tensor(xi, plan, "xi")
    out_shape = _lead(xi) + (plan.info["n_out"],)
    _check_tensor(s, plan, "s", shape=out_shape)
    _check_tensor(s_bar, plan, "s_bar", shape=out_shape)
    for t, name in ((s_levels, "s_levels"), (sbar_levels, "sbar_levels")):
        _check_numel(t, plan, name, batch * plan.info["workspace_elems"])
    if grad is None:
        grad = torch.empty((batch, 2), dtype=torch.float64, device=xi.device)
    if workspace is None:
        workspace = torch.empty((batch, max(plan.info["hypergrad_workspace_elems"], 1)), dtype=torch.float64,
                                device=xi.device)
    _check_numel(grad, plan, "grad", 2 * batch, dtype=torch.float64)
    _check_numel(workspace, plan, "workspace", batch * plan.info["hypergrad_workspace_elems"],
                 dtype=torch.float64)
    _check(load_library().icr_hyper_grad(plan.handle, batch, xi.data_ptr(), s.data_ptr(), s_levels.data_ptr(),
                                         s_bar.data_ptr(), sbar_levels.data_ptr(), grad.data_ptr(),
                                         workspace.data_ptr(), _stream_handle(stream)))
    return grad


def hyper_grad(plan: Plan, xi, s_bar, stream=None):
    """Forward, adjoint and icr_hyper_grad in one call: returns (s, xi_bar, grad)."""
    batch = _batch_of(xi, plan.info["n_xi"])
    ws_f = workspace_for(plan, batch)
    ws_a = workspace_for(plan, batch)
    s = icr_forward(plan, xi, workspace=ws_f, stream=stream)
    xi_bar = icr_adjoint(plan, s_bar, workspace=ws_a, stream=stream)
    grad = icr_hyper_grad(plan, xi, s, ws_f, s_bar, ws_a, stream=stream)
    return s, xi_bar, grad


def _level_sizes(plan: Plan, level: int):
    """(coarse, fine) element counts of refinement `level` (level -1: level 0 alone)."""
    offs = plan.info["level_offsets"]
    depth = plan.info["depth"]
    if not -1 <= level < depth:
        raise ValueError(f"level must be in -1 .. {depth - 1}")
    fine = offs[level + 2] - offs[level + 1]
    coarse = 0 if level < 0 else offs[level + 1] - offs[level]
    return coarse, fine


def _check_level_view(t, plan, name, size, batch):
    """A (batch, size) view (rows may be strided) or a (size,) vector for batch 1."""
    if t is None:
        return
    shape = (size,) if t.dim() == 1 else (batch, size)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    if not t.is_cuda or t.dtype != plan.dtype:
        raise ValueError(f"{name} must be a device tensor of {plan.dtype}")
    if t.stride(-1) != 1:
        raise ValueError(f"{name} rows must be contiguous")


def icr_forward_level(plan: Plan, level: int, s_coarse, xi_fine, s_fine, stream=None):
    """One forward level on (batch, size) views; level -1 is the level-0 factor."""
    batch = xi_fine.shape[0] if xi_fine.dim() > 1 else 1
    n_c, n_f = _level_sizes(plan, level)
    _check_level_view(xi_fine, plan, "xi_fine", n_f, batch)
    _check_level_view(s_fine, plan, "s_fine", n_f, batch)
    if level >= 0:
        if s_coarse is None:
            raise ValueError("s_coarse is required for a refinement level")
        _check_level_view(s_coarse, plan, "s_coarse", n_c, batch)
    _check(load_library().icr_forward_level(plan.handle, level, batch, _ptr(s_coarse), _stride(s_coarse),
                                            _ptr(xi_fine), xi_fine.stride(0) if xi_fine.dim() > 1 else xi_fine.numel(),
                                            _ptr(s_fine), s_fine.stride(0) if s_fine.dim() > 1 else s_fine.numel(),
                                            _stream_handle(stream)))
    return s_fine


def icr_adjoint_level(plan: Plan, level: int, y_fine, xi_bar_fine, s_bar_coarse, stream=None):
    """One adjoint level on (batch, size) views; level -1 is the level-0 factor."""
    batch = y_fine.shape[0] if y_fine.dim() > 1 else 1
    n_c, n_f = _level_sizes(plan, level)
    _check_level_view(y_fine, plan, "y_fine", n_f, batch)
    _check_level_view(xi_bar_fine, plan, "xi_bar_fine", n_f, batch)
    if level >= 0:
        if s_bar_coarse is None:
            raise ValueError("s_bar_coarse is required for a refinement level")
        _check_level_view(s_bar_coarse, plan, "s_bar_coarse", n_c, batch)
    st = lambda t: 0 if t is None else (t.stride(0) if t.dim() > 1 else t.numel())
    _check(load_library().icr_adjoint_level(plan.handle, level, batch, _ptr(y_fine), st(y_fine),
                                            _ptr(xi_bar_fine), st(xi_bar_fine), _ptr(s_bar_coarse),
                                            st(s_bar_coarse), _stream_handle(stream)))
    return xi_bar_fine


def icr_cg_workspace_bytes(plan: Plan, batch: int) -> int:
    out = ctypes.c_int64()
    _check(load_library().icr_cg_workspace_bytes(plan.handle, batch, ctypes.byref(out)))
    return out.value


def icr_cg_metric(plan: Plan, w, b, iterations: int, x=None, residual_norms=False, workspace=None,
                  stream=None, absdelta=None, iterations_done=None):
    """Solve (L^T W L + 1) x = b by `iterations` CG steps on the device (x_0 = 0).

    With absdelta (> 0) a sample stops after the first step that lowers the CG energy
    x.Mx/2 - b.x by less than absdelta, `iterations` being the maximum
    (icr_cg_metric_sl); iterations_done, an int32 device tensor (batch,), then receives
    the steps each sample took. Returns x, or (x, norms) with
    norms[batch][iterations + 1] = |r_k| when asked."""
    import torch
    batch = _batch_of(b, plan.info["n_xi"])
    _check_tensor(b, plan, "b")
    w_stride = _weights(plan, w, batch)
    if x is None:
        x = _empty(b.shape, plan)
    _check_tensor(x, plan, "x", shape=tuple(b.shape))
    if iterations < 0:
        raise ValueError("iterations must be >= 0")
    if workspace is None:
        workspace = torch.empty(icr_cg_workspace_bytes(plan, batch), dtype=torch.uint8, device="cuda")
    _check_bytes(workspace, "workspace", icr_cg_workspace_bytes(plan, batch))
    norms = torch.empty((batch, iterations + 1), dtype=torch.float64, device="cuda") if residual_norms else None
    if absdelta is None:
        if iterations_done is not None:
            raise ValueError("iterations_done needs absdelta")
        _check(load_library().icr_cg_metric(plan.handle, batch, w.data_ptr(), w_stride, b.data_ptr(), x.data_ptr(),
                                            iterations, _ptr(norms), workspace.data_ptr(), _stream_handle(stream)))
    else:
        if iterations_done is not None:
            _check_tensor(iterations_done, plan, "iterations_done", shape=(batch,), dtype=torch.int32)
        _check(load_library().icr_cg_metric_sl(plan.handle, batch, w.data_ptr(), w_stride, b.data_ptr(),
                                               x.data_ptr(), float(absdelta), iterations, _ptr(iterations_done),
                                               _ptr(norms), workspace.data_ptr(), _stream_handle(stream)))
    return (x, norms) if residual_norms else x


def _weights(plan, w, batch):
    """Batch stride of the weights: (n_out,) is shared by every sample (stride 0),
    (batch, n_out) gives each sample its own row."""
    n_out = plan.info["n_out"]
    if w.dim() == 1:
        if w.numel() != n_out:
            raise ValueError(f"w must have {n_out} elements, got {w.numel()}")
        stride = 0
    elif tuple(w.shape) == (batch, n_out):
        stride = n_out
    else:
        raise ValueError(f"w must have shape ({n_out},) or ({batch}, {n_out}), got {tuple(w.shape)}")
    if w.dtype != plan.acc_dtype or not w.is_cuda or not w.is_contiguous():
        raise ValueError(f"w must be a contiguous device tensor of {plan.acc_dtype}")
    return stride


def icr_weighted_adjoint(plan: Plan, w, y, add=None, half=True, out=None, workspace=None, stream=None):
    """out = L^T (w^(1/2 if half else 1) * y) + add (add may be None)."""
    batch = _batch_of(y, plan.info["n_out"])
    _check_tensor(y, plan, "y")
    w_stride = _weights(plan, w, batch)
    xi_shape = _lead(y) + (plan.info["n_xi"],)
    if add is not None:
        _check_tensor(add, plan, "add", shape=xi_shape)
    if out is None:
        out = _empty(xi_shape, plan)
    _check_tensor(out, plan, "out", shape=xi_shape)
    if workspace is None:
        workspace = workspace_for(plan, batch, metric=True)
    _check_numel(workspace, plan, "workspace", batch * plan.info["metric_workspace_elems"])
    _check(load_library().icr_weighted_adjoint(plan.handle, batch, w.data_ptr(), w_stride, 1 if half else 0,
                                               y.data_ptr(), _ptr(add), out.data_ptr(), workspace.data_ptr(),
                                               _stream_handle(stream)))
    return out


def icr_mgvi_workspace_bytes(plan: Plan, batch: int) -> int:
    out = ctypes.c_int64()
    _check(load_library().icr_mgvi_workspace_bytes(plan.handle, batch, ctypes.byref(out)))
    return out.value


def icr_mgvi_newton_step(plan: Plan, w, b, mean, iterations: int, residual_norms=False, workspace=None,
                         stream=None):
    """mean <- mean - M^-1 (M mean - b) in place (CG with `iterations` steps); returns mean
    (and the CG residual norms when asked)."""
    import torch
    batch = _batch_of(mean, plan.info["n_xi"])
    _check_tensor(mean, plan, "mean")
    _check_tensor(b, plan, "b", shape=tuple(mean.shape))
    w_stride = _weights(plan, w, batch)
    if iterations < 0:
        raise ValueError("iterations must be >= 0")
    if workspace is None:
        workspace = torch.empty(icr_mgvi_workspace_bytes(plan, batch), dtype=torch.uint8, device="cuda")
    _check_bytes(workspace, "workspace", icr_mgvi_workspace_bytes(plan, batch))
    norms = torch.empty((batch, iterations + 1), dtype=torch.float64, device="cuda") if residual_norms else None
    _check(load_library().icr_mgvi_newton_step(plan.handle, batch, w.data_ptr(), w_stride, b.data_ptr(),
                                               mean.data_ptr(), iterations, _ptr(norms), workspace.data_ptr(),
                                               _stream_handle(stream)))
    return (mean, norms) if residual_norms else mean


def mgvi(plan: Plan, w, d, n_pairs: int = 3, n_iterations: int = 3, sample_iterations: int = 100,
         newton_iterations: int = 35, seed: int = 0, mean=None, stream=None, absdelta=None):
    """MGVI with antithetic samples: per iteration draw n_pairs sample displacements
    delta = M^-1 (eta + L^T (sqrt(w) eta')) (CG) around the current mean, then one
    Newton-CG step of the mean. The samples' CG runs sample_iterations steps, or with
    absdelta stops by the energy-change rule with sample_iterations as its maximum.
    Random numbers come from numpy's PCG64 with `seed` and are uploaded; every arithmetic
    step runs in the library. Returns (mean, deltas); the samples are mean + deltas and
    mean - deltas."""
    import numpy as _np
    import torch
    n_xi, n_out = plan.info["n_xi"], plan.info["n_out"]
    rng = _np.random.default_rng(seed)
    b = icr_weighted_adjoint(plan, w, d.reshape(1, n_out), half=False, stream=stream)
    mean = torch.zeros((1, n_xi), dtype=plan.dtype, device="cuda") if mean is None else mean.reshape(1, n_xi)
    deltas = None
    for _ in range(n_iterations):
        eta = torch.from_numpy(rng.standard_normal((n_pairs, n_xi))).to("cuda").to(plan.dtype)
        eta_d = torch.from_numpy(rng.standard_normal((n_pairs, n_out))).to("cuda").to(plan.dtype)
        deltas = mgvi_step(plan, w, b, mean, eta, eta_d, sample_iterations, newton_iterations, stream=stream,
                           absdelta=absdelta)
    return mean[0], deltas


def mgvi_step(plan: Plan, w, b, mean, eta, eta_d, sample_iterations: int, newton_iterations: int,
              workspaces=None, stream=None, absdelta=None, iterations_done=None):
    """The device work of one MGVI iteration for given standard-normal draws eta
    (pairs, n_xi) and eta_d (pairs, n_out): the sample displacements (returned) and the
    Newton-CG step of `mean` (updated in place); b = L^T W d. workspaces: optional
    (weighted-adjoint, CG, Newton) workspaces to reuse. absdelta: stop the samples' CG
    by the energy-change rule (sample_iterations is then the maximum)."""
    ws_a, ws_cg, ws_n = workspaces if workspaces is not None else (None, None, None)
    r = icr_weighted_adjoint(plan, w, eta_d, add=eta, half=True, workspace=ws_a, stream=stream)
    deltas = icr_cg_metric(plan, w, r, sample_iterations, workspace=ws_cg, stream=stream, absdelta=absdelta,
                           iterations_done=iterations_done)
    icr_mgvi_newton_step(plan, w, b, mean, newton_iterations, workspace=ws_n, stream=stream)
    return deltas


def icr_plan_destroy(plan: Plan):
    if plan.handle:
        h, plan.handle = plan.handle, None
        _check(load_library().icr_plan_destroy(h))


def icr_version() -> int:
    return int(load_library().icr_version())
