"""Python binding of the 27-point model-problem solver (include/fv27.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``libfmg.so``; torch supplies device memory and the current stream.  Arrays
are float64 CUDA tensors of shape (n2, n1, n0) indexed [z, y, x].
"""
import ctypes

import torch

from . import fmg
from .fmg import FMGError, FMG_EINVAL

SYMBOLS = ["fv27_check_params", "fv27_plan_create", "fv27_plan_execute", "fv27_plan_destroy",
           "fv27_plan_workspace_bytes", "fv27_plan_model", "fv27_op_apply", "fv27_op_cheb",
           "fv27_op_prolong", "fv27_last_error"]


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("h", ctypes.c_double),
        ("levels", ctypes.c_int32),
        ("sr_levels", ctypes.c_int32),
        ("segments", ctypes.c_int32 * 3),
        ("buffer_schedule", ctypes.POINTER(ctypes.c_int32)),
        ("cheb_pre", ctypes.c_int32),
        ("cheb_post", ctypes.c_int32),
        ("cheb_fmg", ctypes.c_int32),
    ]


_bound = None


def lib():
    global _bound
    L = fmg.lib()
    if _bound is L:
        return L
    vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    pp = ctypes.POINTER(_Params)
    ip = ctypes.POINTER(ctypes.c_int32)
    L.fv27_check_params.argtypes = [pp]
    L.fv27_plan_create.argtypes = [pp, i32, ctypes.POINTER(vp)]
    L.fv27_plan_execute.argtypes = [vp, vp, vp, vp]
    L.fv27_plan_destroy.argtypes = [vp]
    L.fv27_plan_workspace_bytes.argtypes = [vp]
    L.fv27_plan_workspace_bytes.restype = ctypes.c_int64
    L.fv27_plan_model.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(d)]
    L.fv27_op_apply.argtypes = [vp, ip, d, vp, vp]
    L.fv27_op_cheb.argtypes = [vp, vp, ip, d, i32, vp]
    L.fv27_op_prolong.argtypes = [vp, ip, vp, vp]
    L.fv27_last_error.argtypes = []
    L.fv27_last_error.restype = ctypes.c_char_p
    for name in ("fv27_check_params", "fv27_plan_create", "fv27_plan_execute", "fv27_plan_destroy",
                 "fv27_plan_model", "fv27_op_apply", "fv27_op_cheb", "fv27_op_prolong"):
        getattr(L, name).restype = i32
    _bound = L
    return L


def _check(st):
    if st != 0:
        raise FMGError(st, lib().fv27_last_error().decode())


def make_params(n, h, levels, sr_levels=0, segments=(1, 1, 1), buffers=(), degrees=(2, 2, 1)):
    """fv27_params; n = (n0, n1, n2) finest extents (x first); buffers finest
    first; degrees = (pre, post, fmg) Chebyshev degrees.  Returns (params,
    keepalive)."""
    J = (ctypes.c_int32 * max(1, len(buffers)))(*buffers)
    p = _Params((ctypes.c_int32 * 3)(*n), float(h), levels, sr_levels,
                (ctypes.c_int32 * 3)(*segments),
                ctypes.cast(J, ctypes.POINTER(ctypes.c_int32)) if len(buffers) else None,
                degrees[0], degrees[1], degrees[2])
    return p, J


def check_params(**kw):
    p, keep = make_params(**kw)
    st = lib().fv27_check_params(ctypes.byref(p))
    return st, (lib().fv27_last_error().decode() if st else "")


def _dev(t, shape=None):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise FMGError(FMG_EINVAL, "expected a contiguous float64 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise FMGError(FMG_EINVAL, "expected shape %s" % (tuple(shape),))
    return ctypes.c_void_p(t.data_ptr())


def _ext(t):
    return (ctypes.c_int32 * 3)(t.shape[2], t.shape[1], t.shape[0])


class Plan:
    """A plan for the model problem: validated parameters and all workspace."""

    def __init__(self, n, h, levels, sr_levels=0, segments=(1, 1, 1), buffers=(),
                 degrees=(2, 2, 1), device=None):
        self.n = tuple(n)
        self.shape = (n[2], n[1], n[0])
        self._p, self._keep = make_params(n, h, levels, sr_levels, segments, buffers, degrees)
        dev = torch.cuda.current_device() if device is None else device
        h_ = ctypes.c_void_p()
        _check(lib().fv27_plan_create(ctypes.byref(self._p), dev, ctypes.byref(h_)))
        self._h = h_

    @property
    def workspace_bytes(self):
        return lib().fv27_plan_workspace_bytes(self._h)

    def model(self):
        """(launches, algorithmic bytes) of one execute."""
        n = ctypes.c_int64(0)
        b = ctypes.c_double(0.0)
        _check(lib().fv27_plan_model(self._h, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def execute(self, f, u=None, stream=None):
        if u is None:
            u = torch.empty_like(f)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().fv27_plan_execute(self._h, _dev(f, self.shape), _dev(u, self.shape),
                                       ctypes.c_void_p(s.cuda_stream)))
        return u

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fv27_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(f, h, levels, sr_levels=0, segments=(1, 1, 1), buffers=(), degrees=(2, 2, 1)):
    n = (f.shape[2], f.shape[1], f.shape[0])
    plan = Plan(n, h, levels, sr_levels, segments, buffers, degrees, device=f.device.index)
    u = plan.execute(f)
    torch.cuda.current_stream().synchronize()
    plan.close()
    return u


def op_apply(u, h):
    out = torch.empty_like(u)
    _check(lib().fv27_op_apply(_dev(u), _ext(u), float(h), _dev(out),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def op_cheb(u, rhs, h, degree):
    u = u.clone()
    _check(lib().fv27_op_cheb(_dev(u), _dev(rhs, u.shape), _ext(u), float(h), int(degree),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return u


def op_prolong(v):
    out = torch.empty(tuple(2 * s for s in v.shape), dtype=torch.float64, device=v.device)
    _check(lib().fv27_op_prolong(_dev(v), _ext(v), _dev(out),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out
