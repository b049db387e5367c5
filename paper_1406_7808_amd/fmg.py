"""Python binding of the HIP solver library (include/fmg.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``libfmg.so``.  torch supplies device memory and the current stream.  There
is no fallback: if the library is missing, importing a function raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.environ.get("FMG_LIB") or os.path.join(_HERE, "libfmg.so")

FMG_OK, FMG_EINVAL, FMG_ENOMEM, FMG_EHIP, FMG_ENOTSUP = 0, -1, -2, -3, -4
PRECISION = {"fp64": 0, "fp32_refined": 1}


class FMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fmg status %d: %s" % (status, msg))
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("sr_levels", ctypes.c_int32),
        ("segments_per_dim", ctypes.c_int32),
        ("buffer_schedule", ctypes.POINTER(ctypes.c_int32)),
        ("nu_pre", ctypes.c_int32),
        ("nu_post", ctypes.c_int32),
        ("alpha", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
    ]


class _ScheduleStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("bytes", ctypes.c_double),
                ("workspace_bytes", ctypes.c_int64)]


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class Tuning(ctypes.Structure):
    """fmg_tuning: performance knobs of a plan (see include/fmg.h)."""
    _fields_ = [("max_stages", ctypes.c_int32), ("seg_inplace", ctypes.c_int32),
                ("box", ctypes.c_int32), ("target_blocks", ctypes.c_int32),
                ("tile_x", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
SYMBOLS = ["fmg_check_params", "fmg_plan_create", "fmg_plan_execute", "fmg_plan_vcycles",
           "fmg_plan_checkpoints", "fmg_plan_get_tuning", "fmg_plan_set_tuning",
           "fmg_plan_destroy", "fmg_solve", "fmg_plan_workspace_bytes", "fmg_plan_profile",
           "fmg_plan_profile_read", "fmg_schedule_model", "fmg_batch_create", "fmg_batch_execute",
           "fmg_batch_capture", "fmg_batch_replay", "fmg_batch_workspace_bytes",
           "fmg_batch_destroy", "fmg_last_error", "fmg_residual_norms", "fmg_diff_norms",
           "fmg_residual_norms_noalloc", "fmg_op_apply", "fmg_op_smooth", "fmg_op_restrict",
           "fmg_op_interp"]


def lib():
    """Load libfmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise ImportError("HIP library %s is missing: run __graft_entry__.build()" % _SO)
    L = ctypes.CDLL(_SO)
    vp, i32, pp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Params)
    L.fmg_check_params.argtypes = [i32, pp]
    L.fmg_check_params.restype = i32
    L.fmg_plan_create.argtypes = [i32, pp, i32, ctypes.POINTER(vp)]
    L.fmg_plan_create.restype = i32
    L.fmg_plan_execute.argtypes = [vp, vp, vp, vp]
    L.fmg_plan_execute.restype = i32
    L.fmg_plan_vcycles.argtypes = [vp, vp, vp, ctypes.c_double, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double), vp]
    L.fmg_plan_vcycles.restype = i32
    L.fmg_plan_checkpoints.argtypes = [vp, ctypes.POINTER(vp)]
    L.fmg_plan_checkpoints.restype = i32
    L.fmg_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.fmg_plan_get_tuning.restype = i32
    L.fmg_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.fmg_plan_set_tuning.restype = i32
    L.fmg_batch_create.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(_Params),
                                   ctypes.POINTER(Tuning), i32, i32, ctypes.POINTER(vp)]
    L.fmg_batch_create.restype = i32
    L.fmg_batch_execute.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.fmg_batch_execute.restype = i32
    L.fmg_batch_capture.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.fmg_batch_capture.restype = i32
    L.fmg_batch_replay.argtypes = [vp, vp]
    L.fmg_batch_replay.restype = i32
    L.fmg_batch_workspace_bytes.argtypes = [vp]
    L.fmg_batch_workspace_bytes.restype = ctypes.c_int64
    L.fmg_batch_destroy.argtypes = [vp]
    L.fmg_batch_destroy.restype = i32
    L.fmg_plan_destroy.argtypes = [vp]
    L.fmg_plan_destroy.restype = i32
    L.fmg_solve.argtypes = [vp, i32, pp, vp, vp]
    L.fmg_solve.restype = i32
    L.fmg_plan_workspace_bytes.argtypes = [vp]
    L.fmg_plan_workspace_bytes.restype = ctypes.c_int64
    L.fmg_plan_profile.argtypes = [vp, i32]
    L.fmg_plan_profile.restype = i32
    L.fmg_plan_profile_read.argtypes = [vp, ctypes.POINTER(_KernelStat), i32,
                                        ctypes.POINTER(i32)]
    L.fmg_plan_profile_read.restype = i32
    L.fmg_schedule_model.argtypes = [i32, pp, ctypes.POINTER(_ScheduleStat)]
    L.fmg_schedule_model.restype = i32
    L.fmg_last_error.argtypes = []
    L.fmg_last_error.restype = ctypes.c_char_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.fmg_residual_norms.argtypes = [vp, vp, i32, dp, vp]
    L.fmg_diff_norms.argtypes = [vp, vp, i32, dp, vp]
    L.fmg_residual_norms_noalloc.argtypes = [vp, vp, i32, vp, vp]
    L.fmg_op_apply.argtypes = [vp, i32, vp, vp]
    L.fmg_op_smooth.argtypes = [vp, vp, i32, i32, vp]
    L.fmg_op_restrict.argtypes = [vp, i32, vp, vp]
    L.fmg_op_interp.argtypes = [vp, i32, vp, vp]
    for name in ("fmg_residual_norms", "fmg_diff_norms", "fmg_residual_norms_noalloc",
                 "fmg_op_apply", "fmg_op_smooth",
                 "fmg_op_restrict", "fmg_op_interp"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(st):
    if st != FMG_OK:
        raise FMGError(st, lib().fmg_last_error().decode())


def make_params(levels, sr_levels=0, segments=1, buffers=(), sweeps=(2, 2, 1), precision="fp64",
                refine_iters=2):
    """fmg_params; sweeps = (nu_pre, nu_post, alpha); buffers finest first.
    Returns (params, keepalive) -- keep the second alive while params is used."""
    J = (ctypes.c_int32 * max(1, len(buffers)))(*buffers)
    p = _Params(levels, sr_levels, segments,
                ctypes.cast(J, ctypes.POINTER(ctypes.c_int32)) if len(buffers) else None,
                sweeps[0], sweeps[1], sweeps[2], PRECISION[precision], refine_iters)
    return p, J


def check_params(N, **kw):
    """Host-only validation; returns (status, message)."""
    p, keep = make_params(**kw)
    st = lib().fmg_check_params(N, ctypes.byref(p))
    return st, (lib().fmg_last_error().decode() if st else "")


def schedule_model(N, **kw):
    """Host-only walk of one solve's launches: (launches, algorithmic bytes,
    workspace bytes).  Raises FMGError on invalid parameters."""
    p, keep = make_params(**kw)
    st = _ScheduleStat()
    _check(lib().fmg_schedule_model(N, ctypes.byref(p), ctypes.byref(st)))
    return st.launches, st.bytes, st.workspace_bytes


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, N=None):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise FMGError(FMG_EINVAL, "expected a contiguous float64 CUDA tensor")
    if N is not None and tuple(t.shape) != (N, N, N):
        raise FMGError(FMG_EINVAL, "expected shape (%d, %d, %d)" % (N, N, N))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A solver plan: validated parameters plus all device workspace."""

    def __init__(self, N, levels, sr_levels=0, segments=1, buffers=(), sweeps=(2, 2, 1),
                 precision="fp64", refine_iters=2, device=None):
        self.N = N
        self.levels = levels
        self._ck = None
        self._p, self._keep = make_params(levels, sr_levels, segments, buffers, sweeps, precision,
                                          refine_iters)
        dev = torch.cuda.current_device() if device is None else device
        self.device = torch.device("cuda", dev)
        h = ctypes.c_void_p()
        _check(lib().fmg_plan_create(N, ctypes.byref(self._p), dev, ctypes.byref(h)))
        self._h = h

    @property
    def workspace_bytes(self):
        return lib().fmg_plan_workspace_bytes(self._h)

    def execute(self, f, u=None, stream=None):
        """Enqueue u <- FMG(f) on the stream (default: torch's current)."""
        if u is None:
            u = torch.empty_like(f)
        _check(lib().fmg_plan_execute(self._h, _dev(f, self.N), _dev(u, self.N), _stream(stream)))
        return u

    def level_edges(self):
        return [self.N >> (self.levels - 1 - l) for l in range(self.levels)]

    def set_checkpoints(self, bufs):
        """Per-level checkpoint arrays (a list of `levels` float64 CUDA
        tensors of shape (n_l,)*3, or None entries); None clears them."""
        if bufs is None:
            self._ck = None
            _check(lib().fmg_plan_checkpoints(self._h, None))
            return
        edges = self.level_edges()
        arr = (ctypes.c_void_p * self.levels)()
        for l, b in enumerate(bufs):
            arr[l] = None if b is None else _dev(b, edges[l]).value
        self._ck = list(bufs)  # keep them alive while set
        _check(lib().fmg_plan_checkpoints(self._h, arr))

    @property
    def tuning(self):
        t = Tuning()
        _check(lib().fmg_plan_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change performance knobs (max_stages, seg_inplace, box, target_blocks, tile_x)."""
        t = Tuning(**{**self.tuning, **kw})
        _check(lib().fmg_plan_set_tuning(self._h, ctypes.byref(t)))

    def vcycles(self, f, u, rtol=1e-4, maxit=50, stream=None, residual=True):
        """V(nu1, nu2) cycles from the guess in u (updated in place) until
        max|f - L u| <= rtol max|f| or maxit cycles; returns (cycles, relres).
        Global FP64 plans only.  Synchronizes the stream once per cycle;
        rtol=0 runs exactly maxit cycles with one residual check at the end;
        rtol=0 with residual=False only enqueues the cycles (no residual, no
        synchronization, capturable into a graph) and returns (maxit, None)."""
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        _check(lib().fmg_plan_vcycles(self._h, _dev(f, self.N), _dev(u, self.N), float(rtol),
                                      int(maxit), ctypes.byref(it),
                                      ctypes.byref(rr) if residual else None, _stream(stream)))
        return it.value, (rr.value if residual else None)

    def profile(self, enable=True):
        """Start (or stop) per-launch event timing; clears pending records."""
        _check(lib().fmg_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms, algorithmic bytes)} since the last read."""
        cap = 64
        buf = (_KernelStat * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().fmg_plan_profile_read(self._h, buf, cap, ctypes.byref(cnt)))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].bytes)
                for i in range(min(cnt.value, cap))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fmg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent solves of possibly different sizes, run side by side on
    internal streams; capture() records them into one HIP graph, replay()
    launches it.  problems: dicts of Plan's keyword arguments plus "N";
    tunings: None or one dict (or None) per problem."""

    def __init__(self, problems, streams=4, tunings=None, device=None):
        self.count = len(problems)
        self.N = [int(p["N"]) for p in problems]
        params = (_Params * self.count)()
        self._keep = []
        for i, p in enumerate(problems):
            kw = {k: v for k, v in p.items() if k != "N"}
            levels = kw.pop("levels")
            buffers = kw.pop("buffers", ())
            segments = kw.pop("segments", 1)
            pp, keep = make_params(levels, buffers=buffers, segments=segments, **kw)
            params[i] = pp
            self._keep.append(keep)
        tun = None
        if tunings is not None:
            tun = (Tuning * self.count)()
            for i, t in enumerate(tunings):
                tun[i] = Tuning(**{**DEFAULT_TUNING, **(t or {})})
        Ns = (ctypes.c_int32 * self.count)(*self.N)
        dev = torch.cuda.current_device() if device is None else device
        h = ctypes.c_void_p()
        _check(lib().fmg_batch_create(self.count, Ns, params, tun, streams, dev, ctypes.byref(h)))
        self._h = h
        self._io = None

    @property
    def workspace_bytes(self):
        return lib().fmg_batch_workspace_bytes(self._h)

    def _ptrs(self, fs, us):
        if len(fs) != self.count or len(us) != self.count:
            raise FMGError(FMG_EINVAL, "expected %d right-hand sides and solutions" % self.count)
        F = (ctypes.c_void_p * self.count)(*[_dev(f, n).value for f, n in zip(fs, self.N)])
        U = (ctypes.c_void_p * self.count)(*[_dev(u, n).value for u, n in zip(us, self.N)])
        return F, U

    def execute(self, fs, us, stream=None):
        F, U = self._ptrs(fs, us)
        _check(lib().fmg_batch_execute(self._h, F, U, _stream(stream)))
        return us

    def capture(self, fs, us, stream):
        """Record the batch for these tensors (kept alive) into one graph."""
        F, U = self._ptrs(fs, us)
        _check(lib().fmg_batch_capture(self._h, F, U, _stream(stream)))
        self._io = (list(fs), list(us))

    def replay(self, stream=None):
        _check(lib().fmg_batch_replay(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DEFAULT_TUNING = {"max_stages": 4, "seg_inplace": 1, "box": 1, "target_blocks": 0, "tile_x": 0}


def solve(f, levels, sr_levels=0, segments=1, buffers=(), sweeps=(2, 2, 1), precision="fp64",
          refine_iters=2):
    """u = FMG(f) for a (N, N, N) float64 CUDA tensor f (synchronous)."""
    N = f.shape[0]
    u = torch.empty_like(f)
    p, keep = make_params(levels, sr_levels, segments, buffers, sweeps, precision, refine_iters)
    _check(lib().fmg_solve(_dev(f, N), N, ctypes.byref(p), _dev(u, N), _stream(None)))
    return u


def residual_norms(f, u, stream=None):
    """(max |f - L u|, sqrt(h^3 sum (f - L u)^2)) over the N^3 grid."""
    N = f.shape[0]
    out = (ctypes.c_double * 2)()
    _check(lib().fmg_residual_norms(_dev(f, N), _dev(u, N), N, out, _stream(stream)))
    return out[0], out[1]


def residual_norms_noalloc(f, u, out, stream=None):
    """The same norms into `out` (a float64 CUDA tensor of 2 entries), with
    no allocation and no synchronization: only two kernels are enqueued."""
    N = f.shape[0]
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            and out.numel() >= 2):
        raise FMGError(FMG_EINVAL, "out must be a contiguous float64 CUDA tensor of 2 entries")
    _check(lib().fmg_residual_norms_noalloc(_dev(f, N), _dev(u, N), N,
                                            ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def diff_norms(u, v, stream=None):
    """(max |u - v|, sqrt(h^3 sum (u - v)^2)) over the N^3 grid."""
    N = u.shape[0]
    out = (ctypes.c_double * 2)()
    _check(lib().fmg_diff_norms(_dev(u, N), _dev(v, N), N, out, _stream(stream)))
    return out[0], out[1]


def op_apply(u):
    out = torch.empty_like(u)
    _check(lib().fmg_op_apply(_dev(u, u.shape[0]), u.shape[0], _dev(out), _stream(None)))
    return out


def op_smooth(u, rhs, nu):
    """nu red-black sweeps on u in place."""
    _check(lib().fmg_op_smooth(_dev(u, u.shape[0]), _dev(rhs, u.shape[0]), u.shape[0], nu,
                               _stream(None)))
    return u


def op_restrict(v):
    n = v.shape[0]
    out = torch.empty((n // 2,) * 3, dtype=v.dtype, device=v.device)
    _check(lib().fmg_op_restrict(_dev(v, n), n, _dev(out), _stream(None)))
    return out


def op_interp(v):
    n = v.shape[0]
    out = torch.empty((2 * n,) * 3, dtype=v.dtype, device=v.device)
    _check(lib().fmg_op_interp(_dev(v, n), n, _dev(out), _stream(None)))
    return out
