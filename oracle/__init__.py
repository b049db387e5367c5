"""Plain FP64 CPU oracle for segmental-refinement FMG (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path
(``paper_1406_7808_amd``) never imports it and shares no code with it.

``build()`` compiles ``fmg_oracle.c`` with gcc; ``lib()`` loads it.  The
wrappers take and return numpy float64 arrays of shape (N, N, N) indexed
[z, y, x] (x fastest), the same layout as the HIP library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmg_oracle.c")
_SO = os.path.join(_HERE, "libfmg_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(verbose=False):
    """Compile the oracle into oracle/libfmg_oracle.so (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    global _lib
    _lib = None


def build_native(out_dir, verbose=False):
    """The timing build: the same source with -O3 -march=native for the CPU
    it is compiled on (so it is built where it runs, never shipped), into
    out_dir/libfmg_oracle_native.so.  ISO C11 mode keeps gcc from contracting
    multiply-adds, so its results equal the test build's.  Returns the path."""
    so = os.path.join(out_dir, "libfmg_oracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", so + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(so + ".tmp", so)
    return so


def use_library(path):
    """Load the oracle from another build of the same source (the timing
    build); later calls of this module go to it."""
    global _lib
    _lib = None
    _bind(ctypes.CDLL(path))
    return _lib


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    return _bind(ctypes.CDLL(_SO))


def _bind(L):
    global _lib
    i, d = ctypes.c_int, ctypes.c_double
    L.orc_fmg.argtypes = [_dp, i, i, i, i, i, _dp]
    L.orc_srfmg.argtypes = [_dp, i, i, i, i, _ip, i, i, i, _dp]
    L.orc_srfmg_refined.argtypes = [_dp, i, i, i, i, _ip, i, i, i, i, _dp]
    L.orc_vcycles.argtypes = [_dp, i, i, i, i, d, i, _dp, _dp]
    L.orc_apply.argtypes = [_dp, i, _dp]
    L.orc_apply.restype = None
    L.orc_gs_half.argtypes = [_dp, _dp, i, i]
    L.orc_gs_half.restype = None
    L.orc_smooth.argtypes = [_dp, _dp, i, i]
    L.orc_smooth.restype = None
    L.orc_restrict.argtypes = [_dp, i, _dp]
    L.orc_restrict.restype = None
    L.orc_prolong.argtypes = [_dp, i, _dp]
    L.orc_prolong.restype = None
    L.orc_interp.argtypes = [_dp, i, _dp]
    L.orc_interp.restype = None
    L.orc_coarse_solve.argtypes = [_dp, i, _dp]
    L.orc_threads.argtypes = []
    L.orc_set_threads.argtypes = [i]
    L.orc_set_threads.restype = None
    _lib = L
    return L


def _p(a):
    return a.ctypes.data_as(_dp)


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _check(st):
    if st < 0:
        raise ValueError("oracle rejected the parameters (status %d)" % st)
    return st


def threads():
    return lib().orc_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def fmg(f, levels, alpha=1, nu1=2, nu2=2):
    """Global FMG F(alpha, nu1, nu2) on an N^3 right-hand side."""
    f = _arr(f)
    N = f.shape[0]
    u = np.zeros_like(f)
    _check(lib().orc_fmg(_p(f), N, levels, alpha, nu1, nu2, _p(u)))
    return u


def srfmg(f, levels, sr_levels, segments, buffers, alpha=1, nu1=2, nu2=2):
    """FMG with segmental refinement on the finest sr_levels levels.
    buffers: sr_levels buffer widths, finest level first."""
    f = _arr(f)
    N = f.shape[0]
    u = np.zeros_like(f)
    J = (ctypes.c_int * max(1, len(buffers)))(*buffers)
    _check(lib().orc_srfmg(_p(f), N, levels, sr_levels, segments, J, alpha, nu1, nu2, _p(u)))
    return u


def srfmg_refined(f, levels, sr_levels, segments, buffers, iters=2, alpha=1, nu1=2, nu2=2):
    """u = SRFMG(f), then `iters` FP64 residual corrections u += SRFMG(f - L u)."""
    f = _arr(f)
    N = f.shape[0]
    u = np.zeros_like(f)
    J = (ctypes.c_int * max(1, len(buffers)))(*buffers)
    _check(lib().orc_srfmg_refined(_p(f), N, levels, sr_levels, segments, J, alpha, nu1, nu2,
                                   iters, _p(u)))
    return u


def vcycles(f, levels, nu1=2, nu2=2, rtol=1e-13, maxit=60, u0=None):
    """Iterated global FAS V(nu1,nu2) cycles; returns (u, cycles, relres)."""
    f = _arr(f)
    N = f.shape[0]
    u = np.zeros_like(f) if u0 is None else _arr(u0).copy()
    rr = ctypes.c_double(0.0)
    it = _check(lib().orc_vcycles(_p(f), N, levels, nu1, nu2, rtol, maxit, _p(u), ctypes.byref(rr)))
    return u, it, rr.value


def apply(u):
    u = _arr(u)
    out = np.empty_like(u)
    lib().orc_apply(_p(u), u.shape[0], _p(out))
    return out


def gs_half(u, rhs, colour):
    u = _arr(u).copy()
    rhs = _arr(rhs)
    lib().orc_gs_half(_p(u), _p(rhs), u.shape[0], colour)
    return u


def smooth(u, rhs, nu):
    u = _arr(u).copy()
    rhs = _arr(rhs)
    lib().orc_smooth(_p(u), _p(rhs), u.shape[0], nu)
    return u


def restrict(v):
    v = _arr(v)
    n = v.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict(_p(v), n, _p(out))
    return out


def prolong(v):
    v = _arr(v)
    n = v.shape[0]
    out = np.empty((2 * n,) * 3)
    lib().orc_prolong(_p(v), n, _p(out))
    return out


def interp(v):
    v = _arr(v)
    n = v.shape[0]
    out = np.empty((2 * n,) * 3)
    lib().orc_interp(_p(v), n, _p(out))
    return out


def coarse_solve(rhs):
    rhs = _arr(rhs)
    u = np.empty_like(rhs)
    _check(lib().orc_coarse_solve(_p(rhs), rhs.shape[0], _p(u)))
    return u
