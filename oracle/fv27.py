"""Wrappers of the 27-point finite volume oracle (``fv27_oracle.c``): the
paper's own model problem (Sec. 5.1) -- Chebyshev smoothers, linear
prolongation, boxes of cubic cells.  Test infrastructure, like the rest of
``oracle``.

Arrays are float64 of shape (n2, n1, n0) indexed [z, y, x] (x fastest); the
extents are passed as (n0, n1, n2) and the finest cell size as h.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fv27_oracle.c")
_SO = os.path.join(_HERE, "libfv27_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(verbose=False):
    """Compile fv27_oracle.c into oracle/libfv27_oracle.so (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    global _lib
    _lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    i, d = ctypes.c_int, ctypes.c_double
    L.orc27_apply.argtypes = [_dp, _ip, d, _dp]
    L.orc27_apply.restype = None
    L.orc27_cheb.argtypes = [_dp, _dp, _ip, d, i]
    L.orc27_cheb.restype = None
    L.orc27_prolong.argtypes = [_dp, _ip, _dp]
    L.orc27_prolong.restype = None
    L.orc27_coarse_solve.argtypes = [_dp, _ip, d, _dp]
    L.orc27_fmg.argtypes = [_dp, _ip, d, i, i, i, i, _dp]
    L.orc27_vcycles.argtypes = [_dp, _ip, d, i, i, i, d, i, _dp, _dp]
    L.orc27_srfmg.argtypes = [_dp, _ip, d, i, i, _ip, _ip, i, i, i, _dp]
    L.orc27_threads.argtypes = []
    _lib = L
    return L


def _p(a):
    return a.ctypes.data_as(_dp)


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ext(a):
    """(n0, n1, n2) of an array indexed [z, y, x]."""
    return (ctypes.c_int * 3)(a.shape[2], a.shape[1], a.shape[0])


def _check(st):
    if st < 0:
        raise ValueError("oracle rejected the parameters (status %d)" % st)
    return st


def apply(u, h):
    u = _arr(u)
    out = np.empty_like(u)
    lib().orc27_apply(_p(u), _ext(u), h, _p(out))
    return out


def cheb(u, rhs, h, degree):
    u = _arr(u).copy()
    lib().orc27_cheb(_p(u), _p(_arr(rhs)), _ext(u), h, degree)
    return u


def prolong(v):
    v = _arr(v)
    out = np.empty(tuple(2 * s for s in v.shape))
    lib().orc27_prolong(_p(v), _ext(v), _p(out))
    return out


def coarse_solve(rhs, h):
    rhs = _arr(rhs)
    u = np.empty_like(rhs)
    _check(lib().orc27_coarse_solve(_p(rhs), _ext(rhs), h, _p(u)))
    return u


def fmg(f, h, levels, degrees=(2, 2, 1)):
    """Global FMG; degrees = (pre, post, fmg) Chebyshev degrees."""
    f = _arr(f)
    u = np.zeros_like(f)
    _check(lib().orc27_fmg(_p(f), _ext(f), h, levels, degrees[0], degrees[1], degrees[2], _p(u)))
    return u


def vcycles(f, h, levels, degrees=(2, 2), rtol=1e-12, maxit=60, u0=None):
    f = _arr(f)
    u = np.zeros_like(f) if u0 is None else _arr(u0).copy()
    rr = ctypes.c_double(0.0)
    it = _check(lib().orc27_vcycles(_p(f), _ext(f), h, levels, degrees[0], degrees[1], rtol, maxit,
                                    _p(u), ctypes.byref(rr)))
    return u, it, rr.value


def srfmg(f, h, levels, sr_levels, segments, buffers, degrees=(2, 2, 1)):
    """SR-FMG on the sr_levels finest levels; segments = (s0, s1, s2);
    buffers: sr_levels widths, finest level first."""
    f = _arr(f)
    u = np.zeros_like(f)
    S = (ctypes.c_int * 3)(*segments)
    J = (ctypes.c_int * max(1, len(buffers)))(*buffers)
    _check(lib().orc27_srfmg(_p(f), _ext(f), h, levels, sr_levels, S, J, degrees[0], degrees[1],
                             degrees[2], _p(u)))
    return u
