"""Seeded synthetic inputs for the solver (host, numpy, FP64).

This module generates right-hand sides and the continuous solutions they
come from.  It holds none of the solver's arithmetic: it only samples
analytic fields at cell centers x_i = (i + 1/2) / N of the unit cube
(cell-centered grid, boundary on cell faces; Sec. 2 of the paper).  Both the
HIP path and the CPU oracle are fed from here.

Arrays are float64 of shape (N, N, N) indexed [z, y, x] (x fastest).

Workloads
---------
* ``sine(N)``: u = sin(pi x) sin(pi y) sin(pi z), f = -3 pi^2 u.
* ``fourier(N, modes=64, kmax=16, seed=14067808)``: f = sum_m a_m
  prod_d sin(pi k_md x_d) with k_md ~ U{1..kmax} and a_m = z_m / |k_m|^2,
  z_m ~ N(0,1); k (modes x 3) is drawn first, then z.
* ``polynomial(N)``: u = x(1-x) y(1-y) z(1-z) e^{x+y+z} and its Laplacian.
* ``batch(...)``: many Fourier right-hand sides with edges drawn from a set.
"""
import math

import numpy as np

FOURIER_SEED = 14067808


def centers(N):
    return (np.arange(N, dtype=np.float64) + 0.5) / N


def _outer3(vz, vy, vx):
    return vz[:, None, None] * vy[None, :, None] * vx[None, None, :]


def sine(N):
    """Manufactured u = prod sin(pi x_d); returns (f, u_continuous)."""
    s = np.sin(math.pi * centers(N))
    u = _outer3(s, s, s)
    return -3.0 * math.pi ** 2 * u, u


def fourier_modes(modes=64, kmax=16, seed=FOURIER_SEED):
    """Wavenumbers k (modes x 3, columns x, y, z) and amplitudes a."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(modes, 3))
    z = rng.standard_normal(modes)
    a = z / np.sum(k.astype(np.float64) ** 2, axis=1)
    return k, a


def fourier_field(N, k, coef):
    """sum_m coef_m prod_d sin(pi k_md x_d) at the cell centers.

    Evaluated as one (N*N x M) @ (M x N) product: row (z, y) holds
    coef_m sin(pi k_mz z) sin(pi k_my y), column x holds sin(pi k_mx x)."""
    x = centers(N)
    k = np.asarray(k)
    sx = np.sin(math.pi * k[:, 0:1] * x[None, :])  # (M, N)
    sy = np.sin(math.pi * k[:, 1:2] * x[None, :])
    sz = np.sin(math.pi * k[:, 2:3] * x[None, :])
    zy = (np.asarray(coef)[:, None, None] * sz[:, :, None] * sy[:, None, :]).reshape(len(coef), N * N)
    return np.ascontiguousarray((zy.T @ sx).reshape(N, N, N))


def fourier(N, modes=64, kmax=16, seed=FOURIER_SEED):
    """Random smooth right-hand side; returns (f, u_continuous, (k, a))."""
    k, a = fourier_modes(modes, kmax, seed)
    f = fourier_field(N, k, a)
    ucont = fourier_field(N, k, -a / (math.pi ** 2 * np.sum(k.astype(np.float64) ** 2, axis=1)))
    return f, ucont, (k, a)


def polynomial(N):
    """u = x(1-x) y(1-y) z(1-z) e^{x+y+z}; returns (f = Laplacian u, u)."""
    x = centers(N)
    e = np.exp(x)
    p = x * (1.0 - x) * e            # q(x) e^x with q = x(1-x)
    # d2/dx2 [x(1-x) e^x] = e^x (q'' + 2 q' + q) = e^x (-x^2 - 3x) = -x (x+3) e^x
    d2 = -x * (x + 3.0) * e
    u = _outer3(p, p, p)
    f = _outer3(p, p, d2) + _outer3(p, d2, p) + _outer3(d2, p, p)
    return f, u


def random_field(N, seed):
    """Uniform(-1, 1) values, for operator-level checks."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(N, N, N))


def batch(count=96, sizes=(64, 96, 128), modes=16, kmax=8, seed=14067809):
    """Right-hand sides with edges drawn uniformly from `sizes`."""
    rng = np.random.default_rng(seed)
    edges = rng.choice(np.asarray(sizes), size=count)
    out = []
    for b in range(count):
        k = rng.integers(1, kmax + 1, size=(modes, 3))
        z = rng.standard_normal(modes)
        a = z / np.sum(k.astype(np.float64) ** 2, axis=1)
        out.append((int(edges[b]), k, a))
    return out
