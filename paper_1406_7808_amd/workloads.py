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


def paper_model(m, R=(2.0, 1.0, 1.0)):
    """The model problem of the paper (Sec. 5.1) on [0,2] x [0,1] x [0,1]
    with cubic cells h = 1/m (2m x m x m cells): u = prod_i (x_i^4 - R_i^2
    x_i^2), zero on the boundary, and f = Laplacian u, both at cell centers.
    Returns (f, u, h), arrays indexed [z, y, x] of shape (m, m, 2m)."""
    h = 1.0 / m
    x = (np.arange(2 * m, dtype=np.float64) + 0.5) * h
    y = (np.arange(m, dtype=np.float64) + 0.5) * h
    g = [x ** 4 - R[0] ** 2 * x ** 2, y ** 4 - R[1] ** 2 * y ** 2, y ** 4 - R[2] ** 2 * y ** 2]
    d2 = [12.0 * x ** 2 - 2.0 * R[0] ** 2, 12.0 * y ** 2 - 2.0 * R[1] ** 2,
          12.0 * y ** 2 - 2.0 * R[2] ** 2]
    u = _outer3(g[2], g[1], g[0])
    f = _outer3(g[2], g[1], d2[0]) + _outer3(g[2], d2[1], g[0]) + _outer3(d2[2], g[1], g[0])
    return np.ascontiguousarray(f), np.ascontiguousarray(u), h


def buffer_schedule(A, B, K):
    """Eq. 5: J_k = 2 floor((A + B (K - k)) / 2) for the SR levels k = 1..K,
    returned finest level (k = K) first."""
    return [2 * ((A + B * (K - k)) // 2) for k in range(K, 0, -1)]


def max_buffer_schedule(J1, K):
    """The maximum buffer schedule (Sec. 5.2): J_1 on the coarsest SR level and
    every finer compute region the refinement of the next coarser one,
    J_k = 2^(k-1) J_1; finest level first."""
    return [J1 * 2 ** (k - 1) for k in range(K, 0, -1)]


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
