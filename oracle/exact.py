"""Exact discrete solutions of the cell-centered 7-point Dirichlet problem.

Test infrastructure (same rules as the rest of ``oracle``).  The sine modes
prod_d sin(pi k_d x_d) sampled at cell centers are eigenvectors of the
discrete operator with eigenvalue

    lambda_h(k) = -(4 / h^2) sum_d sin^2(k_d pi h / 2),

so a right-hand side given as a sum of modes has a closed-form discrete
solution, and any right-hand side is solved by the type-II discrete sine
transform (whose basis is exactly these modes).
"""
import math

import numpy as np
import scipy.fft


def eigenvalue(k, N):
    h = 1.0 / N
    k = np.asarray(k, dtype=np.float64)
    return -(4.0 / h ** 2) * np.sum(np.sin(k * math.pi * h / 2.0) ** 2, axis=-1)


def dst_solve(f):
    """u = L_h^{-1} f via DST-II along every axis (any N)."""
    N = f.shape[0]
    F = scipy.fft.dstn(f, type=2, norm="ortho", workers=-1)
    k = np.arange(1, N + 1, dtype=np.float64)
    s = np.sin(k * math.pi / (2.0 * N)) ** 2
    lam = -(4.0 * N * N) * (s[:, None, None] + s[None, :, None] + s[None, None, :])
    return scipy.fft.idstn(F / lam, type=2, norm="ortho", workers=-1)


def sine_discrete(N):
    """Discrete solution for f = -3 pi^2 prod sin(pi x_d): the continuous
    solution times (pi h / 2)^2 / sin^2(pi h / 2)."""
    h = 1.0 / N
    return (math.pi * h / 2.0) ** 2 / math.sin(math.pi * h / 2.0) ** 2


def modes_discrete(N, k, a):
    """Coefficients a_m / lambda_h(k_m) of the discrete solution."""
    return a / eigenvalue(k, N)
