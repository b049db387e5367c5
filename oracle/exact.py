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


# --- the 27-point finite volume operator of the paper's model problem -------
#
# On a box of n0 x n1 x n2 cubic cells of size h with odd-reflection ghosts,
# the operator is h^-2 sum_d D2_d W_e W_f with the 1D second difference D2
# and the face-average weights W = (1/24, 11/12, 1/24).  Both 1D factors have
# the sine modes sin(k pi (i + 1/2) / n), k = 1..n, as eigenvectors, with
# eigenvalues -4 sin^2(k pi / (2n)) and 11/12 + (1/12) cos(k pi / n).

FV27_W0 = 11.0 / 12.0
FV27_W1 = 1.0 / 24.0


def fv27_factors(k, n, h):
    """1D eigenvalues (second difference / h^2, face weights) of mode k on n cells."""
    k = np.asarray(k, dtype=np.float64)
    mu = -(4.0 / h ** 2) * np.sin(k * math.pi / (2.0 * n)) ** 2
    om = FV27_W0 + 2.0 * FV27_W1 * np.cos(k * math.pi / n)
    return mu, om


def fv27_eigenvalue(k, n, h):
    """Eigenvalue of the mode with wavenumbers k = (k0, k1, k2) on extents n."""
    m0, o0 = fv27_factors(k[0], n[0], h)
    m1, o1 = fv27_factors(k[1], n[1], h)
    m2, o2 = fv27_factors(k[2], n[2], h)
    return m0 * o1 * o2 + o0 * m1 * o2 + o0 * o1 * m2


def fv27_dst_solve(f, h):
    """u = L^{-1} f for the 27-point operator, f indexed [z, y, x], by DST-II."""
    n2, n1, n0 = f.shape
    F = scipy.fft.dstn(f, type=2, norm="ortho", workers=-1)
    m0, o0 = fv27_factors(np.arange(1, n0 + 1), n0, h)
    m1, o1 = fv27_factors(np.arange(1, n1 + 1), n1, h)
    m2, o2 = fv27_factors(np.arange(1, n2 + 1), n2, h)
    lam = (m0[None, None, :] * o1[None, :, None] * o2[:, None, None]
           + o0[None, None, :] * m1[None, :, None] * o2[:, None, None]
           + o0[None, None, :] * o1[None, :, None] * m2[:, None, None])
    return scipy.fft.idstn(F / lam, type=2, norm="ortho", workers=-1)
