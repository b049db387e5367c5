"""Pins of the 27-point finite volume oracle (the paper's model problem,
Sec. 5.1) against facts other than itself: closed-form eigenpairs, exactness
on quadratics, the dense solve, the Chebyshev polynomial evaluated
independently, second-order convergence on the manufactured solution, the
special cases where segmental refinement reduces to global FMG, and the
trends of Tables 1-3 (the paper's values are for its own sizes; only the
direction of change is pinned)."""
import math

import numpy as np
import pytest

import oracle.exact as ex
from oracle import fv27
from paper_1406_7808_amd import workloads as W

SEG = (4, 2, 2)  # the paper's 4 x 2 x 2 process grid as segments


def _mode(k, n):
    c = [(np.arange(m) + 0.5) / m for m in n]
    return (np.sin(math.pi * k[2] * c[2])[:, None, None] * np.sin(math.pi * k[1] * c[1])[None, :, None]
            * np.sin(math.pi * k[0] * c[0])[None, None, :])


@pytest.mark.parametrize("n,h", [((8, 4, 4), 0.25), ((6, 6, 2), 0.5), ((3, 5, 7), 0.1)])
def test_operator_sine_modes_are_eigenvectors(n, h):
    rng = np.random.default_rng(sum(n))
    for _ in range(6):
        k = tuple(int(rng.integers(1, m + 1)) for m in n)
        v = _mode(k, n)
        lam = ex.fv27_eigenvalue(k, n, h)
        assert np.abs(fv27.apply(v, h) - lam * v).max() <= 1e-13 * abs(lam)


def test_operator_exact_on_quadratics_away_from_walls():
    n, h = (10, 9, 8), 0.125
    z, y, x = np.meshgrid(*[(np.arange(m) + 0.5) * h for m in n[::-1]], indexing="ij")
    u = 1.5 * x * x - 2.0 * y * y + 0.75 * z * z + x * y - 3.0 * y * z + 0.5 * x + 2.0
    lap = 2 * 1.5 - 2 * 2.0 + 2 * 0.75
    got = fv27.apply(u, h)[1:-1, 1:-1, 1:-1]
    assert np.abs(got - lap).max() <= 1e-10


def test_assembled_matrix_is_symmetric_with_the_closed_form_spectrum():
    n, h = (4, 2, 2), 0.5
    m = n[0] * n[1] * n[2]
    A = np.empty((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        A[:, c] = fv27.apply(e.reshape(n[::-1]), h).ravel()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    lam = sorted(ex.fv27_eigenvalue((a, b, c), n, h) for a in range(1, n[0] + 1)
                 for b in range(1, n[1] + 1) for c in range(1, n[2] + 1))
    assert np.allclose(np.linalg.eigvalsh(A), lam, rtol=1e-12, atol=0)
    assert max(lam) < 0


@pytest.mark.parametrize("n", [(2, 1, 1), (4, 2, 2), (8, 4, 4)])
def test_dense_solve_equals_dst(n):
    h = 1.0 / n[1]
    f = np.random.default_rng(7).standard_normal(n[::-1])
    u = fv27.coarse_solve(f, h)
    ref = ex.fv27_dst_solve(f, h)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()


def _cheb_residual_poly(t, k, a=48 / 121, b=200 / 121):
    """The Chebyshev polynomial of [a, b], normalized to 1 at 0, evaluated
    with numpy's Chebyshev series (not the root form the oracle applies)."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    T = np.polynomial.chebyshev.chebval
    return T((b + a - 2 * t) / (b - a), c) / T((b + a) / (b - a), c)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_chebyshev_smoother_is_the_chebyshev_polynomial(k):
    n, h = (16, 8, 8), 1.0 / 8
    d = (121.0 / 24.0) / h ** 2
    for kk in [(1, 1, 1), (9, 2, 3), (16, 8, 8), (12, 7, 1)]:
        v = _mode(kk, n)
        lam = -ex.fv27_eigenvalue(kk, n, h) / d  # spectrum of A/d, A = -L
        got = fv27.cheb(v, np.zeros_like(v), h, k)
        want = _cheb_residual_poly(lam, k) * v
        assert np.abs(got - want).max() <= 1e-13


def test_chebyshev_interval_bounds_the_spectrum():
    # the symbol of A/d over all frequencies lies in (0, 200/121]; the modes a
    # grid twice as coarse cannot represent lie in [48/121, 200/121]
    t = np.linspace(0, math.pi, 97)
    c = np.cos(t)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    w = lambda q: 11 / 12 + q / 12  # noqa: E731
    sym = ((2 - 2 * X) * w(Y) * w(Z) + w(X) * (2 - 2 * Y) * w(Z) + w(X) * w(Y) * (2 - 2 * Z)) / (121 / 24)
    assert sym.max() <= 200 / 121 + 1e-12
    T3 = np.meshgrid(t, t, t, indexing="ij")
    hf = np.maximum(np.maximum(T3[0], T3[1]), T3[2]) >= math.pi / 2 - 1e-12
    assert abs(sym[hf].min() - 48 / 121) <= 1e-12


def test_prolongation_exact_on_linear_fields_away_from_walls():
    n = (6, 4, 4)
    H = 1.0 / n[1]
    zc, yc, xc = np.meshgrid(*[(np.arange(m) + 0.5) * H for m in n[::-1]], indexing="ij")
    v = 0.3 + 1.2 * xc - 0.7 * yc + 2.1 * zc
    fine = fv27.prolong(v)
    h = H / 2
    zf, yf, xf = np.meshgrid(*[(np.arange(2 * m) + 0.5) * h for m in n[::-1]], indexing="ij")
    want = 0.3 + 1.2 * xf - 0.7 * yf + 2.1 * zf
    assert np.abs(fine - want)[1:-1, 1:-1, 1:-1].max() <= 1e-14
    # a fine cell next to one wall gets half its in-line coarse value (linear to 0)
    c = np.ones(n[::-1])
    f1 = fv27.prolong(c)
    assert abs(f1[4, 4, 0] - 0.5) <= 1e-15 and abs(f1[4, 4, 5] - 1.0) <= 1e-15


def test_vcycles_converge_to_the_discrete_solution():
    n = (32, 16, 16)
    h = 1.0 / 16
    f = np.random.default_rng(3).uniform(-1, 1, n[::-1])
    u, it, rr = fv27.vcycles(f, h, 5, rtol=1e-12, maxit=80)
    ref = ex.fv27_dst_solve(f, h)
    assert rr <= 1e-12 and it < 80
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()


def test_fmg_is_second_order_on_the_model_problem():
    errs = []
    for m in (8, 16, 32, 64):
        f, u, h = W.paper_model(m)
        L = int(math.log2(m)) + 1
        ug = fv27.fmg(f, h, L)
        ud = ex.fv27_dst_solve(f, h)
        e_disc = np.abs(ud - u).max()
        assert np.abs(ug - ud).max() <= 0.6 * e_disc
        errs.append(np.abs(ug - u).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(rates) >= 1.85, rates


def test_sr_reduces_to_global_fmg():
    f, u, h = W.paper_model(32)
    L = 6
    g = fv27.fmg(f, h, L)
    assert np.array_equal(fv27.srfmg(f, h, L, 0, SEG, []), g)
    # buffers covering every level: no frozen ghost is left inside the domain
    assert np.abs(fv27.srfmg(f, h, L, 3, SEG, [128, 64, 32]) - g).max() <= 1e-14 * np.abs(g).max()


def test_sr_error_ratio_trends_of_table_1():
    # 2^2 genuine transition cells per segment, K = 4 (Table 1's smallest column
    # shape, at a quarter of its size): e_r falls as A grows and as B grows
    p0, K = 2, 4
    m = 2 * p0 * 2 ** K
    f, u, h = W.paper_model(m)
    L = int(math.log2(m)) + 1
    e_conv = np.abs(fv27.fmg(f, h, L) - u).max()

    def e_r(J):
        return np.abs(fv27.srfmg(f, h, L, K, SEG, J) - u).max() / e_conv

    by_a = [e_r(W.buffer_schedule(A, 0, K)) for A in (2, 4, 6, 8)]
    by_b = [e_r(W.buffer_schedule(2, B, K)) for B in (0, 1, 2)]
    assert all(by_a[i + 1] <= by_a[i] for i in range(3)), by_a
    assert all(by_b[i + 1] <= by_b[i] for i in range(2)), by_b
    assert by_a[0] >= 2.0 and min(by_a + by_b) >= 0.9
    # the maximum buffer schedule with J_1 = 4 is at least as accurate as J = 4
    # on every level
    assert e_r(W.max_buffer_schedule(4, K)) <= by_a[1]


def test_sr_error_ratio_falls_with_transition_segment_size():
    # Tables 2 and 3: a larger genuine transition region per segment gives a
    # smaller e_r, with a constant buffer (A = 2, B = 0) and with the maximum
    # buffer schedule (J_1 = 2)
    K = 3
    const, mbs = [], []
    for p0 in (2, 4):
        m = 2 * p0 * 2 ** K
        f, u, h = W.paper_model(m)
        L = int(math.log2(m)) + 1
        e_conv = np.abs(fv27.fmg(f, h, L) - u).max()
        for out, J in ((const, W.buffer_schedule(2, 0, K)), (mbs, W.max_buffer_schedule(2, K))):
            out.append(np.abs(fv27.srfmg(f, h, L, K, SEG, J) - u).max() / e_conv)
    assert const[0] > const[1] > 1.0, const
    assert mbs[0] > mbs[1] > 1.0, mbs
