"""Pins of the FP64 CPU oracle against what mathematics and the paper fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a brute-force reformulation or a special case that reduces to a
textbook routine.  Section and figure numbers refer to the paper
(arXiv:1406.7808).
"""
import math
import os

import numpy as np
import pytest

import oracle
import oracle.exact as ex
import sr_sets
from paper_1406_7808_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mode(N, k):
    x = W.centers(N)
    s = [np.sin(math.pi * k[d] * x) for d in range(3)]
    return s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]


# --- operator (Sec. 2, Eq. 2) --------------------------------------------------

@pytest.mark.parametrize("N", [4, 8, 16])
def test_operator_sine_modes_are_eigenvectors(N):
    for k in [(1, 1, 1), (2, 1, 3), (N, 1, 2), (N - 1, N, 1)]:
        v = _mode(N, k)
        lam = ex.eigenvalue(k, N)
        Lv = oracle.apply(v)
        assert np.abs(Lv - lam * v).max() <= 1e-12 * abs(lam) * np.abs(v).max()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_operator_matrix_is_kronecker_sum(n):
    """Dense matrix of L_h equals the Kronecker sum of the 1D cell-centered
    Dirichlet matrix (diagonal -2, corners -3, off-diagonal 1) / h^2."""
    m = n ** 3
    A = np.zeros((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        A[:, c] = oracle.apply(e.reshape(n, n, n)).reshape(-1)
    T = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    T[0, 0] -= 1.0
    T[-1, -1] -= 1.0
    I = np.eye(n)
    K3 = np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)
    assert np.array_equal(A, K3 * n * n)
    assert np.array_equal(A, A.T)


# --- coarsest solve (Fig. 1, k = 0) ------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 8])
def test_coarse_solve_equals_dst(n):
    f = W.random_field(n, 11 + n)
    u = oracle.coarse_solve(f)
    ref = ex.dst_solve(f)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()


# --- red-black Gauss-Seidel ---------------------------------------------------

def test_gs_half_zeroes_residual_on_its_colour():
    N = 8
    u = W.random_field(N, 1)
    f = W.random_field(N, 2) * 100.0
    idx = np.indices((N, N, N)).sum(axis=0) % 2
    scale = np.abs(f).max() + np.abs(oracle.apply(u)).max()
    u1 = oracle.gs_half(u, f, 0)
    r1 = f - oracle.apply(u1)
    assert np.abs(r1[idx == 0]).max() <= 1e-12 * scale
    assert not np.allclose(r1[idx == 1], 0.0)
    # red half-sweep leaves black cells alone
    assert np.array_equal(u1[idx == 1], u[idx == 1])
    u2 = oracle.gs_half(u1, f, 1)
    r2 = f - oracle.apply(u2)
    assert np.abs(r2[idx == 1]).max() <= 1e-12 * scale


def test_gs_sweep_matches_dense_rowwise_gauss_seidel():
    """Brute force: Gauss-Seidel on the assembled matrix, all red rows then
    all black rows, one row at a time."""
    n = 4
    m = n ** 3
    A = np.zeros((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        A[:, c] = oracle.apply(e.reshape(n, n, n)).reshape(-1)
    u = W.random_field(n, 3).reshape(-1)
    f = W.random_field(n, 4).reshape(-1) * 10.0
    col = (np.indices((n, n, n)).sum(axis=0) % 2).reshape(-1)
    x = u.copy()
    for sweep in range(2):
        for colour in (0, 1):
            for r in np.nonzero(col == colour)[0]:
                x[r] = (f[r] - A[r] @ x + A[r, r] * x[r]) / A[r, r]
    y = oracle.smooth(u.reshape(n, n, n), f.reshape(n, n, n), 2).reshape(-1)
    assert np.abs(x - y).max() <= 1e-13 * np.abs(x).max()


# --- transfers (Sec. 3.1, Sec. 3.2) -------------------------------------------

def test_restriction_and_prolongation():
    v = W.random_field(6, 5)
    # the 8 equal children are summed one by one, so identity holds to rounding
    assert np.abs(oracle.restrict(oracle.prolong(v)) - v).max() <= 4e-16 * np.abs(v).max()
    c = np.full((8, 8, 8), 2.5)
    assert np.array_equal(oracle.restrict(c), np.full((4, 4, 4), 2.5))
    w = W.random_field(8, 6)
    assert abs(w.sum() - 8.0 * oracle.restrict(w).sum()) <= 1e-12 * np.abs(w).sum()
    # each child carries its parent's value
    p = oracle.prolong(v)
    assert np.array_equal(p[1::2, 0::2, 1::2], v)


def test_fmg_interpolation_is_linear_with_zero_walls():
    nc = 8
    n = 2 * nc
    Xc = W.centers(nc)
    xf = W.centers(n)
    # constant 1: 1 inside, 1/2 per wall dimension at wall-adjacent cells
    one = oracle.interp(np.ones((nc,) * 3))
    fac = np.ones(n)
    fac[0] = fac[-1] = 0.5
    assert np.abs(one - fac[:, None, None] * fac[None, :, None] * fac[None, None, :]).max() <= 1e-15
    # linear ramp in x, constant in y, z: exact at cells away from the x walls
    a, b = 0.3, -1.7
    ramp = np.broadcast_to(a + b * Xc[None, None, :], (nc, nc, nc))
    out = oracle.interp(ramp)
    want = (a + b * xf)[None, None, :] * fac[:, None, None] * fac[None, :, None]
    assert np.abs(out[:, :, 1:-1] - want[:, :, 1:-1]).max() <= 1e-14
    # at the x walls: linear interpolation between zero on the face and the
    # nearest coarse value (fine center at h/2, coarse center at h)
    assert np.abs(out[:, :, 0] - 0.5 * ramp[0, 0, 0] * (fac[:, None] * fac[None, :])).max() <= 1e-14
    assert np.abs(out[:, :, -1] - 0.5 * ramp[0, 0, -1] * (fac[:, None] * fac[None, :])).max() <= 1e-14


# --- V-cycle and FMG (Figs. 1 and 2) -------------------------------------------

def _golden_edisc():
    out = {}
    with open(os.path.join(GOLDEN, "sine_edisc.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            N, e = line.split()
            out[int(N)] = float(e)
    return out


def test_vcycles_converge_to_the_discrete_solution():
    N, L = 16, 4
    f = W.random_field(N, 7)
    u, it, rr = oracle.vcycles(f, L, rtol=1e-13, maxit=40)
    assert rr <= 1e-13 and it < 25
    ref = ex.dst_solve(f)
    assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("N,L", [(8, 3), (16, 4), (32, 5), (64, 6)])
def test_discretization_error_matches_closed_form(N, L):
    f, uc = W.sine(N)
    u, _, _ = oracle.vcycles(f, L, rtol=1e-14, maxit=60)
    e = np.abs(u - uc).max()
    assert abs(e - _golden_edisc()[N]) <= 1e-6 * _golden_edisc()[N]


def test_fmg_is_second_order_and_within_discretization_error():
    ed = _golden_edisc()
    etot = {}
    for N, L in [(16, 4), (32, 5), (64, 6), (128, 7)]:
        f, uc = W.sine(N)
        u = oracle.fmg(f, L)
        ud = uc * ex.sine_discrete(N)
        ealg = np.abs(u - ud).max()
        assert ealg <= 0.6 * ed[N]
        etot[N] = np.abs(u - uc).max()
    for N in (16, 32, 64):
        assert etot[N] / etot[2 * N] >= 3.6


def test_fmg_fourier_rhs_against_closed_form_discrete_solution():
    N, L = 64, 6
    f, uc, (k, a) = W.fourier(N)
    u = oracle.fmg(f, L)
    ud = W.fourier_field(N, k, ex.modes_discrete(N, k, a))
    edisc = np.abs(ud - uc).max()
    assert np.abs(u - ud).max() <= 1.0 * edisc


def test_gamma_r_relation():
    """Sec. 3.2: a per-level solver with error reduction Gamma < 1/4 gives an
    FMG algebraic-to-discretization error ratio r with Gamma = r/(4r+3)."""
    N, L = 64, 6
    u = W.random_field(N, 5)
    z = np.zeros((N, N, N))
    norms = [np.abs(u).max()]
    for _ in range(10):
        u, _, _ = oracle.vcycles(z, L, u0=u, maxit=1, rtol=0.0)
        norms.append(np.abs(u).max())
    G = float(np.mean(np.array(norms[-3:]) / np.array(norms[-4:-1])))
    assert G < 0.25
    r_pred = 3.0 * G / (1.0 - 4.0 * G)
    f, uc = W.sine(N)
    ud = uc * ex.sine_discrete(N)
    r_meas = np.abs(oracle.fmg(f, L) - ud).max() / np.abs(ud - uc).max()
    assert r_pred / 2.5 <= r_meas <= r_pred * 2.5


def test_residual_is_first_order():
    """Sec. 7: the FMG residual decreases at first order only."""
    res = {}
    for N, L in [(32, 5), (64, 6), (128, 7)]:
        f, _ = W.sine(N)
        res[N] = np.abs(f - oracle.apply(oracle.fmg(f, L))).max()
    for N in (32, 64):
        assert 1.6 <= res[N] / res[2 * N] <= 2.5


# --- segmental refinement (Sec. 4, Figs. 5 and 6) ----------------------------

def test_sr_degenerate_cases_equal_global_fmg():
    N, L = 32, 5
    f = W.random_field(N, 8)
    g = oracle.fmg(f, L)
    assert np.array_equal(oracle.srfmg(f, L, 0, 4, []), g)
    assert np.array_equal(oracle.srfmg(f, L, 2, 1, [2, 2]), g)
    assert np.array_equal(oracle.srfmg(f, L, 3, 1, [0, 0, 0]), g)


@pytest.mark.parametrize("K,S,J", [(2, 2, [16, 8]), (3, 2, [16, 8, 4]), (2, 4, [24, 12])])
def test_sr_with_ample_buffers_equals_global_fmg(K, S, J):
    """When every compute region covers its whole level nothing is frozen and
    no tau correction is lost, so SR reproduces global FMG."""
    N, L = 32, 5
    f = W.random_field(N, 9)
    assert np.array_equal(oracle.srfmg(f, L, K, S, J), oracle.fmg(f, L))


@pytest.mark.parametrize("N,L,K,S,J", [
    (16, 4, 2, 2, [2, 2]),
    (32, 5, 2, 2, [2, 2]),
    (32, 5, 3, 2, [2, 4, 6]),
    (32, 5, 2, 2, [4, 2]),
    (32, 5, 1, 4, [0]),
    (32, 5, 4, 2, [2, 2, 2, 2]),
])
def test_sr_matches_set_algebra_reformulation(N, L, K, S, J):
    f = W.random_field(N, 10 + K)
    a = sr_sets.srfmg(f, L, K, S, J)
    assert not np.isnan(a).any()
    b = oracle.srfmg(f, L, K, S, J)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_sr_set_algebra_matches_global_fmg():
    f = W.random_field(16, 12)
    g = sr_sets.fmg(f, 4).u[3][1:-1, 1:-1, 1:-1]
    assert np.abs(g - oracle.fmg(f, 4)).max() <= 1e-13 * np.abs(g).max()


def test_sr_departure_shrinks_as_buffers_grow():
    """Tables 1-3 trend: larger buffers bring SR closer to the conventional
    solver, and ample buffers reproduce it."""
    N, L, K, S = 64, 6, 2, 2
    f, _, _ = W.fourier(N)
    g = oracle.fmg(f, L)
    d = [np.abs(oracle.srfmg(f, L, K, S, [j, j]) - g).max() for j in (2, 4, 6, 8, 12)]
    assert all(d[i + 1] < d[i] for i in range(len(d) - 1))
    assert np.array_equal(oracle.srfmg(f, L, K, S, [32, 16]), g)


def test_sr_error_falls_with_transition_segment_size():
    """Tables 2-3 trend: at fixed K and J, larger genuine regions on the
    transition level give a smaller error ratio."""
    N, L, K, J = 64, 6, 2, [4, 4]
    f, uc = W.sine(N)
    econv = np.abs(oracle.fmg(f, L) - uc).max()
    er = {S: np.abs(oracle.srfmg(f, L, K, S, J) - uc).max() / econv for S in (4, 2)}
    assert er[2] < er[4]
    assert er[2] >= 1.0


def test_sr_error_is_second_order():
    """Sec. 7: SR keeps second-order accuracy (same segment shape per level)."""
    e = {}
    for N, L in [(32, 5), (64, 6), (128, 7)]:
        f, uc = W.sine(N)
        e[N] = np.abs(oracle.srfmg(f, L, 2, N // 16, [4, 4]) - uc).max()
    for N in (32, 64):
        assert e[N] / e[2 * N] >= 3.0


def test_sr_refinement_approaches_discrete_solution():
    N, L, K, S, J = 32, 5, 2, 2, [2, 2]
    f, uc, (k, a) = W.fourier(N)
    ud = W.fourier_field(N, k, ex.modes_discrete(N, k, a))
    e0 = np.abs(oracle.srfmg(f, L, K, S, J) - ud).max()
    e2 = np.abs(oracle.srfmg_refined(f, L, K, S, J, iters=2) - ud).max()
    assert e2 < 0.2 * e0


def test_oracle_rejects_invalid_parameters():
    f = np.zeros((32, 32, 32))
    with pytest.raises(ValueError):
        oracle.srfmg(f, 5, 2, 2, [3, 2])      # odd buffer
    with pytest.raises(ValueError):
        oracle.srfmg(f, 5, 2, 2, [8, 2])      # J_{k-1} < J_k / 2
    with pytest.raises(ValueError):
        oracle.srfmg(f, 5, 2, 3, [2, 2])      # segments do not divide the grid
    with pytest.raises(ValueError):
        oracle.fmg(f, 2)                      # coarsest level too large
