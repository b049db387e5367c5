"""The differentiable solve and the level checkpoints, against the FP64 oracle.

loss(f) = 1/2 ||M f - u_t||^2 with M the FMG map and u_t a seeded Fourier
field.  The backward applies the same solve to grad_u = M f - u_t; it must
equal the oracle's M grad_u (FP64 bar 1e-12).  The loss is exactly quadratic
in f, so a central difference along v is <grad_u, M v> up to rounding; it must
equal the oracle's value to 1e-8.  The backward's <M grad_u, v> differs from
it by the asymmetry of M, which the oracle measures the same way.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1406_7808_amd import autograd as fad
from paper_1406_7808_amd import fmg
from paper_1406_7808_amd import workloads as W

pytestmark = pytest.mark.gpu

TARGET_SEED = 14067810


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _target(N):
    k, a = W.fourier_modes(seed=TARGET_SEED)
    return W.fourier_field(N, k, a / 100.0)


CASES = [(32, 5, 2, 2, [2, 2]), (32, 5, 0, 1, [])]


@pytest.mark.parametrize("N,L,K,S,J", CASES)
def test_backward_and_finite_differences(N, L, K, S, J):
    print("autograd", N, L, K, S, J, flush=True)
    kw = dict(sr_levels=K, segments=S, buffers=J)
    ref = (lambda x: oracle.srfmg(x, L, K, S, J)) if K else (lambda x: oracle.fmg(x, L))
    plan = fmg.Plan(N, L, **kw)
    f_np = W.random_field(N, 1000 + N) * N
    ut = _target(N)
    f = _gpu(f_np).requires_grad_(True)
    u = fad.solve(f, plan)
    loss = 0.5 * ((u - _gpu(ut)) ** 2).sum()
    loss.backward()
    g = ref(f_np) - ut  # oracle grad_u
    mg = ref(g)
    assert _rel(f.grad, mg) <= 1e-12

    rng = np.random.default_rng(TARGET_SEED + N + K)
    gf = f.grad.detach().cpu().numpy()
    for _ in range(8):
        v = rng.standard_normal((N, N, N))
        eps = 1.0  # the loss is quadratic: the central difference is exact but for rounding
        with torch.no_grad():
            lp = 0.5 * ((plan.execute(_gpu(f_np + eps * v)) - _gpu(ut)) ** 2).sum().item()
            lm = 0.5 * ((plan.execute(_gpu(f_np - eps * v)) - _gpu(ut)) ** 2).sum().item()
        fd = (lp - lm) / (2.0 * eps)
        mv = ref(v)
        want = float((g * mv).sum())       # <grad_u, M v>
        assert abs(fd - want) <= 1e-8 * abs(want)
        back = float((gf * v).sum())       # <M grad_u, v>
        asym_o = float((mg * v).sum()) - want
        assert abs((back - fd) - asym_o) <= 1e-8 * abs(want)
    plan.close()


def test_backward_256_sr():
    """The 256^3 differentiable workload: SR on the 3 finest levels."""
    N, L, K, S, J = 256, 8, 3, 8, [2, 4, 6]
    print("autograd 256", flush=True)
    plan = fmg.Plan(N, L, sr_levels=K, segments=S, buffers=J)
    f_np, _, _ = W.fourier(N)
    ut = _target(N)
    f = _gpu(f_np).requires_grad_(True)
    u = fad.solve(f, plan)
    (0.5 * ((u - _gpu(ut)) ** 2).sum()).backward()
    g = oracle.srfmg(f_np, L, K, S, J) - ut
    assert _rel(f.grad, oracle.srfmg(g, L, K, S, J)) <= 1e-12
    plan.close()


@pytest.mark.parametrize("N,L,K,S,J", [(64, 6, 2, 2, [2, 2]), (64, 6, 0, 1, []),
                                        (32, 4, 0, 1, [])])
def test_level_checkpoints(N, L, K, S, J):
    """Level l's state after its stage equals the oracle's (SR-)FMG run with
    top level l on the restricted right-hand side."""
    print("checkpoints", N, L, K, S, J, flush=True)
    T = L - 1 - K
    f_np = W.random_field(N, 1100 + N + K)
    plan = fmg.Plan(N, L, sr_levels=K, segments=S, buffers=J)
    u, levels = fad.solve(_gpu(f_np), plan, keep_levels=True)
    fl = [None] * L
    fl[L - 1] = f_np
    for l in range(L - 1, 0, -1):
        fl[l - 1] = oracle.restrict(fl[l])
    for l in range(L):
        if l <= T:
            ref = oracle.fmg(fl[l], l + 1)
        else:
            ref = oracle.srfmg(fl[l], l + 1, l - T, S, J[L - 1 - l:])
        assert _rel(levels[l], ref) <= 1e-12, l
    assert torch.equal(levels[L - 1], u)
    # checkpoints are off again: a plain solve still works and matches
    assert torch.equal(plan.execute(_gpu(f_np)), u)
    plan.close()
