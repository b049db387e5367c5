"""Bound on the distance between an FP32-refined GPU solve and the oracle's
FP64 run of the same outer iteration.

The FP32-refined solve is u_0 = FMG32(f), then n corrections
u_{i+1} = u_i + FMG32(f - L u_i) with the residual in FP64; the oracle runs
the same iteration in FP64 (o_i).  Write M for one FMG solve and a_i for the
oracle's algebraic error after i corrections (a_{i+1} = (I - M L) a_i).  The
gap g_i = u_i - o_i obeys

    g_{i+1} = (I - M L) g_i + d_{i+1},

where d_{i+1} is the FP32 rounding of correction solve i+1.  Two readings
fix its size:
  * the FP32 rounding of a solve is proportional to the size of what it
    computes, with the first solve's relative gap rho = |g_0| / |u| (mostly
    smooth error: coarse-level FP32 solutions interpolated up), so
    |d_{i+1}| <~ rho |a_i| (correction i+1 removes a_i);
  * I - M L contracts g_0 like it contracts a_0: |(I - M L)^n g_0| <~
    |g_0| |a_n| / |a_0|.
Not contracting the d terms (conservative):
    |g_n| <= 2 rho (|u| |a_n| / |a_0| + sum_{i<n} |a_i|),
with a factor 2 of margin.  Measured on MI355X the gap stays 1.8-40x below
this bound (Fourier right-hand sides of 16 and 64 modes, plain FMG and SR,
64^3 to 512^3).
"""
import numpy as np
import torch

import oracle
from paper_1406_7808_amd import fmg


def _oracle_iterates(f, L, K, S, J, iters):
    """The oracle's FP64 refinement, every iterate: the steps of
    oracle.srfmg_refined (r = f - L u, u += SRFMG(r)) from its own parts."""
    u = oracle.srfmg(f, L, K, S, J) if K else oracle.fmg(f, L)
    out = [u]
    for _ in range(iters):
        r = f - oracle.apply(u)
        u = u + (oracle.srfmg(r, L, K, S, J) if K else oracle.fmg(r, L))
        out.append(u)
    return out


def check(f, ud, u_n, L, K, S, J, iters=2):
    """Assert the bound for u_n (the GPU's FP32-refined solve after `iters`
    corrections, numpy) on right-hand side f with exact discrete solution ud.
    Returns (gap_0, gap_n, bound) relative to max|ud|."""
    fg = torch.from_numpy(np.ascontiguousarray(f)).to("cuda")
    u_0 = fmg.solve(fg, L, sr_levels=K, segments=S, buffers=J, precision="fp32_refined",
                    refine_iters=0).cpu().numpy()
    o = _oracle_iterates(f, L, K, S, J, iters)
    a = [np.abs(oi - ud).max() for oi in o]
    um = np.abs(ud).max()
    gap_0 = np.abs(u_0 - o[0]).max()
    gap_n = np.abs(u_n - o[iters]).max()
    rho = gap_0 / um
    bound = 2.0 * rho * (um * a[iters] / a[0] + sum(a[:iters]))
    print("fp32r gap: first solve %.3e, after %d corrections %.3e, bound %.3e (of max|u|)"
          % (gap_0 / um, iters, gap_n / um, bound / um), flush=True)
    assert gap_n <= bound, (gap_0, gap_n, bound)
    return gap_0 / um, gap_n / um, bound / um
