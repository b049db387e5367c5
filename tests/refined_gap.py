"""Bound on the distance between an FP32-refined GPU solve and the oracle's
FP64 run of the same outer iteration.

The FP32-refined solve is u_0 = FMG32(f), then n corrections
u_{i+1} = u_i + FMG32(f - L u_i) with the residual in FP64.  The oracle runs
the same iteration in FP64.  The FP32 rounding of the first solve leaves a
gap g_0 = |u_0 - o_0| (mostly smooth: coarse-level FP32 solutions
interpolated up), and every FP64-residual correction applies the same
iteration operator I - M L to it that it applies to the oracle's algebraic
error.  So after n corrections the gap is bounded by g_0 times the
contraction of the oracle's algebraic error over the same n corrections,
e_alg(n) / e_alg(0), plus the FP32 rounding of the last correction itself,
which is far smaller.  Measured on MI355X (Fourier right-hand sides), the
gap contracts at least 3x faster than that for plain FMG and SR (64^3 K=2:
3.2x; 128^3 K=3: 17x; 256^3 K=3: 42x; plain FMG 64^3 and 128^3: 25x);
the bound allows a factor 2 on the contraction.
"""
import numpy as np
import torch

import oracle
from paper_1406_7808_amd import fmg


def check(f, ud, u_n, L, K, S, J, iters=2):
    """Assert the bound for u_n (the GPU's FP32-refined solve after `iters`
    corrections, numpy) on right-hand side f with exact discrete solution ud.
    Returns (gap_0, gap_n, bound) relative to max|ud|."""
    fg = torch.from_numpy(np.ascontiguousarray(f)).to("cuda")
    u_0 = fmg.solve(fg, L, sr_levels=K, segments=S, buffers=J, precision="fp32_refined",
                    refine_iters=0).cpu().numpy()
    o_0 = oracle.srfmg_refined(f, L, K, S, J, iters=0)
    o_n = oracle.srfmg_refined(f, L, K, S, J, iters=iters)
    gap_0 = np.abs(u_0 - o_0).max()
    gap_n = np.abs(u_n - o_n).max()
    bound = 2.0 * gap_0 * np.abs(o_n - ud).max() / np.abs(o_0 - ud).max()
    um = np.abs(ud).max()
    print("fp32r gap: first solve %.3e, after %d corrections %.3e, bound %.3e (of max|u|)"
          % (gap_0 / um, iters, gap_n / um, bound / um), flush=True)
    assert gap_n <= bound, (gap_0, gap_n, bound)
    return gap_0 / um, gap_n / um, bound / um
