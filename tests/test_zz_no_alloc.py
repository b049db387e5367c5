"""The allocation-free residual norms entry point against the allocating one.

Both run the same two kernels with the same launch shape, so the results must
be identical.  Two calls in a row, the second on a smaller grid, check that
the shared static scratch keeps no state between calls."""
import numpy as np
import pytest
import torch

from paper_1406_7808_amd import fmg
from paper_1406_7808_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_residual_norms_match_allocating_entry_point():
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    for n, seed in ((130, 11), (37, 12)):
        print("noalloc norms", n, flush=True)
        f = torch.from_numpy(W.random_field(n, seed) * n * n).cuda()
        u = torch.from_numpy(W.random_field(n, seed + 100)).cuda()
        out.fill_(float("nan"))
        fmg.residual_norms_noalloc(f, u, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = fmg.residual_norms(f, u)
        assert got[0] == ref[0] and got[1] == ref[1], (n, got, ref)
        assert np.isfinite(got).all()


def test_noalloc_residual_norms_rejects_aliasing():
    f = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(fmg.FMGError) as e:
        fmg.residual_norms_noalloc(f, f, out)
    assert e.value.status == fmg.FMG_EINVAL
