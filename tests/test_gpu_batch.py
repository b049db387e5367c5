"""Batched solves, graph capture and the tuning knobs, against the FP64 oracle.

A graph is replayed several times with eager work and synchronizations in
between, and every replay must reproduce the eager result exactly.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import oracle.exact as ex
import refined_gap
from paper_1406_7808_amd import batched
from paper_1406_7808_amd import fmg
from paper_1406_7808_amd import tune
from paper_1406_7808_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _oracle(f, p):
    if p.get("precision", "fp64") != "fp64":
        return oracle.srfmg_refined(f, p["levels"], p["sr_levels"], p["segments"],
                                    list(p["buffers"]), iters=2)
    if p["sr_levels"]:
        return oracle.srfmg(f, p["levels"], p["sr_levels"], p["segments"], list(p["buffers"]))
    return oracle.fmg(f, p["levels"])


SMALL = [
    {"N": 32, "levels": 5, "sr_levels": 2, "segments": 2, "buffers": (2, 2)},
    {"N": 48, "levels": 5, "sr_levels": 2, "segments": 2, "buffers": (2, 2)},
    {"N": 64, "levels": 6, "sr_levels": 2, "segments": 4, "buffers": (2, 2)},
    {"N": 32, "levels": 5, "sr_levels": 0, "segments": 1, "buffers": ()},
    {"N": 48, "levels": 5, "sr_levels": 2, "segments": 2, "buffers": (2, 2)},
    {"N": 64, "levels": 6, "sr_levels": 2, "segments": 4, "buffers": (2, 2),
     "precision": "fp32_refined"},
]


@pytest.mark.parametrize("streams", [1, 3])
def test_batch_execute_and_graph_replay(streams):
    print("batch", streams, flush=True)
    fs_np = [W.random_field(p["N"], 1200 + i) for i, p in enumerate(SMALL)]
    b = fmg.Batch(SMALL, streams=streams)
    fs = [_gpu(f) for f in fs_np]
    us = [torch.empty_like(f) for f in fs]
    b.execute(fs, us)
    torch.cuda.synchronize()
    for i, p in enumerate(SMALL):
        ref = _oracle(fs_np[i], p)
        if p.get("precision", "fp64") == "fp64":
            assert _rel(us[i], ref) <= TOL, i
        else:
            refined_gap.check(fs_np[i], ex.dst_solve(fs_np[i]), us[i].cpu().numpy(), p["levels"],
                              p["sr_levels"], p["segments"], list(p["buffers"]),
                              iters=p.get("refine_iters", 2))
    eager = [u.clone() for u in us]
    side = torch.cuda.Stream()
    gu = [torch.full_like(f, float("nan")) for f in fs]
    b.capture(fs, gu, side)
    for rep in range(3):
        for u in gu:
            u.fill_(float("nan"))
        torch.cuda.synchronize()
        b.replay(side)
        side.synchronize()
        for i in range(len(SMALL)):
            assert torch.equal(gu[i], eager[i]), (rep, i)
        # eager work between replays
        b.execute(fs, us)
        torch.cuda.synchronize()
    b.close()


def test_batch_rejects_bad_problem():
    bad = [dict(SMALL[0]), dict(SMALL[1], buffers=(3, 2))]
    with pytest.raises(fmg.FMGError) as e:
        fmg.Batch(bad)
    assert e.value.status == fmg.FMG_EINVAL and "problem 1" in str(e.value)


@pytest.mark.parametrize("ms", [2, 4])
def test_transition_into_a_column_level(ms):
    """SR whose transition level (32^3, global) runs in the column smoother:
    its first pre-smoothing pass forms the FAS right-hand side and t, and with
    max_stages=2 a second pass restricts."""
    print("transition", ms, flush=True)
    N, L, K, S, J = 128, 7, 2, 4, [2, 4]
    f = W.random_field(N, 1400 + ms)
    plan = fmg.Plan(N, L, sr_levels=K, segments=S, buffers=J)
    plan.set_tuning(max_stages=ms)
    assert _rel(plan.execute(_gpu(f)), oracle.srfmg(f, L, K, S, J)) <= TOL
    plan.close()


@pytest.mark.parametrize("kw", [dict(max_stages=2), dict(seg_inplace=0), dict(box=0),
                                dict(target_blocks=256), dict(max_stages=4, seg_inplace=0, box=0),
                                dict(max_stages=2, seg_inplace=0, box=0), dict(tile_x=16),
                                dict(tile_x=64, seg_inplace=0, box=0), dict(tile_x=8),
                                dict(tile_x=256, max_stages=2)])
def test_tuning_knobs_keep_the_solution(kw):
    print("tuning", kw, flush=True)
    N, L, K, S, J = 128, 7, 3, 4, [2, 4, 6]
    f = W.random_field(N, 1300)
    plan = fmg.Plan(N, L, sr_levels=K, segments=S, buffers=J)
    plan.set_tuning(**kw)
    assert all(plan.tuning[k] == v for k, v in kw.items())
    u = plan.execute(_gpu(f))
    assert _rel(u, oracle.srfmg(f, L, K, S, J)) <= TOL
    g = fmg.Plan(N, L)
    g.set_tuning(**kw)
    assert _rel(g.execute(_gpu(f)), oracle.fmg(f, L)) <= TOL
    with pytest.raises(fmg.FMGError):
        plan.set_tuning(max_stages=3)
    with pytest.raises(fmg.FMGError):
        plan.set_tuning(tile_x=7)
    plan.close()
    g.close()


def test_autotuner_cache(tmp_path):
    path = str(tmp_path / "tuning.json")
    cands = tune.CANDIDATES[:3]
    best, ms = tune.tune(64, 6, sr_levels=2, segments=4, buffers=(2, 2), reps=2, cache=path,
                         candidates=cands)
    # a candidate, or a candidate with one of the tile widths
    assert {**best, "tile_x": 0} in cands and best["tile_x"] in (0,) + tune.TILE_WIDTHS
    assert ms > 0 and os.path.exists(path)
    again = tune.tune(64, 6, sr_levels=2, segments=4, buffers=(2, 2), cache=path, candidates=cands)
    assert again == (best, ms)


def test_batch96_sampled(tmp_path):
    """The 96-right-hand-side workload (edges 64/96/128, SR on the 2 finest
    levels) in one graph launch; every solution against the oracle."""
    print("batch96", flush=True)
    items = W.batch()
    edges = [N for N, _, _ in items]
    b, probs = batched.build(edges, cache=str(tmp_path / "t.json"))
    fs = [_gpu(W.fourier_field(N, k, a)) for N, k, a in items]
    us = [torch.empty_like(f) for f in fs]
    side = torch.cuda.Stream()
    b.capture(fs, us, side)
    b.replay(side)
    side.synchronize()
    for i in range(len(items)):  # every problem of the batch
        ref = _oracle(fs[i].cpu().numpy(), probs[i])
        assert _rel(us[i], ref) <= TOL, i
    b.close()


def test_batch96_fp32_refined():
    """The 96-right-hand-side workload in the FP32-refined variant (two FP64
    residual corrections), one graph launch: every solution within the
    discretization error of the exact discrete solution, and the distance to
    the oracle's FP64 run of the same outer iteration bounded by the
    contraction of the oracle's algebraic error (every 8th problem)."""
    print("batch96 fp32r", flush=True)
    items = W.batch()
    edges = [N for N, _, _ in items]
    b, probs = batched.build(edges, precision="fp32_refined", tuned=False)
    fs = [_gpu(W.fourier_field(N, k, a)) for N, k, a in items]
    us = [torch.empty_like(f) for f in fs]
    side = torch.cuda.Stream()
    b.capture(fs, us, side)
    b.replay(side)
    side.synchronize()
    worst, gaps = 0.0, []
    for i, (N, k, a) in enumerate(items):
        ud = W.fourier_field(N, k, ex.modes_discrete(N, k, a))
        uc = W.fourier_field(N, k, -a / (np.pi ** 2 * np.sum(k.astype(np.float64) ** 2, axis=1)))
        edisc = np.abs(ud - uc).max()
        u = us[i].cpu().numpy()
        r = np.abs(u - ud).max() / edisc
        worst = max(worst, r)
        assert r <= 1.0, (i, N, r)
        if i % 8 == 0:
            p = probs[i]
            g0, gn, bound = refined_gap.check(fs[i].cpu().numpy(), ud, u, p["levels"],
                                              p["sr_levels"], p["segments"], list(p["buffers"]))
            gaps.append((i, N, gn))
    print("batch96 fp32r worst e_alg/e_disc %.3f; gaps %s" % (worst, gaps), flush=True)
    b.close()
