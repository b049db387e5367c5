"""The batched workload: many right-hand sides of uneven sizes in one graph.

Each size gets the deepest hierarchy whose coarsest edge is 2 or 3, and
segmental refinement on its two finest levels with 4^3 segments and buffer
widths (2, 2).  Problems with equal configurations share a tuning, found by
the autotuner (tune.py) and cached.
"""
from . import fmg
from . import tune as _tune


def levels_for(N):
    """Levels so that the coarsest edge is 2 or 3."""
    L, n = 1, N
    while n % 2 == 0 and n // 2 >= 2:
        n //= 2
        L += 1
    if n > 3:
        raise ValueError("edge %d does not reduce to a coarsest edge of 2 or 3" % N)
    return L


def problem(N, precision="fp64", sr_levels=2, segments=4, buffers=(2, 2)):
    return {"N": N, "levels": levels_for(N), "sr_levels": sr_levels, "segments": segments,
            "buffers": tuple(buffers), "precision": precision}


def build(edges, precision="fp64", streams=8, tuned=True, cache=None, fs=None, us=None):
    """A fmg.Batch for problems of the given edges.  With tuned and the
    batch's tensors (fs, us), the knobs are tuned on the batch graph itself;
    with tuned alone, per solve."""
    probs = [problem(N, precision) for N in edges]
    tunings = None
    if tuned and fs is not None:
        tunings = _tune.tune_batch(probs, fs, us, streams=streams, cache=cache)[0]
    elif tuned:
        best = {}
        for p in probs:
            key = p["N"]
            if key not in best:
                kw = {k: v for k, v in p.items() if k not in ("N", "levels")}
                best[key] = _tune.tune(p["N"], p["levels"], cache=cache, **kw)[0]
        tunings = [best[p["N"]] for p in probs]
    return fmg.Batch(probs, streams=streams, tunings=tunings), probs
