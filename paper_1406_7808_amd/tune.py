"""Autotuner for the solver's performance knobs (fmg_tuning).

For one problem configuration (N, levels, segmentation, sweeps, precision)
it times every candidate setting of the knobs on the device -- passes of 2 or
4 half-sweeps, in-place segment smoothing, the box-resident smoother, the
workgroup count a streaming pass aims for -- checks that each candidate's
solution agrees with the default's (every setting computes the same solve up
to rounding), and keeps the fastest; then it tries the tile widths of
TILE_WIDTHS for the streaming passes on that setting (the tile shape, which
the library otherwise takes from its cost model).  Segment counts and
buffer widths are not tuned: they change the segmental-refinement solution
itself (its algebraic error), so they belong to the caller.  Results persist in a JSON cache keyed
by the device, the library build and the configuration, so a batch of many
right-hand sides tunes each distinct configuration once.

Solves that run side by side compete for the GPU, so the fastest setting of
a solve alone is not always the fastest inside a batch; tune_batch times the
whole batch graph instead, one configuration at a time (coordinate descent
over the distinct configurations, the others held at their current best).
"""
import hashlib
import itertools
import json
import os

import torch

from . import fmg

CANDIDATES = [{"max_stages": ms, "seg_inplace": ip, "box": bx, "target_blocks": tb, "tile_x": 0}
              for ms, ip, bx, tb in itertools.product((2, 4), (1, 0), (1, 0), (0, 512, 1024, 2048))]
TILE_WIDTHS = (16, 32, 64, 128)


def default_cache_path():
    return os.environ.get("FMG_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1406_7808_amd", "tuning.json")


def library_id():
    """Hash of the built library, so a rebuilt solver is tuned again."""
    h = hashlib.sha256()
    with open(fmg._SO, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def config_key(N, levels, sr_levels=0, segments=1, buffers=(), sweeps=(2, 2, 1),
               precision="fp64", refine_iters=2, device=None):
    dev = torch.cuda.current_device() if device is None else device
    name = torch.cuda.get_device_properties(dev).gcnArchName
    return "|".join([name, library_id(), "N=%d" % N, "L=%d" % levels, "K=%d" % sr_levels,
                     "S=%d" % segments, "J=%s" % ",".join(map(str, buffers)),
                     "sw=%s" % ",".join(map(str, sweeps)), precision, "r=%d" % refine_iters])


def _load(path):
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def _save(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(plan, f, u, reps):
    s = torch.cuda.current_stream()
    for _ in range(2):
        plan.execute(f, u)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.execute(f, u)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(N, levels, sr_levels=0, segments=1, buffers=(), sweeps=(2, 2, 1), precision="fp64",
         refine_iters=2, reps=5, cache=None, refresh=False, candidates=None,
         tile_widths=TILE_WIDTHS):
    """Best tuning (a dict of fmg_tuning fields) and its ms per solve, from the
    cache or by timing every candidate on a seeded right-hand side, then the
    tile widths on the best candidate."""
    kw = dict(sr_levels=sr_levels, segments=segments, buffers=tuple(buffers), sweeps=tuple(sweeps),
              precision=precision, refine_iters=refine_iters)
    path = cache or default_cache_path()
    key = config_key(N, levels, **kw)
    data = _load(path)
    if key in data and not refresh:
        e = data[key]
        return e["tuning"], e["ms"]
    gen = torch.Generator(device="cpu").manual_seed(N * 7919 + levels)
    f = (torch.rand((N, N, N), generator=gen, dtype=torch.float64) * 2 - 1).cuda()
    u = torch.empty_like(f)
    plan = fmg.Plan(N, levels, **kw)
    ref = plan.execute(f, torch.empty_like(f)).clone()
    scale = float(ref.abs().max())
    tol = 1e-12 if precision == "fp64" else 1e-5
    timings = {}
    best, best_ms = None, None

    def trial(c):
        nonlocal best, best_ms
        plan.set_tuning(**{**fmg.DEFAULT_TUNING, **c})
        ms = _time(plan, f, u, reps)
        err = float((u - ref).abs().max()) / max(scale, 1e-300)
        if err > tol:
            raise RuntimeError("tuning %s changes the solution by %.3g" % (c, err))
        timings[json.dumps(c, sort_keys=True)] = round(ms, 5)
        if best_ms is None or ms < best_ms:
            best, best_ms = dict(c), ms

    for c in candidates or CANDIDATES:
        trial(c)
    for tx in tile_widths:
        trial({**best, "tile_x": tx})
    plan.close()
    data = _load(path)
    data[key] = {"tuning": best, "ms": best_ms, "candidates": timings}
    _save(path, data)
    return best, best_ms


def _graph_ms(batch, fs, us, reps):
    side = torch.cuda.Stream()
    batch.capture(fs, us, side)
    for _ in range(2):
        batch.replay(side)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(side)
    for _ in range(reps):
        batch.replay(side)
    e1.record(side)
    side.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batch(problems, fs, us, streams=8, reps=3, cache=None, refresh=False, candidates=None,
               tile_widths=TILE_WIDTHS):
    """Per-problem tunings for a batch (a list of dicts, one per problem),
    chosen by timing the batch graph on the given right-hand sides."""
    path = cache or default_cache_path()
    classes = []  # distinct configurations, in order of appearance
    for p in problems:
        c = tuple(sorted((k, tuple(v) if isinstance(v, (list, tuple)) else v) for k, v in p.items()))
        if c not in classes:
            classes.append(c)
    cls_of = [classes.index(tuple(sorted((k, tuple(v) if isinstance(v, (list, tuple)) else v)
                                          for k, v in p.items()))) for p in problems]
    comp = hashlib.sha256(json.dumps([classes, cls_of, streams], sort_keys=True,
                                     default=str).encode()).hexdigest()[:16]
    dev = torch.cuda.current_device()
    key = "|".join(["batch", torch.cuda.get_device_properties(dev).gcnArchName, library_id(), comp])
    data = _load(path)
    if key in data and not refresh:
        best = data[key]["tunings"]
        return [best[i] for i in cls_of], data[key]["ms"]
    cands = candidates or CANDIDATES
    best = [dict(fmg.DEFAULT_TUNING) for _ in classes]

    def run(tunings):
        b = fmg.Batch(problems, streams=streams, tunings=[tunings[i] for i in cls_of])
        try:
            return _graph_ms(b, fs, us, reps)
        finally:
            b.close()

    best_ms = run(best)

    def attempt(ci, t):
        nonlocal best, best_ms
        if t == best[ci]:
            return
        trial = [dict(x) for x in best]
        trial[ci] = t
        ms = run(trial)
        if ms < best_ms:
            best, best_ms = trial, ms

    for ci in range(len(classes)):
        for c in cands:
            attempt(ci, {**fmg.DEFAULT_TUNING, **c})
        for tx in tile_widths:  # the tile widths on this class's best setting
            attempt(ci, {**best[ci], "tile_x": tx})
    data = _load(path)
    data[key] = {"tunings": best, "ms": best_ms, "classes": [dict(c) for c in classes],
                 "streams": streams}
    _save(path, data)
    return [best[i] for i in cls_of], best_ms
