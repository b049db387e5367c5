#!/usr/bin/env python3
"""FMG solve throughput on one MI355X.

Workload (the 256^3 case): 3D Poisson, cell-centered 7-point, u = 0 on the
unit cube, FP64; FMG F(1,2,2) with 8 levels (256 -> 2), red-black
Gauss-Seidel, mean-of-8 restriction, piecewise-constant V-cycle
prolongation, trilinear FMG interpolation; right-hand side = 64 seeded random
sine modes (k_d ~ U{1..16}, amplitude z/|k|^2, seed 14067808).

One step = one solve.  Three solvers are timed on the same right-hand side:
  sr     segmental refinement on the 3 finest levels, 8^3 segments, buffer
         widths 2, 4, 6 from the finest level up (the headline `value`);
  global plain global FMG;
  sr32r  the same SR solve with FP32 multigrid and 2 FP64 residual
         corrections.
`value` = N^3 / (time of one SR solve), inputs resident in HBM.  Each solver
also reports its fraction of the HBM peak: algorithmic bytes per solve (the
library's schedule model) and, where committed counter readings of the same
kernel sources exist, measured HBM bytes per solve, each over its time.

Also reported, outside the timed region: the same three solvers on the 32^3
sine and 512^3 polynomial workloads; the paper's own model problem (27-point
finite volume stencil, Chebyshev smoothers, 512 x 256 x 256 cells, global and
SR); the V-cycle solver to a relative
residual of 1e-4; error and residual of every solver for N = 32..256; the
dominant kernel's roofline (HIP events around each of its launches, with the
stream held by a sleep kernel until every launch is queued); the CPU
oracle's throughput on a bounded sample (built for the host CPU, at all
threads and at one); and the accuracy against the closed-form discrete
solution.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N, LEVELS, K, S, J = 256, 8, 3, 8, (2, 4, 6)
METRIC = "FMG solve DOF/s + % HBM peak at 256^3 (global vs SR vs FP32-refined SR)"
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")

# solver variants on an edge-N workload: keyword arguments of fmg.Plan
def variant_specs(levels, sr_levels, segments, buffers):
    return {
        "sr": dict(levels=levels, sr_levels=sr_levels, segments=segments, buffers=buffers),
        "global": dict(levels=levels),
        "sr32r": dict(levels=levels, sr_levels=sr_levels, segments=segments, buffers=buffers,
                      precision="fp32_refined", refine_iters=2),
    }


SPECS = variant_specs(LEVELS, K, S, J)


def source_hash():
    """Hash of the 7-point solver's sources (the model-problem solver,
    fv27.hip, builds none of its kernels)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1406_7808_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.startswith("fv27"):
            continue
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def symbol_pattern(label, dtype="double"):
    """Regular expression for the demangled symbol (as rocprofv3 prints it)
    of the kernel instantiation a profile label stands for."""
    base, _, arg = label.partition("<")
    args = arg.rstrip(">").split(",")
    pro = {"load": 0, "interp": 1, "correct": 2}
    if base == "k_smooth_z":
        ns = int(args[1][2:])
        ry = int(args[2][2:])
        res = 1 if "res" in args[3:] else 0
        return r"fmg::k_smooth_z<%s, %d, %d, 1024, %d, \d+, \d+, %d>" % (dtype, ns, pro[args[0]],
                                                                          ry, res)
    if base == "k_smooth_box":
        return r"fmg::k_smooth_box<%s, %d>" % (dtype, pro[args[0]])
    if base == "k_smooth_cols":
        ns = int(args[1][2:])
        res = 1 if "res" in args[2:] else 0
        return r"fmg::k_smooth_cols<%s, %d, %d, %d, \d+>" % (dtype, ns, pro[args[0]], res)
    return r"fmg::%s[<(]" % base


def load_traffic():
    """profiles/traffic.json if it was taken on the current kernel sources."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    return t


COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read and 1 GiB written


def counter_pass(args):
    """The workload run under rocprofv3 --pmc: `steps` solves of one variant,
    then a plain device-to-device copy of COPY_BYTES whose counter readings
    scale the solver's (FETCH_SIZE / WRITE_SIZE are reported in KiB)."""
    import torch
    from paper_1406_7808_amd import fmg
    from paper_1406_7808_amd import workloads as W
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    f, _, _ = W.fourier(N)
    fd = torch.from_numpy(f).to(dev)
    spec = dict(SPECS[args.variant])
    plan = fmg.Plan(N, spec.pop("levels"), **spec)
    u = torch.empty_like(fd)
    for _ in range(args.steps):
        plan.execute(fd, u)
    torch.cuda.synchronize()
    print("counter pass: %d %s solves done" % (args.steps, args.variant), flush=True)
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("counter pass: 3 copies of %d bytes done" % COPY_BYTES, flush=True)
    plan.close()
    return 0


def _pmc_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _symbol(kernel_name):
    return kernel_name.split("(")[0].replace("void ", "").strip()


def traffic_from(variant, solves, fetch_csv, write_csv, commands):
    """Add `variant` to profiles/traffic.json from two rocprofv3 --pmc runs
    of counter_pass (`solves` solves each): per counter, every fmg:: dispatch
    scaled by the calibration copy's bytes per counted unit (the copy is the
    largest copyBuffer dispatch of the run); HBM bytes per solve, and per
    kernel symbol the mean bytes per launch."""
    res = {}
    per_symbol = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _pmc_rows(path) if r.get("Counter_Name") == counter]
        copies = [r for r in rows if "copyBuffer" in r.get("Kernel_Name", "")]
        if not copies:
            raise SystemExit("traffic: no calibration copy in %s" % path)
        big = max(int(r["Grid_Size"]) for r in copies)
        copy = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        scale = COPY_BYTES / (sum(copy) / len(copy))  # bytes per counted unit
        kern = [r for r in rows if "fmg::" in r.get("Kernel_Name", "")]
        if not kern:
            raise SystemExit("traffic: no fmg:: dispatches in %s" % path)
        total = sum(float(r["Counter_Value"]) for r in kern) * scale
        res[counter] = {"dispatches": len(kern), "copy_mean_counter": sum(copy) / len(copy),
                        "copy_bytes": COPY_BYTES, "bytes_per_unit": scale,
                        "bytes_per_solve": total / solves}
        for r in kern:
            e = per_symbol.setdefault(_symbol(r["Kernel_Name"]), {})
            c = e.setdefault(counter, [0, 0.0])
            c[0] += 1
            c[1] += float(r["Counter_Value"]) * scale
    kernels = {}
    for sym, e in per_symbol.items():
        fe = e.get("FETCH_SIZE", [1, 0.0])
        wr = e.get("WRITE_SIZE", [1, 0.0])
        kernels[sym] = {"launches_per_solve": fe[0] / solves,
                        "fetch_bytes_per_launch": fe[1] / fe[0],
                        "write_bytes_per_launch": wr[1] / wr[0],
                        "bytes_per_launch": fe[1] / fe[0] + wr[1] / wr[0]}
    t = {}
    if os.path.exists(TRAFFIC):
        with open(TRAFFIC) as fh:
            t = json.load(fh)
    if t.get("source_hash") != source_hash() or "variants" not in t:
        t = {"source_hash": source_hash(), "variants": {}}
    t["variants"][variant] = {
        "solves": solves,
        "bytes_per_solve": res["FETCH_SIZE"]["bytes_per_solve"] + res["WRITE_SIZE"]["bytes_per_solve"],
        "counters": res, "kernels": kernels, "commands": commands}
    with open(TRAFFIC, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
    print(json.dumps({"variant": variant, "bytes_per_solve": t["variants"][variant]["bytes_per_solve"]}))
    return 0


def time_graph(run, steps, warmup):
    """ms per call of run() (which enqueues on torch's current stream),
    captured once into a graph and replayed `steps` times."""
    import torch
    for _ in range(max(1, warmup)):
        run()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    graph.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    del graph
    return e0.elapsed_time(e1) / steps


def time_solver(fmg, fd, spec, steps, warmup, graph=True):
    """(ms per solve, plan, u) for a plan of `spec` on fd."""
    import torch
    n = fd.shape[0]
    sp = dict(spec)
    plan = fmg.Plan(n, sp.pop("levels"), **sp)
    u = torch.empty_like(fd)
    if graph:
        ms = time_graph(lambda: plan.execute(fd, u), steps, warmup)
    else:
        for _ in range(max(1, warmup)):
            plan.execute(fd, u)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.execute(fd, u)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    return ms, plan, u


def hbm_fracs(fmg, n, spec, ms, measured=None):
    """Algorithmic bytes per solve (schedule model), measured bytes per solve
    (if given) and their fractions of the HBM peak at ms per solve."""
    sp = dict(spec)
    _, model_bytes, _ = fmg.schedule_model(n, **sp)
    out = {"model_bytes_per_solve": model_bytes,
           "model_B_per_DOF": round(model_bytes / n ** 3, 2),
           "model_GB_per_s": round(model_bytes / (ms * 1e-3) / 1e9, 1),
           "hbm_frac_model": round(model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "measured_bytes_per_solve": measured,
           "hbm_frac_measured": (round(measured / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                 if measured else None)}
    return out


def batch_leg(precision, args):
    """96 right-hand sides of edges 64, 96 and 128 (seeded), SR on the two
    finest levels, solved side by side on 8 streams and replayed as one
    graph; knobs tuned on the batch graph (cached per library build)."""
    import torch
    from paper_1406_7808_amd import batched
    from paper_1406_7808_amd import workloads as W
    items = W.batch()
    edges = [n for n, _, _ in items]
    fs = [torch.from_numpy(W.fourier_field(n, k, a)).cuda() for n, k, a in items]
    us = [torch.empty_like(f) for f in fs]
    b, probs = batched.build(edges, precision=precision, streams=8, tuned=True, fs=fs, us=us)
    side = torch.cuda.Stream()
    b.capture(fs, us, side)
    for _ in range(max(1, args.warmup)):
        b.replay(side)
    side.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(side)
    for _ in range(args.steps):
        b.replay(side)
    e1.record(side)
    side.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    dof = sum(n ** 3 for n in edges)
    out = {"ms": round(ms, 4), "dof_per_s": dof / (ms * 1e-3), "solves": len(edges),
           "edges": {str(n): edges.count(n) for n in sorted(set(edges))}, "streams": 8,
           "graph": True, "workspace_MB": round(b.workspace_bytes / 2 ** 20, 1)}
    b.close()
    return out


def dominant_kernel(fmg, plan, fd, traffic):
    """Per-launch HIP events over 3 solves of the headline plan.  A sleep
    kernel holds the stream first, so every launch and event is queued
    before the GPU reaches them and each bracket holds only its kernel.  The
    dominant kernel is the instantiation (one rocprofv3 symbol) with the
    largest total time among those launched with more than one workgroup (a
    single-workgroup kernel is latency bound and has no HBM roofline)."""
    import torch
    u = torch.empty_like(fd)
    plan.execute(fd, u)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda._sleep(200_000_000)  # ~0.1 s of GPU cycles: the host queues ahead
    for _ in range(3):
        plan.execute(fd, u)
    stats = plan.profile_read()
    plan.profile(False)
    by_kernel, label_of = {}, {}
    for k, v in stats.items():
        name = k.split("@")[0]
        sym = symbol_pattern(name)
        label_of.setdefault(sym, name)
        a = by_kernel.setdefault(sym, [0, 0.0, 0.0])
        for i in range(3):
            a[i] += v[i]
    single = ("k_coarse",)
    cand = {s: v for s, v in by_kernel.items() if not label_of[s].startswith(single)}
    sym = max(cand, key=lambda k: cand[k][1])
    kern = label_of[sym]
    launches, tot_ms, tot_bytes = cand[sym]
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    meas = None
    if traffic and "sr" in traffic.get("variants", {}):
        pat = re.compile(sym)
        for s, e in traffic["variants"]["sr"]["kernels"].items():
            if pat.fullmatch(s) or pat.match(s):
                meas = e["bytes_per_launch"]
    kernels = {k: {"launches": v[0] // 3, "ms_per_solve": round(v[1] / 3, 4),
                   "GB_per_s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
    roofline = {"bound": "hbm", "kernel": kern, "symbol": sym, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": meas, "launches_per_solve": launches // 3,
                "avg_launch_us": round(tot_ms / launches * 1e3, 2),
                "bytes_per_launch": tot_bytes / launches,
                "event_sum_ms_per_solve": round(sum(v[1] for v in stats.values()) / 3, 4)}
    return roofline, kernels


def other_configs(fmg, W, ex, args):
    """The 32^3 sine and 512^3 polynomial workloads: the three solvers each,
    graph-replayed, with their HBM fractions and accuracy."""
    import numpy as np
    import torch
    out = {}
    cfgs = [("poisson3d-32^3-sine", 32, variant_specs(5, 2, 2, (2, 2))),
            ("poisson3d-512^3-polynomial", 512, variant_specs(8, 3, 16, (2, 4, 6)))]
    for name, n, specs in cfgs:
        if n == 32:
            f, uc = W.sine(n)
            ud = uc * ex.sine_discrete(n)
        else:
            f, uc = W.polynomial(n)
            ud = None  # the DST-II solve of 512^3 costs ~1 minute of host time: not here
        fd = torch.from_numpy(f).cuda()
        entry = {}
        for v, spec in specs.items():
            ms, plan, u = time_solver(fmg, fd, spec, args.steps, args.warmup)
            e = {"ms": round(ms, 4), "dof_per_s": n ** 3 / (ms * 1e-3)}
            e.update(hbm_fracs(fmg, n, spec, ms))
            uh = u.cpu().numpy()
            e["e_total"] = float(np.abs(uh - uc).max())
            if ud is not None:
                e["e_alg_over_e_disc"] = float(np.abs(uh - ud).max() / np.abs(ud - uc).max())
            entry[v] = e
            plan.close()
            print("bench: %s %s %.3f ms/solve" % (name, v, ms), file=sys.stderr, flush=True)
        out[name] = entry
        del fd
        torch.cuda.empty_cache()
    return out


def vcycle_leg(fmg, fd, ud, uc, edisc, args):
    """The comparison solver (Sec. 7, Fig. 10) on the 256^3 workload: V(2,2)
    cycles from u = 0 until max|f - L u| <= 1e-4 max|f|; then the same cycle
    count timed as one graph (no residual checks inside)."""
    import numpy as np
    import torch
    plan = fmg.Plan(N, LEVELS)
    u = torch.zeros_like(fd)
    it, rr = plan.vcycles(fd, u, rtol=1e-4, maxit=60)
    uh = u.cpu().numpy()
    w = torch.empty_like(fd)

    def run():
        w.zero_()
        plan.vcycles(fd, w, rtol=0.0, maxit=it, residual=False)

    ms = time_graph(run, max(3, args.steps // 4), 1)
    torch.cuda.synchronize()
    same = bool(torch.equal(w, u))
    out = {"rtol": 1e-4, "cycles": it, "relres_inf": rr, "ms": round(ms, 4),
           "dof_per_s": N ** 3 / (ms * 1e-3), "graph_result_equals_iterated": same,
           "e_alg_over_e_disc": float(np.abs(uh - ud).max() / edisc),
           "e_total": float(np.abs(uh - uc).max())}
    plan.close()
    return out


def convergence_study(fmg, W, ex):
    """Error and residual (max norms) of G, SR and the V-cycle solver to
    rtol 1e-4 for N = 32..256 on the Fourier right-hand side (Sec. 7,
    Figs. 8 and 10): SR with 3 levels, 4^3 segments, buffers 2, 4, 6.  The
    error is against the continuous solution at cell centers."""
    import numpy as np
    import torch
    rows = {"N": [], "global": {"err": [], "res": []}, "sr": {"err": [], "res": []},
            "vcycle": {"err": [], "res": [], "cycles": []}}
    for n in (32, 64, 128, 256):
        L = int(math.log2(n))
        f, uc, _ = W.fourier(n)
        fd = torch.from_numpy(f).cuda()
        rows["N"].append(n)
        for v, kw in (("global", {}), ("sr", dict(sr_levels=3, segments=4, buffers=(2, 4, 6)))):
            u = fmg.solve(fd, L, **kw)
            rows[v]["err"].append(float(np.abs(u.cpu().numpy() - uc).max()))
            rows[v]["res"].append(fmg.residual_norms(fd, u)[0])
        plan = fmg.Plan(n, L)
        u = torch.zeros_like(fd)
        it, _ = plan.vcycles(fd, u, rtol=1e-4, maxit=60)
        plan.close()
        rows["vcycle"]["err"].append(float(np.abs(u.cpu().numpy() - uc).max()))
        rows["vcycle"]["res"].append(fmg.residual_norms(fd, u)[0])
        rows["vcycle"]["cycles"].append(it)
    for v in ("global", "sr", "vcycle"):
        for q in ("err", "res"):
            a = rows[v][q]
            rows[v][q + "_order"] = [round(math.log2(a[i] / a[i + 1]), 3) for i in range(len(a) - 1)]
    return rows


def fv27_leg(args):
    """The paper's own model problem (Sec. 5.1): 27-point finite volume
    stencil, Chebyshev smoothers F(1,2,2), trilinear prolongation, on
    [0,2] x [0,1]^2 with 512 x 256 x 256 cells, u = prod(x_i^4 - R_i^2 x_i^2);
    global FMG and SR with the 4 x 2 x 2 segment grid on the 4 finest levels
    (8^3 genuine transition cells per segment), buffers from Eq. 5 with A = 4,
    B = 1.  Graph-replayed solves; e_r = e_SR / e_conv as in Tables 1-3."""
    import numpy as np
    import torch
    from paper_1406_7808_amd import fv27
    from paper_1406_7808_amd import workloads as W
    m, K, S = 256, 4, (4, 2, 2)
    J = W.buffer_schedule(4, 1, K)
    f, uc, h = W.paper_model(m)
    L = int(math.log2(m)) + 1
    n = (2 * m, m, m)
    fd = torch.from_numpy(f).cuda()
    out = {"cells": 2 * m ** 3, "levels": L, "sr_levels": K, "segments": list(S),
           "buffers_finest_first": J, "degrees": [2, 2, 1]}
    errs = {}
    for name, kw in (("global", {}), ("sr", dict(sr_levels=K, segments=S, buffers=J))):
        plan = fv27.Plan(n, h, L, **kw)
        u = torch.empty_like(fd)
        ms = time_graph(lambda: plan.execute(fd, u), max(3, args.steps // 2), args.warmup)
        launches, model_bytes = plan.model()
        errs[name] = float(np.abs(u.cpu().numpy() - uc).max())
        out[name] = {"ms": round(ms, 4), "dof_per_s": 2 * m ** 3 / (ms * 1e-3),
                     "launches": launches, "model_bytes_per_solve": model_bytes,
                     "model_B_per_DOF": round(model_bytes / (2 * m ** 3), 1),
                     "hbm_frac_model": round(model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "e_total": errs[name],
                     "workspace_MB": round(plan.workspace_bytes / 2 ** 20, 1)}
        plan.close()
        print("bench: fv27 %s %.3f ms/solve" % (name, ms), file=sys.stderr, flush=True)
    out["e_r"] = errs["sr"] / errs["global"]
    return out


def cpu_leg(f, fd_result):
    """The oracle's SR solve of the 256^3 workload, built for this host's CPU
    (-O3 -march=native), at all OpenMP threads for about 12 s and at one
    thread for one solve."""
    import numpy as np
    import oracle
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    so = oracle.build_native(tempfile.mkdtemp(prefix="fmg_oracle_"))
    oracle.use_library(so)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    oracle.set_threads(nthreads)
    ref, reps, tc = None, 0, time.time()
    while reps < 40 and (reps == 0 or time.time() - tc < 12.0):
        ref = oracle.srfmg(f, LEVELS, K, S, list(J))
        reps += 1
    el = time.time() - tc
    oracle.set_threads(1)
    t1 = time.time()
    oracle.srfmg(f, LEVELS, K, S, list(J))
    el1 = time.time() - t1
    oracle.set_threads(nthreads)
    cpu = {"value": reps * N ** 3 / el, "unit": "DOF/s", "cores": nthreads, "kind": "oracle",
           "sample": "%d SR-FMG FP64 solve(s) of the same 256^3 workload in %.1f s at %d threads; "
                     "gcc -O3 -march=native -fopenmp on this host" % (reps, el, nthreads),
           "one_thread_dof_per_s": N ** 3 / el1, "cpu_model": model}
    parity = float(np.abs(fd_result - ref).max() / np.abs(ref).max()) if fd_result is not None else None
    return cpu, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-graph", action="store_true", help="launch kernels directly")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 32^3 / 512^3 workloads, the V-cycle solver and the N sweep")
    ap.add_argument("--variants", default="sr,global,sr32r,batch96,batch96_fp32r")
    ap.add_argument("--counter-pass", action="store_true",
                    help="run one variant for rocprofv3 --pmc (solves + calibration copy)")
    ap.add_argument("--variant", default="sr", choices=sorted(SPECS))
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="add --variant to profiles/traffic.json from two counter-pass CSVs "
                         "(--steps solves each)")
    ap.add_argument("--commands", default="", help="commands recorded in traffic.json")
    ap.add_argument("--fv27-only", action="store_true",
                    help="run only the model-problem leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.traffic_from:
        return traffic_from(args.variant, args.steps, args.traffic_from[0], args.traffic_from[1],
                            args.commands)
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is design-only)" % args.gpus, file=sys.stderr)
        return 2
    if args.counter_pass:
        return counter_pass(args)
    if args.fv27_only:
        print(json.dumps(fv27_leg(args)))
        return 0

    import numpy as np
    import torch

    from paper_1406_7808_amd import fmg
    from paper_1406_7808_amd import workloads as W
    import oracle.exact as ex  # closed forms only (test infrastructure)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    f, ucont, (kk, aa) = W.fourier(N)
    fd = torch.from_numpy(f).to(dev)
    print("bench: inputs ready (%.1fs)" % (time.time() - t0), file=sys.stderr, flush=True)

    traffic = load_traffic()
    names = [v for v in args.variants.split(",") if v]
    batch_names = [v for v in names if v.startswith("batch96")]
    names = [v for v in names if v not in batch_names]
    res, outs, plans = {}, {}, {}
    for name in names:
        ms, plan, u = time_solver(fmg, fd, SPECS[name], args.steps, args.warmup,
                                  graph=not args.no_graph)
        plans[name] = plan
        meas = None
        if traffic and name in traffic.get("variants", {}):
            meas = traffic["variants"][name]["bytes_per_solve"]
        res[name] = {"ms": round(ms, 4), "dof_per_s": N ** 3 / (ms * 1e-3),
                     "workspace_MB": round(plan.workspace_bytes / 2 ** 20, 1),
                     "graph": not args.no_graph}
        res[name].update(hbm_fracs(fmg, N, SPECS[name], ms, meas))
        outs[name] = u.cpu().numpy()
        print("bench: %s %.3f ms/solve" % (name, ms), file=sys.stderr, flush=True)

    for name in batch_names:
        res[name] = batch_leg("fp32_refined" if name.endswith("fp32r") else "fp64", args)
        print("bench: %s %.3f ms per batch" % (name, res[name]["ms"]), file=sys.stderr, flush=True)

    head = names[0]
    roofline, kernels = dominant_kernel(fmg, plans[head], fd, traffic)
    print("bench: dominant kernel %s" % roofline["kernel"], file=sys.stderr, flush=True)

    # accuracy against the closed-form discrete solution
    ud = W.fourier_field(N, kk, ex.modes_discrete(N, kk, aa))
    edisc = float(np.abs(ud - ucont).max())
    acc = {"e_disc": edisc}
    for name, u in outs.items():
        acc[name] = {"e_alg_over_e_disc": float(np.abs(u - ud).max() / edisc),
                     "e_total": float(np.abs(u - ucont).max())}
    if "sr" in outs and "global" in outs:
        acc["e_r_sr_over_global"] = acc["sr"]["e_total"] / acc["global"]["e_total"]

    extra = {}
    if not args.no_extra:
        extra["vcycle_rtol_1e-4"] = vcycle_leg(fmg, fd, ud, ucont, edisc, args)
        print("bench: vcycle leg done", file=sys.stderr, flush=True)
        extra["other_configs"] = other_configs(fmg, W, ex, args)
        extra["convergence_N32_256"] = convergence_study(fmg, W, ex)
        print("bench: convergence study done", file=sys.stderr, flush=True)
        extra["paper_model_fv27"] = fv27_leg(args)

    cpu = None
    if not args.no_cpu:
        cpu, parity = cpu_leg(f, outs.get("sr"))
        if parity is not None:
            acc["sr_parity_rel_vs_oracle"] = parity
        print("bench: cpu leg done", file=sys.stderr, flush=True)

    head_ms = res[head]["ms"]
    out = {
        "metric": METRIC,
        "value": N ** 3 / (head_ms * 1e-3),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson3d-256^3-fp64-srfmg", "N": N, "levels": LEVELS,
                   "sr_levels": K, "segments_per_dim": S, "buffers_finest_first": list(J),
                   "cycle": "F(1,2,2)", "rhs": "64 sine modes, seed 14067808",
                   "headline": head},
        "hbm_frac_per_variant": {v: {"model": res[v]["hbm_frac_model"],
                                     "measured": res[v]["hbm_frac_measured"]} for v in names},
        "variants": res,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "accuracy": acc,
    }
    out.update(extra)
    for p in plans.values():
        p.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
