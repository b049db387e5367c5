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
`value` = N^3 / (time of one SR solve), inputs resident in HBM.

Also reported: the dominant kernel's roofline (HIP events around each of its
launches in a profiled pass, algorithmic bytes from the launch geometry), the
CPU oracle's throughput on a bounded sample, and the accuracy of each solver
against the closed-form discrete solution.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N, LEVELS, K, S, J = 256, 8, 3, 8, (2, 4, 6)
METRIC = "FMG solve DOF/s + % HBM peak at 256^3 (global vs SR vs FP32-refined SR)"


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1406_7808_amd", "csrc")
    for name in sorted(os.listdir(d)):
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
    return r"fmg::%s[<(]" % base


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter
    summaries (profiles/traffic.json), or None when absent or taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash() or t.get("symbol_pattern") != symbol_pattern(kernel):
        return None
    return t.get("bytes_per_launch")


COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read and 1 GiB written


def counter_pass(args):
    """The workload run under rocprofv3 --pmc: a few headline solves, then a
    plain device-to-device copy of COPY_BYTES whose counter readings scale
    the solver's (FETCH_SIZE / WRITE_SIZE are reported in KiB)."""
    import torch
    from paper_1406_7808_amd import fmg
    from paper_1406_7808_amd import workloads as W
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    f, _, _ = W.fourier(N)
    fd = torch.from_numpy(f).to(dev)
    plan = fmg.Plan(N, LEVELS, sr_levels=K, segments=S, buffers=J)
    u = torch.empty_like(fd)
    for _ in range(args.steps):
        plan.execute(fd, u)
    torch.cuda.synchronize()
    print("counter pass: %d solves done" % args.steps, flush=True)
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


def traffic_from(fetch_csv, write_csv, kernel, out_path, commands):
    """profiles/traffic.json from two rocprofv3 --pmc runs of counter_pass:
    mean KiB per dispatch of `kernel`, scaled by the calibration copy's bytes
    per KiB (the copy is the largest copyBuffer dispatch of the run), and the
    same scaled figures for every kernel of the run."""
    pat = re.compile(symbol_pattern(kernel))
    res, table = {}, {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _pmc_rows(path) if r.get("Counter_Name") == counter]
        copies = [r for r in rows if "copyBuffer" in r.get("Kernel_Name", "")]
        if not copies:
            raise SystemExit("traffic: no calibration copy in %s" % path)
        big = max(int(r["Grid_Size"]) for r in copies)
        copy = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        scale = COPY_BYTES / (sum(copy) / len(copy))  # bytes per counted unit
        kern = [float(r["Counter_Value"]) for r in rows if pat.search(r.get("Kernel_Name", ""))]
        if not kern:
            raise SystemExit("traffic: no %s rows for %s in %s" % (counter, kernel, path))
        res[counter] = {"dispatches": len(kern), "mean_counter": sum(kern) / len(kern),
                        "copy_mean_counter": sum(copy) / len(copy),
                        "copy_bytes": COPY_BYTES, "bytes_per_unit": scale,
                        "bytes_per_launch": sum(kern) / len(kern) * scale}
        for r in rows:
            name = r.get("Kernel_Name", "").split("(")[0].replace("void ", "")
            if "fmg::" not in name:
                continue
            key = "%s grid=%s" % (name, r["Grid_Size"])
            e = table.setdefault(key, {"dispatches": 0})
            e["dispatches"] = max(e["dispatches"], e.get("_n" + counter, 0) + 1)
            e["_n" + counter] = e.get("_n" + counter, 0) + 1
            e[counter + "_MB"] = e.get(counter + "_MB", 0.0) + float(r["Counter_Value"]) * scale / 1e6
    for e in table.values():
        n = e.pop("_nFETCH_SIZE", 1)
        e["FETCH_SIZE_MB"] = round(e.get("FETCH_SIZE_MB", 0.0) / n, 2)
        n = e.pop("_nWRITE_SIZE", 1)
        e["WRITE_SIZE_MB"] = round(e.get("WRITE_SIZE_MB", 0.0) / n, 2)
    out = {"kernel": kernel, "symbol_pattern": symbol_pattern(kernel),
           "source_hash": source_hash(),
           "bytes_per_launch": res["FETCH_SIZE"]["bytes_per_launch"]
           + res["WRITE_SIZE"]["bytes_per_launch"],
           "counters": res, "per_dispatch_MB": table, "commands": commands}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "per_dispatch_MB"}))
    return 0


def batch_leg(precision, args):
    """96 right-hand sides of edges 64, 96 and 128 (seeded), SR on the two
    finest levels, solved side by side on 8 streams and replayed as one
    graph; knobs tuned on the batch graph (cached per library build)."""
    import torch
    from paper_1406_7808_amd import batched
    from paper_1406_7808_amd import workloads as W
    items = W.batch()
    edges = [N for N, _, _ in items]
    fs = [torch.from_numpy(W.fourier_field(N, k, a)).cuda() for N, k, a in items]
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
    dof = sum(N ** 3 for N in edges)
    out = {"ms": round(ms, 4), "dof_per_s": dof / (ms * 1e-3), "solves": len(edges),
           "edges": {str(n): edges.count(n) for n in sorted(set(edges))}, "streams": 8,
           "graph": True, "workspace_MB": round(b.workspace_bytes / 2 ** 20, 1)}
    b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-graph", action="store_true", help="launch kernels directly")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--variants", default="sr,global,sr32r,batch96,batch96_fp32r")
    ap.add_argument("--counter-pass", action="store_true",
                    help="run the workload for rocprofv3 --pmc (solves + calibration copy)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two counter-pass CSVs")
    ap.add_argument("--kernel", default="k_smooth_z<load,ns4,ry2>",
                    help="profile label whose traffic --traffic-from extracts")
    ap.add_argument("--commands", default="", help="commands recorded in traffic.json")
    args = ap.parse_args()
    if args.traffic_from:
        return traffic_from(args.traffic_from[0], args.traffic_from[1], args.kernel,
                            os.path.join(ROOT, "profiles", "traffic.json"), args.commands)
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is design-only)" % args.gpus, file=sys.stderr)
        return 2
    if args.counter_pass:
        return counter_pass(args)

    import numpy as np
    import torch

    from paper_1406_7808_amd import fmg
    from paper_1406_7808_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    f, ucont, (kk, aa) = W.fourier(N)
    fd = torch.from_numpy(f).to(dev)
    print("bench: inputs ready (%.1fs)" % (time.time() - t0), file=sys.stderr, flush=True)

    specs = {
        "sr": dict(sr_levels=K, segments=S, buffers=J),
        "global": dict(),
        "sr32r": dict(sr_levels=K, segments=S, buffers=J, precision="fp32_refined",
                      refine_iters=2),
    }
    names = [v for v in args.variants.split(",") if v]
    batch_names = [v for v in names if v.startswith("batch96")]
    names = [v for v in names if v not in batch_names]
    res, outs, plans = {}, {}, {}
    for name in names:
        plan = fmg.Plan(N, LEVELS, **specs[name])
        plans[name] = plan
        u = torch.empty_like(fd)
        for _ in range(max(1, args.warmup)):
            plan.execute(fd, u)
        torch.cuda.synchronize()
        graph = None
        if not args.no_graph:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                plan.execute(fd, u)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                plan.execute(fd, u)
            graph.replay()
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            if graph is not None:
                graph.replay()
            else:
                plan.execute(fd, u)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = {"ms": round(ms, 4), "dof_per_s": N ** 3 / (ms * 1e-3),
                     "workspace_MB": round(plan.workspace_bytes / 2 ** 20, 1),
                     "graph": graph is not None}
        outs[name] = u.cpu().numpy()
        print("bench: %s %.3f ms/solve" % (name, ms), file=sys.stderr, flush=True)
        del graph

    for name in batch_names:
        res[name] = batch_leg("fp32_refined" if name.endswith("fp32r") else "fp64", args)
        print("bench: %s %.3f ms per batch" % (name, res[name]["ms"]), file=sys.stderr, flush=True)

    # dominant kernel of the headline solve: event-timed launches
    head = names[0]
    plan = plans[head]
    plan.profile(True)
    u = torch.empty_like(fd)
    for _ in range(3):
        plan.execute(fd, u)
    stats = plan.profile_read()
    plan.profile(False)
    # the dominant kernel: the instantiation (one rocprofv3 symbol) with the
    # largest total time over all its levels and labels
    by_kernel, label_of = {}, {}
    for k, v in stats.items():
        name = k.split("@")[0]
        sym = symbol_pattern(name)
        label_of.setdefault(sym, name)
        a = by_kernel.setdefault(sym, [0, 0.0, 0.0])
        for i in range(3):
            a[i] += v[i]
    sym = max(by_kernel, key=lambda k: by_kernel[k][1])
    kern = label_of[sym]
    launches, tot_ms, tot_bytes = by_kernel[sym]
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    traffic = measured_traffic(kern)
    kernels = {k: {"launches": v[0] // 3, "ms_per_solve": round(v[1] / 3, 4),
                   "GB_per_s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
    roofline = {"bound": "hbm", "kernel": kern, "symbol": symbol_pattern(kern), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "launches_per_solve": launches // 3,
                "avg_launch_us": round(tot_ms / launches * 1e3, 2),
                "bytes_per_launch": tot_bytes / launches}

    # accuracy against the closed-form discrete solution
    import oracle.exact as ex  # closed forms only (test infrastructure)
    ud = W.fourier_field(N, kk, ex.modes_discrete(N, kk, aa))
    edisc = float(np.abs(ud - ucont).max())
    acc = {"e_disc": edisc}
    for name, u in outs.items():
        acc[name] = {"e_alg_over_e_disc": float(np.abs(u - ud).max() / edisc),
                     "e_total": float(np.abs(u - ucont).max())}
    if "sr" in outs and "global" in outs:
        acc["e_r_sr_over_global"] = acc["sr"]["e_total"] / acc["global"]["e_total"]

    cpu = None
    if not args.no_cpu:
        import oracle
        ref, reps, tc = None, 0, time.time()
        # a bounded sample: whole solves until about 12 s have passed
        while reps < 40 and (reps == 0 or time.time() - tc < 12.0):
            ref = oracle.srfmg(f, LEVELS, K, S, list(J))
            reps += 1
        el = time.time() - tc
        cpu = {"value": reps * N ** 3 / el, "unit": "DOF/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": "%d SR-FMG FP64 solve(s) of the same 256^3 workload, %.1f s" % (reps, el)}
        if "sr" in outs:
            acc["sr_parity_rel_vs_oracle"] = float(np.abs(outs["sr"] - ref).max()
                                                   / np.abs(ref).max())

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
        "variants": res,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "accuracy": acc,
    }
    for p in plans.values():
        p.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
