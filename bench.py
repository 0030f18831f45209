#!/usr/bin/env python3
"""Throughput of the QSL Squasher hot path on one MI355X.

One step = one whole photospheric Q / length / FLEDGE map of a 4-charge
potential field on a 256x256x128 FP32 grid: 1024^2 base lines traced both ways
(adaptive Cash-Karp 5(4), FP32 stepping, FP64 landing and Q), the Sobel FLEDGE
map, FLL-jump refinement along the Hilbert curve to 4x the base resolution
(two levels, every pass on the device), and the array converter.  Inputs are
resident in HBM before timing starts.

Printed (one JSON line): lines traced with Q per second, the stepping
kernel's achieved FLOP rate against the VALU ceiling, the oracle's throughput
on the host cores on a bounded sample, and the median relative log10 Q error
against the FP64 oracle at tolerance 1e-10 on a fixed set of lines.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "field lines traced with Q per sec (1 GPU) + % HBM/L2 roofline at fixed log10 Q err"

# Algorithmic FLOPs of the stepping kernel (FMA = 2), counted from the method:
#  per RHS evaluation: trilinear value + grid-unit gradient of 3 components via
#  the 7-lerp tree (33 each), 9 scalings to physical units, J.dx1 and J.dx2
#  (30), direction sign (9)                                            -> 147
#  per step attempt: Cash-Karp stage inputs for stages 2..6 on 9 components
#  (378), 5th-order combination (63), error combination (81), update (18),
#  error norm (54), controller (6)                                     -> 600
FLOP_PER_EVAL = 147
FLOP_PER_ATTEMPT = 600
# VALU ceiling for this kernel: 256 CUs x 4 SIMD x 16 lanes x 2 FLOP (FMA) x
# 2.4 GHz; packed FP32 is disabled in the build, so the packed-FP32 rate
# (157.3 TFLOP/s) is out of reach and is not the ceiling.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-4, help="stepping rtol = atol")
    ap.add_argument("--base-level", type=int, default=10)
    ap.add_argument("--refine-levels", type=int, default=2)
    ap.add_argument("--threshold", type=float, default=0.02)
    ap.add_argument("--cpu-level", type=int, default=9, help="base level of the oracle's sample map")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy leg")
    ap.add_argument("--accuracy-lines", type=int, default=256)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1609_00724_amd as q
    import synth
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import MapSpec, Profiler, QMapPlan, make_opts

    dev = torch.device("cuda:0")
    w = synth.charges_c2()
    h = min(w["spacing"])
    b = [torch.from_numpy(c).to(dev) for c in w["b"]]
    field = q.field_init(*b, w["origin"], w["spacing"], storage="f32")
    m, r = args.base_level, args.refine_levels
    spec = MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, args.threshold)
    plan = QMapPlan(spec, 4 ** m * 4, dev)
    opts = make_opts(args.tol, args.tol, h_init=0.1 * h, h_max=h, step_dtype="f32")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.run(field, opts)
    torch.cuda.synchronize()
    plan.work.zero_()
    with Profiler() as prof:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t0.record(stream)
        for _ in range(args.steps):
            plan.run(field, opts)
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms_total = t0.elapsed_time(t1)
        n_step, ms_step = prof.read(A.KERNEL_STEP)
        n_land, ms_land = prof.read(A.KERNEL_LAND)
        n_asm, ms_asm = prof.read(A.KERNEL_ASSEMBLE)
    Profiler.reset()
    res = plan.result()
    lines = res["count"]
    work = plan.work.cpu().numpy().astype(np.int64)
    attempts, evals, stepped, landed = (int(v) for v in work)
    ms_per_step = ms_total / args.steps
    value = lines / (ms_per_step / 1e3)

    flops = FLOP_PER_EVAL * evals + FLOP_PER_ATTEMPT * attempts
    achieved = flops / (ms_step / 1e3) / 1e12 if ms_step > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "lines/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"photospheric Q/FLL/FLEDGE map, 4-charge potential field on a 256x256x128 FP32 grid, "
                         f"{1 << m}^2 base lines + FLL-jump Hilbert refinement r={r} thr={args.threshold}, "
                         f"CK54 FP32 stepping tol={args.tol:g}, FP64 landing and Q"),
            "lines_per_step": lines,
            "base_lines": 4 ** m,
            "grid": [256, 256, 128],
            "tol": args.tol,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_trace (adaptive stepping)",
            "achieved": achieved,
            "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / VALU_PEAK_TFLOPS,
            "traffic": None,
            "launches": n_step,
            "avg_launch_ms": ms_step / max(n_step, 1),
            "algorithmic_flops_per_step": flops / args.steps,
            "rhs_evals_per_step": evals / args.steps,
            "attempts_per_step": attempts / args.steps,
        },
        "kernel_ms_per_step": {"step": ms_step / args.steps, "land": ms_land / args.steps,
                               "assemble": ms_asm / args.steps},
        "wall_s_timed": wall,
    }

    if not args.no_accuracy:
        out["accuracy"] = accuracy(args, field, w, h)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args, w, h)
    print(json.dumps(out), flush=True)


def _oracle_field(w):
    import numpy as np
    import oracle
    return oracle.Field.grid(*(c.astype(np.float64) for c in w["b"]), w["origin"], w["spacing"])


def accuracy(args, field, w, h):
    """Median relative log10 Q error of the GPU (bench settings) against the FP64
    oracle at tolerance 1e-10, on a fixed seeded set of photospheric lines."""
    import numpy as np
    import torch

    import oracle
    import paper_1609_00724_amd as q
    import synth
    seeds = synth.random_seeds(2024, args.accuracy_lines, z=0.0)
    g = q.trace(field, torch.from_numpy(seeds).cuda(), rtol=args.tol, atol=args.tol,
                h_init=0.1 * h, h_max=h, step_dtype="f32")
    torch.cuda.synchronize()
    qg = g["q_perp"].cpu().numpy()
    o = oracle.trace(_oracle_field(w), seeds, rtol=1e-10, atol=1e-10, h_init=0.1 * h, h_max=h)
    qo = o["q_perp"]
    m = np.isfinite(qo) & np.isfinite(qg) & (qo < 1e6) & (g["status"].cpu().numpy() == o["status"])
    rel = np.abs(np.log10(qg[m]) - np.log10(qo[m])) / np.abs(np.log10(qo[m]))
    return {"median_rel_log10q_err": float(np.median(rel)), "p90": float(np.percentile(rel, 90)),
            "p99": float(np.percentile(rel, 99)), "max": float(rel.max()),
            "lines": int(m.sum()), "reference": "FP64 oracle, tol 1e-10", "target_median": 1e-3}


def cpu_baseline(args, w, h):
    """The oracle (FP64 C + numpy refinement) on a bounded sample: the same map
    recipe at a coarser base level, on the host cores."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    fo = _oracle_field(w)
    plane = oracle.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)

    def fn(p):
        t = oracle.trace(fo, p, rtol=args.tol, atol=args.tol, h_init=0.1 * h, h_max=h, nthreads=threads)
        return {"fll": t["fll"], "q": t["q_perp"]}

    t0 = time.perf_counter()
    keys, _, _ = oracle.refine_slice(plane, args.cpu_level, args.refine_levels, args.threshold, fn)
    dt = time.perf_counter() - t0
    return {"value": keys.size / dt, "unit": "lines/s", "cores": threads, "kind": "oracle",
            "sample": (f"same field, tolerance and refinement rule; {1 << args.cpu_level}^2 base map "
                       f"({keys.size} lines, {dt:.1f} s)")}


if __name__ == "__main__":
    main()
