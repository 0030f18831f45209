#!/usr/bin/env python3
"""Throughput of the QSL Squasher hot path on one MI355X.

One step (default workload) = one whole refined 3D Q / length / FLEDGE volume
of a twisted flux rope over a 6-charge potential background on a 384x384x256
FP32 grid: 256^3 base cells traced both ways (adaptive Cash-Karp 5(4), FP32
stepping, FP64 landing and Q), the 3D Sobel FLEDGE map, FLL-jump refinement
along the 3D Hilbert curve to 4x the base resolution per axis (every pass on
the device), and the array converter.  Inputs are resident in HBM before
timing starts.  `--workload map` runs the photospheric 1024^2 map of a
4-charge field on a 256x256x128 grid instead.

Fixed-error protocol: on a fixed seeded set of lines, the GPU tracer at each
candidate setting (tolerance x largest step; Euler: step size) is compared
with the FP64 oracle at tolerance 1e-10 on the same gridded field; among the
settings whose median relative log10 Q error is <= 1e-3 the fastest map is
timed.  Printed (one JSON line): lines traced with Q per second at that
setting, the stepping kernel's achieved FLOP rate from the work of the kept
samples against the FP32 vector peak, the oracle's throughput on the host
cores (all allotted and one) on a bounded sample, and the sweep itself.
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
#  per explicit Euler step: the update of 9 components (18)            -> 18
FLOP_PER_EVAL = 147
#  per RHS evaluation with the K-node-per-axis stencils (K = 3 triquadratic,
#  4 tricubic): kernel weights and derivative weights of the 3 axes (45 / 90),
#  per component the separable sums -- along x 2 K^3 FMA, along y 3 K^2, along
#  z 4 K -- (186 / 384 FLOP, x 3 components), scalings, J.dx1, J.dx2 and the
#  sign (48)                                                   -> 651 / 1290
FLOP_PER_EVAL_ORDER = {"linear": FLOP_PER_EVAL, "quadratic": 651, "cubic": 1290}
FLOP_PER_ATTEMPT = 600
FLOP_PER_EULER_STEP = 18
# Published FP32 vector peak of the MI355X: 256 CUs x 4 SIMD x 16 lanes x
# 2 FLOP (FMA) x 2 (packed FP32, two lanes of work per instruction) x 2.4 GHz.
FP32_PEAK_TFLOPS = 157.3
# The same without packed FP32, which this build does not emit: the ceiling
# of one FP32 FMA per lane per clock.
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# fixed-error protocol
TARGET_MEDIAN = 1e-3
SWEEP_TOLS = (1e-2, 3e-3, 1e-3, 3e-4, 1e-4)
SWEEP_HMAX_CELLS = (1.0, 2.0, 3.0, 4.0, 6.0, 8.0)
SWEEP_EULER_DIVS = (5, 10, 20)     # Euler step = one grid cell / this


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("volume", "map", "batch", "learned"), default="volume",
                    help="volume: 3D Q/FLL/FLEDGE volume of a flux-rope field (default); map: photospheric map "
                         "of one field; batch: 64 fields in one batched trace; learned: the CNN proposer")
    ap.add_argument("--tol", type=float, default=None,
                    help="stepping rtol = atol; given with --hmax-cells it replaces the fixed-error sweep")
    ap.add_argument("--hmax-cells", type=float, default=None, help="largest step, in grid cells")
    ap.add_argument("--stepper", choices=("ck54", "euler"), default="ck54",
                    help="map / volume: adaptive Cash-Karp 5(4), or explicit Euler with fixed steps")
    ap.add_argument("--euler-div", type=int, default=None, help="Euler step = one cell / this (with --stepper euler)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the fixed-error sweep (settings from --tol / --hmax-cells, else 1e-4 and 1 cell)")
    ap.add_argument("--base-level", type=int, default=10, help="map workload: 2^m x 2^m base pixels")
    ap.add_argument("--volume-level", type=int, default=8, help="volume workload: 2^m cells a side")
    ap.add_argument("--refine-levels", type=int, default=2)
    ap.add_argument("--threshold", type=float, default=0.02)
    ap.add_argument("--refine-batch", type=int, default=0, help="refinement levels per device round (0: tuned)")
    ap.add_argument("--cpu-level", type=int, default=None,
                    help="base level of the oracle's sample (default: map 8, volume 5)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch shape")
    ap.add_argument("--launch", type=int, default=0, help="launch-shape word with --no-tune (0: library default)")
    ap.add_argument("--order", choices=("linear", "quadratic", "cubic"), default="linear",
                    help="map / volume: interpolation kernel (trilinear, Dodgson triquadratic, Keys tricubic)")
    ap.add_argument("--cell-records", action="store_true",
                    help="add the field's cell records (8 corner records per cell) and let the tuner try them")
    ap.add_argument("--no-bricks", action="store_true",
                    help="do not add the field's brick records (2x2x2 node bricks) for the tuner to try")
    ap.add_argument("--no-dirs", action="store_true",
                    help="do not add the field's direction records (96 bytes per cell) for the tuner to try")
    ap.add_argument("--accuracy-lines", type=int, default=2048)
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy and BF16 legs after the timed region (counter runs)")
    ap.add_argument("--batch-fields", type=int, default=64)
    ap.add_argument("--learn-fields", type=int, default=2000,
                    help="learned workload: maps generated (1/4 flux-rope slices)")
    ap.add_argument("--learn-epochs", type=int, default=40)
    ap.add_argument("--learn-streams", type=int, default=4, help="learned workload: streams the scored maps use")
    ap.add_argument("--learn-batch", type=int, default=256, help="learned workload: tiles per training step")
    ap.add_argument("--learn-group", type=int, default=8, help="learned workload: maps in flight at once")
    ap.add_argument("--train-only", action="store_true",
                    help="learned workload: only time the network's training step and forward pass on seeded "
                         "random 64x64 tiles at each of --train-batches tiles")
    ap.add_argument("--train-batches", default="64,128,256,512,1024",
                    help="with --train-only: comma-separated batch sizes (tiles)")
    ap.add_argument("--cpu-fraction", type=float, default=0.25,
                    help="batch workload: fraction of each field's seeds the oracle traces")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    ap.add_argument("--summarize-pmc", nargs=5,
                    metavar=("NAME", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/k_trace_traffic_NAME.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE "
                         "csv outputs of this benchmark (workload NAME) and of --calibrate-copy")
    ap.add_argument("--pmc-launch", type=int, default=None,
                    help="with --summarize-pmc: the launch word the counter runs used (recorded in the summary)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.summarize_pmc:
        return summarize_pmc(*args.summarize_pmc, launch=args.pmc_launch)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "learned":
        return bench_train_only(args) if args.train_only else bench_learned(args)
    return bench_field_map(args)


# ---------------------------------------------------------------------------
# fixed-error protocol
# ---------------------------------------------------------------------------

def rel_log10_err(qg, sg, ref):
    """Relative log10 Q error per line against the oracle reference, on lines
    whose exit faces agree and whose reference Q is finite and < 1e6."""
    import numpy as np
    qo = ref["q_perp"]
    m = np.isfinite(qo) & np.isfinite(qg) & (qo < 1e6) & (sg == ref["status"])
    return np.abs(np.log10(qg[m]) - np.log10(qo[m])) / np.abs(np.log10(qo[m]))


class Setting:
    """One point of the sweep: stepper, stepping precision, tolerance and
    largest step (CK54), or step size (Euler), in grid cells."""

    def __init__(self, stepper, step_dtype, tol=None, hmax_cells=None, euler_div=None):
        self.stepper, self.step_dtype = stepper, step_dtype
        self.tol, self.hmax_cells, self.euler_div = tol, hmax_cells, euler_div

    def opts(self, h, launch=0):
        from paper_1609_00724_amd.api import make_opts
        if self.stepper == "euler":
            o = make_opts(1e-3, 1e-3, h_init=h / self.euler_div, step_dtype=self.step_dtype, stepper="euler")
        else:
            o = make_opts(self.tol, self.tol, h_init=0.1 * h, h_max=self.hmax_cells * h,
                          step_dtype=self.step_dtype)
        o.launch = launch
        return o

    def oracle_kw(self, h):
        if self.stepper == "euler":
            return dict(rtol=1e-3, atol=1e-3, h_init=h / self.euler_div, h_max=h / self.euler_div, stepper="euler")
        return dict(rtol=self.tol, atol=self.tol, h_init=0.1 * h, h_max=self.hmax_cells * h)

    def describe(self):
        if self.stepper == "euler":
            return {"stepper": "euler", "step_dtype": self.step_dtype, "step_cells": 1.0 / self.euler_div}
        return {"stepper": "ck54", "step_dtype": self.step_dtype, "tol": self.tol, "h_max_cells": self.hmax_cells}

    def text(self):
        if self.stepper == "euler":
            return f"explicit Euler {self.step_dtype.upper()} stepping, fixed step 1/{self.euler_div} cell"
        return (f"CK54 {self.step_dtype.upper()} stepping tol={self.tol:g} h_max={self.hmax_cells:g} cell")


def sweep_settings(variant):
    stepper, dt = variant
    if stepper == "euler":
        return [Setting("euler", dt, euler_div=d) for d in SWEEP_EULER_DIVS]
    return [Setting("ck54", dt, tol=t, hmax_cells=c) for c in SWEEP_HMAX_CELLS for t in SWEEP_TOLS]


def accuracy_of(field, seeds_dev, ref, setting, h):
    """Median / p90 relative log10 Q error of the GPU tracer at `setting` on
    the accuracy lines."""
    import numpy as np
    import torch

    from paper_1609_00724_amd.api import TracePlan
    plan = TracePlan(seeds_dev.shape[1], seeds_dev.device, want=("q_perp",))
    out = plan.run(field, seeds_dev, setting.opts(h))
    torch.cuda.synchronize()
    e = rel_log10_err(out["q_perp"].cpu().numpy(), out["status"].cpu().numpy(), ref)
    return {"median": float(np.median(e)), "p90": float(np.percentile(e, 90)), "lines": int(e.size)}


def time_map(plan, field, opts, reps=1):
    """Milliseconds of one map (the fastest of `reps`, after one untimed run)."""
    import torch
    plan.run(field, opts)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run(field, opts)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def fixed_error(plan, field, seeds_dev, ref, h, variants, log):
    """For each variant, every sweep setting's accuracy; the settings that
    meet the target are timed on the map itself and the fastest is chosen.
    Returns ({variant: chosen row or None}, all rows)."""
    rows, chosen = [], {}
    for var in variants:
        best = None
        for st in sweep_settings(var):
            acc = accuracy_of(field, seeds_dev, ref, st, h)
            row = dict(st.describe(), **acc, meets_target=acc["median"] <= TARGET_MEDIAN)
            if row["meets_target"]:
                row["map_ms"] = time_map(plan, field, st.opts(h))
                row["lines_per_s"] = plan.result()["count"] / (row["map_ms"] / 1e3)
                if best is None or row["map_ms"] < best[0]["map_ms"]:
                    best = (row, st)
            rows.append(row)
            log(f"sweep {row}")
        chosen[var] = best
    return chosen, rows


# ---------------------------------------------------------------------------
# map and volume workloads
# ---------------------------------------------------------------------------

def kept_by_level(keys, steps, levels):
    """Kept samples of a refined map by refinement level (0: the base
    lattice) with the step attempts of their lines (both halves).  Keys of
    the regular lattice tell the level: base cells sit at q B^r + B^r / 2
    (B = 2^DIM, B^r = 2^levels), level 1 adds the multiples of B^r and level
    j >= 2 the odd multiples of 2^(levels - j)."""
    import numpy as np
    k = keys.cpu().numpy().astype(np.uint64)
    a = steps.cpu().numpy().astype(np.int64)
    tz = np.zeros(k.shape, np.int64)
    for _ in range(levels):
        even = (k & np.uint64(1)) == 0
        tz += even
        k = np.where(even, k >> np.uint64(1), k)
    lev = np.where(tz >= levels, 1, np.where(tz == levels - 1, 0, levels - tz))
    out = []
    for j in range(levels + 1):
        aj = a[lev == j]
        if aj.size:
            out.append({"level": j, "lines": int(aj.size), "attempts": int(aj.sum()),
                        "mean_attempts": float(aj.mean()), "max_attempts": int(aj.max())})
    return out


def bench_field_map(args):
    """A refined Q / length / FLEDGE map: the 3D volume of the flux-rope field
    (default) or the photospheric slice of the 4-charge field, at the
    fixed-error setting, with the stepping kernel's roofline from the work of
    the kept samples."""
    import numpy as np
    import torch

    import oracle
    import paper_1609_00724_amd as q
    import synth
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import MapSpec, Profiler, QMapPlan, VolumeSpec

    def log(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    volume = args.workload == "volume"
    t_gen = time.perf_counter()
    if volume:
        w = synth.flux_rope_c4(device=dev)
        m = args.volume_level
    else:
        w = synth.charges_c2()
        m = args.base_level
    b = [torch.from_numpy(c).to(dev) for c in w["b"]]
    field = q.field_init(*b, w["origin"], w["spacing"], storage="f32", order=args.order)
    # BF16 node records are offered with the trilinear kernel only
    bf16 = (q.field_init(*b, w["origin"], w["spacing"], storage="bf16")
            if volume and args.order == "linear" else None)
    del b
    if args.cell_records:
        field.add_cells()
    if not args.no_bricks and args.order == "linear":
        field.add_bricks()
    if not args.no_dirs and args.order == "linear":
        field.add_cell_dirs()
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    h = min(w["spacing"])
    r, thr = args.refine_levels, args.threshold
    dims = 3 if volume else 2
    if volume:
        spec = VolumeSpec(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, m, r, m, thr, args.refine_batch)
        cap = 8 ** m * 4
    else:
        spec = MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, thr, args.refine_batch)
        cap = 4 ** (m + r)     # the finest lattice: the map cannot overflow
    plan = QMapPlan(spec, cap, dev, want_steps=True)
    log(f"field ready ({t_gen:.1f} s)")

    # reference lines: FP64 oracle at tolerance 1e-10 on the same gridded field
    acc_seeds = (synth.random_seeds(2025, args.accuracy_lines) if volume
                 else synth.random_seeds(2024, args.accuracy_lines, z=0.0))
    order_n = {"linear": 1, "quadratic": 2, "cubic": 3}[args.order]
    fo = oracle.Field.grid(*(np.asarray(c, np.float64) for c in w["b"]), w["origin"], w["spacing"], order=order_n)
    t_ref = time.perf_counter()
    ref = oracle.trace(fo, acc_seeds, rtol=1e-10, atol=1e-10, h_init=0.1 * h, h_max=h)
    t_ref = time.perf_counter() - t_ref
    log(f"reference lines traced ({t_ref:.1f} s)")
    seeds_dev = torch.from_numpy(np.ascontiguousarray(acc_seeds.T)).to(dev)

    # the setting: the fixed-error sweep, or given on the command line
    variant = (args.stepper, "f32")
    rows, chosen = [], {}
    if args.no_sweep or args.tol is not None or args.euler_div is not None:
        st = (Setting("euler", "f32", euler_div=args.euler_div or 5) if args.stepper == "euler"
              else Setting("ck54", "f32", tol=args.tol or 1e-4, hmax_cells=args.hmax_cells or 1.0))
    else:
        variants = [("ck54", "f32"), ("ck54", "f64"), ("euler", "f32")]
        chosen, rows = fixed_error(plan, field, seeds_dev, ref, h, variants, log)
        if chosen[variant] is None:
            raise SystemExit("no sweep setting meets the fixed-error target")
        st = chosen[variant][1]
    opts = st.opts(h, args.launch)
    log(f"setting: {st.text()}")

    tuned = None
    if not args.no_tune:
        # launch shape and refinement batch timed on the workload itself
        from paper_1609_00724_amd import autotune
        if volume:
            cands = ([A.launch_word(2, 128, A.GATHER_DIRECT), A.launch_word(2, 128, A.GATHER_CACHED)]
                     + autotune.candidates(lanes=(1, 2), wgs=(64, 128, 256), gathers=(A.GATHER_REGS,)))
            if args.cell_records:
                cands += autotune.candidates(lanes=(1, 2, 4), wgs=(64, 256), gathers=(A.GATHER_CELLS,))
            if field.bricks_ws is not None:
                cands += autotune.candidates(lanes=(1, 2), wgs=(64, 128, 256), gathers=(A.GATHER_BRICKS,))
            if field.dirs_ws is not None:
                cands += autotune.candidates(lanes=(1, 2), wgs=(64, 128, 256), gathers=(A.GATHER_DIRS,))
                if field.bricks_ws is not None:
                    # brick records for the base lattice, direction records after it
                    cands += [w | A.launch_word(refine_gather=A.GATHER_DIRS)
                              for w in autotune.candidates(lanes=(2,), wgs=(64, 128, 256), gathers=(A.GATHER_BRICKS,))]
            batches = (args.refine_batch,) if args.refine_batch > 0 else (1, 2, 3)
            (word, batch), table = autotune.tune_map(plan, field, opts, reps=1, cands=cands, batches=batches)
        else:
            batches = (args.refine_batch,) if args.refine_batch > 0 else (1, 2, 3, 4)
            cands = autotune.candidates()
            if field.bricks_ws is not None:
                cands += autotune.candidates(gathers=(A.GATHER_BRICKS,))
            if field.dirs_ws is not None:
                cands += autotune.candidates(gathers=(A.GATHER_DIRS,))
            (word, batch), table = autotune.tune_map(plan, field, opts, reps=2, cands=cands, batches=batches)
        opts.launch = word
        plan.d.refine_batch = batch
        tuned = dict(autotune.describe(word), refine_batch=batch, ms=table[(word, batch)], candidates=len(table),
                     worst_ms=max(table.values()))
        log(f"tuned: {tuned}")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.run(field, opts)
    torch.cuda.synchronize()
    plan.work.zero_()
    with Profiler() as prof:
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t0.record(stream)
        for _ in range(args.steps):
            plan.run(field, opts)
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms_per_step = t0.elapsed_time(t1) / args.steps
        n_step, ms_trace = prof.read(A.KERNEL_STEP)
        n_land, ms_land = prof.read(A.KERNEL_LAND)
        n_asm, ms_asm = prof.read(A.KERNEL_ASSEMBLE)
    Profiler.reset()
    res = plan.result()
    lines = res["count"]
    attempts, evals, stepped, landed = (int(v) for v in plan.work.cpu().numpy())
    kept_attempts = int(res["steps"].to(torch.int64).sum().item()) * args.steps
    per_attempt = FLOP_PER_EULER_STEP if st.stepper == "euler" else FLOP_PER_ATTEMPT
    traced_flops = FLOP_PER_EVAL_ORDER[args.order] * evals + per_attempt * attempts
    # the method's own work: the kept samples' lines (speculative lines the
    # rule drops are traced but are not the method's); evaluations per attempt
    # are taken as equal for kept and dropped lines
    own = kept_attempts / max(attempts, 1)
    own_flops = traced_flops * own
    achieved = own_flops / (ms_trace / 1e3) / 1e12 if ms_trace > 0 else 0.0
    traffic, traffic_word = measured_traffic(args.workload)
    levels = kept_by_level(res["keys"], res["steps"], dims * r)
    grid_txt = "x".join(str(v) for v in w["n"])
    kernel_txt = {"linear": "", "quadratic": " (triquadratic interpolation)",
                  "cubic": " (tricubic interpolation)"}[args.order]
    if volume:
        wl = (f"3D Q/FLL/FLEDGE volume, flux rope over a 6-charge background on a {grid_txt} FP32 grid, "
              f"{1 << m}^3 base cells + FLL-jump 3D Hilbert refinement r={r} thr={thr}{kernel_txt}")
    else:
        wl = (f"photospheric Q/FLL/FLEDGE map, 4-charge potential field on a {grid_txt} FP32 grid, "
              f"{1 << m}^2 base lines + FLL-jump Hilbert refinement r={r} thr={thr}{kernel_txt}")
    out = {
        "metric": METRIC,
        "value": lines / (ms_per_step / 1e3),
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
            "workload": wl + ", " + st.text() + " (fixed-error setting), FP64 landing and Q",
            "lines_per_step": lines,
            "base_lines": (2 ** dims) ** m,
            "grid": list(w["n"]),
            "setting": st.describe(),
            "interpolation": args.order,
            # 0 selects the library's default: 4 levels per round for slices, 1 for volumes
            "refine_batch": plan.d.refine_batch or (1 if volume else max(1, min(dims * r, 4))),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_trace (" + ("explicit Euler" if st.stepper == "euler" else "adaptive") + " stepping)",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_launch_word": traffic_word,
            "launches": n_step,
            "avg_launch_ms": ms_trace / max(n_step, 1),
            "own_flops_per_step": own_flops / args.steps,
            "traced_flops_per_step": traced_flops / args.steps,
            "traced_over_kept_attempts": attempts / max(kept_attempts, 1),
            "attempts_per_step": attempts / args.steps,
            "kept_attempts_per_step": kept_attempts / args.steps,
            "rhs_evals_per_step": evals / args.steps,
            "nonpacked_fp32_ceiling": FP32_NONPACKED_TFLOPS,
            "frac_of_nonpacked_ceiling": achieved / FP32_NONPACKED_TFLOPS,
        },
        "kernel_ms_per_step": {"step": ms_trace / args.steps, "land": ms_land / args.steps,
                               "assemble": ms_asm / args.steps},
        "kept_by_level": levels,
        "launch_shape": tuned,
        "wall_s_timed": wall,
        "setup_s": t_gen,
    }
    if not args.no_accuracy:
        acc = accuracy_of(field, seeds_dev, ref, st, h)
        out["accuracy"] = dict(acc, reference="FP64 oracle on the same grid data, tol 1e-10",
                               target_median=TARGET_MEDIAN)
    if rows:
        out["fixed_error"] = {
            "target_median_rel_log10q_err": TARGET_MEDIAN,
            "chosen": {f"{k[0]}_{k[1]}": (None if v is None else v[0]) for k, v in chosen.items()},
            "sweep": rows,
        }
    if bf16 is not None and not args.no_accuracy:
        plan16 = QMapPlan(spec, cap, dev)
        plan16.d.refine_batch = plan.d.refine_batch
        ms16 = time_map(plan16, bf16, opts)
        r16 = plan16.result()
        acc16 = accuracy_of(bf16, seeds_dev, ref, st, h)
        out["bf16_storage"] = {"ms": ms16, "lines_per_s": r16["count"] / (ms16 / 1e3), "lines": r16["count"],
                               "accuracy": acc16}
        del plan16
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_map(args, fo, st, h, volume)
    print(json.dumps(out), flush=True)


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "cores_allowed": allowed, "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def host_threads():
    """Threads for the oracle: the host cores this process may use, or the
    box's CPU share where OMP_NUM_THREADS states it."""
    info = host_info()
    omp = int(info["omp_num_threads"] or 0)
    return min(omp, info["cores_allowed"]) if omp > 0 else info["cores_allowed"]


def cpu_baseline_map(args, fo, st, h, volume):
    """The oracle (FP64 C + numpy refinement) at the same setting, field,
    refinement rule and threshold on a bounded sample: a 2^l base lattice
    with its refinement, on all the host cores this process may use, and on
    one core.  l starts at 5 for the volume and 8 for the map and grows (to 6
    and 10 at most) while the next level's sample would take under about
    30 s on one core."""
    import oracle
    level = args.cpu_level if args.cpu_level is not None else (5 if volume else 8)
    top = level if args.cpu_level is not None else (6 if volume else 10)
    region = (oracle.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0) if volume
              else oracle.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0))
    kw = st.oracle_kw(h)

    def run(threads):
        def fn(p):
            t = oracle.trace(fo, p, nthreads=threads, **kw)
            return {"fll": t["fll"], "q": t["q_perp"]}
        t0 = time.perf_counter()
        keys, _, _ = oracle.refine_slice(region, level, args.refine_levels, args.threshold, fn)
        return keys.size, time.perf_counter() - t0

    threads = host_threads()
    n_all, dt_all = run(threads)
    while level < top and dt_all * threads * (8 if volume else 4) < 30.0:
        level += 1
        n_all, dt_all = run(threads)
    n_one, dt_one = run(1)
    shape = f"{1 << level}^{3 if volume else 2}"
    return dict({"value": n_all / dt_all, "unit": "lines/s", "cores": threads, "kind": "oracle",
                 "sample": (f"same field, setting and refinement rule on a {shape} base lattice "
                            f"({n_all} lines, {dt_all:.1f} s on {threads} threads; {dt_one:.1f} s on 1)"),
                 "one_core": n_one / dt_one}, **host_info())


def traffic_file(name):
    return os.path.join(ROOT, "profiles", f"k_trace_traffic_{name}.json")


KERNEL_SOURCES = ("paper_1609_00724_amd/csrc/trace.hip", "paper_1609_00724_amd/csrc/qsq_internal.h")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pmc_rows(d, counter):
    import csv
    import glob
    fs = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not fs:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(open(fs[0]))
            if r["Counter_Name"] == counter]


def summarize_pmc(name, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, launch=None):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what they read for a
    plain 1 GiB copy and store the stepping kernel's bytes per launch, keyed by
    the hash of its sources (the benchmark reports null once they change)."""
    gib = float(1 << 30)
    cf = [v for k, v in _pmc_rows(copy_fetch_dir, "FETCH_SIZE") if "copyBuffer" in k]
    cw = [v for k, v in _pmc_rows(copy_write_dir, "WRITE_SIZE") if "copyBuffer" in k]
    fscale = gib / (sum(cf) / len(cf) * 1024.0)
    wscale = gib / (sum(cw) / len(cw) * 1024.0)
    # every stepping launch of the counter runs: they time a fixed launch shape
    # with no tuning and no warm-up maps (`--no-tune --launch W --refine-batch B
    # --warmup 0`), so all of their k_trace dispatches are the timed maps'
    f = [v for k, v in _pmc_rows(fetch_dir, "FETCH_SIZE") if "k_trace<" in k]
    w = [v for k, v in _pmc_rows(write_dir, "WRITE_SIZE") if "k_trace<" in k]
    if not f or len(f) != len(w):
        raise SystemExit(f"stepping dispatches differ between the runs: {len(f)} FETCH_SIZE, {len(w)} WRITE_SIZE")
    npass = len(f)
    out = {"kernel_sources_sha256": kernel_hash(), "passes": npass, "dispatches": len(f),
           "fetch_bytes_per_launch": sum(f) / npass * 1024.0 * fscale,
           "write_bytes_per_launch": sum(w) / npass * 1024.0 * wscale,
           "fetch_scale": fscale, "write_scale": wscale,
           "copy_fetch_kib": sum(cf) / len(cf), "copy_write_kib": sum(cw) / len(cw), "launch_word": launch}
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    with open(traffic_file(name), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def measured_traffic(name):
    """(HBM bytes per stepping-kernel launch, launch word of the counter runs)
    from the committed counter summary of workload `name`, or (None, None) if
    the kernel's sources changed since the counters were taken."""
    try:
        with open(traffic_file(name)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("kernel_sources_sha256") != kernel_hash():
        return None, None
    return t["bytes_per_launch"], t.get("launch_word")


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, three times: a kernel of known
    HBM traffic (1 GiB read + 1 GiB written) for scaling the byte counters."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "launches": 3}))


def bench_batch(args):
    """Many fields of uneven grid size and seed count in one batched trace,
    captured in a HIP graph and replayed; beside it the same sets traced one
    call per field, and FP64 stepping of the same batch."""
    import numpy as np
    import torch

    import paper_1609_00724_amd as q
    import synth
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import Profiler, TraceBatchPlan, TracePlan, make_opts

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    fields, seeds, host = [], [], []
    for f in synth.batch_c3(count=args.batch_fields):
        b = [torch.from_numpy(c).to(dev) for c in f["b"]]
        fields.append(q.field_init(*b, f["origin"], f["spacing"], storage="f32"))
        seeds.append(torch.from_numpy(f["seeds"]).to(dev))
        host.append(dict(origin=f["origin"], spacing=f["spacing"], n=f["n"], charges=f["charges"],
                         seeds=f["seeds"]))
        del b
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    total = sum(int(s.shape[0]) for s in seeds)
    sets = list(zip(fields, seeds))
    # h_init, h_max: 0.1 and 1 cell of each field's own grid
    tol = args.tol or 1e-4
    opts32 = make_opts(tol, tol, step_dtype="f32")
    opts64 = make_opts(tol, tol, step_dtype="f64")
    opts32.launch = args.launch
    plan = TraceBatchPlan(sets, opts32, want_work=True)
    tuned = None
    if not args.no_tune:
        from paper_1609_00724_amd import autotune
        cands = autotune.candidates(lanes=(1, 2, 3, 4), wgs=(64, 128, 256), gathers=(A.GATHER_DIRECT,))
        word, table = autotune.tune_batch(sets, opts32, reps=1, cands=cands)
        opts32.launch = word
        tuned = dict(autotune.describe(word), ms=table[word], candidates=len(table), worst_ms=max(table.values()))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(max(args.warmup, 1)):
            plan.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run()
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for _ in range(args.steps):
        graph.replay()
    e1.record(cur)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps

    # kernel timing and work counts of the same batch, eager, profiled
    plan.work.zero_()
    with Profiler() as prof:
        with torch.cuda.stream(stream):
            plan.run()
        torch.cuda.synchronize()
        n_step, ms_trace = prof.read(A.KERNEL_STEP)
    Profiler.reset()
    attempts, evals, stepped, landed = (int(v) for v in plan.work.cpu().numpy())
    flops = FLOP_PER_EVAL * evals + FLOP_PER_ATTEMPT * attempts
    achieved = flops / (ms_trace / 1e3) / 1e12

    # the same sets, one qsq_trace call per field, back to back on one stream
    plans1 = [TracePlan(int(s.shape[0]), dev) for s in seeds]
    soas = [s.t().contiguous() for s in seeds]
    with torch.cuda.stream(stream):
        for p1, (fg, _), soa in zip(plans1, sets, soas):
            p1.run(fg, soa, opts32)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        s0.record(stream)
        for p1, (fg, _), soa in zip(plans1, sets, soas):
            p1.run(fg, soa, opts32)
        s1.record(stream)
    torch.cuda.synchronize()
    ms_single = s0.elapsed_time(s1)
    del plans1

    # FP64 stepping of the same batch, and the FP32-vs-FP64 difference in Q
    plan64 = TraceBatchPlan(sets, opts64, want_work=True)
    with torch.cuda.stream(stream):
        plan64.run()
        torch.cuda.synchronize()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d0.record(stream)
        plan64.run()
        d1.record(stream)
    torch.cuda.synchronize()
    ms64 = d0.elapsed_time(d1)
    att64 = int(plan64.work.cpu().numpy()[0]) // 2       # two runs of the FP64 batch
    q32 = torch.cat([o["q_perp"] for o in plan.outs]).cpu().numpy()
    q64 = torch.cat([o["q_perp"] for o in plan64.outs]).cpu().numpy()
    st32 = torch.cat([o["status"] for o in plan.outs]).cpu().numpy()
    st64 = torch.cat([o["status"] for o in plan64.outs]).cpu().numpy()
    m = np.isfinite(q32) & np.isfinite(q64) & (q64 < 1e6) & (st32 == st64)
    rel = np.abs(np.log10(q32[m]) - np.log10(q64[m])) / np.abs(np.log10(q64[m]))

    out = {
        "metric": METRIC,
        "value": total / (ms_step / 1e3),
        "unit": "lines/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched trace: {len(fields)} point-charge fields (2-8 charges, grids 64^3 to "
                         f"256x256x128, FP32 storage), 1e4-1e6 random photospheric seeds each, one batched "
                         f"call (one persistent stepping launch) replayed as a HIP graph, CK54 FP32 stepping "
                         f"tol={tol:g}, h_max 1 cell of each grid, FP64 landing and Q"),
            "fields": len(fields),
            "lines_per_step": total,
            "tol": tol,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_trace (batched, adaptive stepping)",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "nonpacked_fp32_ceiling": FP32_NONPACKED_TFLOPS,
            "frac_of_nonpacked_ceiling": achieved / FP32_NONPACKED_TFLOPS,
            "traffic": None,
            "launches": n_step,
            "avg_launch_ms": ms_trace / max(n_step, 1),
            "rhs_evals": evals,
            "attempts": attempts,
        },
        "launch_shape": tuned,
        "one_call_per_field_ms": ms_single,
        "batch_speedup_vs_one_call_per_field": ms_single / ms_step,
        "fp64_stepping": {"ms": ms64, "lines_per_s": total / (ms64 / 1e3), "attempts": att64,
                          "median_rel_log10q_diff_fp32_vs_fp64": float(np.median(rel)),
                          "p99": float(np.percentile(rel, 99)),
                          "status_agreement": float((st32 == st64).mean())},
        "setup_s": t_gen,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(args, host)
    print(json.dumps(out), flush=True)


def learned_item(k):
    """Map k of the learned workload.  Three of every four are point-charge
    fields (256x256x128 FP32 nodes, 2-8 charges, seeds 5000-6499, slice
    z = 0); the fourth a flux-rope field (384x384x256, the rope of the volume
    workload over its two leg charges and four drawn with seed 6500-6999),
    sliced at z0 ~ U[0.01, 0.3].  The test maps are those with seed % 10 == 0."""
    import synth
    if k % 4 == 3:
        seed = 6500 + k // 4
        return dict(rope=True, seed=seed, n=(384, 384, 256), charges=synth.rope_charges(seed),
                    z0=float(synth.rng(1_000_000 + seed).uniform(0.01, 0.3)))
    seed = 5000 + 3 * (k // 4) + k % 4
    return dict(rope=False, seed=seed, n=(256, 256, 128), z0=0.0,
                charges=synth.point_charges(seed, int(synth.rng(seed).integers(2, 9))))


def map_error(q, ref, qsl=1e3, cap=2.0):
    """Per-pixel |log10 Q - log10 Q_ref| on the finest raster (capped at `cap`
    dex, a missing or non-finite Q counting as `cap`) over the pixels where the
    reference is finite: mean, fraction above 1e-3 relative, and the fraction
    of the reference's QSL pixels (Q > qsl) not shown above qsl."""
    import torch
    lr = torch.log10(ref.double())
    ok = torch.isfinite(lr)
    lq = torch.log10(q.double())
    e = torch.where(torch.isfinite(lq), (lq - lr).abs(), torch.full_like(lr, cap)).clamp(max=cap)[ok]
    rel = e / lr[ok].abs().clamp(min=1e-30)
    isq = (ref > qsl) & ok
    miss = isq & ~(torch.nan_to_num(q, nan=0.0) > qsl)
    return dict(mean=float(e.mean()), frac_rel_over_1e3=float((rel > 1e-3).double().mean()),
                qsl_pixels=int(isq.sum()), qsl_missed=int(miss.sum()))


def score_learned(test, make_field, prop, m, r, thr, nstreams, group, dev):
    """Learned pipeline, FLL-jump rule and uniform sampling on held-out maps.

    test: dicts with "item" (what make_field takes) and "mask" (the rule's
    refine mask at the coarse level); make_field(item) -> (field, Bz on the
    coarse raster, trace opts); item["z0"] is the slice height.  Maps run in groups of `group`, map i of a
    group on stream i % nstreams with its own plans; each method's time is
    that of the whole group (events on the default stream around the
    streams' work).  Errors are taken against the finest uniform map.
    Returns (methods, proposal scores)."""
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import learn
    from paper_1609_00724_amd.api import MapSpec, QMapPlan

    side = 1 << m
    fine_side = 1 << (m + r)

    def spec(b, rr):
        return MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, b, rr, b + rr, thr)

    curve_xy = [v.long() for v in q.hilbert2_d2xy(m, torch.arange(4 ** m, device=dev))]
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    ulev = list(range(m + 1, m + r + 1))
    slots = []
    for _ in range(group):
        sl = dict(coarse=QMapPlan(spec(m, 0), 4 ** m, dev), lplan=QMapPlan(spec(m, r), 4 ** (m + r), dev),
                  rule=QMapPlan(spec(m, r), 4 ** (m + r), dev), prop=torch.zeros(4 ** m, dtype=torch.uint8,
                                                                                 device=dev),
                  ws=prop.workspace((side // 64) ** 2, 64, 64))
        for lv in ulev:
            sl[lv] = QMapPlan(spec(lv, 0), 4 ** lv, dev, fledge_map=False)
        sl["lplan"].d.propose = sl["prop"].data_ptr()
        slots.append(sl)
    names = ["learned", "rule"] + [f"uniform_{1 << lv}" for lv in [m] + ulev]
    tot_ms = dict.fromkeys(names, 0.0)
    tot_samples = dict.fromkeys(names, 0)
    tot_att = dict.fromkeys(names, 0)
    err = {k: dict(mean=0.0, frac_rel_over_1e3=0.0, qsl_pixels=0, qsl_missed=0) for k in names}
    tp = fn = fp = prop_px = rule_px = 0
    up = lambda a, f: a.repeat_interleave(f, 0).repeat_interleave(f, 1)   # noqa: E731
    main = torch.cuda.current_stream()

    def learned(sl, fg, bz, opts, st):
        sl["coarse"].run(fg, opts, stream=st)
        with torch.cuda.stream(st):
            x = learn.features(sl["coarse"].fll_grid, sl["coarse"].fledge, bz)
            out = prop.forward(learn.tiles(x), stream=st, ws=sl["ws"])
            pred = learn.untile(out, side, side)[..., 0] > 0
            sl["prop"].copy_(pred[curve_xy[1], curve_xy[0]].to(torch.uint8))
            sl["pred"] = pred
        sl["lplan"].run(fg, opts, stream=st, base_from=sl["coarse"])

    runners = {"learned": learned,
               "rule": lambda sl, fg, bz, opts, st: sl["rule"].run(fg, opts, stream=st),
               f"uniform_{side}": lambda sl, fg, bz, opts, st: sl["coarse"].run(fg, opts, stream=st)}
    for lv in ulev:
        runners[f"uniform_{1 << lv}"] = (lambda lv_: lambda sl, fg, bz, opts, st: sl[lv_].run(fg, opts,
                                                                                              stream=st))(lv)
    for g0 in range(0, len(test), group):
        chunk = test[g0:g0 + group]
        fields = []
        for d in chunk:
            fg, bz, opts = make_field(d["item"])
            fields.append((fg, bz, opts))
        for sl, d in zip(slots, chunk):
            for key, pl in sl.items():
                if isinstance(pl, QMapPlan):
                    pl.d.z0 = d["item"]["z0"]
                    pl.work.zero_()
        torch.cuda.synchronize()
        att = {}
        for name in ("learned", "rule", *runners.keys()):
            if name in att:
                continue
            for sl in slots[:len(chunk)]:
                for key, pl in sl.items():
                    if isinstance(pl, QMapPlan):
                        pl.work.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(main)
            for st in streams:
                st.wait_event(e0)
            for i, (sl, (fg, bz, opts)) in enumerate(zip(slots, fields)):
                runners[name](sl, fg, bz, opts, streams[i % nstreams])
            for st in streams:
                ev = torch.cuda.Event()
                ev.record(st)
                main.wait_event(ev)
            e1.record(main)
            torch.cuda.synchronize()
            tot_ms[name] += e0.elapsed_time(e1)
            used = {"learned": ("coarse", "lplan"), "rule": ("rule",), f"uniform_{side}": ("coarse",)}
            used.update({f"uniform_{1 << lv}": (lv,) for lv in ulev})
            att[name] = sum(int(sl[k].work[0]) for sl in slots[:len(chunk)] for k in used[name])
            if name == "learned":
                # keep the learned maps: the coarse plan is reused by uniform_<side>
                kept = [(sl["lplan"].q_grid.clone(), int(sl["lplan"].count), sl["pred"]) for sl in slots[:len(chunk)]]
        for i, (sl, d) in enumerate(zip(slots, chunk)):
            ref = sl[m + r].q_grid
            qg = {"learned": (kept[i][0], kept[i][1]), "rule": (sl["rule"].q_grid, int(sl["rule"].count)),
                  f"uniform_{side}": (up(sl["coarse"].q_grid, 1 << r), 4 ** m)}
            qg.update({f"uniform_{1 << lv}": (up(sl[lv].q_grid, 1 << (m + r - lv)), 4 ** lv) for lv in ulev})
            for name, (grid, ns) in qg.items():
                e = map_error(grid, ref)
                for key in err[name]:
                    err[name][key] += e[key] / (len(test) if key in ("mean", "frac_rel_over_1e3") else 1)
                tot_samples[name] += ns
            pred, plain = kept[i][2], d["mask"] > 0.5
            tp += int((pred & plain).sum())
            fn += int((~pred & plain).sum())
            fp += int((pred & ~plain).sum())
            prop_px += int(pred.sum())
            rule_px += int(plain.sum())
        for name in names:
            tot_att[name] += att[name]
        del fields
    n = len(test)
    methods = {}
    for k in names:
        methods[k] = dict(ms_per_map=tot_ms[k] / n, samples_per_map=tot_samples[k] / n,
                          step_attempts_per_map=tot_att[k] / n,
                          map_pixels_per_s=fine_side * fine_side * n / (tot_ms[k] / 1e3),
                          mean_abs_log10q_err=err[k]["mean"], frac_rel_err_over_1e3=err[k]["frac_rel_over_1e3"],
                          qsl_pixels=err[k]["qsl_pixels"],
                          qsl_missed_fraction=err[k]["qsl_missed"] / max(err[k]["qsl_pixels"], 1))
    extra = dict(mask_recall=tp / max(tp + fn, 1), mask_precision=tp / max(tp + fp, 1),
                 proposed_pixel_fraction=prop_px / (n * side * side), rule_pixel_fraction=rule_px / (n * side * side))
    return methods, extra


def bench_train_only(args):
    """The network's kernels alone: training steps (forward, loss, backward,
    Adam with the prepared-weight refresh) and forward passes on seeded random
    64x64 tiles, --steps timed after --warmup, HIP events; one JSON line."""
    import torch

    from paper_1609_00724_amd import learn
    dev = torch.device("cuda:0")
    g = torch.Generator().manual_seed(0)
    flop_fwd = 2 * 64 * 64 * sum(9 * ci * co for ci, co in zip(learn.CHANNELS[:-1], learn.CHANNELS[1:]))
    prop = learn.Proposer(learn.init_params(1, dev))
    rows = []
    for bs in (int(b) for b in args.train_batches.split(",")):
        x = torch.randn(bs, 64, 64, 3, generator=g).to(dev)
        mask = (torch.rand(bs, 64, 64, generator=g) < 0.2).float().to(dev)
        logq = torch.randn(bs, 64, 64, generator=g).to(dev)
        for _ in range(args.warmup):
            prop.train_step(x, mask, logq, lr=1e-9)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        for _ in range(args.steps):
            prop.train_step(x, mask, logq, lr=1e-9)
        e[1].record()
        for _ in range(args.steps):
            prop.forward(x)
        e[2].record()
        torch.cuda.synchronize()
        ms, fms = e[0].elapsed_time(e[1]) / args.steps, e[1].elapsed_time(e[2]) / args.steps
        rows.append({"tiles": bs, "train_step_ms": ms, "train_tflops": bs * flop_fwd * 3 / ms / 1e9,
                     "forward_ms": fms, "forward_tflops": bs * flop_fwd / fms / 1e9})
        print(f"bench: {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "learned proposer: BF16-MFMA training step throughput", "unit": "TFLOP/s",
                      "value": next((r["train_tflops"] for r in rows if r["tiles"] == 256), rows[-1]["train_tflops"]),
                      "n_gpus": 1, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
                      "config": {"workload": "seeded random 64x64 tiles, 3 -> 32 -> 32 -> 32 -> 2 channels"},
                      "steps": args.steps, "warmup": args.warmup, "mfma_peak_tflops_bf16": 2500.0,
                      "batches": rows}))


def bench_learned(args):
    """Learned refinement proposer on its full workload: --learn-fields maps
    (see learned_item) give coarse 256^2 inputs (length, FLEDGE, Bz) and
    targets from the same maps refined 4x by the FLL-jump rule (refine mask,
    max log10 Q per pixel); the CNN trains on the maps with seed % 10 != 0
    with the library's kernels.  On the held-out maps the learned pipeline
    (coarse map, network, then the map with the proposals merged first and the
    rule as fallback, which takes the coarse map's samples as its base lattice)
    is timed and scored beside the rule alone and plain uniform sampling at
    256^2, 512^2 and 1024^2, against the 1024^2 uniform map: mean |log10 Q
    error| per finest pixel and the fraction of its QSL pixels missed."""
    import numpy as np
    import torch
    import torch.nn.functional as F

    import paper_1609_00724_amd as q
    import synth
    from paper_1609_00724_amd import learn
    from paper_1609_00724_amd.api import MapSpec, QMapPlan, make_opts

    dev = torch.device("cuda:0")
    m, r, thr = 8, 2, args.threshold
    side = 1 << m
    tol = args.tol or 1e-4

    def opts_for(n):
        origin, spacing = synth.grid_geometry(n)
        h = min(spacing)
        return origin, spacing, make_opts(tol, tol, h_init=0.1 * h, h_max=h, step_dtype="f32")

    rope_n = (384, 384, 256)
    t_gen = time.perf_counter()
    rb, _ = synth.flux_rope_field(rope_n, charges=np.zeros((0, 4)), device=dev, dtype=np.float64)
    rope_base = [torch.from_numpy(c).to(dev) for c in rb]
    del rb

    def make_field(it):
        origin, spacing, opts = opts_for(it["n"])
        b = synth.charges_device(it["charges"], it["n"], dev, base=rope_base if it["rope"] else None)
        fg = q.field_init(*b, origin, spacing, storage="f32")
        kz = min(int(round((it["z0"] - origin[2]) / spacing[2])), it["n"][2] - 1)
        bz = F.interpolate(b[2][kz][None, None], size=(side, side), mode="bilinear", align_corners=False)[0, 0]
        del b
        return fg, bz, opts

    slab = dict(x0=-1.0, x1=1.0, y0=-1.0, y1=1.0)
    coarse = QMapPlan(MapSpec(0.0, **slab, base_level=m, refine_levels=0, out_level=m, threshold=thr), 4 ** m, dev)
    fine = QMapPlan(MapSpec(0.0, **slab, base_level=m, refine_levels=r, out_level=m + r, threshold=thr),
                    4 ** (m + r), dev)
    data = []
    for k in range(args.learn_fields):
        it = learned_item(k)
        fg, bz, opts = make_field(it)
        coarse.d.z0 = fine.d.z0 = it["z0"]
        coarse.run(fg, opts)
        fine.run(fg, opts)
        cres, fres = coarse.result(), fine.result()
        qbase = F.max_pool2d(torch.nan_to_num(fres["q_grid"], nan=0.0)[None, None], 1 << r)[0, 0]
        mask, logq = learn.refine_labels(fres["keys"], m, r, qbase)
        x = learn.features(cres["fll_grid"], cres["fledge"], bz)
        data.append(dict(item=it, x=x, mask=mask, logq=logq))
        del fg
        if k % 100 == 99:
            print(f"learned: {k + 1} maps generated", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    train = [d for d in data if d["item"]["seed"] % 10 != 0]
    test = [d for d in data if d["item"]["seed"] % 10 == 0]
    X = torch.cat([learn.tiles(d["x"]) for d in train])
    M = torch.cat([learn.tiles(d["mask"]) for d in train])
    Lq = torch.cat([learn.tiles(d["logq"]) for d in train])
    for d in train:
        del d["x"], d["mask"], d["logq"]
    prop = learn.Proposer(learn.init_params(1, dev))
    bs = args.learn_batch
    g = torch.Generator(device="cpu").manual_seed(0)
    curve = []
    t_train = time.perf_counter()
    for ep in range(args.learn_epochs):
        perm = torch.randperm(X.shape[0], generator=g).to(dev)
        tot = torch.zeros((), dtype=torch.float64, device=dev)
        nb = 0
        for i0 in range(0, X.shape[0] - bs + 1, bs):
            idx = perm[i0:i0 + bs]
            tot += prop.train_step(X[idx], M[idx], Lq[idx], lr=2e-3, lam=0.1)
            nb += 1
        curve.append(float(tot) / max(nb, 1))
        print(f"learned: epoch {ep + 1} loss {curve[-1]:.4f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    # training throughput of the kernels alone: ten steps on a full batch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        prop.train_step(X[:bs], M[:bs], Lq[:bs], lr=1e-9, lam=0.1)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / 10
    flop_fwd = 2 * 64 * 64 * sum(9 * ci * co for ci, co in zip(learn.CHANNELS[:-1], learn.CHANNELS[1:]))
    del X, M, Lq

    # held-out maps: the learned pipeline against the rule and uniform sampling
    methods, extra = score_learned(test, make_field, prop, m, r, thr, args.learn_streams, args.learn_group, dev)
    match = next(k for k in methods if k.startswith("uniform")
                 and methods[k]["mean_abs_log10q_err"] <= methods["learned"]["mean_abs_log10q_err"])
    fine_name = f"uniform_{1 << (m + r)}"
    out = {
        "metric": "learned refinement pipeline: Q-map throughput at matched log10 Q error",
        "value": methods["learned"]["map_pixels_per_s"],
        "unit": "1024^2 map pixels/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"{len(data)} maps ({sum(not d['item']['rope'] for d in data)} point-charge fields "
                                f"with 2-8 charges on 256x256x128 FP32 grids, {sum(d['item']['rope'] for d in data)} "
                                f"flux-rope slices z0 ~ U[0.01, 0.3] on 384x384x256), coarse 256^2 -> 16 tiles of "
                                f"64^2, targets from the FLL-jump rule with 4x refinement thr={thr}, CK54 FP32 "
                                f"tol={tol:g}"),
                   "train_tiles": 16 * len(train), "test_maps": len(test), "epochs": args.learn_epochs,
                   "batch": bs},
        "methods": methods,
        "matched_uniform": match,
        "speedup_vs_matched_uniform": methods[match]["ms_per_map"] / methods["learned"]["ms_per_map"],
        "speedup_vs_finest_uniform": methods[fine_name]["ms_per_map"] / methods["learned"]["ms_per_map"],
        "streams": args.learn_streams, "maps_in_flight": args.learn_group,
        "training": {"train_step_ms": ms_step, "batch_tiles": bs,
                     "tflops": bs * flop_fwd * 3 / (ms_step / 1e3) / 1e12, "mfma_peak_tflops_bf16": 2500.0,
                     "loss_curve": curve, "train_s": t_train, "data_s": t_gen},
        "proposals_against_rule": extra,
        "note": ("samples = lines in the map (each traced once; speculative traces a round drops are in the "
                 "step attempts and times only); errors against the 1024^2 uniform map of the same stepping; a "
                 "coarser map counts each pixel "
                 "with the value of the sample whose block holds it; learned = coarse map + network + map whose "
                 "base lattice is the coarse map's samples; rule = the FLL-jump rule alone; ms_per_map = the "
                 "time of a group of maps in flight on the streams (each map's calls in order on one stream, no "
                 "host synchronisation) over the maps of the group"),
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(args, host):
    """The oracle on a seeded sample of every field's seeds (the same fields,
    tolerance and per-grid step limits)."""
    import numpy as np

    import oracle
    import synth
    threads = host_threads()
    tol = args.tol or 1e-4
    g = synth.rng(7)
    lines, dt = 0, 0.0
    for f in host:
        m = f["seeds"].shape[0]
        pick = np.sort(g.choice(m, size=max(1, int(m * args.cpu_fraction)), replace=False))
        b = synth.sample_charges(f["charges"], f["n"], dtype=np.float32)
        fo = oracle.Field.grid(*(c.astype(np.float64) for c in b), f["origin"], f["spacing"])
        del b
        h = min(f["spacing"])
        t0 = time.perf_counter()
        oracle.trace(fo, f["seeds"][pick], rtol=tol, atol=tol, h_init=0.1 * h, h_max=h, nthreads=threads)
        dt += time.perf_counter() - t0
        lines += pick.size
        del fo
    return dict({"value": lines / dt, "unit": "lines/s", "cores": threads, "kind": "oracle",
                 "sample": f"{args.cpu_fraction:g} of each field's seeds ({lines} lines, {dt:.1f} s of tracing)"},
                **host_info())


if __name__ == "__main__":
    main()
