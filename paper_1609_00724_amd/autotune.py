"""Launch-shape autotuner for the persistent stepping kernel.

Candidates are QSQ_LAUNCH words (resident-lane target per compute unit,
workgroup size, corner-gather variant).  Each is timed with HIP events on a
sample of the caller's own seeds and the fastest is kept.  Every candidate
computes the same result (a line's arithmetic does not depend on where it
runs), so tuning only moves time.  Choices are cached per (device, grid,
storage, mode, step dtype, tolerance) in memory and, if QSQ_TUNE_CACHE names a
file, in that JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import _abi as A

DEFAULT_LANES = (1, 2, 3, 4, 6, 8, 12)
DEFAULT_WG = (64, 128, 256)

_cache: dict = {}


# The cell-cache variants of the stepping kernel need more than 168 registers
# per lane, so at most 2 waves per SIMD (512 lanes per CU) stay resident: a
# larger lane target launches the same shape.
CACHE_LANES = (1, 2)


def candidates(lanes=DEFAULT_LANES, wgs=DEFAULT_WG, gathers=(A.GATHER_DIRECT, A.GATHER_CACHED, A.GATHER_REGS),
               parts=(False, True)):
    """Launch words over lanes x workgroup x gather, each with the work list in
    one piece and split into per-XCD parts (QSQ_LAUNCH_PARTS)."""
    out = []
    for g in gathers:
        ls = (lanes if g in (A.GATHER_DIRECT, A.GATHER_CELLS)
              else tuple(l for l in lanes if l in CACHE_LANES) or lanes[:1])
        out += [A.launch_word(l, w, g, pt) for pt in parts for w in wgs for l in ls]
    return out


def _key(field, opts, tag):
    d = field.desc
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    return "|".join(str(v) for v in (name, tag, tuple(d.grid.n), d.storage, d.mode, opts.step_dtype, opts.rtol,
                                     opts.atol, opts.h_max))


def _load():
    path = os.environ.get("QSQ_TUNE_CACHE")
    if path and os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))


def _store():
    path = os.environ.get("QSQ_TUNE_CACHE")
    if path:
        with open(path, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)


def _time(run, reps):
    s = torch.cuda.current_stream()
    run()                               # warm-up (first touch, instruction cache)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        run()
        b.record(s)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_trace(field, seeds, opts, reps=3, cands=None, use_cache=True):
    """Fastest launch word for tracing `seeds` ((n, 3) device tensor, a sample
    of the workload) in `field` with `opts`.  Returns (word, {word: ms})."""
    from .api import TracePlan
    key = _key(field, opts, "trace")
    if use_cache:
        _load()
        if key in _cache:
            return int(_cache[key]["word"]), {int(k): v for k, v in _cache[key]["ms"].items()}
    soa = seeds.t().contiguous()
    plan = TracePlan(soa.shape[1], seeds.device)
    saved = opts.launch
    table = {}
    for w in cands or candidates():
        opts.launch = w
        table[w] = _time(lambda: plan.run(field, soa, opts), reps)
    opts.launch = saved
    best = min(table, key=table.get)
    _cache[key] = {"word": best, "ms": {str(k): v for k, v in table.items()}}
    _store()
    return best, table


def tune_batch(sets, opts, reps=3, cands=None):
    """Fastest launch word for a batched trace of `sets` ((field, seeds) pairs;
    the batch uses direct gathers, so only lanes and workgroup size vary)."""
    from .api import TraceBatchPlan
    plan = TraceBatchPlan(sets, opts)
    saved = opts.launch
    table = {}
    for w in cands or candidates(gathers=(A.GATHER_DIRECT,)):
        opts.launch = w
        plan.opts = opts
        table[w] = _time(plan.run, reps)
    opts.launch = saved
    best = min(table, key=table.get)
    return best, table


def describe(word):
    lanes = word & 15 or 8
    wg = {0: 256, 1: 64, 2: 128}[(word >> 4) & 3]
    names = {0: "auto", 1: "direct", 2: "lds-cache", 3: "reg-cache", 4: "cell-records",
             5: "reg-cache-bricks", 6: "reg-cache-dirs"}
    out = {"word": int(word), "lanes_per_cu": lanes * 256, "workgroup": wg, "gather": names[(word >> 6) & 7],
           "xcd_parts": bool(word & A.LAUNCH_PARTS)}
    if (word >> 10) & 7:
        out["refine_gather"] = names[(word >> 10) & 7]
    return out


def tune_map(plan, field, opts, reps=3, cands=None, batches=None):
    """Fastest launch word (and, if `batches` is given, refinement levels per
    device round) for a whole map call (QMapPlan) on `field`: the tuned
    workload is the real one (base lattice, refinement rounds).  Returns
    (word, table) or, with batches, ((word, batch), table); the plan keeps
    its own refine_batch."""
    saved_w, saved_b = opts.launch, plan.d.refine_batch
    table = {}
    for b in batches or (saved_b,):
        plan.d.refine_batch = b
        for w in cands or candidates():
            opts.launch = w
            table[(w, b)] = _time(lambda: plan.run(field, opts), reps)
    opts.launch, plan.d.refine_batch = saved_w, saved_b
    best = min(table, key=table.get)
    if batches is None:
        return best[0], {k[0]: v for k, v in table.items()}
    return best, table
