"""Batched trace: many fields and seed sets of uneven size in one job (one
persistent stepping launch), checked against one-field traces of the same
sets and against the FP64 oracle; capture of the batched call in a HIP graph
and replay.  Same per-seed computation as the one-field trace (QSL Squasher
Sect. 3.1-3.5)."""
import numpy as np
import pytest

import synth
from gpu_util import check_lines, gpu_field, line_ok, parity

pytestmark = pytest.mark.gpu

SMALL_DIMS = ((24, 24, 16), (32, 32, 32), (40, 32, 20), (20, 20, 20), (48, 40, 24))


def _sets(count, dtype, empty=(3,)):
    out = []
    for k, f in enumerate(synth.batch_c3(count=count, first_seed=3000, dims=SMALL_DIMS,
                                         seeds_range=(20, 1500), dtype=dtype)):
        if k in empty:
            f["seeds"] = np.zeros((0, 3))
        out.append(f)
    return out


def _to_np(out):
    r = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("fp_fwd", "fp_bwd"):
        if k in r:
            r[k] = r[k].T.copy()
    return r


def _run_batch(sets, fields, **kw):
    import torch

    import paper_1609_00724_amd as q
    dev = torch.device("cuda:0")
    outs, work = q.trace_batch([(fg, torch.from_numpy(f["seeds"]).to(dev)) for fg, f in zip(fields, sets)],
                               want_steps=True, want_work=True, **kw)
    torch.cuda.synchronize()
    return [_to_np(o) for o in outs], work.cpu().numpy()


def _run_single(sets, fields, **kw):
    import torch

    import paper_1609_00724_amd as q
    dev = torch.device("cuda:0")
    res = []
    for fg, f in zip(fields, sets):
        if f["seeds"].shape[0] == 0:
            res.append(None)
            continue
        o = q.trace(fg, torch.from_numpy(f["seeds"]).to(dev), want_steps=True, **kw)
        torch.cuda.synchronize()
        res.append(_to_np(o))
    return res


def test_batch_fp64_matches_single_and_oracle(oracle_mod):
    sets = _sets(7, np.float64)
    fields = [gpu_field(f["b"], f["origin"], f["spacing"], storage="f64") for f in sets]
    kw = dict(rtol=1e-8, atol=1e-8, step_dtype="f64")      # h_init, h_max: each grid's own defaults
    bat, work = _run_batch(sets, fields, **kw)
    one = _run_single(sets, fields, **kw)
    total_steps = 0
    for k, (f, b, s) in enumerate(zip(sets, bat, one)):
        n = f["seeds"].shape[0]
        assert b["status"].shape == (n,)
        if n == 0:
            continue
        np.testing.assert_array_equal(b["status"], s["status"], err_msg=f"set {k}")
        np.testing.assert_array_equal(b["steps"], s["steps"], err_msg=f"set {k}")
        for key in ("fp_fwd", "fp_bwd", "fll", "q_perp", "q_det", "q_fp"):
            np.testing.assert_allclose(b[key], s[key], rtol=1e-12, atol=1e-14, equal_nan=True,
                                       err_msg=f"set {k} {key}")
        total_steps += int(b["steps"].sum())
        h = min(f["spacing"])
        fo = oracle_mod.Field.grid(*f["b"], f["origin"], f["spacing"])
        o = oracle_mod.trace(fo, f["seeds"], rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
        check_lines(parity(b, o), o, strict=True, max_mismatch_frac=0.0)
    # the batch's work counters sum the step attempts of every half-line
    assert work[0] == total_steps


def test_batch_fp32_matches_single():
    sets = _sets(6, np.float32, empty=(0,))
    fields = [gpu_field(f["b"], f["origin"], f["spacing"], storage="f32") for f in sets]
    kw = dict(rtol=1e-5, atol=1e-5, step_dtype="f32")
    bat, _ = _run_batch(sets, fields, **kw)
    one = _run_single(sets, fields, **kw)
    for k, (f, b, s) in enumerate(zip(sets, bat, one)):
        if f["seeds"].shape[0] == 0:
            assert b["status"].size == 0
            continue
        p = parity(b, s)
        ok = line_ok(p)[p["gate"]]
        print(f"set {k}: n={b['status'].size} status mismatch {p['status_mismatch']} within gates {ok.mean():.4f}")
        assert p["status_mismatch"] <= 0.003 * b["status"].size + 1
        assert ok.mean() >= 0.998


def test_batch_graph_replay():
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import TraceBatchPlan, make_opts
    dev = torch.device("cuda:0")
    sets = _sets(5, np.float32, empty=(2,))
    fields = [gpu_field(f["b"], f["origin"], f["spacing"], storage="f32") for f in sets]
    plan = TraceBatchPlan([(fg, torch.from_numpy(f["seeds"]).to(dev)) for fg, f in zip(fields, sets)],
                          make_opts(1e-4, 1e-4, step_dtype="f32"), want_steps=True, want_work=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run()                                   # eager run (also warms up)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in plan.outs]
    work_ref = plan.work.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run()
    torch.cuda.synchronize()
    for rep in range(3):
        # eager work between replays: poison every output and the counters
        for o in plan.outs:
            for v in o.values():
                v.fill_(-7)
        plan.work.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(plan.outs, ref)):
            for key in r:
                assert torch.equal(o[key], r[key]), f"replay {rep} set {k} {key}"
        assert torch.equal(plan.work, work_ref), f"replay {rep} work"
    assert q.lib.qsq_abi_version() == 4


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_launch_shapes_give_identical_results(storage):
    """The launch shape (lanes per CU, workgroup size) moves no result: every
    line's arithmetic is the same wherever it runs.  The register cell cache
    reads the same node values into the same arithmetic as the direct loads:
    the same results bit for bit.  The LDS cell cache reads the same node
    values; it must agree with them line by line within the FP32 gates.  FP32
    and BF16 node records."""
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd import autotune
    from paper_1609_00724_amd.api import TracePlan, make_opts
    dev = torch.device("cuda:0")
    f = _sets(1, np.float32, empty=())[0]
    fg = gpu_field(f["b"], f["origin"], f["spacing"], storage=storage)
    seeds = torch.from_numpy(synth.random_seeds(77, 5000)).to(dev).t().contiguous()
    plan = TracePlan(seeds.shape[1], dev, want_steps=True)
    res = {}
    # gather 4 before the cell records exist runs the direct loads
    # (lanes, workgroup, gather[, work list in per-XCD parts])
    shapes = [(0, 256, 4), (0, 256, 1), (2, 64, 1), (3, 128, 1), (12, 256, 1), (2, 64, 1, True), (0, 256, 2),
              (2, 64, 2), (6, 128, 2), (1, 256, 2, True), (0, 256, 3), (2, 128, 3), (1, 64, 3), (1, 256, 3, True),
              "cells", (1, 256, 4), (2, 64, 4), (6, 128, 4), (2, 64, 4, True),
              "bricks", (1, 256, 5), (2, 64, 5), (2, 128, 5, True)]
    for shape in shapes:
        if shape == "cells":
            fg.add_cells()
            continue
        if shape == "bricks":
            fg.add_bricks()
            continue
        lanes, wg, gather, *rest = shape
        parts = bool(rest and rest[0])
        key = (lanes, wg, gather, fg.cells_ws is not None, parts)
        opts = make_opts(1e-5, 1e-5, step_dtype="f32", launch=A.launch_word(lanes, wg, gather, parts))
        out = plan.run(fg, seeds, opts)
        torch.cuda.synchronize()
        res[key] = {k: v.clone() for k, v in out.items()}
    # direct loads, the register cache (node or brick records) and the cell records: one group
    group = {1: 1, 2: 2, 3: 1, 4: 1, 5: 1}
    for g in (1, 2):
        ref = next(v for k, v in res.items() if group[k[2]] == g)
        for k, v in res.items():
            if group[k[2]] != g:
                continue
            for key in ref:
                assert torch.equal(torch.nan_to_num(v[key], nan=-1.0), torch.nan_to_num(ref[key], nan=-1.0)), (k, key)
    assert sum(1 for k in res if k[2] == 4 and k[3]) == 4
    assert sum(1 for k in res if k[4]) == 5
    assert sum(1 for k in res if k[2] == 5) == 3
    a, b = res[(0, 256, 1, False, False)], res[(0, 256, 2, False, False)]
    same = (a["status"] == b["status"]).float().mean().item()
    close = ((a["fll"] - b["fll"]).abs() <= 1e-4 * b["fll"].abs().clamp(min=1e-12)).float().mean().item()
    print(f"direct vs cached gathers: status agreement {same:.4f}, lengths within 1e-4: {close:.4f}")
    assert same >= 0.997 and close >= 0.99
    word, table = autotune.tune_trace(fg, seeds.t().contiguous(), make_opts(1e-5, 1e-5, step_dtype="f32"), reps=1,
                                      cands=autotune.candidates(lanes=(2, 8), wgs=(128, 256)), use_cache=False)
    assert word in table and table[word] == min(table.values())
    assert autotune.describe(word)["workgroup"] in (128, 256)


def test_batch_register_cache_word_runs_direct():
    """Batches lay lines of many fields side by side in a wave, so the cell
    caches do not apply: a batched call with the register-cache word runs the
    direct loads and gives the same results bit for bit, FP32 and BF16
    records."""
    import torch

    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TraceBatchPlan, make_opts
    dev = torch.device("cuda:0")
    for storage, dtype in (("f32", np.float32), ("bf16", np.float32)):
        sets = _sets(6, dtype, empty=(4,))
        fields = [gpu_field(f["b"], f["origin"], f["spacing"], storage=storage) for f in sets]
        pairs = [(fg, torch.from_numpy(f["seeds"]).to(dev)) for fg, f in zip(fields, sets)]
        res = []
        for word in (A.launch_word(2, 64, A.GATHER_DIRECT), A.launch_word(2, 64, A.GATHER_REGS),
                     A.launch_word(0, 256, A.GATHER_AUTO), A.launch_word(1, 128, A.GATHER_DIRECT, parts=True)):
            plan = TraceBatchPlan(pairs, make_opts(1e-4, 1e-4, step_dtype="f32", launch=word), want_steps=True)
            plan.run()
            torch.cuda.synchronize()
            res.append([{k: v.clone() for k, v in o.items()} for o in plan.outs])
        for other in res[1:]:
            for k, (a, b) in enumerate(zip(res[0], other)):
                for key in a:
                    assert torch.equal(torch.nan_to_num(a[key], nan=-1.0), torch.nan_to_num(b[key], nan=-1.0)), \
                        (storage, k, key)


def test_full_batch_sampled(oracle_mod):
    """The benchmark's batch at full size (64 point-charge fields on grids of
    64^3 to 256x256x128, 10^4-10^6 random seeds each, FP32 storage and
    stepping at tol 1e-4, one batched call in spatial work order): every
    field's sampled lines against the FP64 oracle on the same FP32-rounded
    field, with the FP32 gates; the converged oracle (tol 1e-10) decides the
    statistical comparison."""
    import torch

    from gpu_util import check_fp32
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TraceBatchPlan, make_opts
    dev = torch.device("cuda:0")
    g = synth.rng(64)
    sets, picks, oracle_out, ref_out = [], [], [], []
    for f in synth.batch_c3(count=64):
        fg = gpu_field(f["b"], f["origin"], f["spacing"], storage="f32")
        n = f["seeds"].shape[0]
        pick = np.sort(g.choice(n, size=min(n, 6), replace=False))
        h = min(f["spacing"])
        kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
        fo = oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in f["b"]), f["origin"], f["spacing"],
                                   store="f32")
        oracle_out.append(oracle_mod.trace(fo, f["seeds"][pick], **kw))
        ref_out.append(oracle_mod.trace(fo, f["seeds"][pick], **dict(kw, rtol=1e-10, atol=1e-10)))
        del fo
        sets.append((fg, torch.from_numpy(f["seeds"]).to(dev)))
        picks.append(pick)
    opts = make_opts(1e-4, 1e-4, step_dtype="f32", launch=A.launch_word(3, 64, 1))
    plan = TraceBatchPlan(sets, opts)
    plan.run()
    torch.cuda.synchronize()
    outs = [_to_np(o) for o in plan.outs]
    cat = lambda rs, key: np.concatenate([r[key] for r in rs])   # noqa: E731
    gsel = [{k: v[p] for k, v in o.items()} for o, p in zip(outs, picks)]
    keys = ("status", "q_perp", "fll", "fp_fwd", "fp_bwd")
    gg = {k: cat(gsel, k) for k in keys}
    oo = {k: cat(oracle_out, k) for k in keys}
    rr = {k: cat(ref_out, k) for k in keys}
    check_fp32(parity(gg, oo), gg, oo, rr)
