"""GPU parity of the HIP tracer (through the C-ABI) against the FP64 oracle.

Per-line gates (lines whose oracle Q < 1e6 and whose exit faces agree):
relative error of log10 Q <= 1e-3, footpoints <= 1e-5 domain units,
field-line length <= 1e-4 relative.  Same seeds, field and tolerance on both
sides.  FP64 stepping meets them on every line.  FP32 stepping is held to the
statistical gates of gpu_util.check_fp32 (most lines within the per-line
gates; error against the converged FP64 answer no worse than FP64 stepping's
at the same tolerance).  QSL Squasher Sect. 3.1-3.5.
"""
import numpy as np
import pytest

import synth
from gpu_util import (FP_TOL, check_fp32, check_lines, gpu_field, gpu_trace, parity, qfp_in_gate, qfp_parity,
                      sensitivity_floor)

pytestmark = pytest.mark.gpu


def _oracle_grid(oracle_mod, b, origin, spacing, mode, store):
    """The oracle on the field the GPU stores: FP32 node storage rounds the
    prepared node values to FP32, and the oracle traces that same field."""
    return oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in b), origin, spacing,
                                 mode=oracle_mod.PAPER if mode == "paper" else oracle_mod.INTERP_NORMALIZE,
                                 store=store)


# ---------------------------------------------------------------------------
# hyperbolic flux tube, 64^3 FP64 grid, 128^2 seeds on z = 0, FP64 stepping at 1e-8
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    return synth.hyperbolic_c1()


@pytest.mark.parametrize("mode", ["interp_normalize", "paper"])
def test_c1_fp64_parity(oracle_mod, c1, mode):
    seeds = c1["seeds"]
    h = min(c1["spacing"])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c1["b"], c1["origin"], c1["spacing"], storage="f64", mode=mode)
    g = gpu_trace(fg, seeds, step_dtype="f64", **kw)
    fo = _oracle_grid(oracle_mod, c1["b"], c1["origin"], c1["spacing"], mode, "f64")
    o = oracle_mod.trace(fo, seeds, **kw)
    p = parity(g, o)
    check_lines(p, o, strict=True, max_mismatch_frac=0.0)
    assert p["gate"].sum() == seeds.shape[0]
    # the top-exit lines of the configuration carry Q_fp = 2 cosh(2k)
    top = (g["status"] & 0xFF) == 5
    assert top.sum() == 18 * 128
    if mode == "interp_normalize":
        assert np.allclose(g["q_fp"][top], 2 * np.cosh(4.0), rtol=1e-6)
    else:
        assert np.allclose(g["q_fp"][top], 2 * np.cosh(4.0), rtol=5e-3)
    assert np.allclose(g["q_det"], o["q_det"], rtol=1e-6)


# ---------------------------------------------------------------------------
# point-charge fields, FP32 node storage
# ---------------------------------------------------------------------------

CH = synth.point_charges(2, 4)


@pytest.fixture(scope="module")
def small_charges():
    n = (97, 97, 49)
    b = synth.sample_charges(CH, n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    return dict(b=b, origin=origin, spacing=spacing, n=n)


def _mixed_seeds(count, seed):
    s = synth.random_seeds(seed, count)
    s[: count // 2, 2] = 0.0            # half on the photosphere, half inside
    return s


@pytest.mark.parametrize("step_dtype,tol", [("f32", 1e-5), ("f32", 1e-4), ("f64", 1e-5), ("f64", 1e-8)])
def test_charges_parity(oracle_mod, small_charges, step_dtype, tol):
    """FP64 stepping: every gated line within the per-line gates, at tol 1e-5
    and 1e-8.  FP32 stepping at tol 1e-4: the statistical gates, with the
    per-line floor measured on the oracle (seeds moved by 1e-7).  FP32 stepping
    at tol 1e-5: the accuracy gates against the converged answer only.  There
    the FP32 rounding of the stage slopes (~1e-7 of |k|) is no longer small
    against the error estimate (~tol), so accept/reject decisions near err = 1
    flip.  Measured: 5.4 % of lines take another step sequence than FP64
    stepping at 1e-5, against 0.2 % at 1e-4.  The oracle with its stage points,
    slopes and states rounded to FP32 changes 1.5 % of the step sequences and
    moves 0.6 % of the lines out of the gates (test_oracle_sensitivity), so
    most flips come from evaluating the slopes in FP32, which rounding their
    FP64 values does not reproduce."""
    c = small_charges
    seeds = _mixed_seeds(1000 + 37, 41)      # ragged: not a multiple of the wave size
    h = min(c["spacing"])
    kw = dict(rtol=tol, atol=tol, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32")
    g = gpu_trace(fg, seeds, step_dtype=step_dtype, **kw)
    fo = _oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32")
    o = oracle_mod.trace(fo, seeds, **kw)
    p = parity(g, o)
    assert p["gate"].mean() > 0.97
    if step_dtype == "f64":
        check_lines(p, o, strict=True)
        _check_qfp(g, o, 1.0)
    elif tol >= 1e-4:
        ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
        floor, _ = sensitivity_floor(oracle_mod, fo, seeds, o, kw)
        check_fp32(p, g, o, ref, min_frac=floor)
        _check_qfp(g, o, sensitivity_floor(oracle_mod, fo, seeds, o, kw, judge=qfp_in_gate)[0])
    else:
        ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
        check_fp32(p, g, o, ref, min_frac=0.0)


def _check_qfp(g, o, floor):
    """The exit-face-plane Q per line against the oracle's, on every line with
    both ends on faces -- the bottom face and the side and top faces -- with
    the Q gate (relative log10 error <= 1e-3): all of them for FP64 stepping,
    at least the sensitivity floor's share for FP32 stepping."""
    m, e = qfp_parity(g, o)
    fwd, bwd = o["status"] & 0xFF, (o["status"] >> 8) & 0xFF
    side = m & ((fwd < 4) | (bwd < 4) | (fwd == 5) | (bwd == 5))
    ok = np.nan_to_num(e, nan=np.inf) <= 1e-3
    print(f"q_fp: {int(m.sum())} lines with two face ends ({int(side.sum())} reach a side or the top), "
          f"{float(ok[m].mean()):.4f} within 1e-3, max {np.nanmax(e[m]):.2e}")
    assert side.sum() >= 20
    assert ok[m].mean() >= floor and ok[side].mean() >= floor


@pytest.mark.parametrize("n", [1, 2047, 2049, 6001])
def test_spatial_order_steps_every_line_once(oracle_mod, small_charges, n):
    """The half-lines are stepped in spatial order (a radix sort of their
    seeds' cells, tiles of 2048 items): whatever the count and however many
    seeds share a cell (equal keys), every line is stepped exactly once and its
    result does not depend on where the sort put it -- the same seeds given in
    reverse and shuffled order give identical per-seed outputs, and statuses
    match the oracle's."""
    c = small_charges
    g0 = synth.rng(90 + n)
    seeds = _mixed_seeds(n, 90 + n)
    if n > 8:
        # a third of the seeds are copies of five points: long runs of equal keys
        k = n // 3
        seeds[:k] = seeds[g0.integers(k, n, size=5)][g0.integers(0, 5, size=k)]
    h = min(c["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32")
    ref = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    for perm in (np.arange(n)[::-1].copy(), g0.permutation(n)):
        out = gpu_trace(fg, seeds[perm], step_dtype="f32", **kw)
        for key in ("status", "fll", "q_perp", "fp_fwd", "fp_bwd"):
            a, b = np.nan_to_num(out[key], nan=-7.0), np.nan_to_num(ref[key][perm], nan=-7.0)
            assert np.array_equal(a, b), key
    if n >= 100:
        fo = _oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32")
        o = oracle_mod.trace(fo, seeds, **kw)
        assert (ref["status"] == o["status"]).mean() >= 0.99


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_cell_cache_gathers_bit_identical_at_long_steps(small_charges, storage):
    """With steps of up to 4 cells most stage points land in another cell, and
    in a wave some lanes move while others stay: the register cell cache
    (corners loaded by the lanes that moved only), its LDS form and, for FP32
    records, the register cache over brick records and over direction records
    give the same outputs as direct corner loads, bit for bit, for FP32 and
    BF16 records."""
    import torch

    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TracePlan, make_opts
    c = small_charges
    h = min(c["spacing"])
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage=storage)
    gathers = [A.GATHER_DIRECT, A.GATHER_REGS, A.GATHER_CACHED]
    if storage == "f32":
        fg.add_bricks()
        fg.add_cell_dirs()
        gathers += [A.GATHER_BRICKS, A.GATHER_DIRS]
    dev = torch.device("cuda:0")
    n = 3000
    seeds = torch.from_numpy(np.ascontiguousarray(_mixed_seeds(n, 77).T)).to(dev)
    res = {}
    for gather in gathers:
        plan = TracePlan(n, dev, want_steps=True)
        opts = make_opts(1e-2, 1e-2, h_init=0.1 * h, h_max=4 * h, step_dtype="f32",
                         launch=A.launch_word(2, 128, gather))
        out = plan.run(fg, seeds, opts)
        torch.cuda.synchronize()
        res[gather] = {k: v.clone() for k, v in out.items()}
    ref = res[A.GATHER_DIRECT]
    for gather, r in res.items():
        for k in ref:
            assert torch.equal(torch.nan_to_num(r[k], nan=-7.0), torch.nan_to_num(ref[k], nan=-7.0)), (gather, k)
    assert int((ref["steps"][0] > 3).sum()) > n // 4


def test_direction_records_on_an_uneven_grid():
    """A grid with a different node count on every axis (so that a cell index
    with the axes swapped would read another cell): the register cache over
    direction records and over brick records, at steps of up to 4 cells,
    give the direct corner loads' outputs bit for bit, with and without the
    per-XCD parts."""
    import torch

    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TracePlan, make_opts
    n = (89, 71, 41)
    b = synth.sample_charges(CH, n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    h = min(spacing)
    fg = gpu_field(b, origin, spacing).add_bricks().add_cell_dirs()
    assert fg.desc.dir_bytes == 96 * 88 * 70 * 40
    dev = torch.device("cuda:0")
    m = 2000
    seeds = torch.from_numpy(np.ascontiguousarray(_mixed_seeds(m, 78).T)).to(dev)
    res = {}
    for word in (A.launch_word(2, 128, A.GATHER_DIRECT), A.launch_word(2, 128, A.GATHER_BRICKS),
                 A.launch_word(2, 128, A.GATHER_DIRS), A.launch_word(1, 64, A.GATHER_DIRS, parts=True)):
        plan = TracePlan(m, dev, want_steps=True)
        opts = make_opts(1e-2, 1e-2, h_init=0.1 * h, h_max=4 * h, step_dtype="f32", launch=word)
        out = plan.run(fg, seeds, opts)
        torch.cuda.synchronize()
        res[word] = {k: v.clone() for k, v in out.items()}
    ref = res[A.launch_word(2, 128, A.GATHER_DIRECT)]
    for word, r in res.items():
        for k in ref:
            assert torch.equal(torch.nan_to_num(r[k], nan=-7.0), torch.nan_to_num(ref[k], nan=-7.0)), (word, k)
    assert int((ref["steps"][0] > 3).sum()) > m // 4


@pytest.mark.parametrize("n", [1, 3, 8, 9, 65, 1000])
def test_xcd_parts_edge_counts(small_charges, n):
    """The work list split into per-XCD parts (QSQ_LAUNCH_PARTS) with fewer
    items than parts, than workgroups, or than one wave: every line is traced
    once and every output equals the single-counter launch's bit for bit, for
    the register cache and for direct loads."""
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TracePlan, make_opts
    c = small_charges
    h = min(c["spacing"])
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32")
    dev = torch.device("cuda:0")
    seeds = torch.from_numpy(np.ascontiguousarray(_mixed_seeds(n, 300 + n).T)).to(dev)
    res = {}
    for gather in (A.GATHER_REGS, A.GATHER_DIRECT):
        for parts in (False, True):
            plan = TracePlan(n, dev, want_steps=True)
            opts = make_opts(1e-4, 1e-4, h_init=0.1 * h, h_max=h, step_dtype="f32",
                             launch=A.launch_word(1, 64, gather, parts))
            out = plan.run(fg, seeds, opts)
            torch.cuda.synchronize()
            res[(gather, parts)] = {k: v.clone() for k, v in out.items()}
    ref = res[(A.GATHER_REGS, False)]
    for key, r in res.items():
        for k in ref:
            assert torch.equal(torch.nan_to_num(r[k], nan=-7.0), torch.nan_to_num(ref[k], nan=-7.0)), (key, k)
    assert int((ref["steps"][0] > 0).sum()) > 0 or n < 3


def test_interp_normalize_fp32(oracle_mod, small_charges):
    c = small_charges
    seeds = _mixed_seeds(500, 5)
    h = min(c["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32", mode="interp_normalize")
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    fo = _oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "interp_normalize", "f32")
    o = oracle_mod.trace(fo, seeds, **kw)
    ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
    check_fp32(parity(g, o), g, o, ref, min_frac=sensitivity_floor(oracle_mod, fo, seeds, o, kw)[0])


# ---------------------------------------------------------------------------
# stops and degenerate inputs
# ---------------------------------------------------------------------------

def test_edge_cases(oracle_mod, small_charges):
    import paper_1609_00724_amd as q
    c = small_charges
    h = min(c["spacing"])
    kw = dict(rtol=1e-6, atol=1e-6, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32")
    fo = _oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32")
    seeds = np.array([
        [0.0, 0.0, -0.01], [1.5, 0.0, 0.5],          # outside
        [-1.0, -1.0, 0.0], [1.0, 1.0, 1.0],          # corners
        [1.0, 0.3, 0.4], [-1.0, 0.2, 0.7],           # side faces
        [0.1, 0.1, 1.0], [0.2, -0.3, 0.0],           # top, bottom
        [0.05, 0.02, 0.3],
    ])
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    o = oracle_mod.trace(fo, seeds, **kw)
    assert np.array_equal(g["status"], o["status"])
    assert np.all((g["status"][:2] & 0xFF) == q._abi.END_SEED_OUTSIDE)
    # a single seed and exactly three seeds take the same path as any count
    for k in (1, 3):
        gk = gpu_trace(fg, seeds[2:2 + k], step_dtype="f32", **kw)
        assert np.array_equal(gk["status"], g["status"][2:2 + k])
        assert np.array_equal(gk["fll"], g["fll"][2:2 + k])
    assert np.all(np.isnan(g["q_perp"][:2])) and np.all(g["fll"][:2] == 0)
    p = parity(g, o)
    assert p["fp"][p["gate"]].max() <= FP_TOL

    # max_length ("local Q") and max_steps
    g = gpu_trace(fg, seeds[2:], step_dtype="f32", max_length=0.05, **kw)
    o = oracle_mod.trace(fo, seeds[2:], max_length=0.05, **kw)
    assert np.array_equal(g["status"], o["status"])
    both = ((g["status"] & 0xFF) == 6) & (((g["status"] >> 8) & 0xFF) == 6)
    assert both.any() and np.all(g["fll"][both] == 0.1)
    g = gpu_trace(fg, seeds[2:], step_dtype="f32", max_steps=1, **kw)
    o = oracle_mod.trace(fo, seeds[2:], max_steps=1, **kw)
    assert np.array_equal(g["status"], o["status"])

    # open-line switch: Q masked for open lines only
    g1 = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    g2 = gpu_trace(fg, seeds, step_dtype="f32", skip_open=True, **kw)
    open_ = (g1["status"] & q._abi.STATUS_OPEN) != 0
    assert np.all(np.isnan(g2["q_perp"][open_]))
    assert np.array_equal(g2["q_perp"][~open_], g1["q_perp"][~open_])


def test_null_region_and_empty(oracle_mod):
    import paper_1609_00724_amd as q
    import torch
    n = (9, 9, 9)
    b = list(synth.sample_linear(*synth.uniform([0, 0, 1.0]), n))
    b[2][3:6, 3:6, 3:6] = 0.0
    origin, spacing = synth.grid_geometry(n)
    fg = gpu_field(b, origin, spacing, storage="f32")
    seeds = np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.1], [0.9, 0.9, 0.1]])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.01, h_max=min(spacing))
    g = gpu_trace(fg, seeds, step_dtype="f64", **kw)
    o = oracle_mod.trace(oracle_mod.Field.grid(*b, origin, spacing, store="f32"), seeds, **kw)
    assert np.array_equal(g["status"], o["status"])
    assert (g["status"][0] & 0xFF) == q._abi.END_NULL
    # zero seeds: nothing enqueued, no error
    out = q.trace(fg, torch.empty((0, 3), dtype=torch.float64, device="cuda"), rtol=1e-6, atol=1e-6)
    assert out["status"].numel() == 0


def test_step_counts_match_oracle(oracle_mod, c1):
    """FP64 stepping takes the oracle's step sequence (attempts per half-line)."""
    seeds = c1["seeds"][::53]
    h = min(c1["spacing"])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c1["b"], c1["origin"], c1["spacing"], storage="f64", mode="paper")
    g = gpu_trace(fg, seeds, step_dtype="f64", want_steps=True, **kw)
    o = oracle_mod.trace(_oracle_grid(oracle_mod, c1["b"], c1["origin"], c1["spacing"], "paper", "f64"), seeds,
                         **kw)
    att_o = o["counts"][:, 0, 0] + o["counts"][:, 0, 1]
    att_g = g["steps"][0]
    moving = o["lam_fwd"] > 0
    close = np.abs(att_g[moving] - att_o[moving]) <= 2
    assert close.mean() > 0.95, (att_g[moving][:10], att_o[moving][:10])


def test_bf16_storage(oracle_mod, small_charges):
    """BF16 node records: the tracer matches the oracle on the same BF16-rounded
    field (FP32 stepping gates), and the storage error itself -- BF16 field
    against the FP64 field -- is measured and bounded."""
    c = small_charges
    seeds = _mixed_seeds(600, 17)
    h = min(c["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="bf16")
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    fo = _oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "bf16")
    o = oracle_mod.trace(fo, seeds, **kw)
    ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
    check_fp32(parity(g, o), g, o, ref, min_frac=sensitivity_floor(oracle_mod, fo, seeds, o, kw)[0])
    # storage error: BF16 field vs the unrounded field
    f64 = oracle_mod.trace(_oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f64"),
                           seeds, **kw)
    p = parity(g, f64)
    m = p["gate"]
    print(f"BF16 storage error: footpoints median {np.median(p['fp'][m]):.2e} p90 {np.percentile(p['fp'][m], 90):.2e}, "
          f"rel log10 Q median {np.nanmedian(p['lq'][m]):.2e} p90 {np.nanpercentile(p['lq'][m], 90):.2e}")
    assert np.median(p["fp"][m]) < 1e-2 and np.nanmedian(p["lq"][m]) < 1e-2


# ---------------------------------------------------------------------------
# twisted flux rope over a 6-charge background (small grid of the volume workload)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rope():
    n = (72, 72, 48)
    b, meta = synth.flux_rope_field(n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    return dict(b=b, origin=origin, spacing=spacing, n=n, **meta)


def test_flux_rope_fp64_parity(oracle_mod, rope):
    """FP64 storage and stepping at tolerance 1e-8 through a twisted rope: every
    gated line meets the per-line gates."""
    seeds = synth.random_seeds(41, 700)
    h = min(rope["spacing"])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    fg = gpu_field(rope["b"], rope["origin"], rope["spacing"], storage="f64")
    g = gpu_trace(fg, seeds, step_dtype="f64", **kw)
    fo = _oracle_grid(oracle_mod, rope["b"], rope["origin"], rope["spacing"], "paper", "f64")
    o = oracle_mod.trace(fo, seeds, **kw)
    p = parity(g, o)
    check_lines(p, o, strict=True)
    _check_qfp(g, o, 1.0)
    # the rope twists lines: some closed lines (both ends on z = 0) are long
    closed = (o["status"] & 0xFFFF) == (4 | (4 << 8))
    assert closed.sum() > 100 and np.percentile(o["fll"][closed], 90) > 0.5


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_flux_rope_fp32_stepping(oracle_mod, rope, storage):
    """FP32 stepping on FP32 and BF16 node records of the rope field against the
    oracle on the same rounded field (statistical FP32 gates)."""
    seeds = synth.random_seeds(43, 700)
    h = min(rope["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = gpu_field(rope["b"], rope["origin"], rope["spacing"], storage=storage)
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    fo = _oracle_grid(oracle_mod, rope["b"], rope["origin"], rope["spacing"], "paper", storage)
    o = oracle_mod.trace(fo, seeds, **kw)
    ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
    check_fp32(parity(g, o), g, o, ref, min_frac=sensitivity_floor(oracle_mod, fo, seeds, o, kw)[0])


# ---------------------------------------------------------------------------
# UNDERFLOW, NONFINITE and non-finite seeds: status parity with the oracle on
# the inputs its pins use (tests/test_oracle_trace.py)
# ---------------------------------------------------------------------------

def test_underflow_at_a_spine_null(oracle_mod):
    """A line run into a null along its spine stops with UNDERFLOW on the GPU
    as in the oracle (FP64 stepping, tol 1e-8): same statuses, ends on the
    spine within 1e-9 of the null, lengths as the oracle's."""
    from test_oracle_trace import SPINE_SEEDS, spine_null
    b, origin, spacing = spine_null()
    h = min(spacing)
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    fg = gpu_field(b, origin, spacing, storage="f64", mode="interp_normalize")
    g = gpu_trace(fg, SPINE_SEEDS, step_dtype="f64", **kw)
    o = oracle_mod.trace(oracle_mod.Field.grid(*b, origin, spacing, mode=oracle_mod.INTERP_NORMALIZE),
                         SPINE_SEEDS, **kw)
    assert np.array_equal(g["status"], o["status"])
    assert np.all((g["status"] & 0xFF) == oracle_mod.UNDERFLOW)
    assert np.all(g["fp_fwd"][:, :2] == 0.0) and np.all(np.abs(g["fp_fwd"][:, 2]) < 1e-9)
    assert np.allclose(g["fll"], o["fll"], rtol=0, atol=1e-8)
    assert np.all(np.isnan(g["q_perp"]))


@pytest.mark.parametrize("value", [np.nan, np.inf])
@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
@pytest.mark.parametrize("storage,step_dtype", [("f64", "f64"), ("f32", "f32")])
def test_nonfinite_node_status_parity(oracle_mod, value, mode, storage, step_dtype):
    """A NaN or Inf node on the line's way: NONFINITE at the last finite state,
    as in the oracle on the same stored field; the other half unaffected."""
    from test_oracle_trace import poisoned_uniform
    b, origin, spacing = poisoned_uniform(value)
    seeds = np.array([[0.0, 0.0, 0.1], [0.5, 0.5, 0.3], [0.0, 0.0, 0.9]])
    h = min(spacing)
    kw = dict(rtol=1e-6, atol=1e-6, h_init=0.1 * h, h_max=h)
    fg = gpu_field(b, origin, spacing, storage=storage, mode=mode)
    g = gpu_trace(fg, seeds, step_dtype=step_dtype, **kw)
    md = oracle_mod.PAPER if mode == "paper" else oracle_mod.INTERP_NORMALIZE
    o = oracle_mod.trace(oracle_mod.Field.grid(*b, origin, spacing, mode=md, store=storage), seeds, **kw)
    assert np.array_equal(g["status"], o["status"]), (g["status"], o["status"])
    assert (g["status"][0] & 0xFF) == oracle_mod.NONFINITE
    assert ((g["status"][2] >> 8) & 0xFF) == oracle_mod.NONFINITE
    tol = 1e-12 if step_dtype == "f64" else 1e-6
    assert np.allclose(g["fp_fwd"], o["fp_fwd"], rtol=0, atol=tol)
    assert np.allclose(g["fp_bwd"], o["fp_bwd"], rtol=0, atol=tol)
    assert np.allclose(g["fll"], o["fll"], rtol=0, atol=tol)
    assert np.isnan(g["q_perp"][0]) and np.isnan(g["q_perp"][2]) and np.isfinite(g["q_perp"][1])


def test_non_finite_seed_is_outside(oracle_mod, small_charges):
    c = small_charges
    seeds = np.array([[np.nan, 0.0, 0.5], [0.0, 0.0, np.inf], [0.1, 0.1, 0.5]])
    h = min(c["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = gpu_field(c["b"], c["origin"], c["spacing"], storage="f32")
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    o = oracle_mod.trace(_oracle_grid(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32"), seeds, **kw)
    assert np.array_equal(g["status"], o["status"])
    assert np.all((g["status"][:2] & 0xFF) == oracle_mod.SEED_OUTSIDE) and np.all(g["fll"][:2] == 0.0)
