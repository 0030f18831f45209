"""Explicit Euler stepping (QSL Squasher Sect. 3.4: fixed steps of the line
and both deviation vectors, the exit step cut at the face in FP64) on the GPU
against the oracle's Euler on the same field, seeds and step.  FP64 stepping
meets the per-line gates on every line and takes the oracle's step counts;
FP32 stepping meets them on nearly every line; straight lines are exact; the
batched launch gives the one-field results bit for bit."""
import numpy as np
import pytest

import synth
from gpu_util import check_lines, gpu_field, gpu_trace, parity

pytestmark = pytest.mark.gpu

CH = synth.point_charges(2, 4)


def _oracle_grid(oracle_mod, b, origin, spacing, store):
    return oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in b), origin, spacing,
                                 mode=oracle_mod.PAPER, store=store)


def test_euler_fp64_matches_oracle(oracle_mod):
    c1 = synth.hyperbolic_c1()
    seeds = c1["seeds"][::4]
    h = min(c1["spacing"]) / 5
    fg = gpu_field(c1["b"], c1["origin"], c1["spacing"], storage="f64", mode="paper")
    g = gpu_trace(fg, seeds, step_dtype="f64", rtol=1e-6, atol=1e-6, h_init=h, stepper="euler",
                  want_steps=True)
    fo = _oracle_grid(oracle_mod, c1["b"], c1["origin"], c1["spacing"], "f64")
    o = oracle_mod.trace(fo, seeds, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, stepper="euler")
    p = parity(g, o)
    check_lines(p, o, strict=True, max_mismatch_frac=0.0)
    assert p["gate"].sum() == seeds.shape[0]
    # moving half-lines take the oracle's number of steps; a seed on a face
    # with the field pointing out ends at the seed pass (length 0, no step),
    # where the oracle records the one step it cuts at length 0
    for half, lam in ((0, o["lam_fwd"]), (1, o["lam_bwd"])):
        moving = np.abs(lam) > 0
        d = np.abs(g["steps"][half].astype(np.int64) - o["counts"][:, half, 0])[moving]
        assert d.size == 0 or (d.max() <= 1 and (d == 0).mean() >= 0.999), half
        assert np.all(g["steps"][half][~moving] == 0)
    assert (np.abs(o["lam_fwd"]) > 0).all()
    assert np.allclose(g["fll"], o["fll"], rtol=1e-9)


@pytest.mark.parametrize("step_dtype", ["f32", "f64"])
def test_euler_charges_parity(oracle_mod, step_dtype):
    n = (97, 97, 49)
    b = synth.sample_charges(CH, n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    seeds = synth.random_seeds(43, 1000 + 29)
    seeds[:500, 2] = 0.0
    h = min(spacing) / 5
    fg = gpu_field(b, origin, spacing, storage="f32")
    g = gpu_trace(fg, seeds, step_dtype=step_dtype, rtol=1e-6, atol=1e-6, stepper="euler")   # default h
    fo = _oracle_grid(oracle_mod, b, origin, spacing, "f32")
    o = oracle_mod.trace(fo, seeds, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, stepper="euler")
    p = parity(g, o)
    assert p["gate"].mean() > 0.97
    check_lines(p, o, strict=step_dtype == "f64")


def test_euler_straight_lines_exact():
    d = np.array([0.3, -0.5, 0.8])
    n = (33, 33, 17)
    b = synth.sample_linear(*synth.uniform(d), n)
    origin, spacing = synth.grid_geometry(n)
    seeds = synth.rng(6).uniform([-0.9, -0.9, 0.05], [0.9, 0.9, 0.95], (300, 3))
    fg = gpu_field(b, origin, spacing, storage="f64", mode="paper")
    g = gpu_trace(fg, seeds, step_dtype="f64", rtol=1e-6, atol=1e-6, stepper="euler")
    u = d / np.linalg.norm(d)
    lo, hi = np.array(synth.LO), np.array(synth.HI)

    def exit_t(v):
        with np.errstate(divide="ignore"):
            t = np.where(v > 0, (hi - seeds) / v, np.where(v < 0, (lo - seeds) / v, np.inf))
        return t.min(axis=1)
    tf, tb = exit_t(u), exit_t(-u)
    assert np.allclose(g["fp_fwd"], seeds + tf[:, None] * u, rtol=0, atol=1e-11)
    assert np.allclose(g["fp_bwd"], seeds - tb[:, None] * u, rtol=0, atol=1e-11)
    assert np.allclose(g["fll"], tf + tb, rtol=1e-11)
    assert np.allclose(g["q_perp"], 2.0, rtol=1e-10)


def test_euler_batch_matches_single():
    import torch

    import paper_1609_00724_amd as q
    dev = torch.device("cuda:0")
    sets = list(synth.batch_c3(count=5, first_seed=3100, dims=((24, 24, 16), (32, 32, 32), (40, 32, 20)),
                               seeds_range=(20, 900), dtype=np.float32))
    fields = [gpu_field(f["b"], f["origin"], f["spacing"], storage="f32") for f in sets]
    kw = dict(rtol=1e-6, atol=1e-6, step_dtype="f32", stepper="euler", want_steps=True)
    outs = q.trace_batch([(fg, torch.from_numpy(f["seeds"]).to(dev)) for fg, f in zip(fields, sets)], **kw)
    torch.cuda.synchronize()
    for k, (fg, f, ob) in enumerate(zip(fields, sets, outs)):
        os_ = q.trace(fg, torch.from_numpy(f["seeds"]).to(dev), **kw)
        torch.cuda.synchronize()
        for key in ob:
            assert torch.equal(torch.nan_to_num(ob[key], nan=-1.0), torch.nan_to_num(os_[key], nan=-1.0)), (k, key)
