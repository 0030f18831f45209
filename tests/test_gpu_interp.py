"""GPU parity of the triquadratic and tricubic interpolation orders (Sect. 3.2,
eq. 3; analytic gradients, Sect. 3.3) against the oracle at the same order:
FP64 stepping line by line within the per-line gates, FP32 stepping within
the statistical FP32 gates, the hyperbolic flux tube's closed forms on the
grid, a refined map, and the argument checks."""
import numpy as np
import pytest

import synth
from gpu_util import check_fp32, check_lines, gpu_trace, parity, sensitivity_floor, torch_dev

pytestmark = pytest.mark.gpu

CH = synth.point_charges(2, 4)
ORDER = {2: "quadratic", 3: "cubic"}


def _field(b, origin, spacing, storage, mode, order):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    bt = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in b]
    return q.field_init(*bt, origin, spacing, storage=storage, mode=mode, order=ORDER[order])


def _oracle(oracle_mod, b, origin, spacing, mode, store, order):
    return oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in b), origin, spacing,
                                 mode=oracle_mod.PAPER if mode == "paper" else oracle_mod.INTERP_NORMALIZE,
                                 store=store, order=order)


@pytest.fixture(scope="module")
def charges():
    n = (65, 65, 33)
    b = synth.sample_charges(CH, n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    return dict(b=b, origin=origin, spacing=spacing)


def _seeds(count, seed):
    s = synth.random_seeds(seed, count)
    s[: count // 2, 2] = 0.0
    return s


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_fp64_parity(oracle_mod, charges, order, mode):
    c = charges
    seeds = _seeds(700 + 13, 51)
    h = min(c["spacing"])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    fg = _field(c["b"], c["origin"], c["spacing"], "f64", mode, order)
    g = gpu_trace(fg, seeds, step_dtype="f64", **kw)
    o = oracle_mod.trace(_oracle(oracle_mod, c["b"], c["origin"], c["spacing"], mode, "f64", order), seeds, **kw)
    p = parity(g, o)
    assert p["gate"].mean() > 0.97
    check_lines(p, o, strict=True)
    # the determinant form of Q within the same per-line Q gate (the GPU's
    # separable stencil sums round differently from the oracle's triple sum)
    both = np.isfinite(o["q_det"]) & (g["status"] == o["status"]) & (o["q_det"] < 1e6)
    lq = np.abs(np.log10(g["q_det"][both]) - np.log10(o["q_det"][both])) / np.log10(o["q_det"][both])
    assert lq.max() <= 1e-3


@pytest.mark.parametrize("order", [2, 3])
def test_fp32_parity(oracle_mod, charges, order):
    c = charges
    seeds = _seeds(700 + 13, 52)
    h = min(c["spacing"])
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    fg = _field(c["b"], c["origin"], c["spacing"], "f32", "paper", order)
    g = gpu_trace(fg, seeds, step_dtype="f32", **kw)
    fo = _oracle(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32", order)
    o = oracle_mod.trace(fo, seeds, **kw)
    ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
    check_fp32(parity(g, o), g, o, ref, min_frac=sensitivity_floor(oracle_mod, fo, seeds, o, kw)[0])


@pytest.mark.parametrize("order", [2, 3])
def test_hyperbolic_closed_form(oracle_mod, order):
    """B = (2x, -2y, 1) is reproduced exactly at every order when B is
    interpolated and then normalised: the top exits carry Q_fp = 2 cosh 4."""
    w = synth.hyperbolic_c1(n=(32, 32, 32))
    h = min(w["spacing"])
    kw = dict(rtol=1e-9, atol=1e-9, h_init=0.1 * h, h_max=h)
    seeds = w["seeds"][::7]
    fg = _field(w["b"], w["origin"], w["spacing"], "f64", "interp_normalize", order)
    g = gpu_trace(fg, seeds, step_dtype="f64", **kw)
    top = (g["status"] & 0xFF) == 5
    assert top.sum() > 50
    assert np.allclose(g["q_fp"][top], 2 * np.cosh(4.0), rtol=1e-6)
    o = oracle_mod.trace(_oracle(oracle_mod, w["b"], w["origin"], w["spacing"], "interp_normalize", "f64", order),
                         seeds, **kw)
    check_lines(parity(g, o), o, strict=True, max_mismatch_frac=0.0)


def test_cubic_map_vs_oracle(oracle_mod, charges):
    """A refined photospheric map with tricubic interpolation and FP64
    stepping: every sample's length and Q against the oracle traced at its
    position with the same kernel."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec
    torch, dev = torch_dev()
    c = charges
    h = min(c["spacing"])
    fg = _field(c["b"], c["origin"], c["spacing"], "f32", "paper", 3)
    m, r, thr = 5, 2, 0.02
    res = q.qmap(fg, MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, thr, 1), 4 ** (m + r), rtol=1e-7, atol=1e-7,
                 h_init=0.1 * h, h_max=h, step_dtype="f64")
    torch.cuda.synchronize()
    n = res["count"]
    assert n > 4 ** m and res["overflow"] == 0
    keys = res["keys"].cpu().numpy()
    plane = oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)
    blk = 4 ** r
    base = keys % blk == blk // 2
    pos = np.empty((n, 3))
    pos[base] = plane.centres(m, *plane.cells(m, keys[base] // blk))
    pos[~base] = oracle_mod.key_positions(plane, m, r, keys[~base])
    o = oracle_mod.trace(_oracle(oracle_mod, c["b"], c["origin"], c["spacing"], "paper", "f32", 3), pos,
                         rtol=1e-7, atol=1e-7, h_init=0.1 * h, h_max=h)
    gg = dict(status=res["status"].cpu().numpy(), q_perp=res["q_perp"].cpu().numpy(), fll=res["fll"].cpu().numpy(),
              fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))
    check_lines(parity(gg, dict(o, fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))), o, strict=True)


def test_unsupported_combinations(charges):
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import trace_batch
    _, dev = torch_dev()
    c = charges
    seeds = torch.from_numpy(_seeds(64, 3)).to(dev)
    fb = _field(c["b"], c["origin"], c["spacing"], "bf16", "paper", 3)
    with pytest.raises(A.QsqError, match="FP32 or FP64"):
        q.trace(fb, seeds, rtol=1e-4, atol=1e-4)
    small = synth.sample_charges(CH, (3, 9, 9), dtype=np.float32)
    o, s = synth.grid_geometry((3, 9, 9))
    with pytest.raises(A.QsqError, match="4 nodes"):
        q.trace(_field(small, o, s, "f32", "paper", 2), seeds, rtol=1e-4, atol=1e-4)
    f3 = _field(c["b"], c["origin"], c["spacing"], "f32", "paper", 3)
    with pytest.raises(A.QsqError):
        trace_batch([(f3, seeds)], rtol=1e-4, atol=1e-4)
    torch.cuda.synchronize()
