"""GPU parity of the general geometry (Sect. 3.1-3.2) against the oracle on the
same gridded data: spherical grids (eq. 2, deviations eq. 6-8) and rectilinear
Cartesian grids (cells with spans of their own); FP64 stepping within the
per-line gates, FP32 stepping within the statistical gates, the monopole's
radial lines and the flux tube's closed forms, a spherical slice map, and the
unsupported combinations."""
import numpy as np
import pytest

import synth
from gpu_util import check_fp32, check_lines, gpu_trace, parity, sensitivity_floor, torch_dev

pytestmark = pytest.mark.gpu

WLO, WHI = (-0.3, -0.3, 1.0), (0.3, 0.3, 1.5)
DIPOLE = np.array([[0.90, 0.06, 0.02, 1.0], [0.91, -0.07, -0.03, -1.0]])


def _gfield(b, origin, spacing, storage="f64", mode="paper", geometry="cartesian", coords=None):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    bt = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in b]
    ct = None if coords is None else [None if c is None else torch.from_numpy(np.asarray(c, np.float64)).to(dev)
                                      for c in coords]
    return q.field_init(*bt, origin, spacing, storage=storage, mode=mode, geometry=geometry, coords=ct)


def _ofield(O, b, origin, spacing, store="f64", mode="paper", geometry="cartesian", coords=None):
    return O.Field.grid(*(np.asarray(c, np.float64) for c in b), origin, spacing,
                        mode=O.PAPER if mode == "paper" else O.INTERP_NORMALIZE, store=store,
                        geometry=geometry, coords=coords)


def _wedge_seeds(seed, n, bottom=True):
    g = synth.rng(seed)
    lo, hi = np.array(WLO), np.array(WHI)
    s = g.uniform(lo + 0.02 * (hi - lo), hi - 0.02 * (hi - lo), size=(n, 3))
    if bottom:
        s[: n // 2, 2] = WLO[2]
    return s


@pytest.fixture(scope="module")
def sph():
    b, origin, spacing = synth.sample_charges_spherical(DIPOLE, (41, 41, 33), WLO, WHI)
    return dict(b=b, origin=origin, spacing=spacing)


@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_spherical_fp64_parity(oracle_mod, sph, mode):
    seeds = _wedge_seeds(1, 500 + 11)
    h = 0.5 * min(sph["spacing"][2], 1.0 * sph["spacing"][0])
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    g = gpu_trace(_gfield(sph["b"], sph["origin"], sph["spacing"], "f64", mode, "spherical"), seeds,
                  step_dtype="f64", **kw)
    o = oracle_mod.trace(_ofield(oracle_mod, sph["b"], sph["origin"], sph["spacing"], "f64", mode, "spherical"),
                         seeds, **kw)
    p = parity(g, o)
    assert p["gate"].mean() > 0.95
    check_lines(p, o, strict=True)


def test_spherical_fp32_parity(oracle_mod, sph):
    seeds = _wedge_seeds(2, 500 + 11)
    h = 0.5 * sph["spacing"][2]
    kw = dict(rtol=1e-4, atol=1e-4, h_init=0.1 * h, h_max=h)
    g = gpu_trace(_gfield(sph["b"], sph["origin"], sph["spacing"], "f32", "paper", "spherical"), seeds,
                  step_dtype="f32", **kw)
    fo = _ofield(oracle_mod, sph["b"], sph["origin"], sph["spacing"], "f32", "paper", "spherical")
    o = oracle_mod.trace(fo, seeds, **kw)
    ref = oracle_mod.trace(fo, seeds, **dict(kw, rtol=1e-10, atol=1e-10))
    check_fp32(parity(g, o), g, o, ref, min_frac=sensitivity_floor(oracle_mod, fo, seeds, o, kw)[0])


def test_spherical_monopole_radial(oracle_mod):
    n = 17
    rr = np.linspace(WLO[2], WHI[2], n)
    br = np.ascontiguousarray(np.broadcast_to(1.0 / rr[:, None, None] ** 2, (n, n, n)))
    z = np.zeros_like(br)
    origin = WLO
    spacing = tuple((WHI[d] - WLO[d]) / (n - 1) for d in range(3))
    seeds = _wedge_seeds(3, 200, bottom=False)
    kw = dict(rtol=1e-10, atol=1e-10, h_init=1e-3, h_max=0.01)
    g = gpu_trace(_gfield((z, z, br), origin, spacing, "f64", "interp_normalize", "spherical"), seeds,
                  step_dtype="f64", **kw)
    assert np.all(g["status"] & 0xFFFF == (5 | (4 << 8)))
    assert np.abs(g["fp_fwd"][:, :2] - seeds[:, :2]).max() < 1e-12
    assert np.abs(g["fp_bwd"][:, 2] - 1.0).max() < 1e-12 and np.abs(g["fp_fwd"][:, 2] - 1.5).max() < 1e-12
    assert np.allclose(g["fll"], 0.5, atol=1e-10)
    o = oracle_mod.trace(_ofield(oracle_mod, (z, z, br), origin, spacing, "f64", "interp_normalize", "spherical"),
                         seeds, **kw)
    assert np.allclose(g["q_perp"], o["q_perp"], rtol=1e-9) and np.all(np.abs(g["q_perp"] - 2) < 0.02)


def _stretched(n, lo, hi, beta):
    u = np.linspace(-1, 1, n)
    v = np.tanh(beta * u) / np.tanh(beta)
    return lo + (hi - lo) * (v + 1) / 2


def _rect_charges():
    xs = _stretched(57, -1.0, 1.0, 1.3)
    ys = _stretched(49, -1.0, 1.0, 0.9)
    zs = np.geomspace(1.0, 2.0, 29) - 1.0
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    B = [np.zeros_like(X) for _ in range(3)]
    for cx, cy, cz, q in synth.point_charges(2, 4):
        dx, dy, dz = X - cx, Y - cy, Z - cz
        inv3 = q / (dx * dx + dy * dy + dz * dz) ** 1.5
        B[0] += dx * inv3
        B[1] += dy * inv3
        B[2] += dz * inv3
    origin = (xs[0], ys[0], zs[0])
    spacing = tuple((c[-1] - c[0]) / (c.size - 1) for c in (xs, ys, zs))
    return B, origin, spacing, (xs, ys, zs)


@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_rectilinear_fp64_parity(oracle_mod, mode):
    B, origin, spacing, coords = _rect_charges()
    seeds = synth.random_seeds(4, 600 + 7)
    seeds[:300, 2] = 0.0
    h = 0.02
    kw = dict(rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    g = gpu_trace(_gfield(B, origin, spacing, "f64", mode, coords=coords), seeds, step_dtype="f64", **kw)
    o = oracle_mod.trace(_ofield(oracle_mod, B, origin, spacing, "f64", mode, coords=coords), seeds, **kw)
    p = parity(g, o)
    assert p["gate"].mean() > 0.95
    check_lines(p, o, strict=True)


def test_rectilinear_flux_tube_closed_form(oracle_mod):
    """B = (2x, -2y, 1) on a stretched grid, interpolate-then-normalise: the
    top exits carry Q_fp = 2 cosh 4."""
    xs = _stretched(33, -1.0, 1.0, 1.5)
    ys = _stretched(33, -1.0, 1.0, 1.1)
    zs = np.geomspace(1.0, 2.0, 25) - 1.0
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    B = [2.0 * X, -2.0 * Y, np.ones_like(X)]
    origin = (xs[0], ys[0], zs[0])
    spacing = tuple((c[-1] - c[0]) / (c.size - 1) for c in (xs, ys, zs))
    seeds = synth.pixel_seeds(128, 128)[::23]
    kw = dict(rtol=1e-9, atol=1e-9, h_init=1e-3, h_max=0.02)
    g = gpu_trace(_gfield(B, origin, spacing, "f64", "interp_normalize", coords=(xs, ys, zs)), seeds,
                  step_dtype="f64", **kw)
    top = (g["status"] & 0xFF) == 5
    assert top.sum() > 10
    assert np.allclose(g["q_fp"][top], 2 * np.cosh(4.0), rtol=1e-6)


def test_spherical_slice_map(oracle_mod, sph):
    """A refined map of the slice r = 1 over the wedge's longitudes and
    latitudes (a spherical slice): every sample's length against the oracle
    traced at its position."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec
    torch, dev = torch_dev()
    fg = _gfield(sph["b"], sph["origin"], sph["spacing"], "f64", "paper", "spherical")
    h = 0.5 * sph["spacing"][2]
    m, r = 5, 2
    res = q.qmap(fg, MapSpec(WLO[2], WLO[0], WHI[0], WLO[1], WHI[1], m, r, m, 0.02, 1), 4 ** (m + r),
                 rtol=1e-7, atol=1e-7, h_init=0.1 * h, h_max=h, step_dtype="f64")
    torch.cuda.synchronize()
    n = res["count"]
    assert n > 4 ** m and res["overflow"] == 0
    keys = res["keys"].cpu().numpy()
    plane = oracle_mod.SlicePlane(WLO[2], WLO[0], WHI[0], WLO[1], WHI[1])
    blk = 4 ** r
    base = keys % blk == blk // 2
    pos = np.empty((n, 3))
    pos[base] = plane.centres(m, *plane.cells(m, keys[base] // blk))
    pos[~base] = oracle_mod.key_positions(plane, m, r, keys[~base])
    o = oracle_mod.trace(_ofield(oracle_mod, sph["b"], sph["origin"], sph["spacing"], "f64", "paper", "spherical"),
                         pos, rtol=1e-7, atol=1e-7, h_init=0.1 * h, h_max=h)
    gg = dict(status=res["status"].cpu().numpy(), q_perp=res["q_perp"].cpu().numpy(), fll=res["fll"].cpu().numpy(),
              fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))
    check_lines(parity(gg, dict(o, fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))), o, strict=True)


def test_unsupported_combinations(sph):
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import trace_batch
    _, dev = torch_dev()
    seeds = torch.from_numpy(_wedge_seeds(5, 64)).to(dev)
    fg = _gfield(sph["b"], sph["origin"], sph["spacing"], "f32", "paper", "spherical")
    with pytest.raises(A.QsqError, match="CK54"):
        q.trace(fg, seeds, rtol=1e-4, atol=1e-4, h_init=1e-3, stepper="euler")
    with pytest.raises(A.QsqError):
        trace_batch([(fg, seeds)], rtol=1e-4, atol=1e-4)
    fb = _gfield(sph["b"], sph["origin"], sph["spacing"], "bf16", "paper", "spherical")
    with pytest.raises(A.QsqError, match="FP32 or FP64"):
        q.trace(fb, seeds, rtol=1e-4, atol=1e-4)
    fc = _gfield(sph["b"], sph["origin"], sph["spacing"], "f32", "paper", "spherical")
    fc.desc.order = A.ORDER_CUBIC
    with pytest.raises(A.QsqError, match="trilinear"):
        q.trace(fc, seeds, rtol=1e-4, atol=1e-4)
    torch.cuda.synchronize()


def test_tilted_slice_map(oracle_mod):
    """A refined map on a planar slice of any orientation (Sect. 2) through
    the flux tube B = (2x, -2y, 1) on a 48^3 grid, interpolate-then-normalise,
    FP64 stepping: the oracle's refinement on a PlaneSlice, replayed on the
    GPU's samples, asks for exactly the GPU's keys, and every sample's Q is
    the closed form of the line through its position."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec
    from test_oracle_trace import _hyp_closed, _hyp_qperp
    torch, dev = torch_dev()
    w = synth.hyperbolic_c1(n=(48, 48, 48))
    fg = _gfield(w["b"], w["origin"], w["spacing"], "f64", "interp_normalize")
    corner, eu, ev = (-0.3, -0.35, 0.2), (0.6, 0.1, 0.3), (-0.1, 0.7, 0.25)
    m, r, thr = 5, 2, 0.05
    h = min(w["spacing"])
    spec = MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, thr, 1, plane=(corner, eu, ev))
    res = q.qmap(fg, spec, 4 ** (m + r), rtol=1e-10, atol=1e-10, h_init=0.1 * h, h_max=h, step_dtype="f64")
    torch.cuda.synchronize()
    n = res["count"]
    assert n > 4 ** m and res["overflow"] == 0
    keys = res["keys"].cpu().numpy()
    fll = res["fll"].cpu().numpy()
    qg = res["q_perp"].cpu().numpy()
    plane = oracle_mod.PlaneSlice(corner, eu, ev)
    lookup = {int(k): i for i, k in enumerate(keys)}
    missing, calls = [], []

    def from_gpu(pts):
        if not calls:
            ks = oracle_mod.base_samples(plane, m, r)[0]
        else:
            # key of a finest-cell centre: solve corner + s eu + t ev = p
            A = np.array([eu, ev]).T
            st = np.linalg.lstsq(A, (pts - np.array(corner)).T, rcond=None)[0].T
            cells = np.floor(st * (1 << (m + r))).astype(np.int64)
            ks = oracle_mod.hilbert2_xy2d(m + r, cells[:, 0], cells[:, 1])
        calls.append(len(ks))
        idx = np.array([lookup.get(int(k), -1) for k in ks])
        missing.extend(int(k) for k in ks[idx < 0])
        idx = np.maximum(idx, 0)
        return {"fll": fll[idx], "q": qg[idx]}

    rk, _, _ = oracle_mod.refine_slice(plane, m, r, thr, from_gpu)
    assert not missing and np.array_equal(rk, keys)
    blk = 4 ** r
    base = keys % blk == blk // 2
    pos = np.empty((n, 3))
    pos[base] = plane.centres(m, *plane.cells(m, keys[base] // blk))
    pos[~base] = oracle_mod.key_positions(plane, m, r, keys[~base])
    for i in range(0, n, 5):
        c = _hyp_closed(*pos[i])
        assert abs(qg[i] / _hyp_qperp(c["xb"], c["zf"], c["zb"]) - 1) < 1e-6, i
