"""Pins of the oracle's map-level steps (QSL Squasher Sect. 3.6): Sobel FLEDGE,
Hilbert ordering, FLL-jump refinement and the array converter."""
import os

import numpy as np
import pytest
from scipy import ndimage

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# FLEDGE: Sobel gradient magnitude
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(7, 9), (16, 16), (5, 6, 7)])
def test_sobel_matches_scipy(oracle_mod, shape):
    f = synth.rng(3).normal(size=shape)
    want = np.sqrt(sum(ndimage.sobel(f, axis=a, mode="reflect") ** 2 for a in range(f.ndim)))
    assert np.allclose(oracle_mod.sobel_magnitude(f), want, atol=1e-12)


def test_sobel_ramp_closed_form(oracle_mod):
    a, b, c = 0.3, -1.7, 0.9
    j, i = np.mgrid[0:12, 0:10]
    s2 = oracle_mod.sobel_magnitude(a * i + b * j)
    assert np.allclose(s2[1:-1, 1:-1], 8 * np.hypot(a, b))
    k, j, i = np.mgrid[0:6, 0:7, 0:8]
    s3 = oracle_mod.sobel_magnitude(a * i + b * j + c * k)
    assert np.allclose(s3[1:-1, 1:-1, 1:-1], 32 * np.sqrt(a * a + b * b + c * c))


def test_sobel_step_profile(oracle_mod):
    f = np.zeros((8, 8))
    f[:, 4:] = 1.0
    s = oracle_mod.sobel_magnitude(f)
    # columns 3 and 4 straddle the step: derivative 1 * (1 + 2 + 1)
    assert np.allclose(s[:, 3], 4.0) and np.allclose(s[:, 4], 4.0)
    assert np.allclose(s[:, :3], 0.0) and np.allclose(s[:, 5:], 0.0)


def test_sobel_brute_force_tiny(oracle_mod):
    f = synth.rng(4).normal(size=(4, 4))
    p = np.pad(f, 1, mode="symmetric")
    gx = np.zeros_like(f)
    gy = np.zeros_like(f)
    for y in range(4):
        for x in range(4):
            w = p[y:y + 3, x:x + 3]
            gx[y, x] = (w[:, 2] - w[:, 0]) @ np.array([1, 2, 1])
            gy[y, x] = (w[2, :] - w[0, :]) @ np.array([1, 2, 1])
    assert np.allclose(oracle_mod.sobel_magnitude(f), np.hypot(gx, gy))


# ---------------------------------------------------------------------------
# Hilbert curve
# ---------------------------------------------------------------------------

def test_hilbert_golden_order2(oracle_mod):
    rows = np.loadtxt(os.path.join(GOLDEN, "hilbert2_order2.txt"), dtype=np.int64)
    x, y = oracle_mod.hilbert2_d2xy(2, rows[:, 0])
    assert np.array_equal(x, rows[:, 1]) and np.array_equal(y, rows[:, 2])


@pytest.mark.parametrize("L", [1, 2, 3, 5, 7])
def test_hilbert_bijection_adjacency_blocks(oracle_mod, L):
    O = oracle_mod
    n = 1 << L
    d = np.arange(n * n, dtype=np.int64)
    x, y = O.hilbert2_d2xy(L, d)
    assert np.unique(y * n + x).size == n * n                     # bijection
    assert np.array_equal(O.hilbert2_xy2d(L, x, y), d)            # inverse
    step = np.abs(np.diff(x)) + np.abs(np.diff(y))
    assert np.all(step == 1)                                      # face-adjacent
    assert (x[0], y[0]) == (0, 0) and (x[-1], y[-1]) == (n - 1, 0)
    for j in range(1, L + 1):                                     # aligned blocks
        bs = 4 ** j
        side = 1 << j
        bx = x.reshape(-1, bs)
        by = y.reshape(-1, bs)
        assert np.all(bx.max(1) - bx.min(1) == side - 1)
        assert np.all(by.max(1) - by.min(1) == side - 1)
        assert np.all(bx.min(1) % side == 0) and np.all(by.min(1) % side == 0)
    # refinement of the curve: the level-(L-1) cell of d is the parent of d's cell
    if L > 1:
        xp, yp = O.hilbert2_d2xy(L - 1, d // 4)
        assert np.array_equal(x // 2, xp) and np.array_equal(y // 2, yp)


# ---------------------------------------------------------------------------
# FLL-jump refinement and the array converter
# ---------------------------------------------------------------------------

PLANE_ARGS = (0.0, -1.0, 1.0, -1.0, 1.0)


def _disc(R=0.5):
    def fn(p):
        inside = (p[:, 0] ** 2 + p[:, 1] ** 2 < R * R).astype(float)
        return {"fll": inside, "q": 2.0 + 100.0 * inside}
    return fn


def test_refine_constant_field_adds_nothing(oracle_mod):
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    keys, vals, passes = O.refine_slice(plane, 4, 2, 0.01,
                                        lambda p: {"fll": np.ones(len(p)), "q": np.full(len(p), 2.0)})
    assert passes == 0 and keys.size == 256
    assert np.array_equal(keys, np.arange(256) * 16 + 8)


def test_refine_disc_clusters_on_the_edge(oracle_mod):
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    m, r, R = 5, 2, 0.5
    keys, vals, passes = O.refine_slice(plane, m, r, 0.5, _disc(R))
    assert np.all(np.diff(keys) > 0)                  # stays in curve order
    assert passes == 4                                # key gap 16 -> 8 -> 4 -> 2 -> 1
    base = keys % 16 == 8
    new = ~base
    assert new.sum() > 0
    pos = O.key_positions(plane, m, r, keys[new])
    fine = 2.0 / (1 << (m + r))
    dist = np.abs(np.hypot(pos[:, 0], pos[:, 1]) - R)
    # every inserted sample lies within one base pixel of the edge
    assert dist.max() < 2.0 / (1 << m) * np.sqrt(2)
    # count scales with the perimeter: doubling the radius ~doubles the insertions
    keys2, _, _ = O.refine_slice(plane, m, r, 0.5, _disc(2 * R * 0.9))
    ratio = (keys2.size - 4 ** m) / (keys.size - 4 ** m)
    assert 1.4 < ratio < 2.6
    # consecutive samples across the edge end up one finest cell apart in key
    fl = vals["fll"]
    jumps = np.nonzero(np.abs(np.diff(fl)) > 0.5)[0]
    assert np.all(keys[jumps + 1] - keys[jumps] == 1)
    assert fine > 0


def test_refine_from_proposals(oracle_mod):
    """Refinement from a merged sample set: (a) proposing the keys the plain
    rule adds reproduces the plain result with no pass; (b) proposing every
    finest cell of every base pixel leaves no gap >= 2 and no pass; (c) a
    partial proposal ends with every proposal kept and no sample the plain
    rule would have been missing near the edge (each jump still ends one
    finest cell apart)."""
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    m, r, R = 5, 2, 0.5
    plain, _, _ = O.refine_slice(plane, m, r, 0.5, _disc(R))
    base = np.arange(4 ** m) * 16 + 8
    extra = np.setdiff1d(plain, base)
    k2, _, p2 = O.refine_slice(plane, m, r, 0.5, _disc(R), extra_keys=extra)
    assert p2 == 0 and np.array_equal(k2, plain)
    allk = np.setdiff1d(np.arange(4 ** (m + r)), base)
    k3, _, p3 = O.refine_slice(plane, m, r, 0.5, _disc(R), extra_keys=allk)
    assert p3 == 0 and np.array_equal(k3, np.arange(4 ** (m + r)))
    g = np.random.Generator(np.random.PCG64(3))
    picked = g.choice(4 ** m, size=100, replace=False)
    prop = np.setdiff1d((picked[:, None] * 16 + np.arange(16)[None, :]).ravel(), base)
    k4, v4, p4 = O.refine_slice(plane, m, r, 0.5, _disc(R), extra_keys=prop)
    assert np.all(np.isin(prop, k4)) and np.all(np.diff(k4) > 0) and p4 <= 4
    fl = v4["fll"]
    jumps = np.nonzero(np.abs(np.diff(fl)) > 0.5)[0]
    assert np.all(k4[jumps + 1] - k4[jumps] == 1)


def test_convert_base_level_is_the_base_map(oracle_mod):
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    m, r = 4, 2
    keys, pts = O.base_samples(plane, m, r)
    v = 2.0 + pts[:, 0] ** 2 + 3 * pts[:, 1]
    grid = O.convert_to_grid(keys, v, m, r, m, log_interp=True)
    n = 1 << m
    c = (np.arange(n) + 0.5) * 2 / n - 1
    want = 2.0 + c[None, :] ** 2 + 3 * c[:, None]
    assert np.allclose(grid, want)


def test_convert_max_and_gap_fill_brute_force(oracle_mod):
    O = oracle_mod
    m, r = 1, 1
    # finest level 2: 16 keys; samples at a few keys
    keys = np.array([1, 2, 3, 9, 14])
    vals = np.array([10.0, 1000.0, 3.0, 100.0, 10.0])
    g = O.convert_to_grid(keys, vals, m, r, 2, log_interp=True)
    x, y = O.hilbert2_d2xy(2, np.arange(16))
    expect = {}
    for k in range(16):
        if k in keys:
            expect[k] = vals[list(keys).index(k)]
        elif k < 1:
            expect[k] = 10.0
        elif k > 14:
            expect[k] = 10.0
        else:
            lo = keys[keys < k].max()
            hi = keys[keys > k].min()
            w = (k - lo) / (hi - lo)
            vlo, vhi = vals[list(keys).index(lo)], vals[list(keys).index(hi)]
            expect[k] = 10 ** ((1 - w) * np.log10(vlo) + w * np.log10(vhi))
    for k in range(16):
        assert g[y[k], x[k]] == pytest.approx(expect[k], rel=1e-12)
    # one level coarser: blocks of 4 keys -> max of their samples
    g1 = O.convert_to_grid(keys, vals, m, r, 1, log_interp=True)
    x1, y1 = O.hilbert2_d2xy(1, np.arange(4))
    assert g1[y1[0], x1[0]] == 1000.0           # keys 1, 2, 3
    assert g1[y1[2], x1[2]] == 100.0            # key 9
    assert g1[y1[3], x1[3]] == 10.0             # key 14
    # block 1 (keys 4..7) is empty: interpolate at its centre key 5.5 between 3 and 9
    w = (5.5 - 3) / 6
    assert g1[y1[1], x1[1]] == pytest.approx(10 ** ((1 - w) * np.log10(3.0) + w * 2.0))


# ---------------------------------------------------------------------------
# volumes: 3D Hilbert curve, refinement and converter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("b", [1, 2, 3, 4, 5])
def test_hilbert3_bijection_adjacency_blocks(oracle_mod, b):
    O = oracle_mod
    n = 1 << b
    d = np.arange(n ** 3, dtype=np.int64)
    x, y, z = O.hilbert3_d2xyz(b, d)
    assert np.unique((z * n + y) * n + x).size == n ** 3
    assert np.array_equal(O.hilbert3_xyz2d(b, x, y, z), d)
    step = np.abs(np.diff(x)) + np.abs(np.diff(y)) + np.abs(np.diff(z))
    assert np.all(step == 1)
    assert (x[0], y[0], z[0]) == (0, 0, 0)
    for j in range(1, b + 1):
        bs, side = 8 ** j, 1 << j
        for c in (x, y, z):
            blk = c.reshape(-1, bs)
            assert np.all(blk.max(1) - blk.min(1) == side - 1)
            assert np.all(blk.min(1) % side == 0)
    if b > 1:   # the level-(b-1) cell of d is the parent of d's cell
        xp, yp, zp = O.hilbert3_d2xyz(b - 1, d // 8)
        assert np.array_equal(x // 2, xp) and np.array_equal(y // 2, yp) and np.array_equal(z // 2, zp)


def test_refine_volume_sphere(oracle_mod):
    O = oracle_mod
    box = O.VolumeBox(-1, 1, -1, 1, 0, 1)
    R = 0.35
    c = np.array([0.1, -0.2, 0.5])

    def fn(p):
        inside = (np.linalg.norm(p - c, axis=1) < R).astype(float)
        return {"fll": inside, "q": 2.0 + 10 * inside}

    m, r = 3, 2
    keys, vals, passes = O.refine_slice(box, m, r, 0.5, fn)
    assert passes == 6                       # key gap 64 halves to 1 in six passes
    assert np.all(np.diff(keys) > 0)
    new = keys % 64 != 32
    assert new.sum() > 0
    pos = O.key_positions(box, m, r, keys[new])
    cell = (box.hi - box.lo) / (1 << m)
    dist = np.abs(np.linalg.norm(pos - c, axis=1) - R)
    assert dist.max() < np.linalg.norm(cell)          # within one base cell of the surface
    jumps = np.nonzero(np.abs(np.diff(vals["fll"])) > 0.5)[0]
    assert np.all(keys[jumps + 1] - keys[jumps] == 1)


def test_convert_volume_brute_force(oracle_mod):
    O = oracle_mod
    m, r = 1, 1
    keys = np.array([3, 4, 20, 40, 41, 63])
    vals = np.array([5.0, 50.0, 2.0, 7.0, 3.0, 9.0])
    g = O.convert_to_grid(keys, vals, m, r, 1, log_interp=True, dims=3)
    x, y, z = O.hilbert3_d2xyz(1, np.arange(8))
    # blocks of 8 finest keys: [0,8) -> 50, [16,24) -> 2, [40,48) -> 7, [56,64) -> 9
    for blk, want in ((0, 50.0), (2, 2.0), (5, 7.0), (7, 9.0)):
        assert g[z[blk], y[blk], x[blk]] == want
    # block 1 ([8,16)) empty: log-interpolated at key 11.5 between keys 4 and 20
    w = (11.5 - 4) / 16
    assert g[z[1], y[1], x[1]] == pytest.approx(10 ** ((1 - w) * np.log10(50) + w * np.log10(2)))


# ---------------------------------------------------------------------------
# shifted-curve re-pass (Sect. 3.6, last paragraph)
# ---------------------------------------------------------------------------

def _quadrant(p):
    """Length 1 in the lower-right quadrant (x > 0, y < 0), 0 elsewhere: its
    edges run along the curve's top-level seams, where spatial neighbours lie
    in the first and last quadrants of the curve, far apart along it."""
    f = ((p[:, 0] > 0) & (p[:, 1] < 0)).astype(float)
    return {"fll": f, "q": 2.0 + f}


def _longest_miss(O, plane, m, r, keys):
    """Longest stretch (in base pixels) along either edge of the quadrant
    (x = 0 for y < -0.1, y = 0 for x > 0.1) with no refined sample within one
    finest cell of the edge."""
    fine, base = 2.0 / (1 << (m + r)), 2.0 / (1 << m)
    pos = O.key_positions(plane, m, r, keys[keys % (1 << (2 * r)) != (1 << (2 * r)) // 2])
    x, y = pos[:, 0], pos[:, 1]
    ys = np.sort(y[(np.abs(x) < fine) & (y < -0.1)])
    xs = np.sort(x[(np.abs(y) < fine) & (x > 0.1)])
    g1 = np.diff(np.concatenate([[-1.0], ys, [-0.1]])).max()
    g2 = np.diff(np.concatenate([[0.1], xs, [1.0]])).max()
    return max(g1, g2) / base


def test_shifted_repass_finds_the_seam_jump(oracle_mod):
    """The jump along the curve's seams: without the re-pass only the one
    curve-successive pair that crosses an edge (where the curve passes from
    the upper-right to the lower-right quadrant) is refined, so the edges are
    missed along nearly their whole length (14 of 14.4 base pixels); the
    re-pass refines both edges with no miss longer than 3 base pixels, and the
    refined set is complete in both orders."""
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    m, r = 5, 2
    plain, _, _ = O.refine_slice(plane, m, r, 0.5, _quadrant)
    keys, vals, cycles = O.refine_shifted(plane, m, r, 0.5, _quadrant, shift=6)
    miss_plain, miss_shift = _longest_miss(O, plane, m, r, plain), _longest_miss(O, plane, m, r, keys)
    print(f"longest miss along the edges: plain {miss_plain:.2f}, shifted re-pass {miss_shift:.2f} base pixels; "
          f"{keys.size} samples, {cycles} cycles")
    assert miss_plain > 10.0 and miss_shift <= 3.0
    assert np.all(np.diff(keys) > 0) and keys.size > plain.size
    _complete_both_orders(O, plane, m, r, keys, vals["fll"], 0.5, 6)


def _complete_both_orders(O, region, m, r, keys, fll, thr, shift):
    """No pair fires along the curve, and every pair that fires along the
    shifted curve has its new cell outside the map."""
    L = m + r
    assert not np.any((np.diff(keys) >= 2) & (np.abs(np.diff(fll)) > thr))
    cells = region.cells(L, keys)
    kp = O._curve_index(region, L + 1, [np.asarray(c) + shift for c in cells])
    o = np.argsort(kp)
    ks, fs = kp[o], fll[o]
    fire = (np.diff(ks) >= 2) & (np.abs(np.diff(fs)) > thr)
    mid = (ks[:-1][fire] + ks[1:][fire]) // 2
    back = [np.asarray(c) - shift for c in region.cells(L + 1, mid)]
    inside = np.ones(mid.size, bool)
    for c in back:
        inside &= (c >= 0) & (c < (1 << L))
    assert not inside.any()


def test_shifted_repass_leaves_a_jump_free_map_alone(oracle_mod):
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    smooth = lambda p: {"fll": 0.01 * p[:, 0] + 0.02 * p[:, 1], "q": np.full(len(p), 2.0)}   # noqa: E731
    keys, _, cycles = O.refine_shifted(plane, 4, 2, 0.05, smooth, shift=6)
    assert cycles == 1 and np.array_equal(keys, np.arange(256) * 16 + 8)


def test_shifted_repass_disc_and_volume(oracle_mod):
    """A disc (no seam-aligned edges): with the re-pass every sample off the
    base lattice still lies within one base pixel of the edge, there are more
    of them, and the set ends complete in both orders; likewise a ball in a
    volume.  (The re-pass's samples split the curve's gaps unevenly, so later
    passes along the curve may pick other midpoints than the plain rule.)"""
    O = oracle_mod
    plane = O.SlicePlane(*PLANE_ARGS)
    m, r, R = 5, 2, 0.5
    plain, _, _ = O.refine_slice(plane, m, r, 0.5, _disc(R))
    keys, vals, cycles = O.refine_shifted(plane, m, r, 0.5, _disc(R), shift=6)
    assert keys.size > plain.size and cycles >= 2
    new = keys[keys % 16 != 8]
    pos = O.key_positions(plane, m, r, new)
    assert np.all(np.abs(np.hypot(pos[:, 0], pos[:, 1]) - R) < 2.0 / (1 << m) * np.sqrt(2))
    _complete_both_orders(O, plane, m, r, keys, vals["fll"], 0.5, 6)
    box = O.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0)
    ball = lambda p: {"fll": (np.sum((p - [0.1, -0.2, 0.45]) ** 2, axis=1) < 0.3 ** 2).astype(float),   # noqa: E731
                      "q": np.full(len(p), 2.0)}
    vk, vv, vc = O.refine_shifted(box, 3, 2, 0.5, ball, shift=3)
    vplain, _, _ = O.refine_slice(box, 3, 2, 0.5, ball)
    assert vk.size > vplain.size
    _complete_both_orders(O, box, 3, 2, vk, vv["fll"], 0.5, 3)


# ---------------------------------------------------------------------------
# planar slices of any orientation (Sect. 2)
# ---------------------------------------------------------------------------

def test_plane_slice_axis_aligned_is_the_horizontal_slice(oracle_mod):
    O = oracle_mod
    a = O.SlicePlane(0.25, -1.0, 0.5, -0.5, 1.0)
    b = O.PlaneSlice((-1.0, -0.5, 0.25), (1.5, 0.0, 0.0), (0.0, 1.5, 0.0))
    d = np.arange(4 ** 5)
    assert np.array_equal(a.centres(5, *a.cells(5, d)), b.centres(5, *b.cells(5, d)))


def test_plane_slice_tilted_through_the_flux_tube(oracle_mod):
    """A refined map on a tilted slice through the analytic flux tube B = (kx,
    -ky, 1): every sample (base and refined) sits on the plane, and its Q is
    the closed form of the line through its position."""
    from test_oracle_trace import K, _hyp_closed, _hyp_qperp
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    F = O.Field.linear(b0, M, synth.LO, synth.HI)
    corner = np.array([-0.3, -0.35, 0.2])
    u = np.array([0.6, 0.1, 0.3])
    v = np.array([-0.1, 0.7, 0.25])
    plane = O.PlaneSlice(corner, u, v)
    m, r = 3, 2
    got = {}

    def fn(p):
        t = O.trace(F, p, rtol=1e-11, atol=1e-11, h_init=1e-3, h_max=0.02)
        for row, f, q in zip(p, t["fll"], t["q_perp"]):
            got[tuple(row)] = q
        return {"fll": t["fll"], "q": t["q_perp"]}

    keys, vals, _ = O.refine_slice(plane, m, r, 0.05, fn)
    assert keys.size > 4 ** m
    normal = np.cross(u, v)
    pts = np.array(list(got))
    assert np.abs((pts - corner) @ normal).max() < 1e-12
    for p, q in list(got.items())[::7]:
        c = _hyp_closed(*p)
        assert abs(q / _hyp_qperp(c["xb"], c["zf"], c["zb"]) - 1) < 1e-7
