"""Pins of the FP64 oracle's tracer and Q assembly against what the paper and the
mathematics fix (closed forms, invariants, independent integrators).

Paper: Tassev & Savcheva 2017, Sect. 3.1-3.5 (eq. 1, 3-5, 9-11), Cash-Karp RK5(4).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synth

LO = np.array(synth.LO)
HI = np.array(synth.HI)


def _opts(tol, hmax, **kw):
    d = dict(rtol=tol, atol=tol, h_init=0.1 * hmax, h_max=hmax)
    d.update(kw)
    return d


def _fwd(st):
    return st & 0xFF


def _bwd(st):
    return (st >> 8) & 0xFF


# ---------------------------------------------------------------------------
# Cash-Karp tableau: Butcher order conditions (Sect. 3.4)
# ---------------------------------------------------------------------------

def test_ck54_order_conditions(oracle_mod):
    c, a, b5, b4 = oracle_mod.ck54_tableau()
    A = np.zeros((6, 6))
    A[:, :5] = a
    # consistency: row sums equal the nodes
    assert np.allclose(A.sum(1), c, atol=1e-15)

    def conds(b):
        e = np.ones(6)
        Ac = A @ c
        return {
            "1": (b @ e, 1.0),
            "2": (b @ c, 1 / 2),
            "3a": (b @ c**2, 1 / 3), "3b": (b @ Ac, 1 / 6),
            "4a": (b @ c**3, 1 / 4), "4b": (b @ (c * Ac), 1 / 8),
            "4c": (b @ (A @ c**2), 1 / 12), "4d": (b @ (A @ Ac), 1 / 24),
            "5a": (b @ c**4, 1 / 5), "5b": (b @ (c**2 * Ac), 1 / 10),
            "5c": (b @ (c * (A @ c**2)), 1 / 15), "5d": (b @ (c * (A @ Ac)), 1 / 30),
            "5e": (b @ (Ac * Ac), 1 / 20), "5f": (b @ (A @ c**3), 1 / 20),
            "5g": (b @ (A @ (c * Ac)), 1 / 40), "5h": (b @ (A @ (A @ c**2)), 1 / 60),
            "5i": (b @ (A @ (A @ Ac)), 1 / 120),
        }

    for k, (v, want) in conds(b5).items():
        assert abs(v - want) < 1e-14, ("b5", k, v, want)
    c4 = conds(b4)
    for k, (v, want) in c4.items():
        if k[0] in "1234":
            assert abs(v - want) < 1e-14, ("b4", k, v, want)
    # the embedded solution is genuinely only 4th order
    assert max(abs(v - w) for k, (v, w) in c4.items() if k[0] == "5") > 1e-4


# ---------------------------------------------------------------------------
# uniform field: straight lines, Q = 2
# ---------------------------------------------------------------------------

def _ray_exit(p, d):
    """distance and face index where the ray p + t d leaves the box."""
    best, face = np.inf, -1
    for ax in range(3):
        if d[ax] > 0:
            t, f = (HI[ax] - p[ax]) / d[ax], 2 * ax + 1
        elif d[ax] < 0:
            t, f = (LO[ax] - p[ax]) / d[ax], 2 * ax
        else:
            continue
        if t < best:
            best, face = t, f
    return best, face


@pytest.mark.parametrize("mode", ["analytic", "paper", "interp_normalize"])
def test_uniform_field_exact(oracle_mod, mode):
    O = oracle_mod
    dirs = [np.array([0.3, -0.5, 0.8]), np.array([-0.9, 0.2, 0.1]), np.array([0.0, 0.0, 1.0])]
    seeds = synth.random_seeds(11, 40)
    n = (9, 9, 5)
    for d in dirs:
        b0, M = synth.uniform(2.5 * d)
        if mode == "analytic":
            F = O.Field.linear(b0, M, synth.LO, synth.HI)
        else:
            bx, by, bz = synth.sample_linear(b0, M, n)
            origin, spacing = synth.grid_geometry(n)
            F = O.Field.grid(bx, by, bz, origin, spacing,
                             mode=O.PAPER if mode == "paper" else O.INTERP_NORMALIZE)
        r = O.trace(F, seeds, **_opts(1e-10, 0.1))
        u = d / np.linalg.norm(d)
        for i, p in enumerate(seeds):
            tf, ff = _ray_exit(p, u)
            tb, fb = _ray_exit(p, -u)
            assert _fwd(r["status"][i]) == ff and _bwd(r["status"][i]) == fb
            assert np.allclose(r["fp_fwd"][i], p + tf * u, atol=1e-11)
            assert np.allclose(r["fp_bwd"][i], p - tb * u, atol=1e-11)
            assert abs(r["fll"][i] - (tf + tb)) < 1e-11
            assert abs(r["q_perp"][i] - 2.0) < 1e-9
            assert abs(r["q_det"][i] - 2.0) < 1e-9
            if ff // 2 == fb // 2:          # parallel exit planes: a pure translation
                assert abs(r["q_fp"][i] - 2.0) < 1e-9


# ---------------------------------------------------------------------------
# hyperbolic flux tube B = (k x, -k y, 1): closed forms
# ---------------------------------------------------------------------------

K = 2.0


def _hyp_closed(x0, y0, z0, k=K):
    """Footpoints, lengths and exit faces of the line through (x0, y0, z0).

    x = x0 e^{k(z-z0)}, y = y0 e^{-k(z-z0)}; dl = sqrt(1 + |d(x,y)/dz|^2) dz.
    """
    # forward (z increasing): |x| grows
    zf = 1.0
    ff = 5
    if x0 != 0 and abs(x0) * np.exp(k * (1 - z0)) > 1:
        zf = z0 + np.log(1 / abs(x0)) / k
        ff = 1 if x0 > 0 else 0
    # backward (z decreasing): |y| grows
    zb = 0.0
    fb = 4
    if y0 != 0 and abs(y0) * np.exp(k * z0) > 1:
        zb = z0 - np.log(1 / abs(y0)) / k
        fb = 3 if y0 > 0 else 2

    def pos(z):
        return np.array([x0 * np.exp(k * (z - z0)), y0 * np.exp(-k * (z - z0)), z])

    def length(za, zb_):
        t, w = np.polynomial.legendre.leggauss(80)
        z = 0.5 * (zb_ - za) * t + 0.5 * (zb_ + za)
        f = np.sqrt(1 + (k * x0 * np.exp(k * (z - z0)))**2 + (k * y0 * np.exp(-k * (z - z0)))**2)
        return 0.5 * (zb_ - za) * (w @ f)

    return dict(xf=pos(zf), xb=pos(zb), lf=length(z0, zf), lb=length(zb, z0), ff=ff, fb=fb, zf=zf, zb=zb)


def _hyp_qperp(xb, zf, zb, k=K):
    """Perpendicular-plane Q between the ends (derived from the horizontal-plane
    map diag(e^{k D}, e^{-k D}) and the projections along B at both ends)."""
    D = zf - zb
    gx, gy = k * xb[0], -k * xb[1]
    r = gx * gx + gy * gy
    s = np.exp(2 * k * D) * gx**2 + np.exp(-2 * k * D) * gy**2
    t = np.exp(4 * k * D) * gx**2 + np.exp(-4 * k * D) * gy**2
    return np.sqrt((1 + s) / (1 + r)) * (2 * np.cosh(2 * k * D) + (s - t) / (1 + s))


def _hyp_seed_set():
    s = synth.pixel_seeds(128, 128)
    return s[::97]


def _check_hyperbolic(O, r, seeds, tol_fp, tol_q, tol_l):
    nside = 0
    for i, p in enumerate(seeds):
        c = _hyp_closed(*p)
        st = r["status"][i]
        assert _fwd(st) == c["ff"] and _bwd(st) == c["fb"], (p, st)
        assert np.abs(r["fp_fwd"][i] - c["xf"]).max() < tol_fp
        assert np.abs(r["fp_bwd"][i] - c["xb"]).max() < tol_fp
        assert abs(r["fll"][i] - (c["lf"] + c["lb"])) < tol_l * (c["lf"] + c["lb"]) + 1e-14
        qperp = _hyp_qperp(c["xb"], c["zf"], c["zb"])
        assert abs(r["q_perp"][i] / qperp - 1) < tol_q, (p, r["q_perp"][i], qperp)
        if c["ff"] == 5:
            qfp = 2 * np.cosh(2 * K * (c["zf"] - c["zb"]))
        else:
            nside += 1
            qfp = K * (p[0]**2 + p[1]**2) + 1 / (K * p[0]**2)
        assert abs(r["q_fp"][i] / qfp - 1) < tol_q, (p, r["q_fp"][i], qfp)
    return nside


def test_hyperbolic_analytic_closed_forms(oracle_mod):
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    F = O.Field.linear(b0, M, synth.LO, synth.HI)
    seeds = _hyp_seed_set()
    r = O.trace(F, seeds, **_opts(1e-11, 1 / 63))
    nside = _check_hyperbolic(O, r, seeds, 1e-9, 1e-8, 1e-9)
    assert 0 < nside < len(seeds)       # both top and side exits are exercised
    # the top-exit value 2 cosh(2k) of the configuration
    top = _fwd(r["status"]) == 5
    assert np.allclose(r["q_fp"][top], 2 * np.cosh(4.0), rtol=1e-8)


@pytest.mark.parametrize("n", [32, 64])
def test_hyperbolic_interp_normalize_grid_exact(oracle_mod, n):
    """Trilinear interpolation reproduces a linear B exactly, so interpolating B
    and then normalising meets the closed forms on any grid."""
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    grid = (n, n, n)
    bx, by, bz = synth.sample_linear(b0, M, grid)
    origin, spacing = synth.grid_geometry(grid)
    F = O.Field.grid(bx, by, bz, origin, spacing, mode=O.INTERP_NORMALIZE)
    seeds = _hyp_seed_set()[::2]
    r = O.trace(F, seeds, **_opts(1e-11, min(spacing)))
    _check_hyperbolic(O, r, seeds, 1e-8, 1e-7, 1e-8)


def test_hyperbolic_interior_seeds(oracle_mod):
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    F = O.Field.linear(b0, M, synth.LO, synth.HI)
    seeds = synth.random_seeds(5, 30)
    r = O.trace(F, seeds, **_opts(1e-11, 1 / 63))
    for i, p in enumerate(seeds):
        c = _hyp_closed(*p)
        assert np.abs(r["fp_fwd"][i] - c["xf"]).max() < 1e-9
        assert np.abs(r["fp_bwd"][i] - c["xb"]).max() < 1e-9
        assert abs(r["lam_fwd"][i] - c["lf"]) < 1e-9
        assert abs(r["lam_bwd"][i] + c["lb"]) < 1e-9
        q = _hyp_qperp(c["xb"], c["zf"], c["zb"])
        assert abs(r["q_perp"][i] / q - 1) < 1e-8


def test_paper_mode_second_order_convergence(oracle_mod):
    """Normalise-then-interpolate (Sect. 3.5 footnote) is a second-order
    approximation of the field direction: footpoint errors fall ~4x per halving."""
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    seeds = _hyp_seed_set()[::3]
    errs = []
    for n in (17, 33, 65):
        grid = (n, n, n)
        bx, by, bz = synth.sample_linear(b0, M, grid)
        origin, spacing = synth.grid_geometry(grid)
        F = O.Field.grid(bx, by, bz, origin, spacing, mode=O.PAPER)
        r = O.trace(F, seeds, **_opts(1e-10, min(spacing)))
        e = []
        for i, p in enumerate(seeds):
            c = _hyp_closed(*p)
            if _fwd(r["status"][i]) != c["ff"]:
                continue
            e.append(np.abs(r["fp_fwd"][i] - c["xf"]).max())
        errs.append(np.sqrt(np.mean(np.square(e))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.8) & (orders < 2.2)), (errs, orders)


# ---------------------------------------------------------------------------
# point-charge fields: an independent integrator and finite-difference Q
# ---------------------------------------------------------------------------

CHARGES = synth.point_charges(2, 4)


def _charges_B(x):
    B = np.zeros(3)
    for cx, cy, cz, q in CHARGES:
        d = x - np.array([cx, cy, cz])
        B += q * d / np.linalg.norm(d) ** 3
    return B


def _scipy_footpoint(p, sign):
    def f(s, x):
        B = _charges_B(x)
        return sign * B / np.linalg.norm(B)

    events = []
    for ax in range(3):
        for bound, direction in ((LO[ax], -1), (HI[ax], +1)):
            def ev(s, x, ax=ax, bound=bound):
                return x[ax] - bound
            ev.terminal = True
            ev.direction = direction      # only leaving the box counts
            events.append(ev)
    sol = solve_ivp(f, (0, 20), p, method="DOP853", rtol=1e-12, atol=1e-13, events=events)
    assert sol.status == 1
    return sol.y[:, -1], sol.t[-1]


def _charge_seeds():
    g = synth.rng(21)
    out = []
    for cx, cy, cz, q in CHARGES:
        if q > 0:
            for _ in range(4):
                rr, th = 0.06 + 0.1 * g.uniform(), 2 * np.pi * g.uniform()
                out.append([cx + rr * np.cos(th), cy + rr * np.sin(th), 0.0])
    return np.array(out)


def test_charges_footpoints_vs_dop853(oracle_mod):
    """Footpoints and lengths agree with SciPy's DOP853 on the analytic field."""
    O = oracle_mod
    F = O.Field.charges(CHARGES, synth.LO, synth.HI)
    seeds = _charge_seeds()
    r = O.trace(F, seeds, **_opts(1e-12, 0.01))
    for i, p in enumerate(seeds):
        xf, lf = _scipy_footpoint(p, +1.0)
        assert np.abs(r["fp_fwd"][i] - xf).max() < 1e-8, (p, r["fp_fwd"][i], xf)
        assert abs(r["lam_fwd"][i] - lf) < 1e-8
        assert _bwd(r["status"][i]) == 4 and r["lam_bwd"][i] == 0.0


def _face_axes(face):
    ax = face // 2
    return [a for a in range(3) if a != ax]


def test_linearised_q_vs_finite_differences(oracle_mod):
    """Q from the linearised deviation equation (eq. 5) equals Q from finite
    differences of neighbouring lines' footpoints (the method it replaces,
    Sect. 3.3), both in the footpoint planes."""
    O = oracle_mod
    F = O.Field.charges(CHARGES, synth.LO, synth.HI)
    seeds = _charge_seeds()
    o = _opts(1e-12, 0.01)
    r = O.trace(F, seeds, **o)
    eps = 1e-5
    for i, p in enumerate(seeds):
        ff = _fwd(r["status"][i])
        ax2 = _face_axes(ff)
        nb = np.array([p + [eps, 0, 0], p - [eps, 0, 0], p + [0, eps, 0], p - [0, eps, 0]])
        rn = O.trace(F, nb, **o)
        assert np.all(_fwd(rn["status"]) == ff)
        fp = rn["fp_fwd"][:, ax2]
        J = np.column_stack([(fp[0] - fp[1]) / (2 * eps), (fp[2] - fp[3]) / (2 * eps)])
        q_fd = (J**2).sum() / abs(np.linalg.det(J))
        assert abs(r["q_fp"][i] / q_fd - 1) < 1e-6, (p, r["q_fp"][i], q_fd)


def test_flux_identity_analytic(oracle_mod):
    """For a divergence-free field, B |a x b| is conserved along the line
    (footnote to eq. 11), so eq. (11) equals the determinant form."""
    O = oracle_mod
    F = O.Field.charges(CHARGES, synth.LO, synth.HI)
    seeds = np.vstack([_charge_seeds(), synth.random_seeds(3, 10)])
    r = O.trace(F, seeds, **_opts(1e-12, 0.01), want_ends=True)
    _, _, B0 = F.eval(seeds)
    for k in range(2):
        e = r["ends"][:, k]
        u, _, Bend = F.eval(e[:, :3])
        u = u / np.linalg.norm(u, axis=1, keepdims=True)
        a = e[:, 3:6] - u * np.sum(u * e[:, 3:6], 1, keepdims=True)
        b = e[:, 6:9] - u * np.sum(u * e[:, 6:9], 1, keepdims=True)
        ident = Bend / B0 * np.linalg.norm(np.cross(a, b), axis=1)
        assert np.allclose(ident, 1.0, atol=1e-8), ident
    assert np.allclose(r["q_perp"], r["q_det"], rtol=1e-8)


# ---------------------------------------------------------------------------
# invariants on a gridded (normalise-then-interpolate) point-charge field
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def charge_grid(oracle_mod):
    n = (65, 65, 33)
    bx, by, bz = synth.sample_charges(CHARGES, n, dtype=np.float64)
    origin, spacing = synth.grid_geometry(n)
    F = oracle_mod.Field.grid(bx, by, bz, origin, spacing)
    return F, (bx, by, bz), origin, spacing


def test_q_det_at_least_two(oracle_mod, charge_grid):
    F, _, _, spacing = charge_grid
    seeds = synth.random_seeds(9, 300)
    r = oracle_mod.trace(F, seeds, **_opts(1e-8, min(spacing)))
    ok = np.isfinite(r["q_det"])
    assert ok.mean() > 0.95
    assert np.all(r["q_det"][ok] >= 2 * (1 - 1e-12))
    # eq. (11) relies on flux conservation, which the normalised interpolant only
    # approximates; it stays close to the determinant form
    rel = np.abs(r["q_perp"][ok] / r["q_det"][ok] - 1)
    assert np.median(rel) < 1e-2


def test_q_same_along_the_line_and_both_ways(oracle_mod, charge_grid):
    """Q is a property of the whole field line: re-seeding at its footpoint or at
    an interior point, flipping the field, or rotating the initial frame leaves
    it unchanged.  Along the line this holds exactly for the determinant form;
    eq. (11) trades the determinants for |B| ratios (flux conservation), which
    the normalised interpolant satisfies only approximately, so Q_perp moves by
    about the flux-conservation error when the seed moves."""
    O = oracle_mod
    F, (bx, by, bz), origin, spacing = charge_grid
    o = _opts(1e-11, min(spacing))
    seeds = synth.random_seeds(13, 12)
    r = O.trace(F, seeds, **o)
    closedish = (_fwd(r["status"]) < 6) & (_bwd(r["status"]) < 6) & (r["q_perp"] < 1e4)
    seeds, sel = seeds[closedish], np.nonzero(closedish)[0]
    assert sel.size >= 6
    q0, qd0, l0 = r["q_perp"][sel], r["q_det"][sel], r["fll"][sel]

    # re-seed at the forward footpoint
    r1 = O.trace(F, r["fp_fwd"][sel], **o)
    assert np.all(r1["lam_fwd"] == 0.0)
    assert np.allclose(r1["q_det"], qd0, rtol=1e-6)
    assert np.allclose(r1["fll"], l0, rtol=1e-8)
    assert np.allclose(r1["fp_bwd"], r["fp_bwd"][sel], atol=1e-8)
    assert np.median(np.abs(r1["q_perp"] / q0 - 1)) < 2e-2

    # re-seed half way along the forward half-line
    half = r["lam_fwd"][sel] * 0.5
    mids = []
    for p, h in zip(seeds, half):
        rr = O.trace(F, p[None], **o, max_length=h)
        assert _fwd(rr["status"][0]) == O.MAX_LENGTH
        mids.append(rr["fp_fwd"][0])
    r2 = O.trace(F, np.array(mids), **o)
    assert np.allclose(r2["q_det"], qd0, rtol=1e-6)
    assert np.allclose(r2["fll"], l0, rtol=1e-8)

    # B -> -B swaps the two half-lines and keeps Q (eq. 11 is symmetric in F, B)
    Fm = O.Field.grid(-bx, -by, -bz, origin, spacing)
    r3 = O.trace(Fm, seeds, **o)
    assert np.allclose(r3["fp_fwd"], r["fp_bwd"][sel], atol=1e-8)
    assert np.allclose(r3["fp_bwd"], r["fp_fwd"][sel], atol=1e-8)
    assert np.allclose(r3["q_perp"], q0, rtol=1e-6)
    assert np.allclose(r3["q_det"], qd0, rtol=1e-6)

    # any orthonormal completion of the frame (eq. 9)
    r4 = O.trace(F, seeds, **o, frame_angle=0.7)
    assert np.allclose(r4["q_perp"], q0, rtol=1e-7)
    assert np.allclose(r4["q_det"], qd0, rtol=1e-7)
    assert np.allclose(r4["q_fp"], r["q_fp"][sel], rtol=1e-7, equal_nan=True)


# ---------------------------------------------------------------------------
# stops and degenerate cases
# ---------------------------------------------------------------------------

def test_statuses(oracle_mod):
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    F = O.Field.linear(b0, M, synth.LO, synth.HI)
    o = _opts(1e-9, 1 / 63)
    # outside the closed box; on the face (inside); corner
    r = O.trace(F, np.array([[0.0, 0.0, -0.01], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]), **o)
    assert _fwd(r["status"][0]) == O.SEED_OUTSIDE and np.isnan(r["q_perp"][0])
    assert _bwd(r["status"][1]) == O.ZLO and r["lam_bwd"][1] == 0.0
    assert _fwd(r["status"][2]) in (O.XHI, O.ZHI) and r["lam_fwd"][2] == 0.0
    # max_steps and max_length ("local Q" option, Sect. 3.5)
    r = O.trace(F, np.array([[0.05, 0.05, 0.5]]), **o, max_steps=1)
    assert _fwd(r["status"][0]) == O.MAX_STEPS
    r = O.trace(F, np.array([[0.05, 0.05, 0.5]]), **o, max_length=0.1)
    assert _fwd(r["status"][0]) == O.MAX_LENGTH and _bwd(r["status"][0]) == O.MAX_LENGTH
    assert r["fll"][0] == pytest.approx(0.2, abs=1e-15)
    assert np.isfinite(r["q_perp"][0]) and r["q_perp"][0] >= 2 * (1 - 1e-9)
    # a null: field vanishes on the grid around the seed
    n = (9, 9, 9)
    bx, by, bz = synth.sample_linear(*synth.uniform([0, 0, 1.0]), n)
    bz[3:6, 3:6, 3:6] = 0.0
    origin, spacing = synth.grid_geometry(n)
    Fz = O.Field.grid(bx, by, bz, origin, spacing)
    r = O.trace(Fz, np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.1]]), **_opts(1e-8, min(spacing)))
    assert _fwd(r["status"][0]) == O.NULL and np.isnan(r["q_perp"][0])
    assert _fwd(r["status"][1]) == O.NULL
    # open-line bit: closed only if both ends are on the bottom face
    assert r["status"][1] & O.OPEN_BIT


def test_node_storage_rounding(oracle_mod):
    """FP32 / BF16 node stores hold the prepared values rounded to the storage
    type; values worked out by hand for Bhat of B = (0.3, -0.5, 0.8):
    0.30304576 -> BF16 155/128 * 2^-2, -0.50507627 -> -129/128 * 2^-1,
    0.80812204 -> 207/128 * 2^-1, |B| = 0.98994949 -> 253/128 * 2^-1."""
    O = oracle_mod
    n = (3, 3, 3)
    b = synth.sample_linear(*synth.uniform([0.3, -0.5, 0.8]), n)
    origin, spacing = synth.grid_geometry(n)
    x = np.array([[0.1, 0.2, 0.3]])
    u, _, m = O.Field.grid(*b, origin, spacing, store="bf16").eval(x)
    # (interpolating equal node values reproduces them up to the weights' rounding)
    assert np.allclose(u[0], [155 / 512, -129 / 256, 207 / 256], rtol=1e-14, atol=0)
    assert m[0] == pytest.approx(253 / 256, rel=1e-14)
    u32, _, m32 = O.Field.grid(*b, origin, spacing, store="f32").eval(x)
    exact = np.array([0.3, -0.5, 0.8]) / np.sqrt(0.98)
    assert np.allclose(u32[0], exact.astype(np.float32).astype(np.float64), rtol=1e-14, atol=0)
    assert not np.allclose(u32[0], exact, rtol=1e-12, atol=0)          # it is rounded
    assert m32[0] == pytest.approx(np.float64(np.float32(np.sqrt(0.98))), rel=1e-14)


# ---------------------------------------------------------------------------
# step underflow and non-finite states (Sect. 3.4 controller; stops the paper
# leaves to the implementation)
# ---------------------------------------------------------------------------

def _charge_grid_33(O, mode=None):
    """The 4-charge field sampled FP64 on 33 x 33 x 17 nodes."""
    n = (33, 33, 17)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float64)
    origin, spacing = synth.grid_geometry(n)
    return O.Field.grid(*b, origin, spacing, **({} if mode is None else dict(mode=mode))), min(spacing)


def spine_null(n=(9, 9, 9)):
    """B = (x, y, -2 z) on [-1, 1]^3 (a 3D null at the origin whose spine is
    the z axis), sampled on n nodes: linear, so the INTERP_NORMALIZE grid
    field is exactly the analytic one."""
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    b = synth.sample_linear(np.zeros(3), np.diag([1.0, 1.0, -2.0]), n, lo=lo, hi=hi)
    origin, spacing = synth.grid_geometry(n, lo, hi)
    return b, origin, spacing


SPINE_SEEDS = np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.3137], [0.0, 0.0, -0.7]])


@pytest.mark.parametrize("n", [(9, 9, 9), (17, 17, 16)])
def test_step_underflow_at_a_spine_null(oracle_mod, n):
    """A line run into a magnetic null along its spine: the unit field on the
    spine is (0, 0, -sign z), so it reverses across the null, and the Jacobian
    of eq. (5) grows like 1/|z| as the null nears.  The embedded error of a
    step near the null stays above the tolerance until the step falls below
    1e-12 of the box extent: the forward half stops with UNDERFLOW within
    1e-9 of the null, on the spine (x = y = 0 exactly: the field has no
    transverse part there), after a length equal to the distance it covered
    (|u| = 1 on the spine); the backward half leaves through the face the
    spine meets; Q is undefined."""
    O = oracle_mod
    b, origin, spacing = spine_null(n)
    F = O.Field.grid(*b, origin, spacing, mode=O.INTERP_NORMALIZE)
    h = min(spacing)
    r = O.trace(F, SPINE_SEEDS, rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    assert np.all(_fwd(r["status"]) == O.UNDERFLOW)
    assert np.array_equal(_bwd(r["status"]), np.where(SPINE_SEEDS[:, 2] > 0, O.ZHI, O.ZLO))
    z = r["fp_fwd"][:, 2]
    assert np.all(r["fp_fwd"][:, :2] == 0.0) and np.all(np.abs(z) < 1e-9)
    assert np.all(np.sign(z) == np.sign(SPINE_SEEDS[:, 2]))
    assert np.allclose(r["lam_fwd"], np.abs(SPINE_SEEDS[:, 2] - z), rtol=0, atol=1e-12)
    assert np.all(r["counts"][:, 0, 1] >= 1) and np.all(np.isnan(r["q_perp"]))
    # the same seeds off the spine pass the null by and leave the box
    off = SPINE_SEEDS + np.array([0.05, -0.03, 0.0])
    r = O.trace(F, off, rtol=1e-8, atol=1e-8, h_init=0.1 * h, h_max=h)
    assert np.all(_fwd(r["status"]) < 6)


def poisoned_uniform(value, mode_name="paper"):
    """Uniform field B = (0, 0, 1) on 9^3 nodes with node (x 4, y 4, z 6) set
    to `value` (NaN or Inf): the cells with z index 5 and 6 around x = y = 0
    hold a non-finite corner."""
    n = (9, 9, 9)
    bx, by, bz = (np.array(c) for c in synth.sample_linear(*synth.uniform([0, 0, 1.0]), n))
    bz[6, 4, 4] = value
    origin, spacing = synth.grid_geometry(n)
    return (bx, by, bz), origin, spacing


@pytest.mark.parametrize("value", [np.nan, np.inf])
@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_nonfinite_node(oracle_mod, value, mode):
    """A line through the poisoned cells: the first trial step with a stage
    point in cell z 5 (z >= 0.625) turns non-finite, so the forward half stops
    with NONFINITE at its last accepted point, on the line x = y = 0 within one
    largest step (0.125) below z = 0.625; its length is that point's height
    less the seed's (the field is uniform).  The backward half never reaches
    the cells and lands on z = 0 as on the clean field.  Q is undefined."""
    O = oracle_mod
    b, origin, spacing = poisoned_uniform(value)
    md = O.PAPER if mode == "paper" else O.INTERP_NORMALIZE
    F = O.Field.grid(*b, origin, spacing, mode=md)
    seed = np.array([[0.0, 0.0, 0.1]])
    kw = _opts(1e-8, min(spacing))
    r = O.trace(F, seed, **kw)
    assert _fwd(r["status"][0]) == O.NONFINITE and _bwd(r["status"][0]) == O.ZLO
    z_end = r["fp_fwd"][0, 2]
    assert 0.625 - 0.125 <= z_end < 0.625
    assert np.allclose(r["fp_fwd"][0, :2], 0.0, atol=1e-14)
    assert r["lam_fwd"][0] == pytest.approx(z_end - 0.1, abs=1e-12)
    assert r["fll"][0] == pytest.approx(z_end, abs=1e-12)
    assert np.isnan(r["q_perp"][0]) and np.isnan(r["q_det"][0])
    clean = O.trace(O.Field.grid(*poisoned_uniform(1.0)[0], origin, spacing, mode=md), seed, **kw)
    assert np.array_equal(r["fp_bwd"], clean["fp_bwd"]) and r["lam_bwd"][0] == clean["lam_bwd"][0]
    # the explicit Euler scheme evaluates the field at the start of each step
    # only: it stops at the first point of its fixed-step lattice inside the
    # poisoned cells (z = 0.1 + 21 * 0.025 = 0.625, up to rounding)
    e = O.trace(F, seed, rtol=1e-8, atol=1e-8, h_init=0.025, h_max=0.025, stepper="euler")
    assert _fwd(e["status"][0]) == O.NONFINITE
    assert e["fp_fwd"][0, 2] == pytest.approx(0.625, abs=1e-12) and e["counts"][0, 0, 0] == 21


def test_non_finite_seed_is_outside(oracle_mod):
    """A seed with a NaN coordinate is not a point of the box: SEED_OUTSIDE on
    both halves, length 0, Q undefined."""
    O = oracle_mod
    F, h = _charge_grid_33(O)
    r = O.trace(F, np.array([[np.nan, 0.0, 0.5], [0.0, 0.0, np.inf]]), **_opts(1e-6, h))
    assert np.all(_fwd(r["status"]) == O.SEED_OUTSIDE) and np.all(_bwd(r["status"]) == O.SEED_OUTSIDE)
    assert np.all(r["fll"] == 0.0) and np.all(np.isnan(r["q_perp"]))
