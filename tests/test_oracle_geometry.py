"""Pins of the oracle's spherical geometry (Sect. 3.1 eq. 2; deviations eq. 6-7,
lengths eq. 8) and rectilinear (non-uniform) grids (Sect. 3.2, the cell span
h_c), against facts fixed by the mathematics:

* a monopole B = r_hat / r^2 has radial field lines: footpoints, lengths and
  Q = 2 exactly (flux through a tube scales as r^2 both ways, and eq. (6) is
  exact for a radial field);
* eq. (2) is exact: field lines traced in spherical coordinates through an
  analytic field end where the same lines traced in Cartesian coordinates end;
* eq. (6) drops terms of the order of the field's length scale over the
  radius: its Q stays close to the Cartesian one;
* a gridded monopole gives radial lines exactly and Q -> 2 at second order;
* a rectilinear grid reproduces linear fields exactly (the flux tube's
  closed forms), and with evenly spaced coordinates it is the uniform grid.
"""
import numpy as np
import pytest

import synth
from test_oracle_trace import K, _check_hyperbolic, _hyp_seed_set, _opts

WEDGE_LO, WEDGE_HI = (-0.3, -0.3, 1.0), (0.3, 0.3, 1.5)


def _sph_to_cart(q):
    q = np.atleast_2d(q)
    ph, th, r = q[:, 0], q[:, 1], q[:, 2]
    return np.stack([r * np.cos(th) * np.cos(ph), r * np.cos(th) * np.sin(ph), r * np.sin(th)], axis=1)


def _wedge_seeds(seed, n):
    g = synth.rng(seed)
    lo, hi = np.array(WEDGE_LO), np.array(WEDGE_HI)
    return g.uniform(lo + 0.05 * (hi - lo), hi - 0.05 * (hi - lo), size=(n, 3))


def test_monopole_analytic_exact(oracle_mod):
    O = oracle_mod
    F = O.Field.charges([[0.0, 0.0, 0.0, 1.0]], WEDGE_LO, WEDGE_HI, geometry="spherical")
    s = _wedge_seeds(1, 40)
    r = O.trace(F, s, **_opts(1e-10, 0.01))
    assert np.all(r["status"] & 0xFFFF == (5 | (4 << 8)))      # out through r = 1.5, back to r = 1
    assert np.allclose(r["fp_fwd"][:, :2], s[:, :2], atol=1e-12) and np.allclose(r["fp_fwd"][:, 2], 1.5)
    assert np.allclose(r["fp_bwd"][:, :2], s[:, :2], atol=1e-12) and np.allclose(r["fp_bwd"][:, 2], 1.0)
    assert np.allclose(r["fll"], 0.5, atol=1e-10)
    for key in ("q_perp", "q_det", "q_fp"):
        assert np.allclose(r[key], 2.0, rtol=1e-9), key


def _dipole():
    # a pair of opposite charges just below r = 1 near (phi, theta) = (0, 0)
    return np.array([[0.90, 0.06, 0.02, 1.0], [0.91, -0.07, -0.03, -1.0]])


def test_field_lines_match_cartesian(oracle_mod):
    """eq. (2): the same lines to the same length end at the same points."""
    O = oracle_mod
    ch = _dipole()
    FS = O.Field.charges(ch, WEDGE_LO, WEDGE_HI, geometry="spherical")
    FC = O.Field.charges(ch, (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = _wedge_seeds(2, 60)
    L = 0.08
    kw = dict(_opts(1e-11, 0.01), max_length=L)
    rs = O.trace(FS, s, **kw)
    rc = O.trace(FC, _sph_to_cart(s), **kw)
    both = ((rs["status"] & 0xFF) == 6) & (((rs["status"] >> 8) & 0xFF) == 6)
    assert both.sum() >= 30
    assert np.all(rc["status"][both] & 0xFFFF == (6 | (6 << 8)))
    assert np.abs(_sph_to_cart(rs["fp_fwd"][both]) - rc["fp_fwd"][both]).max() < 1e-8
    assert np.abs(_sph_to_cart(rs["fp_bwd"][both]) - rc["fp_bwd"][both]).max() < 1e-8
    assert np.allclose(rs["fll"][both], 2 * L)


def test_deviation_equation_close_to_cartesian(oracle_mod):
    """eq. (6) neglects terms of the order of (field length scale) / (radius):
    on this dipole (length scale ~ 0.1 at radius ~ 1) Q along lines of length
    0.16 stays within a few per cent of the exact Cartesian linearisation, and
    the determinant form Q_det >= 2 holds."""
    O = oracle_mod
    ch = _dipole()
    FS = O.Field.charges(ch, WEDGE_LO, WEDGE_HI, geometry="spherical")
    FC = O.Field.charges(ch, (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = _wedge_seeds(2, 60)
    kw = dict(_opts(1e-11, 0.01), max_length=0.08)
    rs = O.trace(FS, s, **kw)
    rc = O.trace(FC, _sph_to_cart(s), **kw)
    both = ((rs["status"] & 0xFF) == 6) & (((rs["status"] >> 8) & 0xFF) == 6)
    rel = np.abs(rs["q_perp"][both] / rc["q_perp"][both] - 1)
    print(f"spherical vs Cartesian Q: median {np.median(rel):.2e}, max {rel.max():.2e}")
    assert np.median(rel) < 0.02 and rel.max() < 0.1
    assert np.all(rs["q_det"][both] >= 2 * (1 - 1e-12))


def _gridded_monopole(O, n, mode):
    phi = np.linspace(WEDGE_LO[0], WEDGE_HI[0], n)
    th = np.linspace(WEDGE_LO[1], WEDGE_HI[1], n)
    rr = np.linspace(WEDGE_LO[2], WEDGE_HI[2], n)
    R = np.broadcast_to(rr[:, None, None], (n, n, n))
    br = 1.0 / R ** 2
    z = np.zeros_like(br)
    origin = (phi[0], th[0], rr[0])
    spacing = (phi[1] - phi[0], th[1] - th[0], rr[1] - rr[0])
    return O.Field.grid(z, z, np.ascontiguousarray(br), origin, spacing, mode=mode, geometry="spherical")


@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_gridded_monopole(oracle_mod, mode):
    O = oracle_mod
    m = O.PAPER if mode == "paper" else O.INTERP_NORMALIZE
    s = _wedge_seeds(3, 30)
    errs = []
    for n in (9, 17, 33):
        F = _gridded_monopole(O, n, m)
        r = O.trace(F, s, **_opts(1e-10, 0.01))
        assert np.all(r["status"] & 0xFFFF == (5 | (4 << 8)))
        assert np.allclose(r["fp_fwd"][:, :2], s[:, :2], atol=1e-12)
        assert np.allclose(r["fll"], 0.5, atol=1e-10)
        errs.append(np.abs(r["q_perp"] - 2.0).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(f"{mode}: |Q - 2| {np.array(errs)}, orders {orders}")
    assert errs[-1] < 2e-3 and np.all(orders > 1.7)


def _stretched(n, lo, hi, beta):
    u = np.linspace(-1, 1, n)
    v = np.tanh(beta * u) / np.tanh(beta)
    return lo + (hi - lo) * (v + 1) / 2


def test_rectilinear_linear_field_exact(oracle_mod):
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    xs = _stretched(21, -1.0, 1.0, 1.6)
    ys = np.sort(np.concatenate([[-1.0, 1.0], synth.rng(5).uniform(-1, 1, 17)]))
    zs = np.geomspace(1.0, 2.0, 15) - 1.0
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    B = [b0[i] + M[i, 0] * X + M[i, 1] * Y + M[i, 2] * Z for i in range(3)]
    F = O.Field.grid(*B, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), mode=O.INTERP_NORMALIZE, coords=(xs, ys, zs))
    seeds = _hyp_seed_set()[::3]
    r = O.trace(F, seeds, **_opts(1e-11, 0.02))
    _check_hyperbolic(O, r, seeds, 1e-8, 1e-7, 1e-8)


def test_rectilinear_even_coords_are_the_uniform_grid(oracle_mod):
    O = oracle_mod
    n = (33, 33, 17)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float64)
    origin, spacing = synth.grid_geometry(n)
    coords = [origin[a] + spacing[a] * np.arange(n[a]) for a in range(3)]
    FU = O.Field.grid(*b, origin, spacing)
    FR = O.Field.grid(*b, origin, spacing, coords=coords)
    s = synth.random_seeds(6, 200)
    kw = _opts(1e-6, min(spacing))
    ru, rr = O.trace(FU, s, **kw), O.trace(FR, s, **kw)
    same = ru["status"] == rr["status"]
    assert same.mean() > 0.99
    assert np.abs(ru["fp_fwd"][same] - rr["fp_fwd"][same]).max() < 1e-9
    assert np.allclose(ru["q_perp"][same], rr["q_perp"][same], rtol=1e-6)


def test_rectilinear_arguments(oracle_mod):
    O = oracle_mod
    b = synth.sample_charges(synth.point_charges(2, 4), (5, 5, 5), dtype=np.float64)
    with pytest.raises(ValueError):
        O.Field.grid(*b, (0, 0, 0), (1, 1, 1), coords=(np.array([0, 1, 1, 2, 3.0]), None, None))
    with pytest.raises(ValueError):
        O.Field.grid(*b, (0, 0, 0), (1, 1, 1), order=3, coords=(np.arange(5.0), None, None))
