"""Pins of the oracle's triquadratic (Dodgson 1997) and tricubic (Keys 1981)
interpolation (Sect. 3.2, eq. 3; gradients by the kernels' analytic
derivatives, Sect. 3.3), each against a fact fixed by the mathematics rather
than by the oracle's own formulas:

* both kernels interpolate: at a node the value is the node value;
* both reproduce linear fields exactly, boundary cells included (Keys'
  boundary extrapolation is exact for quadratics), so the hyperbolic flux
  tube's closed forms hold on the grid at every order;
* the cubic kernel reproduces quadratic fields exactly (Keys' third-order
  property); the quadratic kernel does not;
* the gradient is the derivative of the interpolant (central differences);
* on a smooth field the errors fall as h^2 (linear, quadratic) and h^3
  (cubic) per grid halving.
"""
import numpy as np
import pytest

import synth
from test_oracle_trace import K, _check_hyperbolic, _hyp_seed_set, _opts

CH = synth.point_charges(2, 4)


def _box_points(seed, n, margin=0.0):
    g = synth.rng(seed)
    lo, hi = np.array(synth.LO) + margin, np.array(synth.HI) - margin
    return g.uniform(lo, hi, size=(n, 3))


@pytest.mark.parametrize("order", [2, 3])
def test_nodes_are_interpolated(oracle_mod, order):
    O = oracle_mod
    n = (9, 8, 7)
    b = synth.sample_charges(CH, n, dtype=np.float64)
    origin, spacing = synth.grid_geometry(n)
    F = O.Field.grid(*b, origin, spacing, mode=O.INTERP_NORMALIZE, order=order)
    g = synth.rng(4)
    idx = np.column_stack([g.integers(0, n[0], 60), g.integers(0, n[1], 60), g.integers(0, n[2], 60)])
    idx[:6] = [[0, 0, 0], [n[0] - 1, 0, 0], [0, n[1] - 1, n[2] - 1], [n[0] - 1, n[1] - 1, n[2] - 1],
               [3, 0, n[2] - 1], [n[0] - 1, 4, 2]]
    x = np.array(origin) + idx * np.array(spacing)
    u, _, bm = F.eval(x)
    B = np.stack([c[idx[:, 2], idx[:, 1], idx[:, 0]] for c in b], axis=1)
    norm = np.linalg.norm(B, axis=1)
    assert np.allclose(u, B / norm[:, None], rtol=0, atol=1e-13)
    assert np.allclose(bm, norm, rtol=1e-13)


@pytest.mark.parametrize("order", [2, 3])
def test_linear_fields_exact(oracle_mod, order):
    """B = b0 + M x: the interpolated B, and so u = B/|B| and its gradient,
    equal the analytic field's everywhere, boundary cells included."""
    O = oracle_mod
    g = synth.rng(7)
    b0 = np.array([0.3, -0.2, 1.5])
    M = g.normal(scale=0.4, size=(3, 3))
    n = (11, 9, 8)
    bx, by, bz = synth.sample_linear(b0, M, n)
    origin, spacing = synth.grid_geometry(n)
    F = O.Field.grid(bx, by, bz, origin, spacing, mode=O.INTERP_NORMALIZE, order=order)
    A = O.Field.linear(b0, M, synth.LO, synth.HI)
    x = np.concatenate([_box_points(8, 300), _box_points(9, 40) * np.array([1, 1, 0.02])])
    u, J, bm = F.eval(x)
    ua, Ja, ba = A.eval(x)
    assert np.abs(u - ua).max() < 1e-12 and np.abs(J - Ja).max() < 1e-11 and np.abs(bm - ba).max() < 1e-12


def _quadratic_B(C, x):
    """B_i = C[i] . (1, x, y, z, x^2, y^2, z^2, xy, yz, zx)."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    basis = np.stack([np.ones_like(X), X, Y, Z, X * X, Y * Y, Z * Z, X * Y, Y * Z, Z * X], axis=1)
    return basis @ C.T


@pytest.mark.parametrize("order,exact", [(3, True), (2, False)])
def test_quadratic_fields(oracle_mod, order, exact):
    """The cubic kernel reproduces a quadratic B exactly (value and gradient,
    the latter checked against central differences of the analytic unit
    field); the quadratic kernel does not (it is exact for linear fields
    only)."""
    O = oracle_mod
    g = synth.rng(11)
    C = g.normal(scale=0.3, size=(3, 10))
    C[2, 0] = 3.0                                   # keeps |B| away from zero
    n = (12, 10, 9)
    nodes = synth.node_coords(n)
    Z, Y, X = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    B = _quadratic_B(C, pts)
    b = [B[:, k].reshape(X.shape) for k in range(3)]
    origin, spacing = synth.grid_geometry(n)
    F = O.Field.grid(*b, origin, spacing, mode=O.INTERP_NORMALIZE, order=order)
    x = _box_points(12, 200)
    u, J, _ = F.eval(x)
    Ba = _quadratic_B(C, x)
    ua = Ba / np.linalg.norm(Ba, axis=1)[:, None]
    eps = 1e-5
    Jfd = np.empty_like(J)
    for j in range(3):
        e = np.zeros(3)
        e[j] = eps
        up = _quadratic_B(C, x + e)
        um = _quadratic_B(C, x - e)
        up /= np.linalg.norm(up, axis=1)[:, None]
        um /= np.linalg.norm(um, axis=1)[:, None]
        Jfd[:, :, j] = (up - um) / (2 * eps)
    eu = np.abs(u - ua).max()
    eJ = np.abs(J - Jfd).max()
    print(f"order {order}: max |u - u_exact| {eu:.2e}, max |J - J_fd| {eJ:.2e}")
    if exact:
        assert eu < 1e-12 and eJ < 1e-8
    else:
        assert eu > 1e-5 and eu < 0.05


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("mode", ["paper", "interp_normalize"])
def test_gradient_is_the_derivative(oracle_mod, order, mode):
    O = oracle_mod
    n = (13, 12, 9)
    b = synth.sample_charges(CH, n, dtype=np.float64)
    origin, spacing = synth.grid_geometry(n)
    F = O.Field.grid(*b, origin, spacing, mode=O.PAPER if mode == "paper" else O.INTERP_NORMALIZE, order=order)
    x = _box_points(13, 150, margin=0.05)
    u, J, _ = F.eval(x)
    eps = 1e-7
    for j in range(3):
        e = np.zeros(3)
        e[j] = eps
        fd = (F.eval(x + e)[0] - F.eval(x - e)[0]) / (2 * eps)
        scale = np.abs(J[:, :, j]).max() + 1.0
        assert np.abs(fd - J[:, :, j]).max() < 1e-6 * scale, (j, np.abs(fd - J[:, :, j]).max())


def test_convergence_orders(oracle_mod):
    """Interpolating B and then normalising on the 4-charge field, against the
    analytic unit field at 400 interior points: the RMS error falls as h^2 (order 1.7-2.3)
    for the linear and quadratic kernels and at least as h^2.8 for the cubic
    one over the last two grid halvings (17 -> 129 nodes per side)."""
    O = oracle_mod
    A = O.Field.charges(CH, synth.LO, synth.HI)
    x = _box_points(3, 400) * np.array([0.9, 0.9, 0.7]) + np.array([0, 0, 0.2])
    ua = A.eval(x)[0]
    orders = {}
    for order in (1, 2, 3):
        errs = []
        for n in (33, 65, 129):
            grid = (n, n, (n + 1) // 2)
            b = synth.sample_charges(CH, grid, dtype=np.float64)
            origin, spacing = synth.grid_geometry(grid)
            F = O.Field.grid(*b, origin, spacing, mode=O.INTERP_NORMALIZE, order=order)
            errs.append(np.sqrt(np.mean((F.eval(x)[0] - ua) ** 2)))
        orders[order] = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("observed orders:", {k: np.round(v, 2) for k, v in orders.items()})
    for k in (1, 2):
        assert np.all((orders[k] > 1.7) & (orders[k] < 2.3)), orders
    assert np.all(orders[3] > 2.8), orders


@pytest.mark.parametrize("order", [2, 3])
def test_hyperbolic_grid_exact(oracle_mod, order):
    """The flux tube B = (kx, -ky, 1) is linear, so interpolating B and then
    normalising meets its closed forms on the grid at every order."""
    O = oracle_mod
    b0, M = synth.hyperbolic(K)
    grid = (24, 24, 24)
    bx, by, bz = synth.sample_linear(b0, M, grid)
    origin, spacing = synth.grid_geometry(grid)
    F = O.Field.grid(bx, by, bz, origin, spacing, mode=O.INTERP_NORMALIZE, order=order)
    seeds = _hyp_seed_set()[::4]
    r = O.trace(F, seeds, **_opts(1e-11, min(spacing)))
    _check_hyperbolic(O, r, seeds, 1e-8, 1e-7, 1e-8)


def test_order_argument_checked(oracle_mod):
    O = oracle_mod
    b = synth.sample_charges(CH, (3, 5, 5), dtype=np.float64)
    origin, spacing = synth.grid_geometry((3, 5, 5))
    with pytest.raises(ValueError):
        O.Field.grid(*b, origin, spacing, order=3)
    with pytest.raises(ValueError):
        O.Field.grid(*b, origin, spacing, order=4)
