"""Oracle pins of the explicit Euler stepper (QSL Squasher Sect. 3.4: fixed
steps of the line and of both deviation vectors, one right-hand side per
step): exact on straight lines (the exit points of a ray and a box, Q = 2),
first-order convergence to the closed-form field lines of the hyperbolic flux
tube B = (kx, -ky, 1), and the fixed-step bookkeeping of max_steps and
max_length."""
import numpy as np

import synth

LO, HI = np.array(synth.LO), np.array(synth.HI)


def _fwd(st):
    return st & 0xFF


def _bwd(st):
    return (st >> 8) & 0xFF


def _ray_exit(p, v):
    """Parameter t > 0 and face index where p + t v leaves the box."""
    t = np.full(p.shape[0], np.inf)
    face = np.full(p.shape[0], -1)
    for d in range(3):
        for side, wall in ((0, LO[d]), (1, HI[d])):
            with np.errstate(divide="ignore", invalid="ignore"):
                td = (wall - p[:, d]) / v[d]
            ok = (td > 0) & (td < t)
            t = np.where(ok, td, t)
            face = np.where(ok, 2 * d + side, face)
    return t, face


def test_euler_exact_on_a_uniform_field(oracle_mod):
    O = oracle_mod
    d = np.array([0.3, -0.5, 0.8])
    F = O.Field.linear(*synth.uniform(d), synth.LO, synth.HI)
    seeds = synth.rng(5).uniform([-0.9, -0.9, 0.05], [0.9, 0.9, 0.95], (40, 3))
    h = 0.013
    r = O.trace(F, seeds, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, stepper="euler")
    u = d / np.linalg.norm(d)
    tf, ff = _ray_exit(seeds, u)
    tb, fb = _ray_exit(seeds, -u)
    assert np.array_equal(_fwd(r["status"]), ff) and np.array_equal(_bwd(r["status"]), fb)
    assert np.allclose(r["fp_fwd"], seeds + tf[:, None] * u, rtol=0, atol=1e-12)
    assert np.allclose(r["fp_bwd"], seeds - tb[:, None] * u, rtol=0, atol=1e-12)
    assert np.allclose(r["fll"], tf + tb, rtol=1e-12)
    # constant deviations: perpendicular-plane Q of a uniform field is 2
    assert np.allclose(r["q_perp"], 2.0, rtol=1e-12) and np.allclose(r["q_det"], 2.0, rtol=1e-12)
    # one step per h, the last one cut at the face
    assert np.array_equal(r["counts"][:, 0, 0], np.floor(tf / h).astype(np.int64) + 1)
    assert np.array_equal(r["counts"][:, 1, 0], np.floor(tb / h).astype(np.int64) + 1)
    assert not r["counts"][:, :, 1:].any()          # no rejections, no landing iterations


def test_euler_first_order_on_the_hyperbolic_tube(oracle_mod):
    """Forward lines from z = 0 end at (x0 e^k, y0 e^-k, 1) with footpoint Q
    2 cosh(2k); Euler's end-point and Q errors halve with the step."""
    O = oracle_mod
    k = 2.0
    F = O.Field.linear(*synth.hyperbolic(k), synth.LO, synth.HI)
    seeds = np.array([[0.05, 0.3, 0.0], [-0.1, -0.6, 0.0], [0.02, 0.8, 0.0], [0.12, -0.2, 0.0]])
    exact = np.stack([seeds[:, 0] * np.exp(k), seeds[:, 1] * np.exp(-k), np.ones(4)], axis=1)
    errs, qerrs = [], []
    for h in (1 / 100, 1 / 200, 1 / 400, 1 / 800):
        r = O.trace(F, seeds, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, stepper="euler")
        assert np.all(_fwd(r["status"]) == 5)
        errs.append(np.linalg.norm(r["fp_fwd"] - exact, axis=1))
        qerrs.append(np.abs(r["q_fp"] / (2 * np.cosh(2 * k)) - 1))
    errs, qerrs = np.array(errs), np.array(qerrs)
    for e in (errs, qerrs):
        ratio = e[:-1] / e[1:]
        assert np.all((ratio > 1.7) & (ratio < 2.3)), ratio
    assert np.all(errs[-1] < 1e-2) and np.all(qerrs[-1] < 2e-2)


def test_euler_step_budget_and_length_limit(oracle_mod):
    O = oracle_mod
    F = O.Field.linear(*synth.uniform([0.0, 0.0, 1.0]), synth.LO, synth.HI)
    seed = np.array([[0.1, -0.2, 0.5]])
    h = 0.01
    r = O.trace(F, seed, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, max_steps=7, stepper="euler")
    assert _fwd(r["status"][0]) == 7 and _bwd(r["status"][0]) == 7          # max_steps both ways
    assert r["counts"][0, 0, 0] == 7 and abs(r["lam_fwd"][0] - 7 * h) < 1e-15
    assert abs(r["fp_fwd"][0, 2] - (0.5 + 7 * h)) < 1e-14
    r = O.trace(F, seed, rtol=1e-6, atol=1e-6, h_init=h, h_max=h, max_length=0.0234, stepper="euler")
    assert _fwd(r["status"][0]) == 6 and _bwd(r["status"][0]) == 6          # max_length both ways
    assert r["counts"][0, 0, 0] == 3 and r["lam_fwd"][0] == 0.0234
    assert abs(r["fp_fwd"][0, 2] - 0.5234) < 1e-14 and abs(r["fp_bwd"][0, 2] - 0.4766) < 1e-14
