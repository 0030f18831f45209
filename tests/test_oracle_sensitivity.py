"""How many lines the oracle itself moves out of the per-line gates when its
seeds move by about the rounding of FP32 stage arithmetic (1e-7 domain units).

FP32 stepping on the GPU perturbs the stage points by ~1e-7 of a cell; near
cell faces (where the trilinear gradient jumps, Sect. 3.2-3.3) and near
accept/reject decisions at err ~ 1 (Sect. 3.4) a perturbation of that size
sends a few lines down a different, equally valid step sequence.  This test
measures that fraction on the oracle alone, on the fields, seeds and
tolerances of the FP32 GPU parity tests, and checks that the floor the FP32
gate derives from it (``gpu_util.sensitivity_floor``) stays tight: no test may
accept FP32 results that move more lines than the method's own sensitivity
explains, and that sensitivity is a fraction of a percent.
"""
import numpy as np
import pytest

import synth
from gpu_util import FP32_MIN_FRAC, sensitivity_floor


def _mixed_seeds(count, seed):
    s = synth.random_seeds(seed, count)
    s[: count // 2, 2] = 0.0
    return s


def _floor(oracle_mod, fo, seeds, tol, h):
    kw = dict(rtol=tol, atol=tol, h_init=0.1 * h, h_max=h)
    o = oracle_mod.trace(fo, seeds, **kw)
    return sensitivity_floor(oracle_mod, fo, seeds, o, kw, draws=4)


@pytest.mark.parametrize("tol,least", [(1e-4, 0.99), (1e-5, 0.985)])
def test_charges_sensitivity(oracle_mod, tol, least):
    n = (97, 97, 49)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    fo = oracle_mod.Field.grid(*(c.astype(np.float64) for c in b), origin, spacing, store="f32")
    floor, fr = _floor(oracle_mod, fo, _mixed_seeds(1037, 41), tol, min(spacing))
    print(f"charges tol {tol:g}: fractions in the gates {np.round(fr, 4)}, floor {floor:.4f}")
    assert min(fr) >= least              # the method moves under 1.5 % of lines ...
    assert min(fr) < 1.0                 # ... but it does move some
    assert floor >= FP32_MIN_FRAC


def test_rope_sensitivity(oracle_mod):
    n = (72, 72, 48)
    b, _ = synth.flux_rope_field(n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    fo = oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in b), origin, spacing, store="f32")
    floor, fr = _floor(oracle_mod, fo, synth.random_seeds(43, 700), 1e-4, min(spacing))
    print(f"rope tol 1e-4: fractions in the gates {np.round(fr, 4)}, floor {floor:.4f}")
    assert min(fr) >= 0.99 and floor >= FP32_MIN_FRAC


@pytest.mark.parametrize("tol,least", [(1e-4, 0.995), (1e-5, 0.99)])
def test_fp32_rounding_instrument(oracle_mod, tol, least):
    """The oracle with its CK54 stage points, stage slopes and accepted states
    rounded to FP32 (a test instrument; parity references never use it) keeps
    at least 99 % of the charge-field lines inside the per-line gates: the
    roundings FP32 storage of the state forces move few lines, at tol 1e-5 as
    at 1e-4.  With the instrument off the oracle is bit-identical to itself."""
    from gpu_util import _in_gates
    n = (97, 97, 49)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    fo = oracle_mod.Field.grid(*(c.astype(np.float64) for c in b), origin, spacing, store="f32")
    seeds = _mixed_seeds(1037, 41)
    h = min(spacing)
    kw = dict(rtol=tol, atol=tol, h_init=0.1 * h, h_max=h)
    o = oracle_mod.trace(fo, seeds, **kw)
    again = oracle_mod.trace(fo, seeds, round_f32=False, **kw)
    assert np.array_equal(o["q_perp"], again["q_perp"], equal_nan=True)
    e = oracle_mod.trace(fo, seeds, round_f32=True, **kw)
    frac = float(_in_gates(e, o).mean())
    moved = float(np.mean(np.any(e["counts"][:, :, :2] != o["counts"][:, :, :2], axis=(1, 2))))
    print(f"tol {tol:g}: rounded-to-FP32 oracle in the gates {frac:.4f}, step sequences changed {moved:.4f}")
    assert frac >= least and 0.0 < moved < 0.03
