"""The refinement-decision checker (tests/refine_check.py) against planted
mistakes, on the oracle's refinement (Sect. 3.6) of a synthetic length
landscape on a slice and in a volume: identical and rounding-level differing
values pass; a threshold off by 1 %, a key-gap test off by one, a new key
off the midpoint, and decisions taken on values the checker was not told about all fail."""
import numpy as np
import pytest

from refine_check import base_keys, check_refinement

THR = 0.02


def _landscape(p):
    """A length map with a closed ridge (jumps of ~0.6 across a thin ring), a
    slope whose jumps between neighbouring samples sweep through the threshold,
    and a step that crosses the curve's seams."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    r2 = x * x + y * y + (z - 0.5) ** 2
    return 0.5 + 0.3 * np.tanh((r2 - 0.35) / 0.01) + 0.3 * np.sin(4.0 * x + 2.0 * y) + 0.2 * (y > 0.13)


def _region(oracle_mod, dims):
    if dims == 2:
        return oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0), 6, 2
    return oracle_mod.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0), 3, 2


def _refine(oracle_mod, dims, fn, thr=THR):
    region, m, r = _region(oracle_mod, dims)
    keys, vals, _ = oracle_mod.refine_slice(region, m, r, thr, lambda p: {"fll": fn(p), "q": fn(p)})
    return keys, vals["fll"], region, m, r


def _positions(oracle_mod, region, m, r, keys):
    """Sample positions of keys: base keys sit at their base cell's centre,
    the others at the centre of their finest cell."""
    blk = (1 << region.dims) ** r
    base = keys % blk == blk // 2
    pos = np.empty((keys.size, 3))
    pos[base] = region.centres(m, *region.cells(m, keys[base] // blk))
    if (~base).any():
        pos[~base] = oracle_mod.key_positions(region, m, r, keys[~base])
    return pos


def _oracle_at(oracle_mod, region, m, r, keys):
    return _landscape(_positions(oracle_mod, region, m, r, keys))


@pytest.mark.parametrize("dims", [2, 3])
def test_same_values_pass(oracle_mod, dims):
    keys, fll, region, m, r = _refine(oracle_mod, dims, _landscape)
    out = check_refinement(keys, fll, fll, base_keys(m, r, dims), THR, keys_oracle=keys)
    assert out["fired"] > 50 and out["differ"] == 0 and out["symmetric_difference"] == 0


@pytest.mark.parametrize("dims", [2, 3])
def test_rounding_level_differences_pass(oracle_mod, dims):
    """Values moved by 1e-12 (what FP64 stepping differs by): decisions may
    flip only where the jump is within 1e-4 thr of the threshold."""
    noisy = lambda p: _landscape(p) + 1e-12 * np.sin(1e3 * p[:, 0] + 7.0 * p[:, 1])   # noqa: E731
    keys, fll, region, m, r = _refine(oracle_mod, dims, noisy)
    ko, _, _, _, _ = _refine(oracle_mod, dims, _landscape)
    fo = _oracle_at(oracle_mod, region, m, r, keys)
    check_refinement(keys, fll, fo, base_keys(m, r, dims), THR, keys_oracle=ko)


@pytest.mark.parametrize("dims", [2, 3])
def test_threshold_off_by_one_percent_fails(oracle_mod, dims):
    keys, fll, region, m, r = _refine(oracle_mod, dims, _landscape, thr=1.01 * THR)
    ko, _, _, _, _ = _refine(oracle_mod, dims, _landscape)
    assert keys.size != ko.size
    fo = _oracle_at(oracle_mod, region, m, r, keys)
    with pytest.raises(AssertionError, match="decided against|non-marginal"):
        check_refinement(keys, fll, fo, base_keys(m, r, dims), THR, keys_oracle=ko)


def _plain_rule(oracle_mod, min_gap, offset):
    """The pass-by-pass rule with a planted change: pairs fire at key gaps >=
    min_gap, and the new key is floor((k1 + k2) / 2) + offset."""
    region, m, r = _region(oracle_mod, 2)
    keys = base_keys(m, r, 2)
    vals = _landscape(_positions(oracle_mod, region, m, r, keys))
    for _ in range(2 * r):
        gap, jump = np.diff(keys), np.abs(np.diff(vals))
        i = np.nonzero((gap >= min_gap) & (jump > THR))[0]
        if i.size == 0:
            break
        newk = (keys[i] + keys[i + 1]) // 2 + offset
        keys = np.insert(keys, i + 1, newk)
        vals = np.insert(vals, i + 1, _landscape(oracle_mod.key_positions(region, m, r, newk)))
    return keys, vals, m, r


def test_planted_rule_mistakes_fail(oracle_mod):
    """The unchanged rule passes; a gap test of > 2 instead of >= 2 (the last
    level never refined) and a new key one cell past the midpoint both fail."""
    keys, vals, m, r = _plain_rule(oracle_mod, 2, 0)
    check_refinement(keys, vals, vals, base_keys(m, r, 2), THR)
    keys, vals, m, r = _plain_rule(oracle_mod, 3, 0)
    with pytest.raises(AssertionError, match="decided against"):
        check_refinement(keys, vals, vals, base_keys(m, r, 2), THR)
    keys, vals, m, r = _plain_rule(oracle_mod, 2, 1)
    with pytest.raises(AssertionError, match="cannot reach|not strictly increasing"):
        check_refinement(keys, vals, vals, base_keys(m, r, 2), THR)


def test_hidden_value_errors_fail_and_told_errors_pass(oracle_mod):
    """Decisions taken on lengths that differ from the oracle's by 0.01 at a
    few keys pass when the checker sees those lengths (the band includes the
    length error), and fail when it is handed the oracle's lengths as the
    set's own."""
    region, m, r = _region(oracle_mod, 2)
    bump = lambda p: _landscape(p) + 0.01 * (np.abs(p[:, 0] - 0.3) < 0.05)   # noqa: E731
    keys, fll, _, _, _ = _refine(oracle_mod, 2, bump)
    ko, _, _, _, _ = _refine(oracle_mod, 2, _landscape)
    fo = _oracle_at(oracle_mod, region, m, r, keys)
    assert keys.size != ko.size
    check_refinement(keys, fll, fo, base_keys(m, r, 2), THR, keys_oracle=ko)
    with pytest.raises(AssertionError):
        check_refinement(keys, fo, fo, base_keys(m, r, 2), THR, keys_oracle=ko)
