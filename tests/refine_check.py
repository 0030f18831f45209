"""Checks of FLL-jump refinement decisions (QSL Squasher Sect. 3.6).

A refined sample set is checked in three steps, from the final arrays alone:

1. Replay.  Starting from the base keys (plus any proposed keys), the
   pass-by-pass rule is replayed: a curve-successive pair (k1, k2) with
   k2 - k1 >= 2 fired iff its midpoint floor((k1 + k2) / 2) is a sample (no
   other route can put a key strictly between two samples that stay
   curve-successive).  The replay must reach exactly the final set, and each
   examined pair must have fired iff the set's own lengths differ by more than
   the threshold there: the set is the rule applied to its own values.
2. Decisions against the oracle.  For every examined pair the oracle's
   lengths at the same keys decide too.  Where the two decisions differ, the
   oracle's jump must lie within a band of the threshold that the two sides'
   length differences explain: | |dFLL_oracle| - thr | <= rel_band * thr +
   |e(k1)| + |e(k2)|, e = FLL - FLL_oracle at that key.  With FP64 stepping
   the e's are at rounding level, so the band is rel_band * thr.
3. Sample sets.  Every key in the symmetric difference between this set and
   the oracle's own refinement lies strictly inside a pair where the
   decisions differed (step 2): all differences descend from marginal
   decisions.
"""
from __future__ import annotations

import numpy as np


def base_keys(m: int, r: int, dims: int) -> np.ndarray:
    """Keys q B^r + B^r / 2 of the 2^(dims m) base cells (B = 2^dims)."""
    blk = (1 << dims) ** r
    return np.arange((1 << dims) ** m, dtype=np.int64) * blk + blk // 2


def replay(keys, start):
    """Pass-by-pass history of a final sample set from the start keys.

    Returns (reached keys, k1, k2, fired) over the distinct pairs examined."""
    keys = np.unique(np.asarray(keys, np.int64))
    cur = np.unique(np.asarray(start, np.int64))
    seen = set()
    K1, K2, F = [], [], []
    while True:
        k1, k2 = cur[:-1], cur[1:]
        c = (k2 - k1) >= 2
        k1, k2 = k1[c], k2[c]
        mid = (k1 + k2) // 2
        fired = np.isin(mid, keys)
        new = np.array([(a, b) not in seen for a, b in zip(k1.tolist(), k2.tolist())], dtype=bool)
        seen.update(zip(k1[new].tolist(), k2[new].tolist()))
        K1.append(k1[new])
        K2.append(k2[new])
        F.append(fired[new])
        if not fired.any():
            break
        cur = np.union1d(cur, mid[fired])
    cat = lambda xs, dt: np.concatenate(xs) if xs else np.zeros(0, dt)   # noqa: E731
    return cur, cat(K1, np.int64), cat(K2, np.int64), cat(F, bool)


def _at(keys, vals, k):
    i = np.searchsorted(keys, k)
    assert np.all(i < keys.size) and np.all(keys[np.minimum(i, keys.size - 1)] == k)
    return vals[i]


def check_refinement(keys, fll, fll_oracle, start, thr, keys_oracle=None, rel_band=1e-4):
    """Run the three checks above on a refined set (keys sorted, fll per key),
    with the oracle's lengths at the same keys (fll_oracle) and optionally the
    oracle's own refined key set.  Returns a dict of counts; raises
    AssertionError naming the first violation."""
    keys = np.asarray(keys, np.int64)
    fll = np.asarray(fll, np.float64)
    fo = np.asarray(fll_oracle, np.float64)
    assert np.all(np.diff(keys) > 0), "keys not strictly increasing"
    reached, k1, k2, fired = replay(keys, start)
    missing = np.setdiff1d(keys, reached)
    assert missing.size == 0, f"{missing.size} samples the rule cannot reach, e.g. {missing[:5]}"
    # 1. the set applies the rule to its own values
    jump = np.abs(_at(keys, fll, k1) - _at(keys, fll, k2))
    own = jump > thr
    bad = np.nonzero(own != fired)[0]
    assert bad.size == 0, (f"{bad.size} pairs decided against the set's own lengths, e.g. "
                           f"({k1[bad[0]]}, {k2[bad[0]]}) jump {jump[bad[0]]!r} fired {bool(fired[bad[0]])}")
    # 2. decisions against the oracle's lengths at the same keys
    jo = np.abs(_at(keys, fo, k1) - _at(keys, fo, k2))
    e1 = np.abs(_at(keys, fll, k1) - _at(keys, fo, k1))
    e2 = np.abs(_at(keys, fll, k2) - _at(keys, fo, k2))
    differ = (jo > thr) != fired
    band = rel_band * thr + e1 + e2
    margin = np.abs(jo - thr)
    wrong = differ & (margin > band)
    if wrong.any():
        i = np.nonzero(wrong)[0][0]
        raise AssertionError(f"{int(wrong.sum())} non-marginal decisions, e.g. pair ({k1[i]}, {k2[i]}): "
                             f"oracle jump {jo[i]!r}, thr {thr!r}, band {band[i]:.3e}, fired {bool(fired[i])}")
    out = dict(pairs=int(k1.size), fired=int(fired.sum()), differ=int(differ.sum()),
               differ_fp_level=int((differ & (margin <= rel_band * thr)).sum()))
    # 3. every difference of the sample sets descends from a differing decision
    if keys_oracle is not None:
        ko = np.asarray(keys_oracle, np.int64)
        sym = np.setxor1d(keys, ko)
        lo, hi = k1[differ], k2[differ]
        order = np.argsort(lo)
        lo, hi = lo[order], hi[order]
        # pairs where decisions differ are disjoint or nested intervals; a key
        # is covered if some interval with lo < key has hi > key
        run_hi = np.maximum.accumulate(hi) if hi.size else hi
        j = np.searchsorted(lo, sym, side="left") - 1
        covered = (j >= 0) & (run_hi[np.maximum(j, 0)] > sym) if hi.size else np.zeros(sym.size, bool)
        assert covered.all(), (f"{int((~covered).sum())} of {sym.size} differing samples do not descend from a "
                               f"marginal decision, e.g. {sym[~covered][:5]}")
        out["symmetric_difference"] = int(sym.size)
    return out
