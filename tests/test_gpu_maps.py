"""GPU parity of the map-level path (QSL Squasher Sect. 3.6) against the oracle:
Sobel FLEDGE, Hilbert ordering, FLL-jump refinement and the array converter,
on a small map and on the full photospheric map the benchmark times."""
import numpy as np
import pytest

import synth
from gpu_util import check_lines, parity, torch_dev
from refine_check import base_keys, check_refinement

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------------------
# FLEDGE and Hilbert (bit-exact / FP32 rounding)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (3, 700), (257, 129), (33, 17, 9)])
def test_fledge_vs_oracle(oracle_mod, shape):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    f = synth.rng(8).normal(size=shape).astype(np.float32)
    g = q.fledge(torch.from_numpy(f).to(dev)).cpu().numpy()
    o = oracle_mod.sobel_magnitude(f.astype(np.float64))
    assert np.allclose(g, o, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("L", [1, 2, 5, 10, 12])
def test_hilbert_vs_oracle_all(oracle_mod, L):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    d = np.arange(4 ** L, dtype=np.int64)
    x, y = q.hilbert2_d2xy(L, torch.from_numpy(d).to(dev))
    xo, yo = oracle_mod.hilbert2_d2xy(L, d)
    assert np.array_equal(x.cpu().numpy(), xo) and np.array_equal(y.cpu().numpy(), yo)
    dd = q.hilbert2_xy2d(L, x, y).cpu().numpy()
    assert np.array_equal(dd, d)


@pytest.mark.parametrize("L", [16, 24, 31])
def test_hilbert_vs_oracle_sampled(oracle_mod, L):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    d = synth.rng(L).integers(0, 4 ** L, size=5000, dtype=np.int64)
    x, y = q.hilbert2_d2xy(L, torch.from_numpy(d).to(dev))
    xo, yo = oracle_mod.hilbert2_d2xy(L, d)
    assert np.array_equal(x.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, xo)
    assert np.array_equal(y.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, yo)


# ---------------------------------------------------------------------------
# slice maps with refinement
# ---------------------------------------------------------------------------

CHARGES = synth.point_charges(2, 4)
TOL = 1e-4   # stepping tolerance of the photospheric map workload


@pytest.fixture(scope="module")
def c2(oracle_mod):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    w = synth.charges_c2()
    b = w["b"]
    fg = q.field_init(*(torch.from_numpy(c).to(dev) for c in b), w["origin"], w["spacing"], storage="f32")
    fo = oracle_mod.Field.grid(*(c.astype(np.float64) for c in b), w["origin"], w["spacing"], store="f32")
    return dict(w=w, fg=fg, fo=fo, h=min(w["spacing"]))


def _run_map(c2, m, r, thr, out_level, capacity, step_dtype="f32", batch=0):
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec
    torch, dev = torch_dev()
    spec = MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, out_level, thr, batch)
    res = q.qmap(c2["fg"], spec, capacity, rtol=TOL, atol=TOL, h_init=0.1 * c2["h"], h_max=c2["h"],
                 step_dtype=step_dtype)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}
    return out


def _positions(oracle_mod, m, r, keys):
    plane = oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)
    blk = 4 ** r
    base = keys % blk == blk // 2
    pos = np.empty((keys.size, 3))
    q = keys[base] // blk
    ix, iy = oracle_mod.hilbert2_d2xy(m, q)
    pos[base] = plane.centres(m, ix, iy)
    if (~base).any():
        pos[~base] = oracle_mod.key_positions(plane, m, r, keys[~base])
    return pos, base


def _check_complete(res, thr):
    k, f = res["keys"], res["fll"]
    assert np.all(np.diff(k) > 0)
    open_pair = (np.diff(k) >= 2) & (np.abs(np.diff(f)) > thr)
    assert not open_pair.any()


def _oracle_trace(oracle_mod, c2, pts):
    return oracle_mod.trace(c2["fo"], pts, rtol=TOL, atol=TOL, h_init=0.1 * c2["h"], h_max=c2["h"])


def _sample_parity(oracle_mod, c2, res, idx, m, r, strict=False):
    pos, _ = _positions(oracle_mod, m, r, res["keys"][idx])
    o = _oracle_trace(oracle_mod, c2, pos)
    g = dict(status=res["status"][idx], q_perp=res["q_perp"][idx], fll=res["fll"][idx],
             fp_fwd=np.zeros((idx.size, 3)), fp_bwd=np.zeros((idx.size, 3)))
    o2 = dict(o)
    o2["fp_fwd"] = np.zeros((idx.size, 3))
    o2["fp_bwd"] = np.zeros((idx.size, 3))
    check_lines(parity(g, o2), o, strict=strict)
    return o


@pytest.mark.parametrize("step_dtype", ["f32", "f64"])
def test_small_map_vs_oracle(oracle_mod, c2, step_dtype):
    m, r, thr = 6, 2, 0.02
    res = _run_map(c2, m, r, thr, m + r, 4 ** (m + r), step_dtype)
    n = res["count"]
    assert res["overflow"] == 0 and n > 4 ** m
    _check_complete(res, thr)
    # every sample re-traced by the oracle at the same key position
    o = _sample_parity(oracle_mod, c2, res, np.arange(n), m, r, strict=step_dtype == "f64")
    # the oracle's own refinement reaches the same sample set (up to marginal jumps)
    plane = oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)

    def fn(p):
        t = _oracle_trace(oracle_mod, c2, p)
        return {"fll": t["fll"], "q": t["q_perp"]}

    ok, ov, _ = oracle_mod.refine_slice(plane, m, r, thr, fn)
    # every decision follows the rule on the map's own lengths; where it
    # differs from the oracle's decision on the oracle's lengths at the same
    # keys, the jump is within the band the length differences explain, and
    # every sample the two sets do not share descends from such a decision
    out = check_refinement(res["keys"][:n], res["fll"][:n], o["fll"], base_keys(m, r, 2), thr, keys_oracle=ok)
    print("refinement decisions:", out)
    # converter: the oracle's converter applied to the GPU's samples
    want_q = oracle_mod.convert_to_grid(res["keys"], res["q_perp"], m, r, m + r, log_interp=True)
    want_f = oracle_mod.convert_to_grid(res["keys"], res["fll"], m, r, m + r, log_interp=False)
    assert np.allclose(res["q_grid"], want_q, rtol=2e-6, equal_nan=True)
    assert np.allclose(res["fll_grid"], want_f, rtol=2e-6, atol=1e-6)
    # FLEDGE of the base length map
    base = res["keys"] % 16 == 8
    ix, iy = oracle_mod.hilbert2_d2xy(m, res["keys"][base] // 16)
    img = np.zeros((1 << m, 1 << m))
    img[iy, ix] = res["fll"][base]
    assert np.allclose(res["fledge"], oracle_mod.sobel_magnitude(img.astype(np.float32).astype(np.float64)),
                       rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("step_dtype", ["f32", "f64"])
def test_map_with_proposals(oracle_mod, c2, step_dtype):
    """Proposed base pixels get every finest cell as a sample before the
    FLL-jump rule runs; the rule then refines the rest (fallback).  Same result
    as the oracle's refinement from the same merged sample set."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec
    torch, dev = torch_dev()
    m, r, thr = 6, 2, 0.02
    picked = synth.rng(9).choice(4 ** m, size=300, replace=False)
    prop = torch.zeros(4 ** m, dtype=torch.uint8, device=dev)
    prop[torch.from_numpy(picked).to(dev)] = 1
    spec = MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m + r, thr, 0, propose=prop)
    res = q.qmap(c2["fg"], spec, 4 ** (m + r), rtol=TOL, atol=TOL, h_init=0.1 * c2["h"], h_max=c2["h"],
                 step_dtype=step_dtype)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}
    n = res["count"]
    assert res["overflow"] == 0
    _check_complete(res, thr)
    base = np.arange(4 ** m) * 16 + 8
    extra = np.setdiff1d((picked[:, None] * 16 + np.arange(16)[None, :]).ravel(), base)
    assert np.all(np.isin(extra, res["keys"]))
    o = _sample_parity(oracle_mod, c2, res, np.arange(n), m, r, strict=step_dtype == "f64")
    plane = oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)

    def fn(p):
        t = _oracle_trace(oracle_mod, c2, p)
        return {"fll": t["fll"], "q": t["q_perp"]}

    ok, _, _ = oracle_mod.refine_slice(plane, m, r, thr, fn, extra_keys=extra)
    start = np.union1d(base, extra)
    out = check_refinement(res["keys"][:n], res["fll"][:n], o["fll"], start, thr, keys_oracle=ok)
    print("refinement decisions:", out)
    # without proposals the same call is the plain map, and it holds fewer samples
    plain = _run_map(c2, m, r, thr, m + r, 4 ** (m + r), step_dtype)
    assert plain["count"] < n


def test_map_without_refinement(oracle_mod, c2):
    """refine_levels = 0: the base lattice only, key q + 0 (B^0 / 2 = 0 with
    integer halving is the cell itself), every sample a base sample."""
    m = 6
    res = _run_map(c2, m, 0, 0.02, m, 4 ** m)
    assert res["count"] == 4 ** m and res["overflow"] == 0
    assert np.array_equal(res["keys"], np.arange(4 ** m))
    _sample_parity(oracle_mod, c2, res, np.arange(0, 4 ** m, 7), m, 0)


@pytest.mark.parametrize("r,tight", [(2, False), (3, False), (2, True), (3, True)])
def test_refine_batches_give_identical_maps(c2, r, tight):
    """Deciding several refinement levels per device round (tracing every key
    those levels could insert, then applying the rule) keeps exactly the
    samples of the pass-by-pass rule: every batch size gives the same arrays.
    With the full finest lattice as capacity one round can take every level;
    with a capacity of exactly the refined sample count the rounds are planned
    for fewer levels each, so rounds run with fewer levels than the batch or
    as no-ops at the end; the arrays stay the same."""
    m, thr = 6, 0.02
    ref = _run_map(c2, m, r, thr, m + r, 4 ** (m + r), batch=1)
    assert ref["count"] > 4 ** m and ref["overflow"] == 0
    cap = 4 ** (m + r)
    if tight:
        cap = ref["count"]
        assert cap < 15 * 4 ** m            # the first round cannot be planned for 4 levels
        tight_ref = _run_map(c2, m, r, thr, m + r, cap, batch=1)
        assert tight_ref["overflow"] == 0
        for k in ("keys", "fll", "q_perp", "status", "q_grid"):
            assert np.array_equal(tight_ref[k], ref[k], equal_nan=True), k
    for b in (2, 3, 4, 5):
        res = _run_map(c2, m, r, thr, m + r, cap, batch=b)
        assert res["overflow"] == 0, b
        assert res["count"] == ref["count"], b
        for k in ("keys", "fll", "q_perp", "status"):
            assert np.array_equal(res[k], ref[k], equal_nan=True), (b, k)
        assert np.array_equal(res["q_grid"], ref["q_grid"], equal_nan=True)


@pytest.mark.parametrize("dims", [2, 3])
def test_kept_sample_steps(oracle_mod, c2, dims):
    """Per-sample step attempts of a refined map (the method's own work): with
    one level per round every traced line is kept, so they sum to the traced
    attempts; with four speculative levels per round the kept samples are the
    same, carry the same attempts, and sum to less than what was traced; and
    each equals the attempts of its line re-traced on its own at the sample's
    position (forward + backward)."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec, QMapPlan, VolumeSpec, make_opts
    torch, dev = torch_dev()
    h = c2["h"]
    m, r, thr = (6, 2, 0.02) if dims == 2 else (4, 2, 0.02)
    opts = make_opts(TOL, TOL, h_init=0.1 * h, h_max=h, step_dtype="f32")
    got = {}
    for batch in (1, 4):
        spec = (MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, thr, batch) if dims == 2
                else VolumeSpec(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, m, r, m, thr, batch))
        plan = QMapPlan(spec, (2 ** dims) ** (m + r), dev, want_steps=True)
        plan.run(c2["fg"], opts)
        torch.cuda.synchronize()
        res = plan.result()
        got[batch] = (res["keys"].cpu().numpy(), res["steps"].cpu().numpy().astype(np.int64),
                      int(plan.work[0].item()))
    k1, s1, w1 = got[1]
    k4, s4, w4 = got[4]
    print(f"dims {dims}: kept attempts {s1.sum()}, traced at 1 level/round {w1}, at 4 levels/round {w4}")
    assert np.array_equal(k1, k4) and np.array_equal(s1, s4)
    assert s1.sum() == w1 and s4.sum() < w4
    # re-trace a sample of positions alone
    blk = (2 ** dims) ** r
    idx = np.arange(0, k1.size, max(1, k1.size // 500))
    k = k1[idx]
    base = k % blk == blk // 2
    pos = np.empty((idx.size, 3))
    if dims == 2:
        plane = oracle_mod.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0)
        pos[base] = plane.centres(m, *oracle_mod.hilbert2_d2xy(m, k[base] // blk))
        pos[~base] = oracle_mod.key_positions(plane, m, r, k[~base])
    else:
        box = oracle_mod.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0)
        pos[base] = box.centres(m, *oracle_mod.hilbert3_d2xyz(m, k[base] // blk))
        pos[~base] = oracle_mod.key_positions(box, m, r, k[~base])
    t = q.trace(c2["fg"], torch.from_numpy(pos).to(dev), rtol=TOL, atol=TOL, h_init=0.1 * h, h_max=h,
                step_dtype="f32", want_steps=True)
    torch.cuda.synchronize()
    alone = t["steps"].cpu().numpy().astype(np.int64).sum(0)
    assert np.array_equal(alone, s1[idx])


def _keys_of_points(O, region, L, pts):
    """Finest-level curve keys of sample positions (cell centres)."""
    if region.dims == 2:
        ext = [(region.x0, region.x1), (region.y0, region.y1)]
        cols = [pts[:, 0], pts[:, 1]]
    else:
        ext = [(region.lo[a], region.hi[a]) for a in range(3)]
        cols = [pts[:, a] for a in range(3)]
    n = 1 << L
    cells = [np.floor((c - lo) / (hi - lo) * n).astype(np.int64) for c, (lo, hi) in zip(cols, ext)]
    return O._curve_index(region, L, cells)


@pytest.mark.parametrize("dims,shift", [(2, 6), (2, 37), (3, 3)])
def test_shifted_repass_vs_oracle(oracle_mod, c2, dims, shift):
    """The shifted-curve re-pass (Sect. 3.6, last paragraph) on the device,
    FP64 stepping: (1) the oracle's refine_shifted replayed on the GPU's own
    sample values (its sample function looks each requested key up among the
    GPU's samples) asks for exactly the GPU's keys and ends with the same set,
    so every decision of both passes in every cycle matches the rule; (2) each
    sample's length and Q match the oracle traced at its position; (3) the
    re-pass adds samples the plain rule does not; (4) the set is complete in
    both orders (no gap left that either pass would fire)."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd.api import MapSpec, QMapPlan, VolumeSpec, make_opts
    O = oracle_mod
    torch, dev = torch_dev()
    h = c2["h"]
    m, r, thr = (6, 2, 0.02) if dims == 2 else (4, 2, 0.02)
    L = m + r
    opts = make_opts(1e-6, 1e-6, h_init=0.1 * h, h_max=h, step_dtype="f64")
    res = {}
    for sh in (0, shift):
        spec = (MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, m, r, m, thr, 1, shift=sh) if dims == 2
                else VolumeSpec(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, m, r, m, thr, 1, shift=sh))
        plan = QMapPlan(spec, (2 ** dims) ** L, dev)
        plan.run(c2["fg"], opts)
        torch.cuda.synchronize()
        out = plan.result()
        res[sh] = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    g = res[shift]
    n = g["count"]
    assert g["overflow"] == 0, g["overflow"]
    keys = g["keys"][:n]
    assert np.all(np.diff(keys) > 0)
    region = (O.SlicePlane(0.0, -1.0, 1.0, -1.0, 1.0) if dims == 2 else O.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0))
    lookup = {int(k): i for i, k in enumerate(keys)}
    missing = []
    calls = []

    def from_gpu(pts):
        # the first call is the base lattice (key q B^r + B^r / 2 at the centre
        # of base cell q, which is a corner of finest cells); later calls ask
        # for finest-cell centres
        ks = O.base_samples(region, m, r)[0] if not calls else _keys_of_points(O, region, L, pts)
        calls.append(len(ks))
        idx = np.array([lookup.get(int(k), -1) for k in ks])
        missing.extend(int(k) for k in ks[idx < 0])
        idx = np.maximum(idx, 0)
        return {"fll": g["fll"][:n][idx], "q": g["q_perp"][:n][idx]}

    rk, _, cycles = O.refine_shifted(region, m, r, thr, from_gpu, shift=shift, max_cycles=48)
    print(f"dims {dims} shift {shift}: {n} samples (plain rule {res[0]['count']}), oracle replay {rk.size} "
          f"in {cycles} cycles, keys the GPU lacks {len(missing)}")
    assert not missing
    assert np.array_equal(rk, keys)
    assert n > res[0]["count"]
    # values: the oracle traced at every 8th sample position
    idx = np.arange(0, n, 8)
    k = keys[idx]
    blk = (2 ** dims) ** r
    base = k % blk == blk // 2          # base samples sit at their base cell's centre
    pos = np.empty((idx.size, 3))
    pos[base] = region.centres(m, *region.cells(m, k[base] // blk))
    pos[~base] = O.key_positions(region, m, r, k[~base])
    o = O.trace(c2["fo"], pos, rtol=1e-6, atol=1e-6, h_init=0.1 * h, h_max=h)
    same = g["status"][:n][idx] == o["status"]
    assert same.mean() > 0.995
    assert np.all(np.abs(g["fll"][:n][idx][same] - o["fll"][same]) <= 1e-4 * np.maximum(o["fll"][same], 1e-12))
    # completeness in both orders
    gap = np.diff(keys) >= 2
    jump = np.abs(np.diff(g["fll"][:n])) > thr
    assert not np.any(gap & jump)


def test_volume_map_cell_records_identical(c2):
    """A refined volume map stepped with the cell records (gather 4) equals the
    map stepped with the register cell cache (over node, brick or direction
    records), with direct loads, and with another gather for the refinement
    rounds than for the base lattice, bit for bit: the same corner values
    reach the same arithmetic."""
    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import QMapPlan, VolumeSpec, make_opts
    torch, dev = torch_dev()
    h = c2["h"]
    fg = c2["fg"]
    if fg.cells_ws is None:
        fg.add_cells()
    if fg.bricks_ws is None:
        fg.add_bricks()
    if fg.dirs_ws is None:
        fg.add_cell_dirs()
    spec = VolumeSpec(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, 5, 2, 6, 0.02, 1)
    out = []
    for gather, parts, rg in ((A.GATHER_CELLS, False, 0), (A.GATHER_REGS, False, 0), (A.GATHER_DIRECT, False, 0),
                              (A.GATHER_REGS, True, 0), (A.GATHER_DIRECT, True, 0), (A.GATHER_BRICKS, False, 0),
                              (A.GATHER_BRICKS, True, 0), (A.GATHER_DIRS, False, 0),
                              (A.GATHER_BRICKS, False, A.GATHER_DIRS), (A.GATHER_DIRECT, True, A.GATHER_DIRS)):
        plan = QMapPlan(spec, 8 ** 7, dev, want_steps=True)
        opts = make_opts(1e-2, 1e-2, h_init=0.1 * h, h_max=4 * h, step_dtype="f32",
                         launch=A.launch_word(1, 256, gather, parts, refine_gather=rg))
        plan.run(fg, opts)
        torch.cuda.synchronize()
        r = plan.result()
        out.append({k: v.clone() for k, v in r.items() if hasattr(v, "clone")})
    for other in out[1:]:
        for k in out[0]:
            assert torch.equal(torch.nan_to_num(out[0][k].double(), nan=-1.0),
                               torch.nan_to_num(other[k].double(), nan=-1.0)), k


def test_capacity_overflow_is_flagged(c2):
    m, r = 5, 2
    res = _run_map(c2, m, r, 0.0, m, 4 ** m + 10)
    assert res["overflow"] == 1 and res["count"] == 4 ** m + 10
    assert np.all(np.diff(res["keys"]) > 0)


def test_map_graph_replay_matches_eager(c2):
    """The whole map call (base lattice, device-decided refinement rounds,
    conversion) captured in a HIP graph: every replay, with eager work of
    another map between the replays, reproduces the eager map bit for bit."""
    from paper_1609_00724_amd.api import MapSpec, QMapPlan, make_opts
    torch, dev = torch_dev()
    opts = make_opts(TOL, TOL, h_init=0.1 * c2["h"], h_max=c2["h"], step_dtype="f32")
    plan = QMapPlan(MapSpec(0.0, -1.0, 1.0, -1.0, 1.0, 6, 2, 8, 0.02, 0), 4 ** 6 * 16, dev)
    other = QMapPlan(MapSpec(0.0, -0.5, 0.5, -0.5, 0.5, 5, 1, 6, 0.02, 0), 4 ** 5 * 8, dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.run(c2["fg"], opts, s)
    torch.cuda.synchronize()
    keys = ("keys", "fll", "q_perp", "status", "q_grid", "fll_grid", "fledge")
    first = plan.result()
    ref = {k: first[k].clone() for k in keys}
    count = first["count"]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.run(c2["fg"], opts, s)
    torch.cuda.synchronize()

    def same(a, b):
        if a.is_floating_point():
            return torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))
        return torch.equal(a, b)

    for _ in range(3):
        graph.replay()
        torch.cuda.synchronize()
        res = plan.result()
        assert res["count"] == count
        for k in keys:
            assert same(res[k], ref[k]), k
        with torch.cuda.stream(s):
            other.run(c2["fg"], opts, s)
        torch.cuda.synchronize()


@pytest.mark.parametrize("step_dtype", ["f32", "f64"])
def test_full_photospheric_map_sampled(oracle_mod, c2, step_dtype):
    """The benchmark's workload: 1024^2 base map with 4x (two-level) refinement;
    oracle checks on a sample of lines, converter cells, and the whole FLEDGE.
    FP64 stepping must match the oracle on every sampled line."""
    m, r, thr = 10, 2, 0.02
    res = _run_map(c2, m, r, thr, m, 4 ** (m + r), step_dtype)
    n = res["count"]
    assert res["overflow"] == 0 and n > 4 ** m
    _check_complete(res, thr)
    g = synth.rng(77)
    idx = np.sort(g.choice(n, size=1500, replace=False))
    _sample_parity(oracle_mod, c2, res, idx, m, r, strict=step_dtype == "f64")
    cells = g.choice(4 ** m, size=300, replace=False)
    want = oracle_mod.convert_to_grid(res["keys"], res["q_perp"], m, r, m, log_interp=True, cells=cells)
    cx, cy = oracle_mod.hilbert2_d2xy(m, cells)
    assert np.allclose(res["q_grid"][cy, cx], want, rtol=2e-6, equal_nan=True)
    base = res["keys"] % 16 == 8
    ix, iy = oracle_mod.hilbert2_d2xy(m, res["keys"][base] // 16)
    img = np.zeros((1 << m, 1 << m))
    img[iy, ix] = res["fll"][base]
    assert np.allclose(res["fledge"], oracle_mod.sobel_magnitude(img.astype(np.float32).astype(np.float64)),
                       rtol=1e-5, atol=1e-5)


# ---------------------------------------------------------------------------
# volumes (3D Hilbert refinement, 3D converter and FLEDGE)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("b", [1, 2, 4, 6])
def test_hilbert3_vs_oracle_all(oracle_mod, b):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    d = np.arange(8 ** b, dtype=np.int64)
    x, y, z = q.hilbert3_d2xyz(b, torch.from_numpy(d).to(dev))
    xo, yo, zo = oracle_mod.hilbert3_d2xyz(b, d)
    assert np.array_equal(x.cpu().numpy(), xo) and np.array_equal(y.cpu().numpy(), yo)
    assert np.array_equal(z.cpu().numpy(), zo)
    assert np.array_equal(q.hilbert3_xyz2d(b, x, y, z).cpu().numpy(), d)


@pytest.mark.parametrize("b", [10, 21])
def test_hilbert3_vs_oracle_sampled(oracle_mod, b):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    d = synth.rng(b).integers(0, 8 ** b, size=5000, dtype=np.int64)
    x, y, z = q.hilbert3_d2xyz(b, torch.from_numpy(d).to(dev))
    xo, yo, zo = oracle_mod.hilbert3_d2xyz(b, d)
    for g_, o_ in ((x, xo), (y, yo), (z, zo)):
        assert np.array_equal(g_.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, o_)


BOX = (-1.0, 1.0, -1.0, 1.0, 0.0, 1.0)


def _run_vmap(c2, m, r, thr, out_level, capacity, step_dtype="f32", batch=0):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    spec = q.VolumeSpec(*BOX, m, r, out_level, thr, batch)
    res = q.qmap(c2["fg"], spec, capacity, rtol=TOL, atol=TOL, h_init=0.1 * c2["h"], h_max=c2["h"],
                 step_dtype=step_dtype)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


def _vpositions(oracle_mod, m, r, keys):
    box = oracle_mod.VolumeBox(*BOX)
    blk = 8 ** r
    base = keys % blk == blk // 2
    pos = np.empty((keys.size, 3))
    pos[base] = box.centres(m, *oracle_mod.hilbert3_d2xyz(m, keys[base] // blk))
    if (~base).any():
        pos[~base] = oracle_mod.key_positions(box, m, r, keys[~base])
    return pos, base


@pytest.mark.parametrize("step_dtype", ["f32", "f64"])
def test_volume_map_vs_oracle(oracle_mod, c2, step_dtype):
    m, r, thr = 4, 2, 0.02
    res = _run_vmap(c2, m, r, thr, m + 1, 8 ** (m + 1) * 4, step_dtype)   # the oracle's refinement keeps ~101K
    n = res["count"]
    assert res["overflow"] == 0 and n > 8 ** m
    _check_complete(res, thr)
    pos, base = _vpositions(oracle_mod, m, r, res["keys"])
    o = _oracle_trace(oracle_mod, c2, pos)
    g = dict(status=res["status"], q_perp=res["q_perp"], fll=res["fll"],
             fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))
    o2 = dict(o, fp_fwd=np.zeros((n, 3)), fp_bwd=np.zeros((n, 3)))
    check_lines(parity(g, o2), o, strict=step_dtype == "f64")
    # the oracle's own volume refinement reaches the same sample set
    box = oracle_mod.VolumeBox(*BOX)

    def fn(p):
        t = _oracle_trace(oracle_mod, c2, p)
        return {"fll": t["fll"], "q": t["q_perp"]}

    ok, _, passes = oracle_mod.refine_slice(box, m, r, thr, fn)
    assert passes <= 3 * r
    out = check_refinement(res["keys"][:n], res["fll"][:n], o["fll"], base_keys(m, r, 3), thr, keys_oracle=ok)
    print("refinement decisions:", out)
    # converter at level m + 1 on sampled cells, and the 3D FLEDGE of the base lengths
    cells = synth.rng(5).choice(8 ** (m + 1), size=300, replace=False)
    want = oracle_mod.convert_to_grid(res["keys"], res["q_perp"], m, r, m + 1, log_interp=True,
                                      cells=cells, dims=3)
    cx, cy, cz = oracle_mod.hilbert3_d2xyz(m + 1, cells)
    assert np.allclose(res["q_grid"][cz, cy, cx], want, rtol=2e-6, equal_nan=True)
    bx, by, bz = oracle_mod.hilbert3_d2xyz(m, res["keys"][base] // 64)
    img = np.zeros((1 << m,) * 3)
    img[bz, by, bx] = res["fll"][base]
    assert np.allclose(res["fledge"], oracle_mod.sobel_magnitude(img.astype(np.float32).astype(np.float64)),
                       rtol=1e-5, atol=1e-5)


def test_volume_refine_batches_identical(c2):
    m, r, thr = 3, 2, 0.02
    ref = _run_vmap(c2, m, r, thr, m + r, 8 ** (m + r), batch=1)
    assert ref["count"] > 8 ** m
    for b in (3, 4, 5):
        res = _run_vmap(c2, m, r, thr, m + r, 8 ** (m + r), batch=b)
        for k in ("keys", "fll", "q_perp", "status"):
            assert np.array_equal(res[k], ref[k], equal_nan=True), (b, k)


def test_full_rope_volume_sampled(oracle_mod):
    """The benchmark's volume at full size: flux rope over a 6-charge
    background on a 384x384x256 FP32 grid, 256^3 base cells and two levels of
    3D FLL-jump refinement, FP32 stepping at tol 1e-4 with the LDS cell cache.
    The refinement is complete (no curve-successive pair left open), and 400
    sampled lines match the FP64 oracle on the same FP32-rounded field within
    the FP32 gates; the 3D FLEDGE on a sampled block of the base lattice."""
    import paper_1609_00724_amd as q
    from gpu_util import check_fp32
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import QMapPlan, make_opts
    torch, dev = torch_dev()
    w = synth.flux_rope_c4(device=dev)
    b = [torch.from_numpy(c).to(dev) for c in w["b"]]
    fg = q.field_init(*b, w["origin"], w["spacing"], storage="f32")
    del b
    h = min(w["spacing"])
    m, r, thr = 8, 2, 0.02
    spec = q.VolumeSpec(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, m, r, m, thr, 0)
    plan = QMapPlan(spec, 8 ** m * 4, dev)
    opts = make_opts(TOL, TOL, h_init=0.1 * h, h_max=h, step_dtype="f32", launch=A.launch_word(8, 128, 2))
    plan.run(fg, opts)
    torch.cuda.synchronize()
    res = plan.result()
    n = res["count"]
    assert res["overflow"] == 0 and n > 8 ** m
    keys = res["keys"].cpu().numpy()
    fll = res["fll"].cpu().numpy()
    _check_complete(dict(keys=keys, fll=fll), thr)
    g = synth.rng(81)
    idx = np.sort(g.choice(n, size=400, replace=False))
    box = oracle_mod.VolumeBox(-1.0, 1.0, -1.0, 1.0, 0.0, 1.0)
    blk = 8 ** r
    k = keys[idx]
    base = k % blk == blk // 2
    pos = np.empty((idx.size, 3))
    pos[base] = box.centres(m, *oracle_mod.hilbert3_d2xyz(m, k[base] // blk))
    pos[~base] = oracle_mod.key_positions(box, m, r, k[~base])
    fo = oracle_mod.Field.grid(*(np.asarray(c, np.float64) for c in w["b"]), w["origin"], w["spacing"], store="f32")
    kw = dict(rtol=TOL, atol=TOL, h_init=0.1 * h, h_max=h)
    o = oracle_mod.trace(fo, pos, **kw)
    ref = oracle_mod.trace(fo, pos, **dict(kw, rtol=1e-10, atol=1e-10))
    gg = dict(status=res["status"].cpu().numpy()[idx], q_perp=res["q_perp"].cpu().numpy()[idx], fll=fll[idx],
              fp_fwd=np.zeros((idx.size, 3)), fp_bwd=np.zeros((idx.size, 3)))
    oz = dict(o, fp_fwd=np.zeros((idx.size, 3)), fp_bwd=np.zeros((idx.size, 3)))
    check_fp32(parity(gg, oz), gg, oz, ref)
    # FLEDGE of the base lengths on an interior block (the Sobel stencil only
    # reaches one cell beyond the block)
    allbase = keys % blk == blk // 2
    bx, by, bz = oracle_mod.hilbert3_d2xyz(m, keys[allbase] // blk)
    img = np.zeros((1 << m,) * 3)
    img[bz, by, bx] = fll[allbase]
    lo, hi = 100, 132
    sub = img[lo - 1:hi + 1, lo - 1:hi + 1, lo - 1:hi + 1].astype(np.float32).astype(np.float64)
    want = oracle_mod.sobel_magnitude(sub)[1:-1, 1:-1, 1:-1]
    got = res["fledge"].cpu().numpy()[lo:hi, lo:hi, lo:hi]
    assert np.allclose(got, want, rtol=1e-5, atol=1e-5)
