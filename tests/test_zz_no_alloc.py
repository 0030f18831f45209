"""qsq_trace_noalloc (the entry point for callers that cannot allocate: its
scratch is a fixed library-owned device array) against qsq_trace with caller
scratch: two calls in a row, the second with fewer seeds, so the second call
runs on the array the first one left behind.  Same kernels, same arithmetic:
every output must agree bit for bit (NaN where the other has NaN)."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_field

pytestmark = pytest.mark.gpu


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_noalloc_matches_trace_on_two_calls():
    import torch

    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TracePlan, make_opts
    dev = torch.device("cuda:0")
    n = (65, 65, 33)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    fg = gpu_field(b, origin, spacing, storage="f32")
    h = min(spacing)
    opts = make_opts(1e-4, 1e-4, h_init=0.1 * h, h_max=h, step_dtype="f32")
    for count, seed in ((5000 + 17, 3), (1200 + 5, 4)):     # second call smaller, both ragged
        s = synth.random_seeds(seed, count)
        s[: count // 3, 2] = 0.0
        soa = torch.from_numpy(np.ascontiguousarray(s.T)).to(dev)
        print(f"noalloc vs trace: {count} seeds", flush=True)
        ref = _host(TracePlan(count, dev, want_steps=True).run(fg, soa, opts))
        got = _host(TracePlan(count, dev, want_steps=True, noalloc=True).run(fg, soa, opts))
        torch.cuda.synchronize()
        assert set(ref) == set(got)
        for k in ref:
            assert np.array_equal(ref[k], got[k], equal_nan=True), k
        moving = ref["steps"].sum(0) > 0
        assert moving.mean() > 0.5


def test_noalloc_rejects_too_many_seeds():
    import torch

    import paper_1609_00724_amd as q
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd.api import TracePlan, make_opts
    dev = torch.device("cuda:0")
    n = (9, 9, 9)
    b = synth.sample_charges(synth.point_charges(2, 4), n, dtype=np.float32)
    origin, spacing = synth.grid_geometry(n)
    fg = gpu_field(b, origin, spacing, storage="f32")
    plan = TracePlan(A.TRACE_NOALLOC_MAX_SEEDS + 1, dev, want=(), noalloc=True)
    soa = torch.zeros((3, A.TRACE_NOALLOC_MAX_SEEDS + 1), dtype=torch.float64, device=dev)
    with pytest.raises(A.QsqError, match="noalloc"):
        plan.run(fg, soa, make_opts(1e-4, 1e-4))
    assert q.lib.qsq_trace_scratch_bytes(A.TRACE_NOALLOC_MAX_SEEDS) <= 64 << 20
