"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qsq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qsq_[a-z0-9_]+)\s*\(", src)) - {"qsq_STATUS"})


@pytest.fixture(scope="module")
def qsq():
    import paper_1609_00724_amd as q
    return q


def test_exports_every_declared_symbol(qsq):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(qsq.lib, n), n
    from paper_1609_00724_amd import _abi
    assert sorted(_abi.EXPORTS) == names


def test_version_and_strings(qsq):
    from paper_1609_00724_amd import _abi as A
    assert qsq.lib.qsq_abi_version() == 1
    for code in range(12):
        assert qsq.lib.qsq_status_string(code) != b"unknown code"
    for code in (A.ERR_INVALID_ARG, A.ERR_UNSUPPORTED, A.ERR_WORKSPACE_TOO_SMALL, A.ERR_HIP, A.ERR_COUNT_OVERFLOW):
        assert qsq.lib.qsq_status_string(code) != b"unknown code"


def test_sizes(qsq):
    from paper_1609_00724_amd import _abi as A
    g = A.Grid()
    g.n[:] = (256, 256, 128)
    assert qsq.lib.qsq_field_bytes(C.byref(g), A.F32) == 256 * 256 * 128 * 16
    assert qsq.lib.qsq_field_bytes(C.byref(g), A.F64) == 256 * 256 * 128 * 32
    assert qsq.lib.qsq_trace_scratch_bytes(1000) >= 1000 * 2 * (11 * 8 + 8)
    d = A.MapDesc()
    d.base_level, d.refine_levels, d.out_level = 10, 2, 10
    assert qsq.lib.qsq_qmap_scratch_bytes(C.byref(d), 4 ** 11) > 4 ** 11 * 24
    assert qsq.lib.qsq_qmap_scratch_bytes(C.byref(d), 0) == 0


def _fake(n):
    return C.c_void_p(0x100000 * n)   # never dereferenced: validation fails first


def test_invalid_arguments_rejected_before_launch(qsq):
    from paper_1609_00724_amd import _abi as A
    L = qsq.lib
    g = A.Grid()
    g.n[:] = (8, 8, 1)          # n < 2
    g.spacing[:] = (0.1, 0.1, 0.1)
    out = A.FieldDesc()
    rc = L.qsq_field_init(C.byref(g), _fake(1), _fake(2), _fake(3), A.F32, A.F32, A.INTERP_PAPER,
                          _fake(4), 1 << 30, None, C.byref(out))
    assert rc == A.ERR_INVALID_ARG and b"n[2]" in L.qsq_last_error()
    g.n[:] = (8, 8, 8)
    rc = L.qsq_field_init(C.byref(g), _fake(1), _fake(2), _fake(3), A.F32, A.F32, A.INTERP_PAPER,
                          _fake(4), 100, None, C.byref(out))
    assert rc == A.ERR_WORKSPACE_TOO_SMALL
    rc = L.qsq_field_init(C.byref(g), _fake(1), _fake(2), _fake(3), A.F32, A.BF16, A.INTERP_PAPER,
                          _fake(4), 1 << 30, None, C.byref(out))
    assert rc == A.ERR_UNSUPPORTED
    # a field descriptor that validates, used with bad trace options
    f = A.FieldDesc()
    f.grid = g
    f.storage, f.mode, f.nodes = A.F32, A.INTERP_PAPER, _fake(5)
    f.bytes = L.qsq_field_bytes(C.byref(g), A.F32)
    o = A.TraceOpts()
    o.rtol, o.atol = 0.0, 1e-6
    t = A.TraceOut()
    t.status = _fake(6)
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
        A.ERR_INVALID_ARG
    o.rtol = 1e-6
    o.step_dtype = A.BF16
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
        A.ERR_UNSUPPORTED
    o.step_dtype = A.F32
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 16, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    assert L.qsq_trace(C.byref(f), _fake(7), (1 << 30) + 1, C.byref(o), C.byref(t), _fake(8), 1 << 20,
                       None) == A.ERR_COUNT_OVERFLOW
    t.status = None
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
        A.ERR_INVALID_ARG
    assert L.qsq_trace(None, _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
        A.ERR_INVALID_ARG
    # maps
    d = A.MapDesc()
    d.x0, d.x1, d.y0, d.y1 = -1, 1, -1, 1
    d.base_level, d.refine_levels, d.out_level, d.threshold = 4, 2, 7, 0.1
    mo = A.MapOut()
    assert L.qsq_qmap(C.byref(f), C.byref(d), C.byref(o), C.byref(mo), _fake(9), 1 << 30, None) == \
        A.ERR_INVALID_ARG
    # FLEDGE: overlapping buffers, bad rank
    shp = (C.c_int64 * 2)(16, 16)
    assert L.qsq_fledge(_fake(1), 2, shp, C.c_void_p(0x100000 + 64), None) == A.ERR_INVALID_ARG
    assert L.qsq_fledge(_fake(1), 4, shp, _fake(2), None) == A.ERR_INVALID_ARG
    assert L.qsq_hilbert2_d2xy(0, _fake(1), 4, _fake(2), _fake(3), None) == A.ERR_INVALID_ARG
    n = C.c_int64()
    ms = C.c_double()
    assert L.qsq_profile_read(7, C.byref(n), C.byref(ms)) == A.ERR_INVALID_ARG
