"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="qsq.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
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
    cnn = _declared("qsq_cnn.h")
    for n in cnn:
        assert hasattr(qsq.lib, n), n
    assert sorted(_abi.CNN_EXPORTS) == cnn
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["qsq.h", "qsq_cnn.h"]


def test_version_and_strings(qsq):
    from paper_1609_00724_amd import _abi as A
    assert qsq.lib.qsq_abi_version() == 4
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
    assert qsq.lib.qsq_field_bytes(C.byref(g), A.BF16) == 256 * 256 * 128 * 8
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
    rc = L.qsq_field_init(C.byref(g), _fake(1), _fake(2), _fake(3), A.F32, 7, A.INTERP_PAPER,
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
    for bad in (0x30, 0x2000, 0x1c0, 0x1c00):   # workgroup code 3; bits above the word; gather 7; refine gather 7
        o.launch = bad
        assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
            A.ERR_INVALID_ARG
        assert b"launch word" in L.qsq_last_error()
    o.launch = A.launch_word(2, 64, A.GATHER_REGS)   # valid: fails later, on the workspace
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 16, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    o.launch = 0
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 16, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    o.stepper = 2                                     # no such stepper
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 1 << 20, None) == \
        A.ERR_UNSUPPORTED
    o.stepper = A.STEPPER_EULER                       # valid: fails later, on the workspace
    assert L.qsq_trace(C.byref(f), _fake(7), 10, C.byref(o), C.byref(t), _fake(8), 16, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    o.stepper = A.STEPPER_CK54
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
    assert b"out_level" in L.qsq_last_error()
    # capacities past 2^30 samples: the trace records are addressed with int32
    d.out_level = 6
    mo.capacity = (1 << 30) + 1
    assert L.qsq_qmap(C.byref(f), C.byref(d), C.byref(o), C.byref(mo), _fake(9), 1 << 62, None) == \
        A.ERR_COUNT_OVERFLOW
    vd = A.VolumeDesc()
    vd.x0, vd.x1, vd.y0, vd.y1, vd.z0, vd.z1 = -1, 1, -1, 1, 0, 1
    vd.base_level, vd.refine_levels, vd.out_level, vd.threshold = 4, 2, 4, 0.1
    assert L.qsq_vmap(C.byref(f), C.byref(vd), C.byref(o), C.byref(mo), _fake(9), 1 << 62, None) == \
        A.ERR_COUNT_OVERFLOW
    mo.capacity = 1 << 30                  # the largest allowed: fails later, on the arrays
    assert L.qsq_vmap(C.byref(f), C.byref(vd), C.byref(o), C.byref(mo), _fake(9), 1 << 62, None) == \
        A.ERR_INVALID_ARG
    assert b"sample arrays" in L.qsq_last_error()
    # FLEDGE: overlapping buffers, bad rank
    shp = (C.c_int64 * 2)(16, 16)
    assert L.qsq_fledge(_fake(1), 2, shp, C.c_void_p(0x100000 + 64), None) == A.ERR_INVALID_ARG
    assert L.qsq_fledge(_fake(1), 4, shp, _fake(2), None) == A.ERR_INVALID_ARG
    assert L.qsq_hilbert2_d2xy(0, _fake(1), 4, _fake(2), _fake(3), None) == A.ERR_INVALID_ARG
    n = C.c_int64()
    ms = C.c_double()
    assert L.qsq_profile_read(7, C.byref(n), C.byref(ms)) == A.ERR_INVALID_ARG


def test_batch_arguments_rejected_before_launch(qsq):
    from paper_1609_00724_amd import _abi as A
    L = qsq.lib
    g = A.Grid()
    g.n[:] = (8, 8, 8)
    g.spacing[:] = (0.1, 0.1, 0.1)
    sets = (A.TraceSet * 3)()
    for k, t in enumerate(sets):
        t.field.grid = g
        t.field.storage, t.field.mode, t.field.nodes = A.F32, A.INTERP_PAPER, _fake(1 + k)
        t.field.bytes = L.qsq_field_bytes(C.byref(g), A.F32)
        t.seeds = _fake(10 + k)
        t.n = 100 * (k + 1)
        t.out.status = _fake(20 + k)
    o = A.TraceOpts()
    o.rtol, o.atol = 1e-6, 1e-6
    o.step_dtype = A.F32
    need = L.qsq_trace_batch_scratch_bytes(3, 600)
    assert need >= L.qsq_trace_scratch_bytes(600)
    assert L.qsq_trace_batch(sets, 0, C.byref(o), None, _fake(30), need, None) == A.ERR_INVALID_ARG
    assert L.qsq_trace_batch(None, 3, C.byref(o), None, _fake(30), need, None) == A.ERR_INVALID_ARG
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, _fake(30), need - 1, None) == A.ERR_WORKSPACE_TOO_SMALL
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, C.c_void_p(0x100000 + 8), need, None) == A.ERR_INVALID_ARG
    sets[1].field.storage = A.F64
    sets[1].field.bytes = L.qsq_field_bytes(C.byref(g), A.F64)
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, _fake(30), need, None) == A.ERR_INVALID_ARG
    assert b"set 1" in L.qsq_last_error()
    sets[1].field.storage = A.F32
    sets[2].out.status = None
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, _fake(30), need, None) == A.ERR_INVALID_ARG
    assert b"set 2" in L.qsq_last_error()
    sets[2].field.grid.n[1] = 1
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, _fake(30), need, None) == A.ERR_INVALID_ARG
    assert b"set 2" in L.qsq_last_error() and b"n[1]" in L.qsq_last_error()
    # a batch without seeds enqueues nothing and needs no scratch
    for t in sets:
        t.n = 0
    sets[2].field.grid.n[1] = 8
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, None, 0, None) == A.OK
    sets[0].n = -1
    assert L.qsq_trace_batch(sets, 3, C.byref(o), None, None, 0, None) == A.ERR_INVALID_ARG


def test_cnn_arguments_rejected_before_launch(qsq):
    from paper_1609_00724_amd import _abi as A
    L = qsq.lib
    assert A.CNN_PARAMS == 19970
    assert L.qsq_cnn_prep_bytes() >= 2 * (1024 + 2 * 9216 + 4608) + 4 * 4 * 32
    need = L.qsq_cnn_workspace_bytes(4, 64, 64)
    assert need >= 4 * 64 * 64 * (3 * 64 + 8 + 4 + 2 * 64)
    assert L.qsq_cnn_forward(_fake(1), _fake(2), 4, 64, 48, _fake(3), _fake(4), need, None) == A.ERR_INVALID_ARG
    assert L.qsq_cnn_forward(_fake(1), _fake(2), 0, 64, 64, _fake(3), _fake(4), need, None) == A.ERR_INVALID_ARG
    assert L.qsq_cnn_forward(_fake(1), _fake(2), 4, 64, 64, _fake(3), _fake(4), need - 1, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    assert L.qsq_cnn_forward(_fake(1), _fake(2), 1 << 20, 64, 64, _fake(3), _fake(4), 1 << 62, None) == \
        A.ERR_COUNT_OVERFLOW
    # one tile above 2^24 pixels: its tensors would not fit 32-bit byte offsets
    assert L.qsq_cnn_forward(_fake(1), _fake(2), 1, 4096, 4128, _fake(3), _fake(4), 1 << 62, None) == \
        A.ERR_COUNT_OVERFLOW
    assert L.qsq_cnn_train_step(_fake(1), _fake(2), _fake(3), 0, 1e-3, _fake(4), _fake(5), _fake(6), 4, 64, 64, 0.1,
                                _fake(7), None, None, _fake(8), need, None) == A.ERR_INVALID_ARG
    assert L.qsq_cnn_layer_forward(4, _fake(1), _fake(2), 4, 64, 64, _fake(3), None) == A.ERR_INVALID_ARG
    s = L.qsq_cnn_layer_scratch_bytes(4, 64, 64)
    assert L.qsq_cnn_layer_backward(0, _fake(1), _fake(2), _fake(3), 4, 64, 64, _fake(4), _fake(5), _fake(6),
                                    _fake(7), s, None) == A.ERR_INVALID_ARG     # layer 0 has no input gradient


def test_noalloc_limits(qsq):
    """qsq_trace_noalloc rejects a seed count beyond its fixed scratch before
    touching the device, and its limit fits the 64 MiB array."""
    from paper_1609_00724_amd import _abi as A
    assert qsq.lib.qsq_trace_scratch_bytes(A.TRACE_NOALLOC_MAX_SEEDS) <= 64 << 20
    f = A.FieldDesc()
    o = A.TraceOpts()
    rc = qsq.lib.qsq_trace_noalloc(C.byref(f), None, A.TRACE_NOALLOC_MAX_SEEDS + 1, C.byref(o), None, None)
    assert rc == A.ERR_WORKSPACE_TOO_SMALL
    assert b"noalloc" in qsq.lib.qsq_last_error()


def test_shifted_repass_arguments_rejected(qsq):
    """Shift outside (0, 2^(m+r)), too many cycles, or proposals together
    with the re-pass are refused before anything is enqueued."""
    from paper_1609_00724_amd import _abi as A
    d = A.MapDesc()
    d.x0, d.x1, d.y0, d.y1 = -1.0, 1.0, -1.0, 1.0
    d.base_level, d.refine_levels, d.out_level, d.threshold = 4, 2, 4, 0.02
    # a well-formed descriptor (its node pointer is never dereferenced: the
    # call fails on the map description first)
    f = A.FieldDesc()
    f.grid.n[:] = (8, 8, 8)
    f.grid.spacing[:] = (1.0, 1.0, 1.0)
    f.storage, f.mode, f.nodes, f.bytes = A.F32, A.INTERP_PAPER, 256, 8 ** 3 * 16
    o = A.TraceOpts()
    for shift, cycles, prop, code in ((-1, 0, None, A.ERR_INVALID_ARG), (64, 0, None, A.ERR_INVALID_ARG),
                                      (5, 49, None, A.ERR_INVALID_ARG), (5, 0, 1, A.ERR_UNSUPPORTED)):
        d.shift, d.max_cycles, d.propose = shift, cycles, prop
        rc = qsq.lib.qsq_qmap(C.byref(f), C.byref(d), C.byref(o), None, None, 0, None)
        assert rc == code, (shift, cycles, rc, qsq.lib.qsq_last_error())
        assert any(w in qsq.lib.qsq_last_error() for w in (b"shift", b"proposals", b"max_cycles"))
    d.shift, d.max_cycles, d.propose = 5, 0, None
    assert qsq.lib.qsq_qmap_scratch_bytes(C.byref(d), 4 ** 6) > 0


def test_base_given_flag_checked(qsq):
    """base_given takes 0 or 1; any other value is refused before anything is
    enqueued."""
    from paper_1609_00724_amd import _abi as A
    d = A.MapDesc()
    d.x0, d.x1, d.y0, d.y1 = -1.0, 1.0, -1.0, 1.0
    d.base_level, d.refine_levels, d.out_level, d.threshold = 4, 2, 4, 0.02
    f = A.FieldDesc()
    f.grid.n[:] = (8, 8, 8)
    f.grid.spacing[:] = (1.0, 1.0, 1.0)
    f.storage, f.mode, f.nodes, f.bytes = A.F32, A.INTERP_PAPER, 256, 8 ** 3 * 16
    o = A.TraceOpts()
    d.base_given = 2
    rc = qsq.lib.qsq_qmap(C.byref(f), C.byref(d), C.byref(o), None, None, 0, None)
    assert rc == A.ERR_INVALID_ARG and b"base_given" in qsq.lib.qsq_last_error()


def test_brick_record_sizes_and_limits(qsq):
    """Brick records: 8 records per 2x2x2 brick of the (padded) grid; fields
    other than trilinear, Cartesian and uniform are refused before any work."""
    from paper_1609_00724_amd import _abi as A
    g = A.Grid()
    g.n[:] = (5, 4, 3)
    assert qsq.lib.qsq_field_brick_bytes(C.byref(g), A.F32) == 8 * 16 * 3 * 2 * 2
    assert qsq.lib.qsq_field_brick_bytes(C.byref(g), A.BF16) == 8 * 8 * 3 * 2 * 2
    assert qsq.lib.qsq_field_brick_bytes(C.byref(g), A.F64) == 8 * 32 * 3 * 2 * 2
    f = A.FieldDesc()
    f.grid.n[:] = (8, 8, 8)
    f.grid.spacing[:] = (1.0, 1.0, 1.0)
    f.storage, f.mode, f.nodes, f.bytes = A.F32, A.INTERP_PAPER, 256, 8 ** 3 * 16
    f.order = A.ORDER_CUBIC
    rc = qsq.lib.qsq_field_add_bricks(C.byref(f), 256, 1 << 20, None)
    assert rc == A.ERR_UNSUPPORTED and b"brick" in qsq.lib.qsq_last_error()
    f.order = A.ORDER_LINEAR
    rc = qsq.lib.qsq_field_add_bricks(C.byref(f), 256, 16, None)
    assert rc == A.ERR_WORKSPACE_TOO_SMALL


def test_direction_record_sizes_and_limits(qsq):
    """Direction records: 96 bytes per cell for FP32 fields and none for other
    storage; other storage, higher orders, a short workspace and a descriptor
    claiming fewer direction bytes than the grid's cells need are refused
    before any work."""
    from paper_1609_00724_amd import _abi as A
    g = A.Grid()
    g.n[:] = (5, 4, 3)
    assert qsq.lib.qsq_field_cell_dir_bytes(C.byref(g), A.F32) == 96 * 4 * 3 * 2
    assert qsq.lib.qsq_field_cell_dir_bytes(C.byref(g), A.BF16) == 0
    assert qsq.lib.qsq_field_cell_dir_bytes(C.byref(g), A.F64) == 0
    f = A.FieldDesc()
    f.grid.n[:] = (8, 8, 8)
    f.grid.spacing[:] = (1.0, 1.0, 1.0)
    f.storage, f.mode, f.nodes, f.bytes = A.BF16, A.INTERP_PAPER, 256, 8 ** 3 * 8
    rc = qsq.lib.qsq_field_add_cell_dirs(C.byref(f), 256, 1 << 20, None)
    assert rc == A.ERR_UNSUPPORTED and b"direction" in qsq.lib.qsq_last_error()
    f.storage, f.bytes = A.F32, 8 ** 3 * 16
    f.order = A.ORDER_CUBIC
    rc = qsq.lib.qsq_field_add_cell_dirs(C.byref(f), 256, 1 << 20, None)
    assert rc == A.ERR_UNSUPPORTED
    f.order = A.ORDER_LINEAR
    rc = qsq.lib.qsq_field_add_cell_dirs(C.byref(f), 256, 96 * 7 ** 3 - 1, None)
    assert rc == A.ERR_WORKSPACE_TOO_SMALL
    f.dirs, f.dir_bytes = 256, 96 * 7 ** 3 - 1
    rc = qsq.lib.qsq_field_add_cell_dirs(C.byref(f), 256, 96 * 7 ** 3, None)
    assert rc == A.ERR_INVALID_ARG and b"direction" in qsq.lib.qsq_last_error()
