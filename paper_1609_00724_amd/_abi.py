"""ctypes mirror of include/qsq.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))

# return codes
OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_WORKSPACE_TOO_SMALL = -3
ERR_HIP = -4
ERR_COUNT_OVERFLOW = -5

F64, F32, BF16 = 0, 1, 2
INTERP_PAPER, INTERP_NORMALIZE = 0, 1
STEPPER_CK54 = 0
STEPPER_EULER = 1
ORDER_LINEAR, ORDER_QUADRATIC, ORDER_CUBIC = 1, 2, 3
GEOMETRY_CARTESIAN, GEOMETRY_SPHERICAL = 0, 1
FLAG_SKIP_OPEN = 1

END_XLO, END_XHI, END_YLO, END_YHI, END_ZLO, END_ZHI = range(6)
END_MAX_LENGTH, END_MAX_STEPS, END_NULL, END_UNDERFLOW, END_SEED_OUTSIDE, END_NONFINITE = range(6, 12)
STATUS_OPEN = 1 << 16

# every entry point include/qsq.h declares
EXPORTS = ["qsq_abi_version", "qsq_status_string", "qsq_last_error", "qsq_field_bytes",
           "qsq_field_init", "qsq_field_cell_bytes", "qsq_field_add_cells", "qsq_field_brick_bytes",
           "qsq_field_add_bricks", "qsq_field_cell_dir_bytes", "qsq_field_add_cell_dirs", "qsq_trace_scratch_bytes",
           "qsq_trace", "qsq_fledge",
           "qsq_hilbert2_d2xy", "qsq_hilbert2_xy2d", "qsq_qmap_scratch_bytes", "qsq_qmap",
           "qsq_profile_enable", "qsq_profile_reset", "qsq_profile_read",
           "qsq_hilbert3_d2xyz", "qsq_hilbert3_xyz2d", "qsq_vmap_scratch_bytes", "qsq_vmap",
           "qsq_trace_batch_scratch_bytes", "qsq_trace_batch", "qsq_trace_noalloc"]

# every entry point include/qsq_cnn.h declares
CNN_EXPORTS = ["qsq_cnn_prep_bytes", "qsq_cnn_prepare", "qsq_cnn_workspace_bytes", "qsq_cnn_layer_scratch_bytes",
               "qsq_cnn_forward", "qsq_cnn_train_step", "qsq_cnn_layer_forward", "qsq_cnn_layer_backward"]
CNN_PARAMS = 19970

MAX_TRACE_SETS = 65536
TRACE_NOALLOC_MAX_SEEDS = 1 << 18

KERNEL_STEP, KERNEL_LAND, KERNEL_ASSEMBLE = 0, 1, 2

WG_CODES = {256: 0, 64: 1, 128: 2}
GATHER_AUTO, GATHER_DIRECT, GATHER_CACHED, GATHER_REGS, GATHER_CELLS, GATHER_BRICKS, GATHER_DIRS = range(7)


LAUNCH_PARTS = 1 << 9


def launch_word(lanes=0, wg=256, gather=GATHER_AUTO, parts=False, refine_gather=0):
    """QSQ_LAUNCH(lanes, wg, gather), with QSQ_LAUNCH_PARTS if parts and
    QSQ_LAUNCH_REFINE_GATHER(refine_gather), of include/qsq.h."""
    if not 0 <= lanes <= 15 or wg not in WG_CODES or gather not in range(7) or refine_gather not in range(7):
        raise ValueError("launch shape outside QSQ_LAUNCH(0..15, 64|128|256, 0..6), refine gather 0..6")
    return ((lanes & 15) | (WG_CODES[wg] << 4) | (gather << 6) | (LAUNCH_PARTS if parts else 0)
            | (refine_gather << 10))


class Grid(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class FieldDesc(C.Structure):
    _fields_ = [("grid", Grid), ("storage", C.c_int32), ("mode", C.c_int32),
                ("nodes", C.c_void_p), ("bytes", C.c_uint64), ("cells", C.c_void_p), ("cell_bytes", C.c_uint64),
                ("order", C.c_int32), ("geometry", C.c_int32), ("coords", C.c_void_p * 3),
                ("bricks", C.c_void_p), ("brick_bytes", C.c_uint64), ("dirs", C.c_void_p),
                ("dir_bytes", C.c_uint64)]


class TraceOpts(C.Structure):
    _fields_ = [("stepper", C.c_int32), ("step_dtype", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("h_init", C.c_double), ("h_max", C.c_double),
                ("max_length", C.c_double), ("max_steps", C.c_int64), ("flags", C.c_int32),
                ("launch", C.c_int32)]


class TraceOut(C.Structure):
    _fields_ = [("fp_fwd", C.c_void_p), ("fp_bwd", C.c_void_p), ("fll", C.c_void_p),
                ("q_perp", C.c_void_p), ("q_det", C.c_void_p), ("q_fp", C.c_void_p),
                ("status", C.c_void_p), ("steps", C.c_void_p), ("work", C.c_void_p)]


class TraceSet(C.Structure):
    _fields_ = [("field", FieldDesc), ("seeds", C.c_void_p), ("n", C.c_int64), ("out", TraceOut)]


class MapDesc(C.Structure):
    _fields_ = [("z0", C.c_double), ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double),
                ("y1", C.c_double), ("base_level", C.c_int32), ("refine_levels", C.c_int32),
                ("out_level", C.c_int32), ("refine_batch", C.c_int32), ("threshold", C.c_double),
                ("propose", C.c_void_p), ("shift", C.c_int32), ("max_cycles", C.c_int32),
                ("tilted", C.c_int32), ("base_given", C.c_int32), ("corner", C.c_double * 3), ("edge_u", C.c_double * 3),
                ("edge_v", C.c_double * 3)]


class VolumeDesc(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("z0", C.c_double), ("z1", C.c_double), ("base_level", C.c_int32),
                ("refine_levels", C.c_int32), ("out_level", C.c_int32), ("refine_batch", C.c_int32),
                ("threshold", C.c_double), ("propose", C.c_void_p), ("shift", C.c_int32),
                ("max_cycles", C.c_int32)]


class MapOut(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("keys", C.c_void_p), ("fll", C.c_void_p),
                ("q_perp", C.c_void_p), ("status", C.c_void_p), ("count", C.c_void_p),
                ("overflow", C.c_void_p), ("q_grid", C.c_void_p), ("fll_grid", C.c_void_p),
                ("fledge", C.c_void_p), ("work", C.c_void_p), ("steps", C.c_void_p)]


class QsqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qsq error {code}: {msg}")
        self.code = code


def _load():
    L = C.CDLL(os.path.join(_HERE, "libqsq.so"))
    P, I64, U64, I = C.c_void_p, C.c_int64, C.c_uint64, C.c_int
    L.qsq_abi_version.restype = I
    L.qsq_status_string.restype = C.c_char_p
    L.qsq_status_string.argtypes = [I]
    L.qsq_last_error.restype = C.c_char_p
    L.qsq_field_bytes.restype = U64
    L.qsq_field_bytes.argtypes = [C.POINTER(Grid), I]
    L.qsq_field_init.restype = I
    L.qsq_field_init.argtypes = [C.POINTER(Grid), P, P, P, I, I, I, P, U64, P, C.POINTER(FieldDesc)]
    L.qsq_trace_scratch_bytes.restype = U64
    L.qsq_field_cell_bytes.restype = U64
    L.qsq_field_cell_bytes.argtypes = [C.POINTER(Grid), I]
    L.qsq_field_add_cells.restype = I
    L.qsq_field_add_cells.argtypes = [C.POINTER(FieldDesc), P, U64, P]
    L.qsq_field_brick_bytes.restype = U64
    L.qsq_field_brick_bytes.argtypes = [C.POINTER(Grid), I]
    L.qsq_field_add_bricks.restype = I
    L.qsq_field_add_bricks.argtypes = [C.POINTER(FieldDesc), P, U64, P]
    L.qsq_field_cell_dir_bytes.restype = U64
    L.qsq_field_cell_dir_bytes.argtypes = [C.POINTER(Grid), I]
    L.qsq_field_add_cell_dirs.restype = I
    L.qsq_field_add_cell_dirs.argtypes = [C.POINTER(FieldDesc), P, U64, P]
    L.qsq_trace_scratch_bytes.argtypes = [I64]
    L.qsq_trace.restype = I
    L.qsq_trace.argtypes = [C.POINTER(FieldDesc), P, I64, C.POINTER(TraceOpts), C.POINTER(TraceOut),
                            P, U64, P]
    L.qsq_trace_batch_scratch_bytes.restype = U64
    L.qsq_trace_noalloc.restype = I
    L.qsq_trace_noalloc.argtypes = [C.POINTER(FieldDesc), P, I64, C.POINTER(TraceOpts), C.POINTER(TraceOut), P]
    L.qsq_trace_batch_scratch_bytes.argtypes = [C.c_int32, I64]
    L.qsq_trace_batch.restype = I
    L.qsq_trace_batch.argtypes = [C.POINTER(TraceSet), C.c_int32, C.POINTER(TraceOpts), P, P, U64, P]
    L.qsq_cnn_prep_bytes.restype = U64
    L.qsq_cnn_prepare.restype = I
    L.qsq_cnn_prepare.argtypes = [P, P, P]
    L.qsq_cnn_workspace_bytes.restype = U64
    L.qsq_cnn_workspace_bytes.argtypes = [I64, I, I]
    L.qsq_cnn_layer_scratch_bytes.restype = U64
    L.qsq_cnn_layer_scratch_bytes.argtypes = [I64, I, I]
    L.qsq_cnn_forward.restype = I
    L.qsq_cnn_forward.argtypes = [P, P, I64, I, I, P, P, U64, P]
    L.qsq_cnn_train_step.restype = I
    L.qsq_cnn_train_step.argtypes = [P, P, P, I64, C.c_float, P, P, P, I64, I, I, C.c_float, P, P, P, P, U64, P]
    L.qsq_cnn_layer_forward.restype = I
    L.qsq_cnn_layer_forward.argtypes = [I, P, P, I64, I, I, P, P]
    L.qsq_cnn_layer_backward.restype = I
    L.qsq_cnn_layer_backward.argtypes = [I, P, P, P, I64, I, I, P, P, P, P, U64, P]
    L.qsq_fledge.restype = I
    L.qsq_fledge.argtypes = [P, I, C.POINTER(C.c_int64), P, P]
    L.qsq_hilbert2_d2xy.restype = I
    L.qsq_hilbert2_d2xy.argtypes = [I, P, I64, P, P, P]
    L.qsq_hilbert2_xy2d.restype = I
    L.qsq_hilbert2_xy2d.argtypes = [I, P, P, I64, P, P]
    L.qsq_qmap_scratch_bytes.restype = U64
    L.qsq_qmap_scratch_bytes.argtypes = [C.POINTER(MapDesc), I64]
    L.qsq_qmap.restype = I
    L.qsq_qmap.argtypes = [C.POINTER(FieldDesc), C.POINTER(MapDesc), C.POINTER(TraceOpts),
                           C.POINTER(MapOut), P, U64, P]
    L.qsq_hilbert3_d2xyz.restype = I
    L.qsq_hilbert3_d2xyz.argtypes = [I, P, I64, P, P, P, P]
    L.qsq_hilbert3_xyz2d.restype = I
    L.qsq_hilbert3_xyz2d.argtypes = [I, P, P, P, I64, P, P]
    L.qsq_vmap_scratch_bytes.restype = U64
    L.qsq_vmap_scratch_bytes.argtypes = [C.POINTER(VolumeDesc), I64]
    L.qsq_vmap.restype = I
    L.qsq_vmap.argtypes = [C.POINTER(FieldDesc), C.POINTER(VolumeDesc), C.POINTER(TraceOpts),
                           C.POINTER(MapOut), P, U64, P]
    L.qsq_profile_enable.restype = I
    L.qsq_profile_enable.argtypes = [I]
    L.qsq_profile_reset.restype = I
    L.qsq_profile_read.restype = I
    L.qsq_profile_read.argtypes = [I, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    return L


lib = _load()


def check(rc: int):
    if rc != OK:
        raise QsqError(rc, lib.qsq_last_error().decode())
