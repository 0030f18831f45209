"""Torch-facing wrappers of the libqsq C-ABI: device buffers and streams come
from PyTorch, every computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import torch

from . import _abi as A
from ._abi import check, lib

_DT = {"f64": A.F64, "f32": A.F32, "bf16": A.BF16}
_MODE = {"paper": A.INTERP_PAPER, "interp_normalize": A.INTERP_NORMALIZE}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        t = t.to(dtype)
    return t.contiguous()


def _bytes_tensor(nbytes, device):
    # int64 elements keep the base 256-byte aligned through the caching allocator
    return torch.empty((max(int(nbytes), 8) + 7) // 8, dtype=torch.int64, device=device)


class Field:
    """A prepared field: node records (and, if added, cell or brick records)
    in torch-owned device workspaces."""

    def __init__(self, desc: A.FieldDesc, ws: torch.Tensor):
        self.desc = desc
        self.ws = ws
        self.cells_ws = None
        self.bricks_ws = None
        self.dirs_ws = None

    def add_cells(self, stream=None):
        """Add cell records (the 8 corner records of every cell, contiguous),
        read by the stepping kernel's gather 4; returns self."""
        nbytes = lib.qsq_field_cell_bytes(C.byref(self.desc.grid), self.desc.storage)
        ws = _bytes_tensor(nbytes, self.ws.device)
        check(lib.qsq_field_add_cells(C.byref(self.desc), _p(ws), ws.numel() * 8, _stream(stream)))
        self.cells_ws = ws
        return self

    def add_bricks(self, stream=None):
        """Add brick records (the node records in 2 x 2 x 2 bricks), read by
        the stepping kernel's gather 5; returns self."""
        nbytes = lib.qsq_field_brick_bytes(C.byref(self.desc.grid), self.desc.storage)
        ws = _bytes_tensor(nbytes, self.ws.device)
        check(lib.qsq_field_add_bricks(C.byref(self.desc), _p(ws), ws.numel() * 8, _stream(stream)))
        self.bricks_ws = ws
        return self

    def add_cell_dirs(self, stream=None):
        """Add direction records (each cell's 8 corner directions, 96
        contiguous bytes; FP32 fields), read by the stepping kernel's gather 6;
        returns self."""
        nbytes = lib.qsq_field_cell_dir_bytes(C.byref(self.desc.grid), self.desc.storage)
        ws = _bytes_tensor(nbytes, self.ws.device)
        check(lib.qsq_field_add_cell_dirs(C.byref(self.desc), _p(ws), ws.numel() * 8, _stream(stream)))
        self.dirs_ws = ws
        return self

    @property
    def n(self):
        return tuple(self.desc.grid.n)

    @property
    def spacing(self):
        return tuple(self.desc.grid.spacing)


_ORDER = {"linear": A.ORDER_LINEAR, "quadratic": A.ORDER_QUADRATIC, "cubic": A.ORDER_CUBIC}


def field_init(bx, by, bz, origin, spacing, storage="f32", mode="paper", stream=None, order="linear",
               geometry="cartesian", coords=None) -> Field:
    """Prepare node records from B component arrays shaped (nz, ny, nx) on the
    device; `order` picks the interpolation kernel (linear, quadratic, cubic);
    geometry "spherical" reads the axes as (longitude, latitude, radius) and
    the arrays as (B_phi, B_theta, B_r); `coords` = (x, y, z) node coordinate
    tensors (None per axis: uniform) makes a rectilinear grid, whose first and
    last coordinates must equal origin and origin + (n - 1) spacing."""
    if bx.dtype not in (torch.float32, torch.float64):
        raise TypeError("B components must be float32 or float64")
    in_dt = A.F64 if bx.dtype == torch.float64 else A.F32
    bx, by, bz = (_dev(b, bx.dtype, "B") for b in (bx, by, bz))
    nz, ny, nx = bx.shape
    g = A.Grid()
    g.n[:] = (nx, ny, nz)
    g.origin[:] = tuple(float(v) for v in origin)
    g.spacing[:] = tuple(float(v) for v in spacing)
    nbytes = lib.qsq_field_bytes(C.byref(g), _DT[storage])
    ws = _bytes_tensor(nbytes, bx.device)
    d = A.FieldDesc()
    check(lib.qsq_field_init(C.byref(g), _p(bx), _p(by), _p(bz), in_dt, _DT[storage], _MODE[mode],
                             _p(ws), ws.numel() * 8, _stream(stream), C.byref(d)))
    d.order = _ORDER[order]
    d.geometry = {"cartesian": A.GEOMETRY_CARTESIAN, "spherical": A.GEOMETRY_SPHERICAL}[geometry]
    keep = []
    for a, c in enumerate(coords or (None, None, None)):
        if c is None:
            continue
        c = _dev(c, torch.float64, "coords")
        if c.numel() != d.grid.n[a]:
            raise ValueError(f"coords[{a}] must hold {d.grid.n[a]} node coordinates")
        d.coords[a] = c.data_ptr()
        keep.append(c)
    f = Field(d, ws)
    f.coords_ws = keep
    return f


_STEPPER = {"ck54": A.STEPPER_CK54, "euler": A.STEPPER_EULER}


def make_opts(rtol, atol, h_init=0.0, h_max=0.0, max_length=0.0, max_steps=0, step_dtype="f32",
              skip_open=False, launch=0, stepper="ck54") -> A.TraceOpts:
    """Trace options.  stepper "ck54": adaptive Cash-Karp 5(4) with rtol, atol,
    first step h_init, largest step h_max; "euler": explicit Euler with the
    fixed step h_init (0: one fifth of the smallest grid spacing)."""
    o = A.TraceOpts()
    o.stepper = _STEPPER[stepper]
    o.step_dtype = _DT[step_dtype]
    o.rtol, o.atol = float(rtol), float(atol)
    o.h_init, o.h_max, o.max_length = float(h_init), float(h_max), float(max_length)
    o.max_steps = int(max_steps)
    o.flags = A.FLAG_SKIP_OPEN if skip_open else 0
    o.launch = int(launch)
    return o


class TracePlan:
    """Preallocated outputs and scratch for repeated traces of n seeds."""

    def __init__(self, n: int, device, want=("fp_fwd", "fp_bwd", "fll", "q_perp", "q_det", "q_fp"),
                 want_steps=False, want_work=False, noalloc=False):
        self.n = int(n)
        self.noalloc = bool(noalloc)   # run through qsq_trace_noalloc (library-owned scratch)
        f64 = dict(dtype=torch.float64, device=device)
        self.out = {}
        for k in want:
            self.out[k] = torch.empty((3, n) if k.startswith("fp_") else (n,), **f64)
        self.out["status"] = torch.empty(n, dtype=torch.int32, device=device)
        if want_steps:
            self.out["steps"] = torch.empty((2, n), dtype=torch.int32, device=device)
        if want_work:
            self.out["work"] = torch.zeros(4, dtype=torch.int64, device=device)
        self.scratch = None if self.noalloc else _bytes_tensor(lib.qsq_trace_scratch_bytes(n), device)
        o = A.TraceOut()
        for k in ("fp_fwd", "fp_bwd", "fll", "q_perp", "q_det", "q_fp", "status", "steps", "work"):
            setattr(o, k, _p(self.out.get(k)))
        self.tout = o

    def run(self, field: Field, seeds_soa: torch.Tensor, opts: A.TraceOpts, stream=None):
        if self.noalloc:
            check(lib.qsq_trace_noalloc(C.byref(field.desc), _p(seeds_soa), self.n, C.byref(opts),
                                        C.byref(self.tout), _stream(stream)))
        else:
            check(lib.qsq_trace(C.byref(field.desc), _p(seeds_soa), self.n, C.byref(opts), C.byref(self.tout),
                                _p(self.scratch), self.scratch.numel() * 8, _stream(stream)))
        return self.out


def trace(field: Field, seeds, *, rtol, atol, h_init=0.0, h_max=0.0, max_length=0.0, max_steps=0,
          step_dtype="f32", skip_open=False, want_steps=False, want_work=False, stream=None, stepper="ck54"):
    """Trace seeds, a device tensor of shape (n, 3) (one row per seed), both ways.

    Returns device tensors: fp_fwd, fp_bwd (3, n) SoA planes; fll, q_perp, q_det,
    q_fp (n,); status (n,) int32; steps (2, n) int32 and work (4,) if asked.
    """
    seeds = _dev(seeds, torch.float64, "seeds")
    if seeds.dim() != 2 or seeds.shape[1] != 3:
        raise ValueError("seeds must have shape (n, 3)")
    soa = seeds.t().contiguous()
    n = soa.shape[1]
    plan = TracePlan(n, seeds.device, want_steps=want_steps, want_work=want_work)
    opts = make_opts(rtol, atol, h_init, h_max, max_length, max_steps, step_dtype, skip_open, stepper=stepper)
    return plan.run(field, soa, opts, stream)


class TraceBatchPlan:
    """A batched trace of several (field, seeds) sets with preallocated outputs
    and scratch.  run() enqueues one qsq_trace_batch call; since every pointer
    stays fixed, the call can be captured in a HIP graph and replayed."""

    def __init__(self, sets, opts: A.TraceOpts, want=("fp_fwd", "fp_bwd", "fll", "q_perp", "q_det", "q_fp"),
                 want_steps=False, want_work=False):
        if not sets:
            raise ValueError("need at least one set")
        self.opts = opts
        self.fields, self.seeds, self.outs = [], [], []
        arr = (A.TraceSet * len(sets))()
        total = 0
        device = None
        for k, (field, seeds) in enumerate(sets):
            seeds = _dev(seeds, torch.float64, "seeds")
            if seeds.dim() != 2 or seeds.shape[1] != 3:
                raise ValueError("seeds must have shape (n, 3)")
            soa = seeds.t().contiguous()
            n = soa.shape[1]
            device = seeds.device
            f64 = dict(dtype=torch.float64, device=device)
            out = {key: torch.empty((3, n) if key.startswith("fp_") else (n,), **f64) for key in want}
            out["status"] = torch.empty(n, dtype=torch.int32, device=device)
            if want_steps:
                out["steps"] = torch.empty((2, n), dtype=torch.int32, device=device)
            t = arr[k]
            t.field = field.desc
            t.seeds = _p(soa)
            t.n = n
            for key in ("fp_fwd", "fp_bwd", "fll", "q_perp", "q_det", "q_fp", "status", "steps"):
                setattr(t.out, key, _p(out.get(key)))
            self.fields.append(field)
            self.seeds.append(soa)
            self.outs.append(out)
            total += n
        self.sets = arr
        self.total = total
        self.work = torch.zeros(4, dtype=torch.int64, device=device) if want_work else None
        self.scratch = _bytes_tensor(lib.qsq_trace_batch_scratch_bytes(len(sets), total), device)

    def run(self, stream=None):
        check(lib.qsq_trace_batch(self.sets, len(self.outs), C.byref(self.opts), _p(self.work), _p(self.scratch),
                                  self.scratch.numel() * 8, _stream(stream)))
        return self.outs


def trace_batch(sets, *, rtol, atol, h_init=0.0, h_max=0.0, max_length=0.0, max_steps=0, step_dtype="f32",
                skip_open=False, want_steps=False, want_work=False, stream=None, stepper="ck54"):
    """Trace several (field, seeds (n, 3)) sets in one batched call; returns one
    output dict per set (as trace()) and, if asked, the summed work counters."""
    opts = make_opts(rtol, atol, h_init, h_max, max_length, max_steps, step_dtype, skip_open, stepper=stepper)
    plan = TraceBatchPlan(sets, opts, want_steps=want_steps, want_work=want_work)
    outs = plan.run(stream)
    return (outs, plan.work) if want_work else outs


def fledge(x: torch.Tensor, stream=None) -> torch.Tensor:
    """Sobel FLEDGE magnitude of a 2D or 3D float32 device map."""
    x = _dev(x, torch.float32, "map")
    out = torch.empty_like(x)
    shape = (C.c_int64 * x.dim())(*x.shape)
    check(lib.qsq_fledge(_p(x), x.dim(), shape, _p(out), _stream(stream)))
    return out


def hilbert2_d2xy(L: int, d: torch.Tensor, stream=None):
    d = _dev(d, torch.int64, "d")
    x = torch.empty(d.shape, dtype=torch.int32, device=d.device)
    y = torch.empty_like(x)
    check(lib.qsq_hilbert2_d2xy(L, _p(d), d.numel(), _p(x), _p(y), _stream(stream)))
    return x, y


def hilbert2_xy2d(L: int, x: torch.Tensor, y: torch.Tensor, stream=None):
    x = _dev(x, torch.int32, "x")
    y = _dev(y, torch.int32, "y")
    d = torch.empty(x.shape, dtype=torch.int64, device=x.device)
    check(lib.qsq_hilbert2_xy2d(L, _p(x), _p(y), x.numel(), _p(d), _stream(stream)))
    return d


def hilbert3_d2xyz(b: int, d: torch.Tensor, stream=None):
    d = _dev(d, torch.int64, "d")
    x, y, z = (torch.empty(d.shape, dtype=torch.int32, device=d.device) for _ in range(3))
    check(lib.qsq_hilbert3_d2xyz(b, _p(d), d.numel(), _p(x), _p(y), _p(z), _stream(stream)))
    return x, y, z


def hilbert3_xyz2d(b: int, x, y, z, stream=None):
    x, y, z = (_dev(v, torch.int32, "cell") for v in (x, y, z))
    d = torch.empty(x.shape, dtype=torch.int64, device=x.device)
    check(lib.qsq_hilbert3_xyz2d(b, _p(x), _p(y), _p(z), x.numel(), _p(d), _stream(stream)))
    return d


@dataclass
class MapSpec:
    z0: float
    x0: float
    x1: float
    y0: float
    y1: float
    base_level: int
    refine_levels: int
    out_level: int
    threshold: float
    refine_batch: int = 0   # refinement levels per device round; 0: all in one round
    propose: Optional[torch.Tensor] = None   # uint8 per base pixel in curve order (device)
    shift: int = 0          # > 0: shifted-curve re-pass by this many finest cells per axis
    max_cycles: int = 0     # re-pass cycles at most (0: library default)
    plane: Optional[tuple] = None   # (corner, edge_u, edge_v): a slice of any orientation

    def desc(self) -> A.MapDesc:
        d = A.MapDesc()
        d.z0, d.x0, d.x1, d.y0, d.y1 = self.z0, self.x0, self.x1, self.y0, self.y1
        d.base_level, d.refine_levels, d.out_level = self.base_level, self.refine_levels, self.out_level
        d.refine_batch = self.refine_batch
        d.threshold = self.threshold
        d.propose = _proposal_ptr(self.propose, 4 ** self.base_level)
        d.shift, d.max_cycles = self.shift, self.max_cycles
        if self.plane is not None:
            corner, eu, ev = self.plane
            d.tilted = 1
            d.corner[:] = tuple(float(v) for v in corner)
            d.edge_u[:] = tuple(float(v) for v in eu)
            d.edge_v[:] = tuple(float(v) for v in ev)
        return d


@dataclass
class VolumeSpec:
    x0: float
    x1: float
    y0: float
    y1: float
    z0: float
    z1: float
    base_level: int
    refine_levels: int
    out_level: int
    threshold: float
    refine_batch: int = 0
    propose: Optional[torch.Tensor] = None   # uint8 per base cell in curve order (device)
    shift: int = 0
    max_cycles: int = 0

    def desc(self) -> A.VolumeDesc:
        d = A.VolumeDesc()
        d.x0, d.x1, d.y0, d.y1, d.z0, d.z1 = self.x0, self.x1, self.y0, self.y1, self.z0, self.z1
        d.base_level, d.refine_levels, d.out_level = self.base_level, self.refine_levels, self.out_level
        d.refine_batch = self.refine_batch
        d.threshold = self.threshold
        d.propose = _proposal_ptr(self.propose, 8 ** self.base_level)
        d.shift, d.max_cycles = self.shift, self.max_cycles
        return d


def _proposal_ptr(t, n):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"propose must be a contiguous uint8 device tensor of {n} entries (curve order)")
    return t.data_ptr()


class QMapPlan:
    """Preallocated sample arrays, grids and scratch for repeated slice maps
    (MapSpec) or volume maps (VolumeSpec)."""

    def __init__(self, spec: MapSpec, capacity: int, device, grids=True, fledge_map=True, want_steps=False):
        """Work counters (step attempts, RHS evaluations, half-lines stepped,
        half-lines landed) accumulate in ``self.work``; zero it to restart.
        want_steps: also keep the step attempts of each kept sample's line."""
        self.spec = spec
        self.capacity = int(capacity)
        self.d = spec.desc()
        self.dims = 3 if isinstance(spec, VolumeSpec) else 2
        cap = self.capacity
        self.keys = torch.empty(cap, dtype=torch.int64, device=device)
        self.fll = torch.empty(cap, dtype=torch.float64, device=device)
        self.q_perp = torch.empty(cap, dtype=torch.float64, device=device)
        self.status = torch.empty(cap, dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        side = 1 << spec.out_level
        bside = 1 << spec.base_level
        gshape, bshape = (side,) * self.dims, (bside,) * self.dims
        self.q_grid = torch.empty(gshape, dtype=torch.float32, device=device) if grids else None
        self.fll_grid = torch.empty(gshape, dtype=torch.float32, device=device) if grids else None
        self.fledge = torch.empty(bshape, dtype=torch.float32, device=device) if fledge_map else None
        self.work = torch.zeros(4, dtype=torch.int64, device=device)
        self.steps = torch.empty(cap, dtype=torch.int32, device=device) if want_steps else None
        sizer = lib.qsq_vmap_scratch_bytes if self.dims == 3 else lib.qsq_qmap_scratch_bytes
        self.scratch = _bytes_tensor(sizer(C.byref(self.d), cap), device)
        o = A.MapOut()
        o.capacity = cap
        o.keys, o.fll, o.q_perp, o.status = _p(self.keys), _p(self.fll), _p(self.q_perp), _p(self.status)
        o.count, o.overflow = _p(self.count), _p(self.overflow)
        o.q_grid, o.fll_grid, o.fledge = _p(self.q_grid), _p(self.fll_grid), _p(self.fledge)
        o.work = _p(self.work)
        o.steps = _p(self.steps)
        self.mout = o

    def run(self, field: Field, opts: A.TraceOpts, stream=None, base_from=None):
        """Enqueue the map.  base_from: a slice plan of the same slice and base
        level with no refinement levels whose result holds the base lattice;
        its samples are copied in and not traced again."""
        fn = lib.qsq_vmap if self.dims == 3 else lib.qsq_qmap
        if base_from is not None:
            if self.dims != 2 or base_from.spec.base_level != self.spec.base_level or base_from.spec.refine_levels:
                raise ValueError("base_from must be an unrefined slice map of the same base level")
            nb = 4 ** self.spec.base_level
            pairs = [(self.fll, base_from.fll), (self.q_perp, base_from.q_perp), (self.status, base_from.status)]
            if self.steps is not None:
                if base_from.steps is None:
                    raise ValueError("base_from must keep the step attempts too")
                pairs.append((self.steps, base_from.steps))
            with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
                for a, b in pairs:
                    a[:nb].copy_(b[:nb])
            self.d.base_given = 1
        try:
            check(fn(C.byref(field.desc), C.byref(self.d), C.byref(opts), C.byref(self.mout),
                     _p(self.scratch), self.scratch.numel() * 8, _stream(stream)))
        finally:
            if self.dims == 2:
                self.d.base_given = 0
        return self

    def result(self):
        n = int(self.count.item())
        return dict(count=n, overflow=int(self.overflow.item()), keys=self.keys[:n], fll=self.fll[:n],
                    q_perp=self.q_perp[:n], status=self.status[:n], q_grid=self.q_grid,
                    fll_grid=self.fll_grid, fledge=self.fledge,
                    steps=None if self.steps is None else self.steps[:n])


def qmap(field: Field, spec, capacity: int, *, rtol, atol, h_init=0.0, h_max=0.0,
         max_length=0.0, max_steps=0, step_dtype="f32", skip_open=False, stream=None, stepper="ck54"):
    plan = QMapPlan(spec, capacity, field.ws.device)
    opts = make_opts(rtol, atol, h_init, h_max, max_length, max_steps, step_dtype, skip_open, stepper=stepper)
    plan.run(field, opts, stream)
    return plan.result()


class Profiler:
    """Event timing of the library's kernels on their own streams (process-wide)."""

    def __enter__(self):
        check(lib.qsq_profile_reset())
        check(lib.qsq_profile_enable(1))
        return self

    def __exit__(self, *exc):
        check(lib.qsq_profile_enable(0))
        return False

    @staticmethod
    def read(kernel: int):
        n = C.c_int64()
        ms = C.c_double()
        check(lib.qsq_profile_read(kernel, C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    @staticmethod
    def reset():
        check(lib.qsq_profile_reset())
