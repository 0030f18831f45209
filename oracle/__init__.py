"""Plain FP64 CPU oracle of the QSL Squasher path (arXiv:1609.00724).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1609_00724_amd``) and never imports it.

Contents, each following the paper (Tassev & Savcheva 2017):
  * ``Field`` / ``trace``      -- C library ``qsl_oracle.c``: Sect. 3.1-3.5,
                                  eq. (1), (3)-(5), (9)-(11), Cash-Karp RK5(4)
  * ``sobel_magnitude``        -- Sect. 3.6: FLEDGE map as the Sobel gradient
                                  magnitude of a field-line-length map
  * ``hilbert2_*``             -- Sect. 3.6: Hilbert ordering of a slice
  * ``refine_slice``           -- Sect. 3.6: FLL-jump refinement along the curve
  * ``refine_shifted``         -- Sect. 3.6: the same with the shifted-curve re-pass
  * ``convert_to_grid``        -- Sect. 3.6: array converter (max per cell,
                                  log Q interpolated along the curve in gaps)
  * ``oracle.cnn``             -- FP64 reference of the learned refinement
                                  proposer (3x3 convolutions, loss, backward,
                                  Adam), an extension beyond the paper
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsl_oracle.c")
_LIB = os.path.join(_HERE, "libqsl_oracle.so")

# status codes of one half-line (exit faces first)
XLO, XHI, YLO, YHI, ZLO, ZHI = range(6)
MAX_LENGTH, MAX_STEPS, NULL, UNDERFLOW, SEED_OUTSIDE, NONFINITE = range(6, 12)
OPEN_BIT = 1 << 16

PAPER, INTERP_NORMALIZE, ANALYTIC = 0, 1, 2
GEOMETRIES = {"cartesian": 0, "spherical": 1}
AN_LINEAR, AN_CHARGES = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-ffp-contract=off", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("analytic", C.c_int32), ("n", C.c_int64 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bx", C.c_void_p), ("by", C.c_void_p), ("bz", C.c_void_p),
                ("lin", C.c_double * 12), ("charges", C.c_void_p), ("ncharges", C.c_int64),
                ("quantize", C.c_int32), ("order", C.c_int32), ("geometry", C.c_int32), ("pad", C.c_int32),
                ("coord", C.c_void_p * 3)]


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_init", C.c_double),
                ("h_max", C.c_double), ("max_length", C.c_double), ("max_steps", C.c_int64),
                ("frame_angle", C.c_double), ("nthreads", C.c_int32), ("stepper", C.c_int32),
                ("round_f32", C.c_int32), ("pad", C.c_int32)]


STEPPERS = {"ck54": 0, "euler": 1}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_field_new.restype = P
        L.or_field_new.argtypes = [C.POINTER(_Desc)]
        L.or_field_free.argtypes = [P]
        L.or_field_eval.argtypes = [P, C.c_int64, P, P, P, P]
        L.or_trace.argtypes = [P, C.POINTER(_Opts), C.c_int64, P] + [P] * 11
        L.or_ck54_tableau.argtypes = [P, P, P, P]
        L.or_hilbert2_xy2d.argtypes = [C.c_int, C.c_int64, P, P, P]
        L.or_hilbert2_d2xy.argtypes = [C.c_int, C.c_int64, P, P, P]
        L.or_hilbert3_d2xyz.argtypes = [C.c_int, C.c_int64, P, P, P, P]
        L.or_hilbert3_xyz2d.argtypes = [C.c_int, C.c_int64, P, P, P, P]
        L.or_version.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Field:
    """A field the oracle can trace through.

    Grid kinds take node arrays of shape (nz, ny, nx) (x fastest) on the
    node-centred grid ``origin + i * spacing``; the box is the node hull.
    """

    def __init__(self, desc: _Desc, keep):
        self._keep = keep
        self.lo = np.array(desc.lo[:])
        self.hi = np.array(desc.hi[:])
        self._h = lib().or_field_new(C.byref(desc))
        if not self._h:
            raise MemoryError("oracle field allocation failed")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_field_free(self._h)
            self._h = None

    @classmethod
    def grid(cls, bx, by, bz, origin, spacing, mode=PAPER, store="f64", order=1, geometry="cartesian",
             coords=None):
        """``store="f32"`` / ``"bf16"`` rounds the prepared node values (Bhat and
        |B| in PAPER mode, B otherwise) to FP32 / BF16 (via FP32, nearest even),
        i.e. traces the field such a node store holds.  ``order`` is the
        interpolation order (Sect. 3.2): 1 trilinear, 2 triquadratic (Dodgson
        1997), 3 tricubic (Keys 1981).  ``geometry="spherical"`` reads the axes as
        (longitude, latitude, radius) and the arrays as (B_phi, B_theta, B_r)
        (Sect. 3.1, eq. 2 and 6-8).  ``coords`` = (x, y, z) node coordinate
        arrays (None per axis: uniform) gives a rectilinear grid whose cells
        have their own spans (Sect. 3.2); trilinear only."""
        bx, by, bz = (np.ascontiguousarray(b, dtype=np.float64) for b in (bx, by, bz))
        nz, ny, nx = bx.shape
        d = _Desc()
        d.kind = mode
        d.n[:] = (nx, ny, nz)
        d.origin[:] = origin
        d.spacing[:] = spacing
        d.lo[:] = origin
        d.hi[:] = [origin[i] + (d.n[i] - 1) * spacing[i] for i in range(3)]
        d.bx, d.by, d.bz = _ptr(bx), _ptr(by), _ptr(bz)
        d.quantize = {"f64": 0, "f32": 1, "bf16": 2}[store]
        if order not in (1, 2, 3) or (order > 1 and min(d.n) < 4):
            raise ValueError("order must be 1, 2 or 3 (2 and 3 need >= 4 nodes per axis)")
        d.order = order
        d.geometry = GEOMETRIES[geometry]
        keep = [bx, by, bz]
        for a, c in enumerate(coords or (None, None, None)):
            if c is None:
                continue
            c = np.ascontiguousarray(c, dtype=np.float64)
            if c.shape != (d.n[a],) or not np.all(np.diff(c) > 0):
                raise ValueError(f"coords[{a}] must be {d.n[a]} increasing node coordinates")
            if order > 1:
                raise ValueError("rectilinear (non-uniform) axes take the trilinear kernel only")
            d.coord[a] = _ptr(c)
            d.lo[a], d.hi[a] = c[0], c[-1]
            keep.append(c)
        return cls(d, tuple(keep))

    @classmethod
    def linear(cls, b0, M, lo, hi):
        """Analytic B = b0 + M x on the closed box [lo, hi]."""
        d = _Desc()
        d.kind = ANALYTIC
        d.analytic = AN_LINEAR
        d.lin[:] = list(np.asarray(b0, float)) + list(np.asarray(M, float).reshape(9))
        d.lo[:] = lo
        d.hi[:] = hi
        return cls(d, ())

    @classmethod
    def charges(cls, charges, lo, hi, geometry="cartesian"):
        """Analytic field of point charges, rows (x, y, z, q).  With
        ``geometry="spherical"`` the box [lo, hi] is in (longitude, latitude,
        radius) and the field is seen in spherical components (a test of the
        spherical equations against the Cartesian ones)."""
        ch = np.ascontiguousarray(charges, dtype=np.float64).reshape(-1, 4)
        d = _Desc()
        d.kind = ANALYTIC
        d.analytic = AN_CHARGES
        d.charges = _ptr(ch)
        d.ncharges = ch.shape[0]
        d.lo[:] = lo
        d.hi[:] = hi
        d.geometry = GEOMETRIES[geometry]
        return cls(d, (ch,))

    def eval(self, x):
        """Bhat (as interpolated), d Bhat_i/d x_j and |B| at points x (n, 3)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        u = np.empty((n, 3))
        J = np.empty((n, 3, 3))
        b = np.empty(n)
        lib().or_field_eval(self._h, n, _ptr(x), _ptr(u), _ptr(J), _ptr(b))
        return u, J, b


def default_opts(field: Field, spacing_min: float, tol: float):
    return dict(rtol=tol, atol=tol, h_init=0.1 * spacing_min, h_max=spacing_min,
                max_length=0.0, max_steps=1 << 22)


def trace(field: Field, seeds, *, rtol, atol, h_init, h_max, max_length=0.0,
          max_steps=1 << 22, frame_angle=0.0, nthreads=0, want_ends=False, stepper="ck54",
          round_f32=False):
    """Trace seeds (n, 3) both ways; return a dict of per-seed arrays.

    stepper "ck54": adaptive Cash-Karp 5(4) (rtol, atol, first step h_init,
    largest step h_max); "euler": explicit Euler with the fixed step h_init
    (rtol, atol, h_max unused), Sect. 3.4.

    round_f32 is a test instrument, off for every parity reference: it rounds
    each CK54 stage point and each accepted state to FP32, so that a test can
    measure how many lines the roundings FP32 stepping cannot avoid move.

    Keys: fp_fwd, fp_bwd (n,3); fll, q_perp (eq. 11), q_det (determinant
    form), q_fp (exit-face planes), lam_fwd, lam_bwd (n,); status (n,) int32
    = fwd | bwd << 8 | OPEN_BIT; counts (n, 2, 3) = (accepted, rejected,
    landing iterations) per half-line; ends (n, 2, 10) if asked.
    """
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    n = seeds.shape[0]
    o = _Opts(rtol, atol, h_init, h_max, max_length, int(max_steps), frame_angle, nthreads, STEPPERS[stepper],
              int(bool(round_f32)), 0)
    out = dict(fp_fwd=np.empty((n, 3)), fp_bwd=np.empty((n, 3)), fll=np.empty(n),
               q_perp=np.empty(n), q_det=np.empty(n), q_fp=np.empty(n),
               lam_fwd=np.empty(n), lam_bwd=np.empty(n),
               status=np.empty(n, np.int32), counts=np.empty((n, 2, 3), np.int64))
    ends = np.empty((n, 2, 10)) if want_ends else None
    lib().or_trace(field._h, C.byref(o), n, _ptr(seeds), _ptr(out["fp_fwd"]), _ptr(out["fp_bwd"]),
                   _ptr(out["fll"]), _ptr(out["q_perp"]), _ptr(out["q_det"]), _ptr(out["q_fp"]),
                   _ptr(out["lam_fwd"]), _ptr(out["lam_bwd"]), _ptr(out["status"]),
                   _ptr(out["counts"]), _ptr(ends))
    if want_ends:
        out["ends"] = ends
    return out


def ck54_tableau():
    c, a, b5, b4 = np.empty(6), np.empty((6, 5)), np.empty(6), np.empty(6)
    lib().or_ck54_tableau(_ptr(c), _ptr(a), _ptr(b5), _ptr(b4))
    return c, a, b5, b4


# --------------------------------------------------------------------------
# Sect. 3.6: FLEDGE map = gradient magnitude of the Sobel operator on an FLL map
# --------------------------------------------------------------------------

def sobel_magnitude(f):
    """sqrt(sum_d G_d^2); G_d = derivative [-1, 0, 1] along axis d convolved
    with smoothing [1, 2, 1] along every other axis; mirror boundary
    (d c b a | a b c d); pixel units.  Works for 2D and 3D arrays."""
    f = np.asarray(f, dtype=np.float64)
    nd = f.ndim
    p = np.pad(f, 1, mode="symmetric")
    total = np.zeros_like(f)
    offsets = [(-1, 1.0), (0, 2.0), (1, 1.0)]
    for d in range(nd):
        g = np.zeros_like(f)
        # loop over the 3^nd stencil taps
        for taps in np.ndindex(*(3,) * nd):
            w = 1.0
            for ax, t in enumerate(taps):
                off = t - 1
                if ax == d:
                    w *= float(off)           # derivative tap: -1, 0, +1
                else:
                    w *= offsets[t][1]        # smoothing tap: 1, 2, 1
            if w == 0.0:
                continue
            sl = tuple(slice(1 + (t - 1), 1 + (t - 1) + f.shape[ax]) for ax, t in enumerate(taps))
            g += w * p[sl]
        total += g * g
    return np.sqrt(total)


# --------------------------------------------------------------------------
# Sect. 3.6: Hilbert curve on a 2^L x 2^L slice
# --------------------------------------------------------------------------

def hilbert2_xy2d(L, x, y):
    x = np.ascontiguousarray(x, dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.int64)
    d = np.empty_like(x)
    lib().or_hilbert2_xy2d(L, x.size, _ptr(x), _ptr(y), _ptr(d))
    return d


def hilbert2_d2xy(L, d):
    d = np.ascontiguousarray(d, dtype=np.int64)
    x = np.empty_like(d)
    y = np.empty_like(d)
    lib().or_hilbert2_d2xy(L, d.size, _ptr(d), _ptr(x), _ptr(y))
    return x, y


def hilbert3_d2xyz(b, d):
    """Cells (x, y, z) of curve indices d on a 2^b cube (Skilling's 3D curve)."""
    d = np.ascontiguousarray(d, dtype=np.int64)
    x, y, z = np.empty_like(d), np.empty_like(d), np.empty_like(d)
    lib().or_hilbert3_d2xyz(b, d.size, _ptr(d), _ptr(x), _ptr(y), _ptr(z))
    return x, y, z


def hilbert3_xyz2d(b, x, y, z):
    x, y, z = (np.ascontiguousarray(v, dtype=np.int64) for v in (x, y, z))
    d = np.empty_like(x)
    lib().or_hilbert3_xyz2d(b, x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(d))
    return d


class SlicePlane:
    """Horizontal slice z = z0 over [x0, x1] x [y0, y1] (Sect. 2: planar slice)."""
    dims = 2

    def __init__(self, z0, x0, x1, y0, y1):
        self.z0, self.x0, self.x1, self.y0, self.y1 = z0, x0, x1, y0, y1

    def centres(self, level, ix, iy):
        n = 1 << level
        px = self.x0 + (np.asarray(ix) + 0.5) * (self.x1 - self.x0) / n
        py = self.y0 + (np.asarray(iy) + 0.5) * (self.y1 - self.y0) / n
        return np.stack([px, py, np.full(px.shape, float(self.z0))], axis=-1)

    def cells(self, level, d):
        return hilbert2_d2xy(level, d)


class PlaneSlice:
    """Planar slice of any orientation (Sect. 2: orientation, centre and axis
    spans): the parallelogram corner + s u + t v, s, t in [0, 1], with edge
    vectors u and v.  Cell (i, j) of level L sits at corner + (i + 1/2) / 2^L u
    + (j + 1/2) / 2^L v.  In spherical geometry a slice at fixed radius over
    longitude and latitude ranges is the plane r = r0 of the coordinates."""
    dims = 2

    def __init__(self, corner, u, v):
        self.corner = np.asarray(corner, float)
        self.u = np.asarray(u, float)
        self.v = np.asarray(v, float)

    def centres(self, level, ix, iy):
        n = 1 << level
        s = (np.asarray(ix, float) + 0.5) / n
        t = (np.asarray(iy, float) + 0.5) / n
        return self.corner + s[..., None] * self.u + t[..., None] * self.v

    def cells(self, level, d):
        return hilbert2_d2xy(level, d)


class VolumeBox:
    """Axis-aligned volume [x0, x1] x [y0, y1] x [z0, z1] (3D maps)."""
    dims = 3

    def __init__(self, x0, x1, y0, y1, z0, z1):
        self.lo = np.array([x0, y0, z0], float)
        self.hi = np.array([x1, y1, z1], float)

    def centres(self, level, ix, iy, iz):
        n = 1 << level
        idx = np.stack([np.asarray(ix), np.asarray(iy), np.asarray(iz)], axis=-1).astype(float)
        return self.lo + (idx + 0.5) * (self.hi - self.lo) / n

    def cells(self, level, d):
        return hilbert3_d2xyz(level, d)


def base_samples(region, m: int, r: int):
    """Base lattice: 2^m cells per axis at their centres in level-m curve order
    q; key of cell q at the finest level m+r is q * B^r + B^r / 2 with
    B = 2^dims (4 for slices, 8 for volumes)."""
    blk = (1 << region.dims) ** r
    q = np.arange((1 << region.dims) ** m, dtype=np.int64)
    keys = q * blk + blk // 2
    return keys, region.centres(m, *region.cells(m, q))


def key_positions(region, m: int, r: int, keys):
    """Centre of the finest-level cell H^-1(key) at level m + r."""
    return region.centres(m + r, *region.cells(m + r, keys))


def refine_slice(region, m: int, r: int, thr: float, sample_fn, max_passes=64, extra_keys=None):
    """FLL-jump refinement along the Hilbert curve (Sect. 3.6), for a slice or
    a volume.

    ``sample_fn(points (n,3)) -> dict`` with at least ``fll`` and ``q``.
    Returns (keys, values dict, passes): samples in curve order.  A new sample
    goes halfway (in key) between curve-successive samples whose FLL differs
    by more than ``thr`` while they are at least two finest cells apart.
    ``extra_keys`` (finest-level keys, none of them a base key) are sampled
    with the base lattice before the first pass: the rule then starts from the
    merged, curve-ordered sample set.
    """
    keys, pts = base_samples(region, m, r)
    if extra_keys is not None and len(extra_keys):
        ek = np.unique(np.asarray(extra_keys, dtype=np.int64))
        assert np.intersect1d(ek, keys).size == 0, "extra keys must not repeat base keys"
        keys = np.concatenate([keys, ek])
        pts = np.concatenate([pts, key_positions(region, m, r, ek)])
        order = np.argsort(keys, kind="stable")
        keys, pts = keys[order], pts[order]
    vals = sample_fn(pts)
    vals = {k: np.asarray(v) for k, v in vals.items()}
    passes = 0
    while passes < max_passes:
        fll = vals["fll"]
        gap = keys[1:] - keys[:-1]
        jump = np.abs(fll[1:] - fll[:-1])
        fire = (gap >= 2) & (jump > thr)
        if not fire.any():
            break
        passes += 1
        idx = np.nonzero(fire)[0]
        newk = (keys[idx] + keys[idx + 1]) // 2
        newv = sample_fn(key_positions(region, m, r, newk))
        # every new key lies strictly between keys[i] and keys[i+1]
        keys = np.insert(keys, idx + 1, newk)
        vals = {k: np.insert(v, idx + 1, np.asarray(newv[k]), axis=0) for k, v in vals.items()}
    return keys, vals, passes


def _curve_index(region, level, cells):
    """Hilbert index at `level` of cells (one array per axis) of the region's
    curve (2D for slices, 3D for volumes)."""
    if region.dims == 2:
        return hilbert2_xy2d(level, cells[0], cells[1])
    return hilbert3_xyz2d(level, cells[0], cells[1], cells[2])


def refine_shifted(region, m: int, r: int, thr: float, sample_fn, shift: int, max_cycles=64):
    """FLL-jump refinement with the shifted-curve re-pass (Sect. 3.6, last
    paragraph: after each refinement step the curve is shifted in space, the
    samples are reordered along it, the refinement step is applied again, and
    the curve is shifted back).

    Each cycle is one pass of the rule along the curve (as refine_slice: a new
    sample at floor((k1 + k2) / 2) between curve-successive samples two or more
    finest cells apart whose lengths differ by more than ``thr``), then one
    pass of the same rule along the shifted curve: every sample's finest cell
    (the cell its key names at level L = m + r) is moved by ``shift`` finest
    cells along every axis into the square (cube) of side 2^(L+1), where the
    order-(L+1) Hilbert curve orders them; curve-successive samples of that
    order whose shifted indices differ by >= 2 and whose lengths differ by more
    than ``thr`` put a new sample in the cell of index floor((k1' + k2') / 2)
    on that curve, moved back by ``shift``, unless the cell lies outside the
    map; the new samples join the key-ordered list.  Cycles repeat until one
    inserts nothing, at most ``max_cycles``.  0 < shift < 2^L.

    Returns (keys, values dict, cycles run)."""
    L = m + r
    if not 0 < shift < (1 << L):
        raise ValueError("shift must lie in (0, 2^(m+r))")
    keys, pts = base_samples(region, m, r)
    vals = {k: np.asarray(v) for k, v in sample_fn(pts).items()}
    cycles = 0
    while cycles < max_cycles:
        cycles += 1
        inserted = 0
        # one pass along the curve
        gap = keys[1:] - keys[:-1]
        fire = (gap >= 2) & (np.abs(vals["fll"][1:] - vals["fll"][:-1]) > thr)
        if fire.any():
            idx = np.nonzero(fire)[0]
            newk = (keys[idx] + keys[idx + 1]) // 2
            newv = sample_fn(key_positions(region, m, r, newk))
            keys = np.insert(keys, idx + 1, newk)
            vals = {k: np.insert(v, idx + 1, np.asarray(newv[k]), axis=0) for k, v in vals.items()}
            inserted += newk.size
        # one pass along the shifted curve
        cells = region.cells(L, keys)
        kp = _curve_index(region, L + 1, [np.asarray(c) + shift for c in cells])
        order = np.argsort(kp, kind="stable")
        ks, fs = kp[order], vals["fll"][order]
        fire = (ks[1:] - ks[:-1] >= 2) & (np.abs(fs[1:] - fs[:-1]) > thr)
        if fire.any():
            j = np.nonzero(fire)[0]
            mid = (ks[j] + ks[j + 1]) // 2
            back = [np.asarray(c) - shift for c in region.cells(L + 1, mid)]
            inside = np.ones(mid.size, dtype=bool)
            for c in back:
                inside &= (c >= 0) & (c < (1 << L))
            newk = _curve_index(region, L, [c[inside] for c in back]) if inside.any() else np.zeros(0, np.int64)
            if newk.size:
                # a cell strictly between two successive samples of the shifted
                # order holds no sample, and distinct pairs give distinct cells
                assert np.unique(newk).size == newk.size and not np.isin(newk, keys).any()
                newv = sample_fn(key_positions(region, m, r, newk))
                keys = np.concatenate([keys, newk])
                vals = {k: np.concatenate([v, np.asarray(newv[k])], axis=0) for k, v in vals.items()}
                o = np.argsort(keys, kind="stable")
                keys = keys[o]
                vals = {k: v[o] for k, v in vals.items()}
                inserted += newk.size
        if inserted == 0:
            break
    return keys, vals, cycles


def convert_to_grid(keys, values, m: int, r: int, level: int, log_interp: bool, cells=None, dims=2):
    """Array converter (Sect. 3.6) to a grid of 2^level cells per axis
    (m <= level <= m+r), for slices (dims 2) and volumes (dims 3).

    A cell is the aligned block of finest keys it contains; its value is the
    largest sample in the block (NaN samples ignored unless all are NaN).  An
    empty cell takes the value interpolated along the curve, linearly in key
    (in log10 when ``log_interp``), between the nearest samples below and above
    the block centre.  Output indexed [iy, ix] or [iz, iy, ix]; with ``cells``
    (curve indices at ``level``) only those cells are computed and returned as
    a 1-D array.
    """
    keys = np.asarray(keys, dtype=np.int64)
    values = np.asarray(values, dtype=np.float64)
    n = 1 << level
    bsize = (1 << dims) ** (m + r - level)
    out = np.empty((n,) * dims)
    todo = range(n ** dims) if cells is None else [int(c) for c in cells]
    picked = []
    for cell in todo:
        lo, hi = cell * bsize, (cell + 1) * bsize
        a = np.searchsorted(keys, lo, side="left")
        b = np.searchsorted(keys, hi, side="left")
        if b > a:
            v = values[a:b]
            v = v[~np.isnan(v)]
            val = v.max() if v.size else np.nan
        else:
            kc = lo + (bsize - 1) / 2.0
            j = a  # first sample above the block
            if j == 0:
                val = values[0]
            elif j == keys.size:
                val = values[-1]
            else:
                k0, k1 = keys[j - 1], keys[j]
                v0, v1 = values[j - 1], values[j]
                w = (kc - k0) / (k1 - k0)
                if log_interp:
                    val = 10.0 ** ((1 - w) * np.log10(v0) + w * np.log10(v1))
                else:
                    val = (1 - w) * v0 + w * v1
        if cells is not None:
            picked.append(val)
            continue
        if dims == 2:
            x, y = hilbert2_d2xy(level, np.array([cell]))
            out[y[0], x[0]] = val
        else:
            x, y, z = hilbert3_d2xyz(level, np.array([cell]))
            out[z[0], y[0], x[0]] = val
    return out if cells is None else np.array(picked)
