"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only builds inputs: magnetic fields sampled on node-centred grids
and seed point sets.  It contains none of the tracing, interpolation, Q,
FLEDGE, Hilbert or refinement arithmetic, which the HIP library and the
oracle each implement on their own.

Domain convention: box [-1, 1]^2 x [0, 1], photosphere at z = 0, node-centred
grids (node (0,0,0) at the lower corner, node n-1 at the upper corner).
Node arrays have shape (nz, ny, nx), x fastest.
"""
from __future__ import annotations

import numpy as np

LO = (-1.0, -1.0, 0.0)
HI = (1.0, 1.0, 1.0)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_geometry(n, lo=LO, hi=HI):
    """origin and spacing of a node-centred grid with n = (nx, ny, nz) nodes."""
    origin = tuple(float(v) for v in lo)
    spacing = tuple((hi[d] - lo[d]) / (n[d] - 1) for d in range(3))
    return origin, spacing


def node_coords(n, lo=LO, hi=HI):
    origin, spacing = grid_geometry(n, lo, hi)
    return [origin[d] + spacing[d] * np.arange(n[d]) for d in range(3)]


def sample_linear(b0, M, n, lo=LO, hi=HI, dtype=np.float64):
    """B = b0 + M x sampled on the nodes."""
    xs, ys, zs = node_coords(n, lo, hi)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    M = np.asarray(M, float)
    out = []
    for i in range(3):
        out.append((b0[i] + M[i, 0] * X + M[i, 1] * Y + M[i, 2] * Z).astype(dtype))
    return out


def hyperbolic(k: float):
    """(b0, M) of the hyperbolic flux-tube field B = (k x, -k y, 1)."""
    return np.array([0.0, 0.0, 1.0]), np.diag([k, -k, 0.0])


def uniform(direction):
    d = np.asarray(direction, float)
    return d, np.zeros((3, 3))


def point_charges(seed: int, count: int, depth=(0.05, 0.15), xy=0.5, q=(0.5, 1.5)):
    """Sub-surface magnetic point charges (rows x, y, z, q), net charge zero.

    (x, y) ~ U[-xy, xy]^2, depth ~ U[depth] below z = 0, |q| ~ U[q]; the first
    ceil(count/2) are positive, the rest negative and rescaled so sum q = 0.
    """
    g = rng(seed)
    pos = g.uniform(-xy, xy, size=(count, 2))
    dep = g.uniform(depth[0], depth[1], size=count)
    mag = g.uniform(q[0], q[1], size=count)
    npos = (count + 1) // 2
    sign = np.array([1.0] * npos + [-1.0] * (count - npos))
    qv = mag * sign
    neg = qv < 0
    if neg.any():
        qv[neg] *= qv[~neg].sum() / (-qv[neg].sum())
    return np.column_stack([pos[:, 0], pos[:, 1], -dep, qv])


def sample_charges(charges, n, lo=LO, hi=HI, dtype=np.float32, zchunk=16):
    """B = sum q (r - r_i)/|r - r_i|^3 on the nodes (FP64 sums, cast at the end)."""
    xs, ys, zs = node_coords(n, lo, hi)
    nx, ny, nz = n
    out = [np.empty((nz, ny, nx), dtype) for _ in range(3)]
    Y2, X2 = np.meshgrid(ys, xs, indexing="ij")
    for z0 in range(0, nz, zchunk):
        zz = zs[z0:z0 + zchunk]
        Z = zz[:, None, None]
        acc = [np.zeros((zz.size, ny, nx)) for _ in range(3)]
        for cx, cy, cz, q in charges:
            dx = X2[None] - cx
            dy = Y2[None] - cy
            dz = Z - cz
            r2 = dx * dx + dy * dy + dz * dz
            inv3 = q / (r2 * np.sqrt(r2))
            acc[0] += dx * inv3
            acc[1] += dy * inv3
            acc[2] += dz * inv3
        for i in range(3):
            out[i][z0:z0 + zz.size] = acc[i].astype(dtype)
    return out


def pixel_seeds(nx, ny, z0=0.0, lo=LO, hi=HI):
    """Pixel centres of an nx x ny raster on the plane z = z0, raster order (x fastest)."""
    px = lo[0] + (np.arange(nx) + 0.5) * (hi[0] - lo[0]) / nx
    py = lo[1] + (np.arange(ny) + 0.5) * (hi[1] - lo[1]) / ny
    Y, X = np.meshgrid(py, px, indexing="ij")
    return np.column_stack([X.ravel(), Y.ravel(), np.full(X.size, float(z0))])


def random_seeds(seed: int, count: int, lo=LO, hi=HI, z=None):
    """Uniform random points in the box (or on the plane z if given)."""
    g = rng(seed)
    p = g.uniform(lo, hi, size=(count, 3))
    if z is not None:
        p[:, 2] = z
    return p


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def hyperbolic_c1(n=(64, 64, 64), k=2.0, dtype=np.float64):
    """Hyperbolic flux tube B = (k x, -k y, 1), k = 2, 64^3 FP64 nodes, 128^2 seeds on z = 0."""
    b0, M = hyperbolic(k)
    bx, by, bz = sample_linear(b0, M, n, dtype=dtype)
    origin, spacing = grid_geometry(n)
    return dict(b=(bx, by, bz), origin=origin, spacing=spacing, n=n,
                seeds=pixel_seeds(128, 128), k=k)


def charges_c2(n=(256, 256, 128), seed=2, count=4, dtype=np.float32):
    """4 sub-surface point charges on a 256x256x128 FP32 grid (photospheric map workload)."""
    ch = point_charges(seed, count)
    bx, by, bz = sample_charges(ch, n, dtype=dtype)
    origin, spacing = grid_geometry(n)
    return dict(b=(bx, by, bz), origin=origin, spacing=spacing, n=n, charges=ch)
