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


def sample_charges(charges, n, lo=LO, hi=HI, dtype=np.float32, zchunk=16, device=None):
    """B = sum q (r - r_i)/|r - r_i|^3 on the nodes (FP64 sums, cast at the end;
    with torch on `device` if given, else numpy)."""
    if device is not None:
        return _sample_charges_torch(charges, n, lo, hi, dtype, device)
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


def _sample_charges_torch(charges, n, lo, hi, dtype, device):
    import torch
    f64 = dict(dtype=torch.float64, device=torch.device(device))
    xs, ys, zs = (torch.tensor(c, **f64) for c in node_coords(n, lo, hi))
    Z, Y, X = torch.meshgrid(zs, ys, xs, indexing="ij")
    acc = [torch.zeros_like(X) for _ in range(3)]
    for cx, cy, cz, q in np.asarray(charges, float):
        dx, dy, dz = X - cx, Y - cy, Z - cz
        inv3 = q * (dx * dx + dy * dy + dz * dz) ** -1.5
        acc[0] += dx * inv3
        acc[1] += dy * inv3
        acc[2] += dz * inv3
    return [a.cpu().numpy().astype(dtype) for a in acc]


def charges_device(charges, n, device, base=None, lo=LO, hi=HI):
    """sample_charges kept on `device`: FP64 sums (plus the FP64 device
    tensors `base`, if given) cast to three FP32 torch tensors (nz, ny, nx)."""
    import torch
    f64 = dict(dtype=torch.float64, device=torch.device(device))
    xs, ys, zs = (torch.tensor(c, **f64) for c in node_coords(n, lo, hi))
    out = []
    for comp in range(3):
        acc = base[comp].clone() if base is not None else torch.zeros((n[2], n[1], n[0]), **f64)
        for z0 in range(0, n[2], 32):
            Z = zs[z0:z0 + 32, None, None]
            for cx, cy, cz, q in np.asarray(charges, float):
                dx, dy, dz = xs[None, None, :] - cx, ys[None, :, None] - cy, Z - cz
                inv3 = q * (dx * dx + dy * dy + dz * dz) ** -1.5
                acc[z0:z0 + 32] += (dx, dy, dz)[comp] * inv3
        out.append(acc.float())
        del acc
    return out


def rope_charges(seed: int, ring_radius=0.3, depth=0.1, leg_charge=1.5):
    """Background charges of a flux-rope field: +leg_charge and -leg_charge
    under the rope's two legs (x = +-sqrt(R^2 - depth^2), z = -depth) and four
    drawn as point_charges(seed, 4)."""
    xleg = float(np.sqrt(ring_radius ** 2 - depth ** 2))
    legs = np.array([[xleg, 0.0, -depth, leg_charge], [-xleg, 0.0, -depth, -leg_charge]])
    return np.vstack([legs, point_charges(seed, 4)])


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


C3_DIMS = ((64, 64, 64), (96, 96, 96), (128, 128, 128), (128, 128, 64), (192, 192, 96), (256, 256, 128))


def batch_c3(count=64, first_seed=3000, dims=C3_DIMS, seeds_range=(1e4, 1e6), dtype=np.float32):
    """Many-field batch: field k uses seed first_seed + k; 2..8 sub-surface
    charges drawn as in point_charges; grid dims cycle through `dims`; seed
    count log-uniform in seeds_range, uniform random points on z = 0.

    Yields one dict per field (b, origin, spacing, n, charges, seeds)."""
    for k in range(count):
        s = first_seed + k
        g = rng(s)
        nch = int(g.integers(2, 9))
        m = int(round(np.exp(g.uniform(np.log(seeds_range[0]), np.log(seeds_range[1])))))
        ch = point_charges(s, nch)
        n = tuple(dims[k % len(dims)])
        origin, spacing = grid_geometry(n)
        yield dict(b=sample_charges(ch, n, dtype=dtype), origin=origin, spacing=spacing, n=n, charges=ch,
                   seeds=random_seeds(s + 100000, m, z=0.0))


def flux_rope_field(n, ring_radius=0.3, depth=0.1, minor=0.08, current=0.5, turns=1.5, leg_charge=1.5,
                    charges=None, quad=96, device=None, dtype=np.float32):
    """Twisted flux rope over a potential background, sampled on the nodes.

    Poloidal part: a circular line current of radius `ring_radius` in the x-z
    plane, centre (0, 0, -depth), by Biot-Savart quadrature (`quad` points,
    trapezoid rule) with the kernel softened over `minor`:
    dB = I dl x r / (|r|^2 + minor^2)^(3/2), the curl of a smooth vector
    potential, so divergence-free.  Toroidal part: B_phi(rho) e_phi with
    B_phi = B0 (1 - rho^2 / minor^2) inside the tube (rho = distance to the
    ring's core circle), e_phi the azimuthal direction about the ring's axis
    (the y axis): axisymmetric, so divergence-free.  B0 gives about `turns`
    turns of twist at rho = minor / 2 over the rope's length above z = 0.
    Background: point charges (rows x, y, z, q) as in sample_charges; by
    default +leg_charge and -leg_charge under the two legs plus four charges
    drawn as in point_charges(4, 4).

    Sums run in FP64 with torch (on `device` if given) and are cast at the end."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cpu")
    f64 = dict(dtype=torch.float64, device=dev)
    R, zc, a = ring_radius, -depth, minor
    if charges is None:
        charges = rope_charges(4, ring_radius, depth, leg_charge)
    th = torch.arange(quad, **f64) * (2 * np.pi / quad)
    px, pz = R * torch.cos(th), zc + R * torch.sin(th)                  # ring points
    tx, tz = -R * torch.sin(th) * (2 * np.pi / quad), R * torch.cos(th) * (2 * np.pi / quad)   # dl

    def ring_b(X, Y, Z):
        bx = torch.zeros_like(X)
        by = torch.zeros_like(X)
        bz = torch.zeros_like(X)
        for k in range(quad):
            rx, rz = X - px[k], Z - pz[k]
            w = current * (rx * rx + Y * Y + rz * rz + a * a) ** -1.5
            # dl = (tx, 0, tz); dl x r = (0*rz - tz*Y, tz*rx - tx*rz, tx*Y - 0*rx)
            bx -= w * tz[k] * Y
            by += w * (tz[k] * rx - tx[k] * rz)
            bz += w * tx[k] * Y
        return bx, by, bz

    def phi_dir(X, Z):
        s = torch.sqrt(X * X + (Z - zc) ** 2)
        return -(Z - zc) / s, X / s, s

    # toroidal amplitude from the poloidal field at rho = a/2 below the apex
    P = torch.tensor([0.0], **f64), torch.tensor([0.0], **f64), torch.tensor([zc + R - a / 2], **f64)
    bp = float(torch.sqrt(sum(c * c for c in ring_b(*P)))[0])
    arc = R * (np.pi - 2 * np.arcsin(-zc / R))
    rho0 = a / 2
    B0 = arc * bp / (2 * np.pi * rho0 * turns * (1 - (rho0 / a) ** 2))

    xs, ys, zs = node_coords(n)
    nx, ny, nz = n
    out = [np.empty((nz, ny, nx), dtype) for _ in range(3)]
    Y2, X2 = torch.meshgrid(torch.tensor(ys, **f64), torch.tensor(xs, **f64), indexing="ij")
    zchunk = max(1, (1 << 22) // (nx * ny))
    for z0 in range(0, nz, zchunk):
        zz = torch.tensor(zs[z0:z0 + zchunk], **f64)
        Z = zz[:, None, None].expand(-1, ny, nx)
        X = X2[None].expand_as(Z)
        Y = Y2[None].expand_as(Z)
        bx, by, bz = ring_b(X, Y, Z)
        ex, ez, s = phi_dir(X, Z)
        rho2 = (s - R) ** 2 + Y * Y
        bt = torch.where(rho2 < a * a, B0 * (1 - rho2 / (a * a)), torch.zeros_like(rho2))
        bx = bx + bt * ex
        bz = bz + bt * ez
        for cx, cy, cz, q in charges:
            dx, dy, dz = X - cx, Y - cy, Z - cz
            r2 = dx * dx + dy * dy + dz * dz
            inv3 = q * r2 ** -1.5
            bx = bx + dx * inv3
            by = by + dy * inv3
            bz = bz + dz * inv3
        for i, c in enumerate((bx, by, bz)):
            out[i][z0:z0 + zz.numel()] = c.cpu().numpy().astype(dtype)
    return out, dict(charges=charges, B0=B0, ring_radius=R, depth=depth, minor=a, current=current)


def flux_rope_c4(n=(384, 384, 256), dtype=np.float32, device=None):
    """Flux rope over a 6-charge background on a 384x384x256 grid (volume workload)."""
    b, meta = flux_rope_field(n, dtype=dtype, device=device)
    origin, spacing = grid_geometry(n)
    return dict(b=b, origin=origin, spacing=spacing, n=n, **meta)


def sample_charges_spherical(charges, n, lo, hi, dtype=np.float64):
    """The point-charge field on a (longitude, latitude, radius) grid of n =
    (n_phi, n_theta, n_r) nodes spanning [lo, hi], as the components (B_phi,
    B_theta, B_r) in the local orthonormal basis, arrays shaped (n_r, n_theta,
    n_phi).  Returns (b, origin, spacing)."""
    axes = [np.linspace(lo[d], hi[d], n[d]) for d in range(3)]
    R, TH, PH = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    X = R * np.cos(TH) * np.cos(PH)
    Y = R * np.cos(TH) * np.sin(PH)
    Z = R * np.sin(TH)
    B = [np.zeros_like(X) for _ in range(3)]
    for cx, cy, cz, q in charges:
        dx, dy, dz = X - cx, Y - cy, Z - cz
        inv3 = q / (dx * dx + dy * dy + dz * dz) ** 1.5
        B[0] += dx * inv3
        B[1] += dy * inv3
        B[2] += dz * inv3
    e_phi = (-np.sin(PH), np.cos(PH), 0.0 * PH)
    e_th = (-np.sin(TH) * np.cos(PH), -np.sin(TH) * np.sin(PH), np.cos(TH))
    e_r = (np.cos(TH) * np.cos(PH), np.cos(TH) * np.sin(PH), np.sin(TH))
    comp = [sum(B[k] * e[k] for k in range(3)).astype(dtype) for e in (e_phi, e_th, e_r)]
    origin = tuple(float(lo[d]) for d in range(3))
    spacing = tuple((hi[d] - lo[d]) / (n[d] - 1) for d in range(3))
    return comp, origin, spacing
