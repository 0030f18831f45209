// Map-level steps of QSL Squasher (Sect. 3.6) for gfx950:
//   - FLEDGE: Sobel gradient magnitude of a 2D/3D length map;
//   - Hilbert ordering of a 2^L x 2^L slice (iterative digit transforms);
//   - FLL-jump refinement along the curve: jump test, device-wide exclusive
//     scan, midpoint seeds, trace, order-preserving merge -- every pass runs
//     with device-side counts, so a whole map is one host-sync-free sequence;
//   - the array converter (max per output cell, log Q interpolated along the
//     curve in empty cells).
#include <math.h>

#include "qsq_internal.h"

namespace qsq {

// ---------------------------------------------------------------------------
// Hilbert curve: curve of order L starts at (0,0) and ends at (2^L-1, 0);
// quadrant digits 0..3 = lower-left (diagonal reflection), upper-left,
// upper-right (translations), lower-right (anti-diagonal reflection).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ void h2_cell(int L, uint64_t d, uint32_t &x, uint32_t &y)
{
    uint32_t cx = 0, cy = 0;   // position inside the sub-curve built so far
    for (int k = 0; k < L; ++k) {
        const uint32_t s = 1u << k;
        const uint32_t q = (uint32_t)(d >> (2 * k)) & 3u;
        uint32_t nx, ny;
        if (q == 0) {
            nx = cy;
            ny = cx;
        } else if (q == 1) {
            nx = cx;
            ny = cy + s;
        } else if (q == 2) {
            nx = cx + s;
            ny = cy + s;
        } else {
            nx = 2 * s - 1 - cy;
            ny = s - 1 - cx;
        }
        cx = nx;
        cy = ny;
    }
    x = cx;
    y = cy;
}

__host__ __device__ __forceinline__ uint64_t h2_index(int L, uint32_t x, uint32_t y)
{
    uint64_t d = 0;
    for (int k = L - 1; k >= 0; --k) {
        const uint32_t s = 1u << k;
        const uint32_t rx = (x >> k) & 1u, ry = (y >> k) & 1u;
        const uint32_t q = rx ? (ry ? 2u : 3u) : (ry ? 1u : 0u);
        d += (uint64_t)q << (2 * k);
        x &= s - 1;
        y &= s - 1;
        if (q == 0) {
            const uint32_t t = x;
            x = y;
            y = t;
        } else if (q == 3) {
            const uint32_t t = x;
            x = s - 1 - y;
            y = s - 1 - t;
        }
    }
    return d;
}

// ---------------------------------------------------------------------------
// Hilbert curve in 3D: Skilling's transpose algorithm (AIP Conf. Proc. 707,
// 2004) on three b-bit axes.  The index holds, most significant first, bit
// b-1 of x, y, z, then bit b-2 of x, y, z, ...
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ void h3_cell(int b, uint64_t d, uint32_t &x, uint32_t &y, uint32_t &z)
{
    uint32_t a0 = 0, a1 = 0, a2 = 0;
    for (int j = 0; j < b; ++j) {
        a0 |= (uint32_t)((d >> (3 * j + 2)) & 1u) << j;
        a1 |= (uint32_t)((d >> (3 * j + 1)) & 1u) << j;
        a2 |= (uint32_t)((d >> (3 * j)) & 1u) << j;
    }
    // Gray decode
    const uint32_t t0 = a2 >> 1;
    a2 ^= a1;
    a1 ^= a0;
    a0 ^= t0;
    // undo the per-level rotations and reflections, finest level first
    const uint32_t top = 2u << (b - 1);
    for (uint32_t Q = 2; Q != top; Q <<= 1) {
        const uint32_t P = Q - 1;
        uint32_t *ax[3] = {&a0, &a1, &a2};
        for (int i = 2; i >= 0; --i) {
            uint32_t &ai = *ax[i];
            if (ai & Q) {
                a0 ^= P;
            } else {
                const uint32_t t = (a0 ^ ai) & P;
                a0 ^= t;
                ai ^= t;
            }
        }
    }
    x = a0;
    y = a1;
    z = a2;
}

__host__ __device__ __forceinline__ uint64_t h3_index(int b, uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t a[3] = {x, y, z};
    const uint32_t M = 1u << (b - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (a[i] & Q) {
                a[0] ^= P;
            } else {
                const uint32_t t = (a[0] ^ a[i]) & P;
                a[0] ^= t;
                a[i] ^= t;
            }
        }
    }
    a[1] ^= a[0];
    a[2] ^= a[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (a[2] & Q) t ^= Q - 1;
    uint64_t d = 0;
    for (int j = 0; j < b; ++j) {
        d |= (uint64_t)(((a[0] ^ t) >> j) & 1u) << (3 * j + 2);
        d |= (uint64_t)(((a[1] ^ t) >> j) & 1u) << (3 * j + 1);
        d |= (uint64_t)(((a[2] ^ t) >> j) & 1u) << (3 * j);
    }
    return d;
}

// cell of a curve index at a level, for slices (DIM 2, z = 0) and volumes
template <int DIM>
__host__ __device__ __forceinline__ void cell_of_key(int level, uint64_t k, uint32_t c[3])
{
    if (DIM == 2) {
        h2_cell(level, k, c[0], c[1]);
        c[2] = 0;
    } else {
        h3_cell(level, k, c[0], c[1], c[2]);
    }
}

template <int DIM>
__host__ __device__ __forceinline__ uint64_t key_of_cell(int level, const uint32_t c[3])
{
    return DIM == 2 ? h2_index(level, c[0], c[1]) : h3_index(level, c[0], c[1], c[2]);
}

__global__ void k_h3_d2xyz(int b, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, uint32_t *z)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        h3_cell(b, d[i], x[i], y[i], z[i]);
}

__global__ void k_h3_xyz2d(int b, const uint32_t *x, const uint32_t *y, const uint32_t *z, int64_t n, uint64_t *d)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = h3_index(b, x[i], y[i], z[i]);
}

__global__ void k_h2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t a, b;
        h2_cell(L, d[i], a, b);
        x[i] = a;
        y[i] = b;
    }
}

__global__ void k_h2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = h2_index(L, x[i], y[i]);
}

static int grid_for(int64_t n, int per_cu = 16)
{
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

hipError_t launch_hilbert2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_h2_d2xy, dim3(grid_for(n)), dim3(256), 0, s, L, d, n, x, y);
    return hipGetLastError();
}

hipError_t launch_hilbert2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_h2_xy2d, dim3(grid_for(n)), dim3(256), 0, s, L, x, y, n, d);
    return hipGetLastError();
}

hipError_t launch_hilbert3_d2xyz(int b, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, uint32_t *z,
                                 hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_h3_d2xyz, dim3(grid_for(n)), dim3(256), 0, s, b, d, n, x, y, z);
    return hipGetLastError();
}

hipError_t launch_hilbert3_xyz2d(int b, const uint32_t *x, const uint32_t *y, const uint32_t *z, int64_t n,
                                 uint64_t *d, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_h3_xyz2d, dim3(grid_for(n)), dim3(256), 0, s, b, x, y, z, n, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FLEDGE: Sobel gradient magnitude, mirror boundary
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t mirror(int64_t i, int64_t n)
{
    return i < 0 ? 0 : (i >= n ? n - 1 : i);   // d c b a | a b c d, one cell deep
}

__global__ void __launch_bounds__(256) k_sobel2(const float *__restrict__ f, int64_t ny, int64_t nx,
                                                float *__restrict__ out)
{
    const int64_t N = nx * ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / nx, x = i - y * nx;
        const int64_t ym = mirror(y - 1, ny), yp = mirror(y + 1, ny);
        const int64_t xm = mirror(x - 1, nx), xp = mirror(x + 1, nx);
        const float a = f[ym * nx + xm], b = f[ym * nx + x], c = f[ym * nx + xp];
        const float d = f[y * nx + xm], e = f[y * nx + xp];
        const float g = f[yp * nx + xm], h = f[yp * nx + x], k = f[yp * nx + xp];
        const float gx = (c - a) + 2.0f * (e - d) + (k - g);
        const float gy = (g - a) + 2.0f * (h - b) + (k - c);
        out[i] = sqrtf(gx * gx + gy * gy);
    }
}

__global__ void __launch_bounds__(256) k_sobel3(const float *__restrict__ f, int64_t nz, int64_t ny,
                                                int64_t nx, float *__restrict__ out)
{
    const int64_t N = nx * ny * nz;
    const float w[3] = {1.0f, 2.0f, 1.0f};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t z = i / (nx * ny), r = i - z * nx * ny, y = r / nx, x = r - y * nx;
        float G[3] = {0.0f, 0.0f, 0.0f};
        for (int c = 0; c < 3; ++c) {
            const int64_t zz = mirror(z + c - 1, nz);
            for (int b = 0; b < 3; ++b) {
                const int64_t yy = mirror(y + b - 1, ny);
                for (int a = 0; a < 3; ++a) {
                    const int64_t xx = mirror(x + a - 1, nx);
                    const float v = f[(zz * ny + yy) * nx + xx];
                    G[0] += (float)(a - 1) * w[b] * w[c] * v;
                    G[1] += w[a] * (float)(b - 1) * w[c] * v;
                    G[2] += w[a] * w[b] * (float)(c - 1) * v;
                }
            }
        }
        out[i] = sqrtf(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    }
}

hipError_t launch_fledge(const float *in, int ndim, const int64_t *shape, float *out, hipStream_t s)
{
    if (ndim == 2) {
        const int64_t N = shape[0] * shape[1];
        hipLaunchKernelGGL(k_sobel2, dim3(grid_for(N, 32)), dim3(256), 0, s, in, shape[0], shape[1], out);
    } else {
        const int64_t N = shape[0] * shape[1] * shape[2];
        hipLaunchKernelGGL(k_sobel3, dim3(grid_for(N, 32)), dim3(256), 0, s, in, shape[0], shape[1], shape[2],
                           out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// slice refinement
// ---------------------------------------------------------------------------
// Sampled region: a horizontal slice (DIM 2, z = lo[2]) or an axis-aligned
// volume (DIM 3); d = cell size at the finest level m + r.
struct Region {
    double lo[3], d[3];
    int m, r, L;                 // base level, refine levels, finest level
    int tilted;                  // slices: 1 = a plane of any orientation (eu, ev below)
    double thr;
    double eu[3], ev[3];         // tilted slices: the finest cell's edge vectors
};

// Position of the centre of cell c at a level whose cells are `f` finest cells
// wide: axis-aligned slices and volumes offset lo along the axes; a tilted
// slice (Sect. 2: orientation, centre and axis spans) offsets it along the
// plane's edge vectors.
template <int DIM>
__device__ __forceinline__ void cell_centre(const Region &rg, const uint32_t c[3], double f, double x[3])
{
    if (DIM == 2 && rg.tilted) {
        const double s = ((double)c[0] + 0.5) * f, t = ((double)c[1] + 0.5) * f;
        for (int a = 0; a < 3; ++a) x[a] = rg.lo[a] + s * rg.eu[a] + t * rg.ev[a];
    } else {
        for (int a = 0; a < 3; ++a) x[a] = (a < DIM) ? rg.lo[a] + ((double)c[a] + 0.5) * f * rg.d[a] : rg.lo[a];
    }
}

struct Samples {
    uint64_t *keys;
    double *fll, *q;
    int32_t *status;
    int32_t *att;      // step attempts of the sample's line (nullable: not kept)
};

// base lattice: cell q of level m at its centre, key q B^r + B^r/2 (B = 2^DIM)
template <int DIM>
__global__ void k_base_seeds(Region rg, int64_t nb, int64_t stride, double *seeds, uint64_t *keys)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[3];
        cell_of_key<DIM>(rg.m, (uint64_t)q, c);
        const double f = (double)(1u << rg.r);   // base cell = f finest cells per axis
        double x[3];
        cell_centre<DIM>(rg, c, f, x);
        for (int a = 0; a < 3; ++a) seeds[a * stride + q] = x[a];
        const uint64_t blk = (uint64_t)1 << (DIM * rg.r);
        keys[q] = (uint64_t)q * blk + blk / 2;
    }
}

// keys of a base lattice given by the caller (samples in level-m curve order)
__global__ void k_base_keys(const Region rg, int64_t nb, uint64_t *keys, int dim)
{
    const uint64_t blk = (uint64_t)1 << (dim * rg.r);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x)
        keys[q] = (uint64_t)q * blk + blk / 2;
}

__global__ void k_set_count(int64_t *c, int64_t v, int32_t *overflow)
{
    *c = v;
    *overflow = 0;
}

// base length map in raster order (x fastest) for the Sobel FLEDGE
template <int DIM>
__global__ void k_fll_raster(Region rg, int64_t nb, const double *fll, float *img)
{
    const int64_t side = (int64_t)1 << rg.m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[3];
        cell_of_key<DIM>(rg.m, (uint64_t)q, c);
        img[((int64_t)c[2] * side + c[1]) * side + c[0]] = (float)fll[q];
    }
}

__device__ __forceinline__ int fires(const Samples &a, int64_t i, int64_t count, double thr)
{
    if (i + 1 >= count) return 0;
    const uint64_t k0 = a.keys[i], k1 = a.keys[i + 1];
    return (k1 - k0 >= 2) && (fabs(a.fll[i + 1] - a.fll[i]) > thr) ? 1 : 0;
}

// fire flag of the gap after each sample
__global__ void k_fire(Samples a, const int64_t *count_in, double thr, int32_t *flag)
{
    const int64_t count = *count_in;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = fires(a, i, count, thr);
}

constexpr int kScanPer = 4;                      // elements per thread
constexpr int kScanBlock = 256 * kScanPer;       // elements per block

// inclusive scan of one value per thread across a 256-thread block
__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t *lds, int64_t &block_total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == 63) lds[w] = v;
    __syncthreads();
    int64_t pre = 0;
    for (int k = 0; k < w; ++k) pre += lds[k];
    block_total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return v + pre;
}

// exclusive scan of v[0..count), three kernels: block sums, block offsets,
// apply.  Arrays are sized for the capacity; only the blocks the device count
// reaches are read or written (the grid strides over them).
__global__ void __launch_bounds__(256) k_scan_sums(const int32_t *v, const int64_t *count_in, int64_t nblocks,
                                                   int64_t *bsum)
{
    __shared__ int64_t lds[4];
    const int64_t count = *count_in;
    for (int64_t blk = blockIdx.x; blk < nblocks && blk * kScanBlock < count; blk += gridDim.x) {
        const int64_t i0 = blk * kScanBlock + (int64_t)threadIdx.x * kScanPer;
        int64_t s = 0;
        for (int k = 0; k < kScanPer; ++k)
            if (i0 + k < count) s += v[i0 + k];
        int64_t tot;
        block_incl_scan(s, lds, tot);
        if (threadIdx.x == 0) bsum[blk] = tot;
    }
}

// block offsets of the blocks the count reaches: each thread sums a
// contiguous run of block sums, one block scan of the 256 run totals, then
// each thread writes its run's offsets
__global__ void __launch_bounds__(256) k_scan_top(const int64_t *count_in, int64_t nblocks_max, int64_t *bsum,
                                                  int64_t *total)
{
    __shared__ int64_t lds[4];
    const int64_t used = (*count_in + kScanBlock - 1) / kScanBlock;
    const int64_t nblocks = used < nblocks_max ? used : nblocks_max;
    const int64_t per = (nblocks + 255) / 256;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    const int64_t b1 = b0 + per < nblocks ? b0 + per : nblocks;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bsum[b];
    int64_t tot;
    int64_t run = block_incl_scan(s, lds, tot) - s;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = bsum[b];
        bsum[b] = run;
        run += x;
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ void __launch_bounds__(256) k_scan_apply(const int32_t *v, const int64_t *count_in, int64_t nblocks,
                                                    const int64_t *boff, int32_t *off)
{
    __shared__ int64_t lds[4];
    const int64_t count = *count_in;
    for (int64_t blk = blockIdx.x; blk < nblocks && blk * kScanBlock < count; blk += gridDim.x) {
        const int64_t i0 = blk * kScanBlock + (int64_t)threadIdx.x * kScanPer;
        int32_t x[kScanPer];
        int64_t s = 0;
        for (int k = 0; k < kScanPer; ++k) {
            x[k] = i0 + k < count ? v[i0 + k] : 0;
            s += x[k];
        }
        int64_t tot;
        const int64_t incl = block_incl_scan(s, lds, tot);
        int64_t run = boff[blk] + incl - s;
        for (int k = 0; k < kScanPer; ++k) {
            if (i0 + k < count) off[i0 + k] = (int32_t)run;
            run += x[k];
        }
    }
}

// A refinement round decides D levels at once: every firing gap (size G keys)
// gets the S = 2^D - 1 keys of its bisection tree of depth D traced -- at
// spacing unit = G / 2^D on the regular lattice, or, where the gaps are
// irregular (after proposals), by repeated integer midpoints (an interval of
// fewer than 2 keys cannot be split: its slot repeats its first key and is
// never kept).
struct Round {
    int D, S;
    uint64_t unit;
    int irregular;
    int pad;
};

// key of node j (1 .. 2^D - 1, in order) of the depth-D bisection tree of the
// gap [k0, k1): integer midpoints, as the pass-by-pass rule inserts them
__device__ __forceinline__ uint64_t tree_key(uint64_t k0, uint64_t k1, int D, int j)
{
    int lo = 0, hi = 1 << D;
    uint64_t s = k0, e = k1;
    for (;;) {
        const int mi = (lo + hi) >> 1;
        const uint64_t mk = s + ((e - s) >> 1);
        if (j == mi) return mk;
        if (j < mi) {
            hi = mi;
            e = mk;
        } else {
            lo = mi;
            s = mk;
        }
    }
}

// Round set-up on the device: rem levels are left; the round decides
// D = min(batch, rem) levels at once, fewer if the firing gaps' speculative
// keys would not fit the trace slots (D = 1 always fits: one key per firing
// gap, and gaps are fewer than samples).  When no gap fires, no gap can fire at
// a finer level either (the samples do not change), so the refinement is over.
__global__ void k_round_setup(const int64_t *n_fire, int batch, int irregular, int64_t slots, int64_t *rem, Round *rd,
                              int64_t *n_eff, int64_t *n_seeds, int32_t *overflow)
{
    const int64_t nf = *n_fire;
    const int rm = (int)*rem;
    Round r{0, 0, 0, irregular, 0};
    int64_t ne = 0;
    if (rm > 0 && nf > 0) {
        int D = batch < rm ? batch : rm;
        while (D > 1 && nf * ((1 << D) - 1) > slots) --D;
        r.D = D;
        r.S = (1 << D) - 1;
        r.unit = ((uint64_t)1 << rm) >> D;
        ne = nf;
        if (ne * r.S > slots) {   // cannot happen while slots >= samples; kept as a guard
            ne = slots / r.S;
            *overflow = 1;
        }
        *rem = rm - D;
    } else {
        *rem = 0;
    }
    *rd = r;
    *n_eff = ne;
    *n_seeds = ne * r.S;
}

template <int DIM>
__global__ void k_spec_seeds(Region rg, const Round *rdp, Samples a, const int64_t *count_in, const int32_t *flag,
                             const int32_t *fpos, const int64_t *n_eff, int64_t stride, double *seeds,
                             uint64_t *nkeys)
{
    const Round rd = *rdp;
    const int64_t count = *count_in, ne = *n_eff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[i] || fpos[i] >= ne) continue;
        const int64_t base = (int64_t)fpos[i] * rd.S;
        const uint64_t k0 = a.keys[i];
        const uint64_t k1 = a.keys[i + 1];
        for (int j = 1; j <= rd.S; ++j) {
            // the regular lattice: k0 + j unit; irregular gaps (any size once
            // proposals were merged): the bisection tree's integer midpoints
            const uint64_t k = rd.irregular || rd.D == 1 ? tree_key(k0, k1, rd.D, j) : k0 + (uint64_t)j * rd.unit;
            uint32_t c[3];
            cell_of_key<DIM>(rg.L, k, c);
            const int64_t p = base + j - 1;
            nkeys[p] = k;
            double x[3];
            cell_centre<DIM>(rg, c, 1.0, x);
            for (int ax = 0; ax < 3; ++ax) seeds[ax * stride + p] = x[ax];
        }
    }
}

// The pass-by-pass rule applied to the traced values of one firing gap: an
// interval at depth d (length 2^(D-d) units) is split iff its parent was split,
// its ends differ in length by more than thr and its key gap is >= 2; the
// midpoints of split intervals are kept.  Bit j-1 of the mask keeps key j.
__device__ __forceinline__ uint32_t keep_mask(const Round &rd, double thr, double f0, double fG, const double *fs,
                                              uint64_t k0, uint64_t kG, const uint64_t *ks)
{
    const int N = 1 << rd.D;
    uint32_t keep = 0, active = 1;   // the whole gap fired
    for (int d = 0; d < rd.D; ++d) {
        const int L = N >> d;
        uint32_t next = 0;
        for (int a = 0; a < (1 << d); ++a) {
            if (!((active >> a) & 1u)) continue;
            const int m = a * L + L / 2;
            keep |= 1u << (m - 1);
            if (d + 1 < rd.D) {
                for (int c = 0; c < 2; ++c) {
                    const int s = a * L + c * (L / 2), e = s + L / 2;
                    const double fs_ = s == 0 ? f0 : fs[s - 1];
                    const double fe_ = e == N ? fG : fs[e - 1];
                    // key gap of the child (L/2 units on the regular lattice)
                    const uint64_t kg = (e == N ? kG : ks[e - 1]) - (s == 0 ? k0 : ks[s - 1]);
                    if (kg >= 2 && fabs(fe_ - fs_) > thr) next |= 1u << (2 * a + c);
                }
            }
        }
        active = next;
    }
    return keep;
}

__global__ void k_select(Region rg, const Round *rdp, Samples a, const int64_t *count_in, const int32_t *flag,
                         const int32_t *fpos, const int64_t *n_eff, const double *nfll, const uint64_t *nkeys,
                         int32_t *kcnt, uint32_t *kmask)
{
    const Round rd = *rdp;
    const int64_t count = *count_in, ne = *n_eff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = 0;
        if (flag[i] && fpos[i] < ne) {
            const int64_t p = fpos[i];
            const uint32_t mk = keep_mask(rd, rg.thr, a.fll[i], a.fll[i + 1], nfll + p * rd.S, a.keys[i],
                                          a.keys[i + 1], nkeys + p * rd.S);
            kmask[p] = mk;
            c = __popc(mk);
        }
        kcnt[i] = c;
    }
}

// order-preserving merge: sample i moves up by the kept samples before it; a
// gap's kept samples follow its first member in key order; kept samples past
// the room left in the caller's arrays are dropped (overflow is flagged)
__global__ void k_merge(const Round *rdp, Samples a, Samples b, Samples nw, const int64_t *count_in,
                        const int32_t *flag, const int32_t *fpos, const int64_t *n_eff, const int32_t *kcnt,
                        const int32_t *koff, const uint32_t *kmask, int64_t capacity)
{
    const Round rd = *rdp;
    const int64_t count = *count_in, ne = *n_eff, room = capacity - count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t off = koff[i];
        const int64_t dst = i + (off < room ? off : room);
        b.keys[dst] = a.keys[i];
        b.fll[dst] = a.fll[i];
        b.q[dst] = a.q[i];
        b.status[dst] = a.status[i];
        if (b.att) b.att[dst] = a.att[i];
        if (kcnt[i] > 0 && flag[i] && fpos[i] < ne) {
            const int64_t p = (int64_t)fpos[i] * rd.S;
            const uint32_t mk = kmask[fpos[i]];
            int64_t t = 0;
            for (int j = 1; j <= rd.S; ++j) {
                if (!((mk >> (j - 1)) & 1u)) continue;
                if (off + t < room) {
                    b.keys[dst + 1 + t] = nw.keys[p + j - 1];
                    b.fll[dst + 1 + t] = nw.fll[p + j - 1];
                    b.q[dst + 1 + t] = nw.q[p + j - 1];
                    b.status[dst + 1 + t] = nw.status[p + j - 1];
                    if (b.att) b.att[dst + 1 + t] = nw.att[p + j - 1];
                }
                ++t;
            }
        }
    }
}

__global__ void k_round_finish(const int64_t *count_in, const int64_t *n_kept, int64_t capacity, int64_t *count_out,
                               int32_t *overflow)
{
    const int64_t count = *count_in, kept = *n_kept, room = capacity - count;
    if (kept > room) *overflow = 1;
    *count_out = count + (kept < room ? kept : room);
}

__global__ void k_copy_count(const int64_t *src, int64_t *dst) { *dst = *src; }

__global__ void k_copy_samples(Samples src, Samples dst, const int64_t *count_in)
{
    const int64_t count = *count_in;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        dst.keys[i] = src.keys[i];
        dst.fll[i] = src.fll[i];
        dst.q[i] = src.q[i];
        dst.status[i] = src.status[i];
        if (dst.att) dst.att[i] = src.att[i];
    }
}

// array converter: output cell = aligned block of finest keys
template <int DIM>
__global__ void __launch_bounds__(256) k_convert(Region rg, int out_level, Samples a, const int64_t *count_in,
                                                 float *qg, float *fg)
{
    const int64_t count = *count_in;
    const int64_t side = (int64_t)1 << out_level;
    int64_t N = side * side;
    if (DIM == 3) N *= side;
    const int sh = DIM * (rg.L - out_level);
    const uint64_t B = (uint64_t)1 << sh;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[3];
        c[0] = (uint32_t)(i % side);
        c[1] = (uint32_t)((i / side) % side);
        c[2] = DIM == 3 ? (uint32_t)(i / (side * side)) : 0u;
        const uint64_t lo = key_of_cell<DIM>(out_level, c) << sh, hi = lo + B;
        // first sample with key >= lo
        int64_t l = 0, h = count;
        while (l < h) {
            const int64_t mid = (l + h) >> 1;
            if (a.keys[mid] < lo) l = mid + 1;
            else h = mid;
        }
        double qv, fv;
        if (l < count && a.keys[l] < hi) {
            double qm = NAN, fm = NAN;
            for (int64_t j = l; j < count && a.keys[j] < hi; ++j) {
                qm = fmax(qm, a.q[j]);     // fmax ignores a NaN operand
                fm = fmax(fm, a.fll[j]);
            }
            qv = qm;
            fv = fm;
        } else if (l == 0) {
            qv = a.q[0];
            fv = a.fll[0];
        } else if (l == count) {
            qv = a.q[count - 1];
            fv = a.fll[count - 1];
        } else {
            const double kc = (double)lo + 0.5 * (double)(B - 1);
            const double k0 = (double)a.keys[l - 1], k1 = (double)a.keys[l];
            const double w = (kc - k0) / (k1 - k0);
            qv = exp10((1.0 - w) * log10(a.q[l - 1]) + w * log10(a.q[l]));
            fv = (1.0 - w) * a.fll[l - 1] + w * a.fll[l];
        }
        if (qg) qg[i] = (float)qv;
        if (fg) fg[i] = (float)fv;
    }
}

// ---------------------------------------------------------------------------
// qmap orchestration (host): scratch layout and the fixed sequence of passes
// ---------------------------------------------------------------------------
static uint64_t al(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

// device scalars of a map: sample counts after each round at [0, kRoundWords),
// four per-round scalars from kRoundWords, the levels left at kRemWord
constexpr int kMaxRounds = 64;
constexpr int kRoundWords = 128;
constexpr int kRemWord = kRoundWords + 4 * kMaxRounds;
constexpr int kPropWords = kRemWord + 8;
// shifted re-pass: per cycle the shifted pass's firing count, the new samples
// kept and the sort's two scalars
constexpr int kMaxCycles = 48;
constexpr int kShiftWords = kPropWords + 8;
constexpr int kCountWords = kShiftWords + 4 * kMaxCycles;

struct QmapLayout {
    uint64_t trace, seeds, bkeys, bfll, bq, bst, batt, nkeys, nfll, nq, nst, natt, flag, fpos, kcnt, koff, kmask,
        bsum, counts, rounds, img;
    // shifted re-pass only: shifted keys and sample indices (and the sort's
    // second buffers), the new key of each shifted gap, the sort's digit counts
    // and scan space, the new samples in key order
    uint64_t skeys, sidx, skeys2, sidx2, nkey, scnt, sscan, gkeys, gfll, gq, gst, gatt, total;
    int64_t tcap, nblocks;
};

static QmapLayout layout(int dims, int m, int64_t cap, bool shifted)
{
    QmapLayout L{};
    const int64_t nb = (int64_t)1 << (dims * m);
    L.tcap = nb > cap ? nb : cap;   // trace slots: base lattice or speculative keys
    L.nblocks = (cap + kScanBlock - 1) / kScanBlock;
    uint64_t o = 0;
    L.trace = o; o += al(256 + records_bytes(L.tcap));
    L.seeds = o; o += al(3 * (uint64_t)L.tcap * 8);
    L.bkeys = o; o += al((uint64_t)cap * 8);
    L.bfll = o; o += al((uint64_t)cap * 8);
    L.bq = o; o += al((uint64_t)cap * 8);
    L.bst = o; o += al((uint64_t)cap * 4);
    L.batt = o; o += al((uint64_t)cap * 4);
    L.nkeys = o; o += al((uint64_t)L.tcap * 8);
    L.nfll = o; o += al((uint64_t)L.tcap * 8);
    L.nq = o; o += al((uint64_t)L.tcap * 8);
    L.nst = o; o += al((uint64_t)L.tcap * 4);
    L.natt = o; o += al((uint64_t)L.tcap * 4);
    L.flag = o; o += al((uint64_t)cap * 4);
    L.fpos = o; o += al((uint64_t)cap * 4);
    L.kcnt = o; o += al((uint64_t)cap * 4);
    L.koff = o; o += al((uint64_t)cap * 4);
    L.kmask = o; o += al((uint64_t)cap * 4);
    L.bsum = o; o += al((uint64_t)(L.nblocks + 1) * 8);
    L.counts = o; o += al(kCountWords * 8);
    L.rounds = o; o += al(kMaxRounds * sizeof(Round));
    L.img = o; o += al((uint64_t)nb * 4);
    if (shifted) {
        const int64_t sc = sort_count_words(L.tcap);
        L.skeys = o; o += al((uint64_t)L.tcap * 8);
        L.sidx = o; o += al((uint64_t)L.tcap * 4);
        L.skeys2 = o; o += al((uint64_t)L.tcap * 8);
        L.sidx2 = o; o += al((uint64_t)L.tcap * 4);
        L.nkey = o; o += al((uint64_t)L.tcap * 8);
        L.scnt = o; o += al((uint64_t)sc * 4);
        L.sscan = o; o += al((uint64_t)scan_tmp_words(sc) * 8);
        L.gkeys = o; o += al((uint64_t)L.tcap * 8);
        L.gfll = o; o += al((uint64_t)L.tcap * 8);
        L.gq = o; o += al((uint64_t)L.tcap * 8);
        L.gst = o; o += al((uint64_t)L.tcap * 4);
        L.gatt = o; o += al((uint64_t)L.tcap * 4);
    }
    L.total = o;
    return L;
}

uint64_t qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity)
{
    return layout(2, d->base_level, capacity, d->shift > 0).total;
}

uint64_t vmap_scratch_bytes(const qsq_volume_desc *d, int64_t capacity)
{
    return layout(3, d->base_level, capacity, d->shift > 0).total;
}

static void launch_scan(const int32_t *v, const int64_t *count_in, int64_t nblocks, int64_t *bsum, int32_t *off,
                        int64_t *total, hipStream_t st)
{
    const unsigned grid = (unsigned)(nblocks < 2048 ? nblocks : 2048);
    hipLaunchKernelGGL(k_scan_sums, dim3(grid), dim3(256), 0, st, v, count_in, nblocks, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, count_in, nblocks, bsum, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid), dim3(256), 0, st, v, count_in, nblocks, bsum, off);
}

int64_t scan_tmp_words(int64_t n_max) { return (n_max + kScanBlock - 1) / kScanBlock + 1; }

void launch_scan_i32(const int32_t *v, const int64_t *n_dev, int64_t n_max, int64_t *tmp, int32_t *off,
                     int64_t *total, hipStream_t st)
{
    const int64_t nblocks = (n_max + kScanBlock - 1) / kScanBlock;
    if (nblocks <= 0) return;
    launch_scan(v, n_dev, nblocks, tmp, off, total, st);
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

// ---------------------------------------------------------------------------
// proposals: every finest cell of a proposed base cell becomes a sample
// ---------------------------------------------------------------------------
__global__ void k_prop_flags(const uint8_t *propose, int64_t nb, int32_t *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = propose[i] ? 1 : 0;
}

// proposed cells whose B^r - 1 new keys fit the trace slots
__global__ void k_prop_setup(const int64_t *n_prop, int64_t per, int64_t slots, int64_t *n_eff, int64_t *n_seeds,
                             int32_t *overflow)
{
    int64_t ne = *n_prop;
    if (ne * per > slots) {
        ne = slots / per;
        *overflow = 1;
    }
    *n_eff = ne;
    *n_seeds = ne * per;
}

// keys q B^r + j, j != B^r / 2 (the base sample), in key order
template <int DIM>
__global__ void k_prop_seeds(Region rg, int64_t nb, const int32_t *flag, const int32_t *fpos, const int64_t *n_eff,
                             int64_t stride, double *seeds, uint64_t *nkeys)
{
    const int64_t ne = *n_eff;
    const uint64_t B = (uint64_t)1 << (DIM * rg.r), per = B - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[i] || fpos[i] >= ne) continue;
        const int64_t base = (int64_t)fpos[i] * (int64_t)per;
        for (uint64_t j = 0, p = 0; j < B; ++j) {
            if (j == B / 2) continue;
            const uint64_t k = (uint64_t)i * B + j;
            uint32_t c[3];
            cell_of_key<DIM>(rg.L, k, c);
            nkeys[base + p] = k;
            double x[3];
            cell_centre<DIM>(rg, c, 1.0, x);
            for (int ax = 0; ax < 3; ++ax) seeds[ax * stride + base + p] = x[ax];
            ++p;
        }
    }
}

__device__ __forceinline__ int64_t lower_bound_key(const uint64_t *keys, int64_t n, uint64_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// merge of two key-sorted sample lists with no key in common: every element
// lands at its own index plus its rank in the other list; beyond capacity it
// is dropped and *overflow set
__global__ void k_merge_sorted(Samples a, const int64_t *na_p, Samples nw, const int64_t *nn_p, Samples b,
                               int64_t capacity, int64_t *count_out, int32_t *overflow)
{
    const int64_t na = *na_p, nn = *nn_p;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (na + nn > capacity) *overflow = 1;
        *count_out = na + nn < capacity ? na + nn : capacity;
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na + nn; t += (int64_t)gridDim.x * blockDim.x) {
        const bool old = t < na;
        const int64_t i = old ? t : t - na;
        const Samples &src = old ? a : nw;
        const uint64_t k = src.keys[i];
        const int64_t dst = i + (old ? lower_bound_key(nw.keys, nn, k) : lower_bound_key(a.keys, na, k));
        if (dst >= capacity) continue;
        b.keys[dst] = k;
        b.fll[dst] = src.fll[i];
        b.q[dst] = src.q[i];
        b.status[dst] = src.status[i];
        if (b.att) b.att[dst] = src.att[i];
    }
}

// ---------------------------------------------------------------------------
// shifted-curve re-pass (Sect. 3.6, last paragraph)
// ---------------------------------------------------------------------------
// Index of every sample on the shifted curve: its finest cell moved by
// `shift` cells along every axis, indexed on the order L+1 curve of the square
// (cube) of side 2^(L+1) that holds the moved map; the sample's own index rides
// along for the sort.
template <int DIM>
__global__ void k_shift_keys(Region rg, int shift, Samples a, const int64_t *count_in, uint64_t *skeys,
                             int32_t *sidx)
{
    const int64_t count = *count_in;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[3];
        cell_of_key<DIM>(rg.L, a.keys[i], c);
        for (int ax = 0; ax < DIM; ++ax) c[ax] += (uint32_t)shift;
        skeys[i] = key_of_cell<DIM>(rg.L + 1, c);
        sidx[i] = (int32_t)i;
    }
}

// The rule along the shifted order: successive samples j, j+1 whose shifted
// indices differ by >= 2 and whose lengths differ by more than thr put a new
// sample in the cell of shifted index floor((k1'+k2')/2), moved back by
// `shift`, if that cell lies inside the map; flag[j] marks it, nkey[j] holds
// its key on the map's own curve.
template <int DIM>
__global__ void k_shift_fire(Region rg, int shift, Samples a, const int64_t *count_in, const uint64_t *skeys,
                             const int32_t *sidx, int32_t *flag, uint64_t *nkey)
{
    const int64_t count = *count_in;
    const int64_t side = (int64_t)1 << rg.L;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
        int32_t f = 0;
        if (j + 1 < count) {
            const uint64_t k0 = skeys[j], k1 = skeys[j + 1];
            if (k1 - k0 >= 2 && fabs(a.fll[sidx[j + 1]] - a.fll[sidx[j]]) > rg.thr) {
                uint32_t c[3];
                cell_of_key<DIM>(rg.L + 1, k0 + ((k1 - k0) >> 1), c);
                bool inside = true;
                for (int ax = 0; ax < DIM; ++ax) {
                    const int64_t v = (int64_t)c[ax] - shift;
                    inside = inside && v >= 0 && v < side;
                    c[ax] = (uint32_t)v;
                }
                if (inside) {
                    nkey[j] = key_of_cell<DIM>(rg.L, c);
                    f = 1;
                }
            }
        }
        flag[j] = f;
    }
}

// new samples that fit the trace slots (the rest set *overflow)
__global__ void k_shift_setup(const int64_t *n_new, int64_t slots, int64_t *n_eff, int32_t *overflow)
{
    int64_t ne = *n_new;
    if (ne > slots) {
        ne = slots;
        *overflow |= 1;
    }
    *n_eff = ne;
}

// seeds of the new samples, compacted in shifted order; nidx = 0, 1, ... for
// the sort into key order that follows the trace
template <int DIM>
__global__ void k_shift_seeds(Region rg, const int64_t *count_in, const int32_t *flag, const int32_t *fpos,
                              const uint64_t *nkey, const int64_t *n_eff, int64_t stride, double *seeds,
                              uint64_t *nkeys, int32_t *nidx)
{
    const int64_t count = *count_in, ne = *n_eff;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[j] || fpos[j] >= ne) continue;
        const int64_t p = fpos[j];
        const uint64_t k = nkey[j];
        uint32_t c[3];
        cell_of_key<DIM>(rg.L, k, c);
        nkeys[p] = k;
        nidx[p] = (int32_t)p;
        double x[3];
        cell_centre<DIM>(rg, c, 1.0, x);
        for (int ax = 0; ax < 3; ++ax) seeds[ax * stride + p] = x[ax];
    }
}

// the traced new samples in key order: dst[t] = src[perm[t]] (keys already sorted)
__global__ void k_gather_samples(Samples src, const int32_t *perm, const uint64_t *sorted_keys, const int64_t *n_p,
                                 Samples dst)
{
    const int64_t n = *n_p;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[t];
        dst.keys[t] = sorted_keys[t];
        dst.fll[t] = src.fll[i];
        dst.q[t] = src.q[i];
        dst.status[t] = src.status[i];
        if (dst.att) dst.att[t] = src.att[i];
    }
}

// bit 1 of *overflow: the last re-pass cycle still inserted samples
__global__ void k_cycle_check(const int64_t *count_before, const int64_t *count_after, int32_t *overflow)
{
    if (*count_after != *count_before) *overflow |= 2;
}

// Rounds to enqueue.  If the trace slots hold 2^batch - 1 keys for every
// possible firing gap (at most one per sample), no round takes fewer than
// batch levels and ceil(levels / batch) rounds suffice; otherwise a round may
// fall back to fewer levels and up to one round per level is enqueued.
// Rounds to enqueue.  A round takes the most levels (up to batch) for which
// the speculative keys of every firing pair fit the trace slots, and a round
// over n samples fires at most n pairs: the first round starts from `first`
// samples, later ones from at most `capacity`.  Enough rounds for the fewest
// levels per round are enqueued; rounds after the last level are no-ops.
static int planned_rounds(int levels, int batch, int64_t slots, int64_t first, int64_t capacity)
{
    if (levels <= 0) return 0;
    auto most = [&](int64_t n) {
        int D = batch < levels ? batch : levels;
        while (D > 1 && (double)n * (double)((1 << D) - 1) > (double)slots) --D;
        return D;
    };
    const int rem = levels - most(first), later = most(capacity);
    return 1 + (rem + later - 1) / later;
}

// One refined map of a slice (DIM 2) or volume (DIM 3): base lattice, trace,
// FLEDGE of the base lengths, refinement rounds, converter.
template <int DIM>
static hipError_t launch_map(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype, Region rg,
                             int out_level, int refine_batch, const uint8_t *propose, int shift, int max_cycles,
                             bool base_given, const qsq_map_out *out, void *scratch, hipStream_t st)
{
    const int64_t cap = out->capacity;
    const int m = rg.m, r = rg.r;
    const QmapLayout Lo = layout(DIM, m, cap, shift > 0);
    char *base = static_cast<char *>(scratch);
    const int64_t nb = (int64_t)1 << (DIM * m);

    double *seeds = reinterpret_cast<double *>(base + Lo.seeds);
    // device scalars (sample counts, per-round scalars, levels left; see kRoundWords)
    int64_t *counts = reinterpret_cast<int64_t *>(base + Lo.counts);
    // per-sample step attempts travel with the samples only if the caller asked
    const bool att = out->steps != nullptr;
    Samples A{out->keys, out->fll, out->q_perp, out->status, out->steps};
    Samples Bs{reinterpret_cast<uint64_t *>(base + Lo.bkeys), reinterpret_cast<double *>(base + Lo.bfll),
               reinterpret_cast<double *>(base + Lo.bq), reinterpret_cast<int32_t *>(base + Lo.bst),
               att ? reinterpret_cast<int32_t *>(base + Lo.batt) : nullptr};
    Samples N{reinterpret_cast<uint64_t *>(base + Lo.nkeys), reinterpret_cast<double *>(base + Lo.nfll),
              reinterpret_cast<double *>(base + Lo.nq), reinterpret_cast<int32_t *>(base + Lo.nst),
              att ? reinterpret_cast<int32_t *>(base + Lo.natt) : nullptr};
    int32_t *flag = reinterpret_cast<int32_t *>(base + Lo.flag);
    int32_t *fpos = reinterpret_cast<int32_t *>(base + Lo.fpos);
    int32_t *kcnt = reinterpret_cast<int32_t *>(base + Lo.kcnt);
    int32_t *koff = reinterpret_cast<int32_t *>(base + Lo.koff);
    uint32_t *kmask = reinterpret_cast<uint32_t *>(base + Lo.kmask);
    int64_t *bsum = reinterpret_cast<int64_t *>(base + Lo.bsum);

    TraceJob job{};
    job.nodes = f->nodes;
    job.cells = f->cells;
    job.bricks = f->bricks;
    job.dirs = static_cast<const float *>(f->dirs);
    job.storage = f->storage;
    job.mode = job_mode(f);
    job.g = g;
    job.o = o;
    job.seeds = seeds;
    job.seed_stride = Lo.tcap;
    carve_records(base + Lo.trace, Lo.tcap, &job.rec, &job.counter);
    job.out_stride = Lo.tcap;
    job.steps_sum = 1;
    job.work = reinterpret_cast<unsigned long long *>(out->work);

    // base lattice (traced here, or given in the caller's arrays)
    hipError_t e = hipSuccess;
    if (base_given) {
        hipLaunchKernelGGL(k_base_keys, dim3(grid_for(nb)), dim3(256), 0, st, rg, nb, A.keys, DIM);
        hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, &counts[0], nb, out->overflow);
    } else {
        hipLaunchKernelGGL((k_base_seeds<DIM>), dim3(grid_for(nb)), dim3(256), 0, st, rg, nb, Lo.tcap, seeds,
                           A.keys);
        hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, &counts[0], nb, out->overflow);
        job.n_host = nb;
        job.n_dev = nullptr;
        job.fll = A.fll;
        job.q_perp = A.q;
        job.status = A.status;
        job.steps = A.att;
        e = launch_trace(job, step_dtype, st);
        if (e != hipSuccess) return e;
    }
    // every stepping launch after the base lattice (proposals, refinement
    // rounds, shifted re-pass) takes the refinement gather, if the word names one
    const int rgather = (o.launch >> 10) & 7;
    if (rgather) job.o.launch = (o.launch & ~(7 << 6)) | (rgather << 6);
    if (out->fledge) {
        float *img = reinterpret_cast<float *>(base + Lo.img);
        hipLaunchKernelGGL((k_fll_raster<DIM>), dim3(grid_for(nb)), dim3(256), 0, st, rg, nb, A.fll, img);
        const int64_t side = (int64_t)1 << m;
        const int64_t shp[3] = {side, side, side};
        e = launch_fledge(img, DIM, shp, out->fledge, st);
        if (e != hipSuccess) return e;
    }

    // refinement rounds: the key gap B^r halves with every level, DIM r levels
    // in all.  Each round takes as many levels as its device set-up decides,
    // so up to DIM r rounds are enqueued; rounds after the last level are
    // no-ops (nothing fires, samples are copied to the other buffer).
    const int levels = DIM * r;
    int batch = refine_batch;
    // default: slices speculate up to 4 levels per round (their rounds are
    // bound by the longest line, so fewer rounds pay); volumes take one level
    // per round (their rounds are bound by throughput, and the speculative
    // lines a round discards cost in full)
    if (batch <= 0) batch = DIM == 2 ? (levels < 4 ? levels : 4) : 1;
    if (batch > 5) batch = 5;
    if (batch < 1) batch = 1;       // no levels: no rounds either
    int64_t *rem = &counts[kRemWord];
    Round *rds = reinterpret_cast<Round *>(base + Lo.rounds);
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, rem, (int64_t)levels);
    Samples cur = A, nxt = Bs;
    int step = 0;      // sample-count slot of the current sample list
    bool irregular = false;   // gaps no longer on the regular lattice (proposals merged)
    if (propose && levels > 0) {
        // proposals first: trace the finest cells of every proposed base cell
        // and merge them in; the gaps are irregular from here on, so the
        // rounds take the bisection trees of the gaps as they are
        int64_t *n_prop = &counts[kPropWords], *n_eff = n_prop + 1, *n_seeds = n_prop + 2;
        hipLaunchKernelGGL(k_prop_flags, dim3(grid_for(nb)), dim3(256), 0, st, propose, nb, flag);
        launch_scan(flag, &counts[0], Lo.nblocks, bsum, fpos, n_prop, st);
        const int64_t per = ((int64_t)1 << (DIM * r)) - 1;
        hipLaunchKernelGGL(k_prop_setup, dim3(1), dim3(1), 0, st, n_prop, per, Lo.tcap, n_eff, n_seeds, out->overflow);
        hipLaunchKernelGGL((k_prop_seeds<DIM>), dim3(grid_for(nb)), dim3(256), 0, st, rg, nb, flag, fpos, n_eff,
                           Lo.tcap, seeds, N.keys);
        job.n_dev = n_seeds;
        job.fll = N.fll;
        job.q_perp = N.q;
        job.status = N.status;
        job.steps = N.att;
        e = launch_trace(job, step_dtype, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_merge_sorted, dim3(grid_for(cap)), dim3(256), 0, st, cur, &counts[0], N, n_seeds, nxt,
                           cap, &counts[1], out->overflow);
        Samples t = cur;
        cur = nxt;
        nxt = t;
        step = 1;
        irregular = true;
    }
    if (shift > 0) {
        // cycles of two passes: the rule along the curve (one new key per
        // firing gap), then along the shifted curve; a cycle that inserts
        // nothing leaves the samples as they are, so later cycles do nothing
        uint64_t *skeys = reinterpret_cast<uint64_t *>(base + Lo.skeys);
        uint64_t *skeys2 = reinterpret_cast<uint64_t *>(base + Lo.skeys2);
        uint64_t *nkey = reinterpret_cast<uint64_t *>(base + Lo.nkey);
        int32_t *sidx = reinterpret_cast<int32_t *>(base + Lo.sidx);
        int32_t *sidx2 = reinterpret_cast<int32_t *>(base + Lo.sidx2);
        int32_t *scnt = reinterpret_cast<int32_t *>(base + Lo.scnt);
        int64_t *sscan = reinterpret_cast<int64_t *>(base + Lo.sscan);
        Samples G{reinterpret_cast<uint64_t *>(base + Lo.gkeys), reinterpret_cast<double *>(base + Lo.gfll),
                  reinterpret_cast<double *>(base + Lo.gq), reinterpret_cast<int32_t *>(base + Lo.gst),
                  att ? reinterpret_cast<int32_t *>(base + Lo.gatt) : nullptr};
        const int cycles = max_cycles > 0 && max_cycles < kMaxCycles ? max_cycles : kMaxCycles;
        int slot = 0;
        for (int cyc = 0; cyc < cycles; ++cyc, slot += 2) {
            int64_t *cin = &counts[slot], *cmid = &counts[slot + 1], *cout = &counts[slot + 2];
            int64_t *n_fire = &counts[kRoundWords + 4 * cyc], *n_eff = n_fire + 1, *n_seeds = n_fire + 2,
                    *n_kept = n_fire + 3;
            int64_t *sw = &counts[kShiftWords + 4 * cyc];   // new samples, kept of them, sort scalars
            // the rule along the curve
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, rem, (int64_t)1);
            hipLaunchKernelGGL(k_fire, dim3(grid_for(cap)), dim3(256), 0, st, cur, cin, rg.thr, flag);
            launch_scan(flag, cin, Lo.nblocks, bsum, fpos, n_fire, st);
            hipLaunchKernelGGL(k_round_setup, dim3(1), dim3(1), 0, st, n_fire, 1, 1, Lo.tcap, rem, &rds[cyc], n_eff,
                               n_seeds, out->overflow);
            hipLaunchKernelGGL((k_spec_seeds<DIM>), dim3(grid_for(cap)), dim3(256), 0, st, rg, &rds[cyc], cur, cin,
                               flag, fpos, n_eff, Lo.tcap, seeds, N.keys);
            job.n_dev = n_seeds;
            job.fll = N.fll;
            job.q_perp = N.q;
            job.status = N.status;
            job.steps = N.att;
            e = launch_trace(job, step_dtype, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_select, dim3(grid_for(cap)), dim3(256), 0, st, rg, &rds[cyc], cur, cin, flag, fpos,
                               n_eff, N.fll, N.keys, kcnt, kmask);
            launch_scan(kcnt, cin, Lo.nblocks, bsum, koff, n_kept, st);
            hipLaunchKernelGGL(k_merge, dim3(grid_for(cap)), dim3(256), 0, st, &rds[cyc], cur, nxt, N, cin, flag,
                               fpos, n_eff, kcnt, koff, kmask, cap);
            hipLaunchKernelGGL(k_round_finish, dim3(1), dim3(1), 0, st, cin, n_kept, cap, cmid, out->overflow);
            Samples t = cur;
            cur = nxt;
            nxt = t;
            // the rule along the shifted curve
            hipLaunchKernelGGL((k_shift_keys<DIM>), dim3(grid_for(cap)), dim3(256), 0, st, rg, shift, cur, cmid, skeys,
                               sidx);
            launch_sort_pairs64(skeys, sidx, skeys2, sidx2, scnt, sscan, &sw[2], cmid, Lo.tcap, DIM * (rg.L + 1), st);
            hipLaunchKernelGGL((k_shift_fire<DIM>), dim3(grid_for(cap)), dim3(256), 0, st, rg, shift, cur, cmid, skeys,
                               sidx, flag, nkey);
            launch_scan(flag, cmid, Lo.nblocks, bsum, fpos, &sw[0], st);
            hipLaunchKernelGGL(k_shift_setup, dim3(1), dim3(1), 0, st, &sw[0], Lo.tcap, &sw[1], out->overflow);
            hipLaunchKernelGGL((k_shift_seeds<DIM>), dim3(grid_for(cap)), dim3(256), 0, st, rg, cmid, flag, fpos, nkey,
                               &sw[1], Lo.tcap, seeds, N.keys, sidx2);
            job.n_dev = &sw[1];
            e = launch_trace(job, step_dtype, st);
            if (e != hipSuccess) return e;
            // the new samples in key order (the shifted keys' buffers are free
            // again and serve as the sort's second buffers), then merged in
            launch_sort_pairs64(N.keys, sidx2, skeys, sidx, scnt, sscan, &sw[2], &sw[1], Lo.tcap, DIM * rg.L, st);
            hipLaunchKernelGGL(k_gather_samples, dim3(grid_for(cap)), dim3(256), 0, st, N, sidx2, N.keys, &sw[1], G);
            hipLaunchKernelGGL(k_merge_sorted, dim3(grid_for(cap)), dim3(256), 0, st, cur, cmid, G, &sw[1], nxt, cap,
                               cout, out->overflow);
            t = cur;
            cur = nxt;
            nxt = t;
        }
        if (slot >= 2)
            hipLaunchKernelGGL(k_cycle_check, dim3(1), dim3(1), 0, st, &counts[slot - 2], &counts[slot], out->overflow);
        step = slot;
    }
    const int rounds = shift > 0 ? 0 : planned_rounds(levels, batch, Lo.tcap, step ? cap : nb, cap);
    int round = 0;
    for (; round < rounds; ++round) {
        int64_t *cin = &counts[step + round], *cout = &counts[step + round + 1];
        int64_t *n_fire = &counts[kRoundWords + 4 * round], *n_eff = n_fire + 1, *n_seeds = n_fire + 2,
                *n_kept = n_fire + 3;
        hipLaunchKernelGGL(k_fire, dim3(grid_for(cap)), dim3(256), 0, st, cur, cin, rg.thr, flag);
        launch_scan(flag, cin, Lo.nblocks, bsum, fpos, n_fire, st);
        hipLaunchKernelGGL(k_round_setup, dim3(1), dim3(1), 0, st, n_fire, batch, irregular ? 1 : 0, Lo.tcap, rem,
                           &rds[round], n_eff, n_seeds, out->overflow);
        hipLaunchKernelGGL((k_spec_seeds<DIM>), dim3(grid_for(cap)), dim3(256), 0, st, rg, &rds[round], cur, cin,
                           flag, fpos, n_eff, Lo.tcap, seeds, N.keys);
        job.n_dev = n_seeds;
        job.fll = N.fll;
        job.q_perp = N.q;
        job.status = N.status;
        job.steps = N.att;
        e = launch_trace(job, step_dtype, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_select, dim3(grid_for(cap)), dim3(256), 0, st, rg, &rds[round], cur, cin, flag, fpos,
                           n_eff, N.fll, N.keys, kcnt, kmask);
        launch_scan(kcnt, cin, Lo.nblocks, bsum, koff, n_kept, st);
        hipLaunchKernelGGL(k_merge, dim3(grid_for(cap)), dim3(256), 0, st, &rds[round], cur, nxt, N, cin, flag, fpos,
                           n_eff, kcnt, koff, kmask, cap);
        hipLaunchKernelGGL(k_round_finish, dim3(1), dim3(1), 0, st, cin, n_kept, cap, cout, out->overflow);
        Samples t = cur;
        cur = nxt;
        nxt = t;
    }
    // leave the samples in the caller's arrays
    const int last = step + round;
    if (last % 2 == 1) {
        hipLaunchKernelGGL(k_copy_samples, dim3(grid_for(cap)), dim3(256), 0, st, cur, A, &counts[last]);
        cur = A;
    }
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, st, &counts[last], out->count);
    if (out->q_grid || out->fll_grid) {
        const int64_t No = (int64_t)1 << (DIM * out_level);
        hipLaunchKernelGGL((k_convert<DIM>), dim3(grid_for(No, 32)), dim3(256), 0, st, rg, out_level, cur,
                           &counts[last], out->q_grid, out->fll_grid);
    }
    return hipGetLastError();
}

hipError_t launch_qmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_map_desc *d, const qsq_map_out *out, void *scratch, hipStream_t st)
{
    Region rg{};
    rg.m = d->base_level;
    rg.r = d->refine_levels;
    rg.L = rg.m + rg.r;
    const double nL = (double)((int64_t)1 << rg.L);
    rg.lo[0] = d->x0;
    rg.lo[1] = d->y0;
    rg.lo[2] = d->z0;
    rg.d[0] = (d->x1 - d->x0) / nL;
    rg.d[1] = (d->y1 - d->y0) / nL;
    rg.d[2] = 0.0;
    rg.thr = d->threshold;
    if (d->tilted) {
        rg.tilted = 1;
        for (int a = 0; a < 3; ++a) {
            rg.lo[a] = d->corner[a];
            rg.eu[a] = d->edge_u[a] / nL;
            rg.ev[a] = d->edge_v[a] / nL;
        }
    }
    return launch_map<2>(f, g, o, step_dtype, rg, d->out_level, d->refine_batch, d->propose, d->shift, d->max_cycles,
                         d->base_given != 0, out, scratch, st);
}

hipError_t launch_vmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_volume_desc *d, const qsq_map_out *out, void *scratch, hipStream_t st)
{
    Region rg{};
    rg.m = d->base_level;
    rg.r = d->refine_levels;
    rg.L = rg.m + rg.r;
    const double nL = (double)((int64_t)1 << rg.L);
    const double lo[3] = {d->x0, d->y0, d->z0}, hi[3] = {d->x1, d->y1, d->z1};
    for (int a = 0; a < 3; ++a) {
        rg.lo[a] = lo[a];
        rg.d[a] = (hi[a] - lo[a]) / nL;
    }
    rg.thr = d->threshold;
    return launch_map<3>(f, g, o, step_dtype, rg, d->out_level, d->refine_batch, d->propose, d->shift, d->max_cycles,
                         false, out, scratch, st);
}

}  // namespace qsq
