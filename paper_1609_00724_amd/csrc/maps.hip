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
struct Slice {
    double z0, x0, y0, dx, dy;   // pixel size at the finest level: dx, dy
    int m, r, L;                 // base level, refine levels, finest level
    double thr;
};

struct Samples {
    uint64_t *keys;
    double *fll, *q;
    int32_t *status;
};

// base lattice: pixel q of level m at its centre, key q*4^r + 4^r/2
__global__ void k_base_seeds(Slice sl, int64_t nb, int64_t stride, double *seeds, uint64_t *keys)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t ix, iy;
        h2_cell(sl.m, (uint64_t)q, ix, iy);
        const double f = (double)(1u << sl.r);   // base pixel = f finest pixels
        seeds[q] = sl.x0 + ((double)ix + 0.5) * f * sl.dx;
        seeds[stride + q] = sl.y0 + ((double)iy + 0.5) * f * sl.dy;
        seeds[2 * stride + q] = sl.z0;
        const uint64_t blk = (uint64_t)1 << (2 * sl.r);
        keys[q] = (uint64_t)q * blk + blk / 2;
    }
}

__global__ void k_set_count(int64_t *c, int64_t v, int32_t *overflow)
{
    *c = v;
    *overflow = 0;
}

// base length map in raster order for the Sobel FLEDGE
__global__ void k_fll_raster(Slice sl, int64_t nb, const double *fll, float *img)
{
    const uint32_t side = 1u << sl.m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t ix, iy;
        h2_cell(sl.m, (uint64_t)q, ix, iy);
        img[(int64_t)iy * side + ix] = (float)fll[q];
    }
}

__device__ __forceinline__ int fires(const Samples &a, int64_t i, int64_t count, double thr)
{
    if (i + 1 >= count) return 0;
    const uint64_t k0 = a.keys[i], k1 = a.keys[i + 1];
    return (k1 - k0 >= 2) && (fabs(a.fll[i + 1] - a.fll[i]) > thr) ? 1 : 0;
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

__global__ void __launch_bounds__(256) k_scan_sums(Samples a, const int64_t *count_in, double thr, int64_t *bsum)
{
    __shared__ int64_t lds[4];
    const int64_t count = *count_in;
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    if (b0 >= count) {
        if (threadIdx.x == 0) bsum[blockIdx.x] = 0;
        return;
    }
    int64_t v = 0;
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kScanPer;
    for (int k = 0; k < kScanPer; ++k) v += fires(a, i0 + k, count, thr);
    int64_t tot;
    block_incl_scan(v, lds, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single block: exclusive offsets of the block sums, new-sample count, capacity
__global__ void __launch_bounds__(256) k_scan_top(int64_t nblocks, int64_t *bsum, const int64_t *count_in,
                                                  int64_t *count_out, int64_t *n_new, int64_t capacity,
                                                  int32_t *overflow)
{
    __shared__ int64_t lds[4];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblocks; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nblocks ? bsum[i] : 0;
        int64_t tot;
        const int64_t incl = block_incl_scan(v, lds, tot);
        if (i < nblocks) bsum[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t cnt = *count_in;
        int64_t add = carry;
        if (cnt + add > capacity) {
            add = capacity - cnt;
            *overflow = 1;
        }
        *n_new = add;
        *count_out = cnt + add;
    }
}

__global__ void __launch_bounds__(256) k_scan_apply(Samples a, const int64_t *count_in, double thr,
                                                    const int64_t *boff, int32_t *pos)
{
    __shared__ int64_t lds[4];
    const int64_t count = *count_in;
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    if (b0 >= count) return;
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kScanPer;
    int f[kScanPer];
    int64_t v = 0;
    for (int k = 0; k < kScanPer; ++k) {
        f[k] = fires(a, i0 + k, count, thr);
        v += f[k];
    }
    int64_t tot;
    const int64_t incl = block_incl_scan(v, lds, tot);
    int64_t run = boff[blockIdx.x] + incl - v;
    for (int k = 0; k < kScanPer; ++k) {
        if (i0 + k < count) pos[i0 + k] = (int32_t)run;
        run += f[k];
    }
}

// midpoint keys and their seeds (centre of the finest cell)
__global__ void k_new_seeds(Slice sl, Samples a, const int64_t *count_in, const int64_t *n_new,
                            const int32_t *pos, int64_t stride, double *seeds, uint64_t *nkeys)
{
    const int64_t count = *count_in, nn = *n_new;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        if (!fires(a, i, count, sl.thr)) continue;
        const int64_t p = pos[i];
        if (p >= nn) continue;
        const uint64_t k = (a.keys[i] + a.keys[i + 1]) >> 1;
        uint32_t ix, iy;
        h2_cell(sl.L, k, ix, iy);
        nkeys[p] = k;
        seeds[p] = sl.x0 + ((double)ix + 0.5) * sl.dx;
        seeds[stride + p] = sl.y0 + ((double)iy + 0.5) * sl.dy;
        seeds[2 * stride + p] = sl.z0;
    }
}

// order-preserving merge: sample i moves up by the insertions before it; an
// inserted sample follows the pair's first member
__global__ void k_merge(Slice sl, Samples a, Samples b, Samples nw, const int64_t *count_in,
                        const int64_t *n_new, const int32_t *pos)
{
    const int64_t count = *count_in, nn = *n_new;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = pos[i];
        const int64_t before = p < nn ? p : nn;
        const int64_t dst = i + before;
        b.keys[dst] = a.keys[i];
        b.fll[dst] = a.fll[i];
        b.q[dst] = a.q[i];
        b.status[dst] = a.status[i];
        if (p < nn && fires(a, i, count, sl.thr)) {
            b.keys[dst + 1] = nw.keys[p];
            b.fll[dst + 1] = nw.fll[p];
            b.q[dst + 1] = nw.q[p];
            b.status[dst + 1] = nw.status[p];
        }
    }
}

__global__ void k_copy_count(const int64_t *src, int64_t *dst) { *dst = *src; }

// array converter: output cell = aligned block of finest keys
__global__ void __launch_bounds__(256) k_convert(Slice sl, int out_level, Samples a, const int64_t *count_in,
                                                 float *qg, float *fg)
{
    const int64_t count = *count_in;
    const uint32_t side = 1u << out_level;
    const int64_t N = (int64_t)side * side;
    const int sh = 2 * (sl.L - out_level);
    const uint64_t B = (uint64_t)1 << sh;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t iy = (uint32_t)(i / side), ix = (uint32_t)(i - (int64_t)iy * side);
        const uint64_t c = h2_index(out_level, ix, iy);
        const uint64_t lo = c << sh, hi = lo + B;
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

struct QmapLayout {
    uint64_t trace, seeds, bkeys, bfll, bq, bst, nkeys, nfll, nq, nst, pos, bsum, counts, img, total;
    int64_t tcap, nblocks;
};

static QmapLayout layout(const qsq_map_desc *d, int64_t cap)
{
    QmapLayout L{};
    const int64_t nb = (int64_t)1 << (2 * d->base_level);
    L.tcap = nb > (cap + 1) / 2 ? nb : (cap + 1) / 2;
    L.nblocks = (cap + kScanBlock - 1) / kScanBlock;
    uint64_t o = 0;
    L.trace = o; o += al(256 + records_bytes(L.tcap));
    L.seeds = o; o += al(3 * (uint64_t)L.tcap * 8);
    L.bkeys = o; o += al((uint64_t)cap * 8);
    L.bfll = o; o += al((uint64_t)cap * 8);
    L.bq = o; o += al((uint64_t)cap * 8);
    L.bst = o; o += al((uint64_t)cap * 4);
    L.nkeys = o; o += al((uint64_t)L.tcap * 8);
    L.nfll = o; o += al((uint64_t)L.tcap * 8);
    L.nq = o; o += al((uint64_t)L.tcap * 8);
    L.nst = o; o += al((uint64_t)L.tcap * 4);
    L.pos = o; o += al((uint64_t)cap * 4);
    L.bsum = o; o += al((uint64_t)(L.nblocks + 1) * 8);
    L.counts = o; o += al(64 * 8);
    L.img = o; o += al((uint64_t)nb * 4);
    L.total = o;
    return L;
}

uint64_t qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity)
{
    return layout(d, capacity).total;
}

hipError_t launch_qmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_map_desc *d, const qsq_map_out *out, void *scratch, hipStream_t st)
{
    const int64_t cap = out->capacity;
    const QmapLayout Lo = layout(d, cap);
    char *base = static_cast<char *>(scratch);
    const int m = d->base_level, r = d->refine_levels;
    const int64_t nb = (int64_t)1 << (2 * m);

    Slice sl;
    sl.z0 = d->z0;
    sl.x0 = d->x0;
    sl.y0 = d->y0;
    sl.m = m;
    sl.r = r;
    sl.L = m + r;
    sl.dx = (d->x1 - d->x0) / (double)((int64_t)1 << sl.L);
    sl.dy = (d->y1 - d->y0) / (double)((int64_t)1 << sl.L);
    sl.thr = d->threshold;

    double *seeds = reinterpret_cast<double *>(base + Lo.seeds);
    int64_t *counts = reinterpret_cast<int64_t *>(base + Lo.counts);   // [0..2r] totals, [32..] n_new
    Samples A{out->keys, out->fll, out->q_perp, out->status};
    Samples Bs{reinterpret_cast<uint64_t *>(base + Lo.bkeys), reinterpret_cast<double *>(base + Lo.bfll),
               reinterpret_cast<double *>(base + Lo.bq), reinterpret_cast<int32_t *>(base + Lo.bst)};
    Samples N{reinterpret_cast<uint64_t *>(base + Lo.nkeys), reinterpret_cast<double *>(base + Lo.nfll),
              reinterpret_cast<double *>(base + Lo.nq), reinterpret_cast<int32_t *>(base + Lo.nst)};
    int32_t *pos = reinterpret_cast<int32_t *>(base + Lo.pos);
    int64_t *bsum = reinterpret_cast<int64_t *>(base + Lo.bsum);

    TraceJob job{};
    job.nodes = f->nodes;
    job.storage = f->storage;
    job.mode = f->mode;
    job.g = g;
    job.o = o;
    job.seeds = seeds;
    job.seed_stride = Lo.tcap;
    carve_records(base + Lo.trace, Lo.tcap, &job.rec, &job.counter);
    job.out_stride = Lo.tcap;
    job.work = reinterpret_cast<unsigned long long *>(out->work);

    // base lattice
    hipLaunchKernelGGL(k_base_seeds, dim3(grid_for(nb)), dim3(256), 0, st, sl, nb, Lo.tcap, seeds, A.keys);
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, &counts[0], nb, out->overflow);
    job.n_host = nb;
    job.n_dev = nullptr;
    job.fll = A.fll;
    job.q_perp = A.q;
    job.status = A.status;
    hipError_t e = launch_trace(job, step_dtype, st);
    if (e != hipSuccess) return e;
    if (out->fledge) {
        float *img = reinterpret_cast<float *>(base + Lo.img);
        hipLaunchKernelGGL(k_fll_raster, dim3(grid_for(nb)), dim3(256), 0, st, sl, nb, A.fll, img);
        const int64_t shp[2] = {(int64_t)1 << m, (int64_t)1 << m};
        e = launch_fledge(img, 2, shp, out->fledge, st);
        if (e != hipSuccess) return e;
    }

    // refinement passes: the key gap 4^r halves each pass, so 2r passes suffice
    Samples cur = A, nxt = Bs;
    const int passes = 2 * r;
    for (int p = 1; p <= passes; ++p) {
        int64_t *cin = &counts[p - 1], *cout = &counts[p], *nn = &counts[32 + p];
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)Lo.nblocks), dim3(256), 0, st, cur, cin, sl.thr, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, Lo.nblocks, bsum, cin, cout, nn, cap,
                           out->overflow);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)Lo.nblocks), dim3(256), 0, st, cur, cin, sl.thr, bsum,
                           pos);
        hipLaunchKernelGGL(k_new_seeds, dim3(grid_for(cap)), dim3(256), 0, st, sl, cur, cin, nn, pos, Lo.tcap,
                           seeds, N.keys);
        job.n_dev = nn;
        job.fll = N.fll;
        job.q_perp = N.q;
        job.status = N.status;
        e = launch_trace(job, step_dtype, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_merge, dim3(grid_for(cap)), dim3(256), 0, st, sl, cur, nxt, N, cin, nn, pos);
        Samples t = cur;
        cur = nxt;
        nxt = t;
    }
    // an even number of passes leaves the samples in the caller's arrays
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, st, &counts[passes], out->count);
    if (out->q_grid || out->fll_grid) {
        const int64_t No = (int64_t)1 << (2 * d->out_level);
        hipLaunchKernelGGL(k_convert, dim3(grid_for(No, 32)), dim3(256), 0, st, sl, d->out_level, cur,
                           &counts[passes], out->q_grid, out->fll_grid);
    }
    return hipGetLastError();
}

}  // namespace qsq
