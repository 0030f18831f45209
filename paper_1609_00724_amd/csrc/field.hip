// Field preparation (Sect. 3.2; footnote to Sect. 3.5): one streaming pass that
// turns three node arrays of B into 4-vector node records (FP64, FP32 or BF16).
// PAPER mode stores (B/|B|, |B|) with the normalisation done in FP64 (zero
// direction where |B| < 1e-30); INTERP_NORMALIZE stores (B, 0).
#include <math.h>

#include "qsq_internal.h"

namespace qsq {

template <typename I>
__device__ __forceinline__ double rd(const void *p, int64_t i)
{
    return (double)static_cast<const I *>(p)[i];
}

__device__ __forceinline__ void store4(float *o, int64_t i, double a, double b, double c, double d)
{
    reinterpret_cast<float4 *>(o)[i] = make_float4((float)a, (float)b, (float)c, (float)d);
}

__device__ __forceinline__ void store4(double *o, int64_t i, double a, double b, double c, double d)
{
    double2 *q = reinterpret_cast<double2 *>(o) + 2 * i;
    q[0] = make_double2(a, b);
    q[1] = make_double2(c, d);
}

// BF16: the value rounded to FP32, then to the nearest BF16 (ties to even)
__device__ __forceinline__ uint32_t bf16_bits(double x)
{
    const uint32_t u = __float_as_uint((float)x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void store4(Bf16 *o, int64_t i, double a, double b, double c, double d)
{
    reinterpret_cast<uint2 *>(o)[i] = make_uint2(bf16_bits(a) | (bf16_bits(b) << 16), bf16_bits(c) | (bf16_bits(d) << 16));
}

template <typename I, typename S, int MODE>
__global__ void __launch_bounds__(256) k_field_init(const void *bx, const void *by, const void *bz,
                                                    S *out, int64_t N)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = rd<I>(bx, i), y = rd<I>(by, i), z = rd<I>(bz, i);
        if (MODE == QSQ_INTERP_PAPER) {
            const double b = sqrt(x * x + y * y + z * z);
            if (b < 1e-30)
                store4(out, i, 0.0, 0.0, 0.0, b);
            else
                store4(out, i, x / b, y / b, z / b, b);
        } else {
            store4(out, i, x, y, z, 0.0);
        }
    }
}

template <typename I, typename S>
static void go(const void *bx, const void *by, const void *bz, int mode, void *ws, int64_t N,
               hipStream_t st)
{
    const int cus = device_cu_count();
    int64_t want = (N + 255) / 256;
    const int blocks = (int)(want < (int64_t)cus * 32 ? want : (int64_t)cus * 32);
    if (mode == QSQ_INTERP_PAPER)
        hipLaunchKernelGGL((k_field_init<I, S, QSQ_INTERP_PAPER>), dim3(blocks), dim3(256), 0, st, bx,
                           by, bz, static_cast<S *>(ws), N);
    else
        hipLaunchKernelGGL((k_field_init<I, S, QSQ_INTERP_NORMALIZE>), dim3(blocks), dim3(256), 0, st,
                           bx, by, bz, static_cast<S *>(ws), N);
}

// cell records: the 8 corner records of every cell, corner a + 2b + 4c =
// node (i+a, j+b, k+c), copied whole (R is one record: 16, 8 or 32 bytes)
template <typename R>
__global__ void __launch_bounds__(256) k_cell_records(const R *__restrict__ nodes, int64_t nx, int64_t ny,
                                                      int64_t ncells, R *__restrict__ cells)
{
    const int64_t cx = nx - 1, cy = ny - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 8 * ncells;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e >> 3;
        const int v = (int)(e & 7);
        const int64_t i = c % cx, j = (c / cx) % cy, k = c / (cx * cy);
        const int64_t n = ((k + (v >> 2)) * ny + j + ((v >> 1) & 1)) * nx + i + (v & 1);
        cells[e] = nodes[n];
    }
}

uint64_t cell_record_bytes(const qsq_grid *g, int storage)
{
    const uint64_t rec = storage == QSQ_F64 ? 32 : storage == QSQ_F32 ? 16 : 8;
    return 8 * rec * (uint64_t)(g->n[0] - 1) * (uint64_t)(g->n[1] - 1) * (uint64_t)(g->n[2] - 1);
}

hipError_t launch_cell_records(const qsq_field *f, void *ws, hipStream_t st)
{
    const int64_t nx = f->grid.n[0], ny = f->grid.n[1];
    const int64_t ncells = (nx - 1) * (ny - 1) * (f->grid.n[2] - 1);
    const int cus = device_cu_count();
    const int64_t want = (8 * ncells + 255) / 256;
    const int blocks = (int)(want < (int64_t)cus * 32 ? want : (int64_t)cus * 32);
    if (f->storage == QSQ_F32)
        hipLaunchKernelGGL(k_cell_records<float4>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const float4 *>(f->nodes), nx, ny, ncells, static_cast<float4 *>(ws));
    else if (f->storage == QSQ_BF16)
        hipLaunchKernelGGL(k_cell_records<uint2>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const uint2 *>(f->nodes), nx, ny, ncells, static_cast<uint2 *>(ws));
    else
        hipLaunchKernelGGL(k_cell_records<double4>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const double4 *>(f->nodes), nx, ny, ncells, static_cast<double4 *>(ws));
    return hipGetLastError();
}

// Brick records: the node records in 2 x 2 x 2 bricks, bricks x fastest,
// node (i, j, k) at ((bk nby + bj) nbx + bi) 8 + 4 (k & 1) + 2 (j & 1) + (i & 1)
// with (bi, bj, bk) = (i, j, k) / 2; the nodes of a brick fill one 128-byte
// line (FP32), so a cell's 8 corners span 1 to 8 lines (3.4 on average)
// rather than the 4 to 8 of the x-fastest layout.  Padding nodes are zero.
template <typename R>
__global__ void __launch_bounds__(256) k_brick_records(const R *__restrict__ nodes, int64_t nx, int64_t ny, int64_t nz,
                                                       int64_t nbx, int64_t nby, int64_t total, R *__restrict__ bricks)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(e & 7);
        const int64_t b = e >> 3;
        const int64_t i = 2 * (b % nbx) + (v & 1), j = 2 * ((b / nbx) % nby) + ((v >> 1) & 1),
                      k = 2 * (b / (nbx * nby)) + (v >> 2);
        R r{};
        if (i < nx && j < ny && k < nz) r = nodes[(k * ny + j) * nx + i];
        bricks[e] = r;
    }
}

// Direction records: for each cell (x fastest) the direction part (3 FP32
// values) of its 8 corner records in the order a + 2b + 4c of corner
// (i+a, j+b, k+c), 96 contiguous bytes, so that a cell's corners come in six
// 16-byte loads from at most two 128-byte lines.  One thread per (cell, corner).
__global__ void __launch_bounds__(256) k_cell_dirs(const float4 *__restrict__ nodes, int64_t nx, int64_t ny,
                                                   int64_t ncells, float *__restrict__ dirs)
{
    const int64_t cx = nx - 1, cy = ny - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 8 * ncells;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e >> 3;
        const int v = (int)(e & 7);
        const int64_t i = c % cx, j = (c / cx) % cy, k = c / (cx * cy);
        const float4 r = nodes[((k + (v >> 2)) * ny + j + ((v >> 1) & 1)) * nx + i + (v & 1)];
        dirs[3 * e] = r.x;
        dirs[3 * e + 1] = r.y;
        dirs[3 * e + 2] = r.z;
    }
}

uint64_t cell_dir_bytes(const qsq_grid *g)
{
    return 96 * (uint64_t)(g->n[0] - 1) * (uint64_t)(g->n[1] - 1) * (uint64_t)(g->n[2] - 1);
}

hipError_t launch_cell_dirs(const qsq_field *f, void *ws, hipStream_t st)
{
    const int64_t nx = f->grid.n[0], ny = f->grid.n[1];
    const int64_t ncells = (nx - 1) * (ny - 1) * (f->grid.n[2] - 1);
    const int cus = device_cu_count();
    const int64_t want = (8 * ncells + 255) / 256;
    const int blocks = (int)(want < (int64_t)cus * 32 ? want : (int64_t)cus * 32);
    hipLaunchKernelGGL(k_cell_dirs, dim3(blocks), dim3(256), 0, st, static_cast<const float4 *>(f->nodes), nx, ny,
                       ncells, static_cast<float *>(ws));
    return hipGetLastError();
}

uint64_t brick_record_bytes(const qsq_grid *g, int storage)
{
    const uint64_t rec = storage == QSQ_F64 ? 32 : storage == QSQ_F32 ? 16 : 8;
    return 8 * rec * (uint64_t)((g->n[0] + 1) / 2) * (uint64_t)((g->n[1] + 1) / 2) * (uint64_t)((g->n[2] + 1) / 2);
}

hipError_t launch_brick_records(const qsq_field *f, void *ws, hipStream_t st)
{
    const int64_t nx = f->grid.n[0], ny = f->grid.n[1], nz = f->grid.n[2];
    const int64_t nbx = (nx + 1) / 2, nby = (ny + 1) / 2, nbz = (nz + 1) / 2;
    const int64_t total = 8 * nbx * nby * nbz;
    const int cus = device_cu_count();
    const int64_t want = (total + 255) / 256;
    const int blocks = (int)(want < (int64_t)cus * 32 ? want : (int64_t)cus * 32);
    if (f->storage == QSQ_F32)
        hipLaunchKernelGGL(k_brick_records<float4>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const float4 *>(f->nodes), nx, ny, nz, nbx, nby, total, static_cast<float4 *>(ws));
    else if (f->storage == QSQ_BF16)
        hipLaunchKernelGGL(k_brick_records<uint2>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const uint2 *>(f->nodes), nx, ny, nz, nbx, nby, total, static_cast<uint2 *>(ws));
    else
        hipLaunchKernelGGL(k_brick_records<double4>, dim3(blocks), dim3(256), 0, st,
                           static_cast<const double4 *>(f->nodes), nx, ny, nz, nbx, nby, total,
                           static_cast<double4 *>(ws));
    return hipGetLastError();
}

hipError_t launch_field_init(const qsq_grid *g, const void *bx, const void *by, const void *bz,
                             int in_dtype, int storage, int mode, void *ws, hipStream_t st)
{
    const int64_t N = g->n[0] * g->n[1] * g->n[2];
    if (in_dtype == QSQ_F64) {
        if (storage == QSQ_F32) go<double, float>(bx, by, bz, mode, ws, N, st);
        else if (storage == QSQ_BF16) go<double, Bf16>(bx, by, bz, mode, ws, N, st);
        else go<double, double>(bx, by, bz, mode, ws, N, st);
    } else {
        if (storage == QSQ_F32) go<float, float>(bx, by, bz, mode, ws, N, st);
        else if (storage == QSQ_BF16) go<float, Bf16>(bx, by, bz, mode, ws, N, st);
        else go<float, double>(bx, by, bz, mode, ws, N, st);
    }
    return hipGetLastError();
}

}  // namespace qsq
