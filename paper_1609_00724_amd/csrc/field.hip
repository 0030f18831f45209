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
