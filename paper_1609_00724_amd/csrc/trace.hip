// Field-line + deviation tracer for gfx950 (QSL Squasher, Sect. 3.1-3.5).
//
// Three kernels per trace call:
//   k_trace    persistent wave64 lanes; each lane owns one half-line (seed x
//              direction), takes adaptive Cash-Karp 5(4) steps of
//              y = (x, dx1, dx2) under eq. (1) and eq. (5) in the stepping
//              precision T, and retires when a trial step leaves the box or a
//              stop condition holds.  Retired lanes are refilled from a device
//              work counter with one atomic per wave (ballot + prefix count).
//   k_land     FP64: re-solves the step that left the box for the step length
//              whose 5th-order end lies on the first face crossed (regula
//              falsi on the signed face distance, Anderson-Bjorck variant),
//              then snaps to it.
//   k_assemble FP64: per seed, projects the deviations perpendicular to the
//              renormalised field at both ends and forms Q by eq. (10)-(11),
//              the determinant form, the exit-face-plane Q and the length.
//
// Field records are 4-vectors per node (x fastest): PAPER mode holds
// (Bhat, |B|) with Bhat = B/|B| formed on the nodes (footnote to Sect. 3.5);
// INTERP_NORMALIZE holds B.  One RHS evaluation gathers the 8 corner records of
// the containing cell (eq. 3-4) and forms the value and the analytic gradient
// of the trilinear interpolant with a lerp tree (Sect. 3.3).
#include <math.h>

#include <mutex>
#include <type_traits>

#include "qsq_internal.h"

namespace qsq {

// ---------------------------------------------------------------------------
// Cash-Karp 5(4) coefficients (Cash & Karp 1990, the stepper of Sect. 3.4)
// ---------------------------------------------------------------------------
namespace ck {
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 3.0 / 10.0, a42 = -9.0 / 10.0, a43 = 6.0 / 5.0;
constexpr double a51 = -11.0 / 54.0, a52 = 5.0 / 2.0, a53 = -70.0 / 27.0, a54 = 35.0 / 27.0;
constexpr double a61 = 1631.0 / 55296.0, a62 = 175.0 / 512.0, a63 = 575.0 / 13824.0,
                 a64 = 44275.0 / 110592.0, a65 = 253.0 / 4096.0;
constexpr double b1 = 37.0 / 378.0, b3 = 250.0 / 621.0, b4 = 125.0 / 594.0, b6 = 512.0 / 1771.0;
// difference between the 5th- and the embedded 4th-order weights
constexpr double e1 = b1 - 2825.0 / 27648.0, e3 = b3 - 18575.0 / 48384.0,
                 e4 = b4 - 13525.0 / 55296.0, e5 = -277.0 / 14336.0, e6 = b6 - 1.0 / 4.0;
}  // namespace ck

// ---------------------------------------------------------------------------
// node loads
// ---------------------------------------------------------------------------
template <typename T>
struct V4 {
    T x, y, z, w;
};

__device__ __forceinline__ V4<float> ld4(const float *__restrict__ p, int64_t i)
{
    float4 v = reinterpret_cast<const float4 *>(p)[i];
    return {v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ V4<double> ld4(const double *__restrict__ p, int64_t i)
{
    const double2 *q = reinterpret_cast<const double2 *>(p) + 2 * i;
    double2 a = q[0], b = q[1];
    return {a.x, a.y, b.x, b.y};
}

// BF16 records: one 8-byte load, each value widened to FP32 exactly
__device__ __forceinline__ V4<float> ld4(const Bf16 *__restrict__ p, int64_t i)
{
    const uint2 v = reinterpret_cast<const uint2 *>(p)[i];
    return {__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u), __uint_as_float(v.y << 16),
            __uint_as_float(v.y & 0xffff0000u)};
}

// value and grid-unit partial derivatives of one trilinear component
template <typename T>
__device__ __forceinline__ void lerp_tree(T v000, T v100, T v010, T v110, T v001, T v101, T v011,
                                          T v111, T tx, T ty, T tz, T &val, T &dx, T &dy, T &dz)
{
    const T d00 = v100 - v000, d10 = v110 - v010, d01 = v101 - v001, d11 = v111 - v011;
    const T a00 = fma(tx, d00, v000), a10 = fma(tx, d10, v010);
    const T a01 = fma(tx, d01, v001), a11 = fma(tx, d11, v011);
    const T e0 = a10 - a00, e1 = a11 - a01;
    const T b0 = fma(ty, e0, a00), b1 = fma(ty, e1, a01);
    const T g0 = fma(ty, d10 - d00, d00), g1 = fma(ty, d11 - d01, d01);
    dz = b1 - b0;
    val = fma(tz, dz, b0);
    dx = fma(tz, g1 - g0, g0);
    dy = fma(tz, e1 - e0, e0);
}

template <typename T>
__device__ __forceinline__ T lerp_val(T v000, T v100, T v010, T v110, T v001, T v101, T v011, T v111,
                                      T tx, T ty, T tz)
{
    const T a00 = fma(tx, v100 - v000, v000), a10 = fma(tx, v110 - v010, v010);
    const T a01 = fma(tx, v101 - v001, v001), a11 = fma(tx, v111 - v011, v011);
    const T b0 = fma(ty, a10 - a00, a00), b1 = fma(ty, a11 - a01, a01);
    return fma(tz, b1 - b0, b0);
}

// Cell of a point given in grid units as integer reference ib plus offset q:
// c = clamp(floor(ib + q), 0, n-2), fraction t = ib + q - c (not clamped, so
// points slightly outside the box extrapolate the boundary cell linearly).
template <typename T>
__device__ __forceinline__ void cell_of(int ib, T q, int n, int &c, T &t)
{
    const T fl = floor(q);
    int ci = ib + (int)fl;
    ci = ci < 0 ? 0 : ci;
    ci = ci > n - 2 ? n - 2 : ci;
    c = ci;
    t = q - (T)(ci - ib);
}

// ---------------------------------------------------------------------------
// Higher interpolation orders (Sect. 3.2): the 27-vertex triquadratic stencil
// (Dodgson 1997) and the 64-vertex tricubic stencil (Keys 1981).  The order
// rides in the MODE template value: bit 0 is the interpolation mode
// (QSQ_INTERP_*), the bits above hold order - 1.
// ---------------------------------------------------------------------------
template <int MODE>
constexpr int interp_order() { return ((MODE >> 1) & 3) + 1; }
template <int MODE>
constexpr bool normalize_first() { return (MODE & 1) == QSQ_INTERP_PAPER; }

// Per-axis stencil of K = order + 1 nodes starting at node s, with the
// weights w of the values and dw of the grid-unit derivative.  Cubic (Keys'
// kernel with a = -1/2): nodes c-1 .. c+2 of the cell c, fraction t.
// Quadratic (Dodgson's interpolating kernel, 1 - 2d^2 within half a spacing,
// d^2 - 5|d|/2 + 3/2 out to 3/2 spacings): the node m nearest the point and
// its two neighbours, offset u = t or t - 1 from m.  A stencil node beyond the
// grid stands for Keys' extrapolation f(-1) = 3 f(0) - 3 f(1) + f(2) (and the
// same at the top end); its weight is folded onto those three nodes and the
// stencil starts at the first node inside.  The last weight is then zero and
// its node index may lie past the grid (the caller clamps it).
template <int K, typename T>
__device__ __forceinline__ void axis_stencil(int c, T t, int n, int &s, T w[K], T dw[K])
{
    if constexpr (K == 4) {
        const T t2 = t * t, t3 = t2 * t;
        w[0] = (T)0.5 * (-t3 + (T)2 * t2 - t);
        w[1] = (T)0.5 * ((T)3 * t3 - (T)5 * t2 + (T)2);
        w[2] = (T)0.5 * ((T)-3 * t3 + (T)4 * t2 + t);
        w[3] = (T)0.5 * (t3 - t2);
        dw[0] = (T)0.5 * ((T)-3 * t2 + (T)4 * t - (T)1);
        dw[1] = (T)0.5 * ((T)9 * t2 - (T)10 * t);
        dw[2] = (T)0.5 * ((T)-9 * t2 + (T)8 * t + (T)1);
        dw[3] = (T)0.5 * ((T)3 * t2 - (T)2 * t);
        s = c - 1;
    } else {
        const bool low = t < (T)0.5;
        const T u = low ? t : t - (T)1;
        w[0] = u * (u - (T)0.5);
        w[1] = (T)1 - (T)2 * u * u;
        w[2] = u * (u + (T)0.5);
        dw[0] = (T)2 * u - (T)0.5;
        dw[1] = (T)-4 * u;
        dw[2] = (T)2 * u + (T)0.5;
        s = low ? c - 1 : c;
    }
    if (s < 0) {
        // node -1 folded onto nodes 0, 1, 2 (weights 3, -3, 1)
        const T a = w[0], da = dw[0];
#pragma unroll
        for (int k = 0; k < K - 1; ++k) {
            w[k] = w[k + 1];
            dw[k] = dw[k + 1];
        }
        w[K - 1] = (T)0;
        dw[K - 1] = (T)0;
        w[0] += (T)3 * a, w[1] -= (T)3 * a, w[2] += a;
        dw[0] += (T)3 * da, dw[1] -= (T)3 * da, dw[2] += da;
        s = 0;
    } else if (s + K - 1 > n - 1) {
        // node n folded onto nodes n-1, n-2, n-3 (weights 3, -3, 1); the
        // stencil then starts at n-3
        const T a = w[K - 1], da = dw[K - 1];
        const int shift = s - (n - 3);   // 0 for the cubic, 1 for the quadratic stencil
        T nw[K], ndw[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            nw[k] = (T)0;
            ndw[k] = (T)0;
        }
#pragma unroll
        for (int k = 0; k < K - 1; ++k) {
            nw[k + shift] += w[k];
            ndw[k + shift] += dw[k];
        }
        nw[0] += a, nw[1] -= (T)3 * a, nw[2] += (T)3 * a;
        ndw[0] += da, ndw[1] -= (T)3 * da, ndw[2] += (T)3 * da;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            w[k] = nw[k];
            dw[k] = ndw[k];
        }
        s = n - 3;
    }
}

// Value and grid-unit gradient of the first NC record components by the
// separable stencil sum: along x per row, then y, then z.
template <int K, int NC, typename T, typename S>
__device__ __forceinline__ void stencil_sum(const S *__restrict__ nodes, const Geom &g, const int s[3],
                                            const T w[3][K], const T dw[3][K], T val[NC], T dx[NC], T dy[NC],
                                            T dz[NC])
{
#pragma unroll
    for (int k = 0; k < NC; ++k) val[k] = dx[k] = dy[k] = dz[k] = (T)0;
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    // rows one at a time (only the K records of a row in flight): unrolling
    // the z and y loops lets the compiler hoist all K^3 loads and spill
#pragma unroll 1
    for (int kz = 0; kz < K; ++kz) {
        const int iz = s[2] + kz < g.n[2] - 1 ? s[2] + kz : g.n[2] - 1;
        T ay[NC], axy[NC], ayy[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) ay[k] = axy[k] = ayy[k] = (T)0;
#pragma unroll 1
        for (int ky = 0; ky < K; ++ky) {
            const int iy = s[1] + ky < g.n[1] - 1 ? s[1] + ky : g.n[1] - 1;
            const int64_t row = (int64_t)iz * sz + (int64_t)iy * sy;
            T rx[NC], drx[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) rx[k] = drx[k] = (T)0;
#pragma unroll
            for (int kx = 0; kx < K; ++kx) {
                const int ix = s[0] + kx < g.n[0] - 1 ? s[0] + kx : g.n[0] - 1;
                const auto v = ld4(nodes, row + ix);
                const T c4[4] = {(T)v.x, (T)v.y, (T)v.z, (T)v.w};
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    rx[k] = fma(w[0][kx], c4[k], rx[k]);
                    drx[k] = fma(dw[0][kx], c4[k], drx[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                ay[k] = fma(w[1][ky], rx[k], ay[k]);
                axy[k] = fma(w[1][ky], drx[k], axy[k]);
                ayy[k] = fma(dw[1][ky], rx[k], ayy[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            val[k] = fma(w[2][kz], ay[k], val[k]);
            dx[k] = fma(w[2][kz], axy[k], dx[k]);
            dy[k] = fma(w[2][kz], ayy[k], dy[k]);
            dz[k] = fma(dw[2][kz], ay[k], dz[k]);
        }
    }
}

// u, the physical gradient rows and |B| from the interpolated components
// (value and grid-unit derivatives; val[3] = interpolated |B| in PAPER mode)
template <typename T, int MODE, bool MAG>
__device__ __forceinline__ void field_finish(const double ih[3], const T val[4], const T dx[4], const T dy[4],
                                             const T dz[4], T u[3], T G[3][3], T &mag)
{
    const T ihx = (T)ih[0], ihy = (T)ih[1], ihz = (T)ih[2];
    if (normalize_first<MODE>()) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i];
            G[0][i] = dx[i] * ihx;
            G[1][i] = dy[i] * ihy;
            G[2][i] = dz[i] * ihz;
        }
        if (MAG) mag = val[3];
    } else {
        // u = B/|B|, grad u = (I - u u^T) grad B / |B|
        const T bb = val[0] * val[0] + val[1] * val[1] + val[2] * val[2];
        const T bn = sqrt(bb);
        const T inv = bn > (T)1e-300 ? (T)1 / bn : (T)0;
        T Gb[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i] * inv;
            Gb[0][i] = dx[i] * ihx;
            Gb[1][i] = dy[i] * ihy;
            Gb[2][i] = dz[i] * ihz;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T ug = u[0] * Gb[j][0] + u[1] * Gb[j][1] + u[2] * Gb[j][2];
#pragma unroll
            for (int i = 0; i < 3; ++i) G[j][i] = (Gb[j][i] - u[i] * ug) * inv;
        }
        if (MAG) mag = bn;
    }
}

// Field value u (Bhat as interpolated) and physical gradient rows
// G[j][i] = d u_i / d x_j at a point; optionally |B| (PAPER: interpolated node
// magnitudes; INTERP_NORMALIZE: magnitude of the interpolated B).
// CELLS: `nodes` points at cell records (the 8 corner records of each cell,
// contiguous, corner a + 2b + 4c) instead of node records; the same values.
template <typename T, typename S, int MODE, bool MAG, bool CELLS = false>
__device__ __forceinline__ void field_at(const S *__restrict__ nodes, const Geom &g, const int ib[3],
                                         const T q[3], T u[3], T G[3][3], T &mag)
{
    int c[3];
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(ib[d], q[d], g.n[d], c[d], t[d]);
    T val[4], dx[4], dy[4], dz[4];
    if constexpr (interp_order<MODE>() > 1) {
        constexpr int K = interp_order<MODE>() + 1;
        int s0[3];
        T w[3][K], dw[3][K];
#pragma unroll
        for (int d = 0; d < 3; ++d) axis_stencil<K, T>(c[d], t[d], g.n[d], s0[d], w[d], dw[d]);
        // |B| is the 4th component in PAPER mode; INTERP_NORMALIZE takes |interpolated B|
        constexpr int NC = (MAG && normalize_first<MODE>()) ? 4 : 3;
        stencil_sum<K, NC, T, S>(nodes, g, s0, w, dw, val, dx, dy, dz);
        field_finish<T, MODE, MAG>(g.ih, val, dx, dy, dz, u, G, mag);
        return;
    }
    int64_t o[8];
    if constexpr (CELLS) {
        const int64_t b = 8 * (((int64_t)c[2] * (g.n[1] - 1) + c[1]) * (g.n[0] - 1) + c[0]);
#pragma unroll
        for (int v = 0; v < 8; ++v) o[v] = b + v;
    } else {
        const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
        const int64_t b = (int64_t)c[2] * sz + (int64_t)c[1] * sy + c[0];
        o[0] = b, o[1] = b + 1, o[2] = b + sy, o[3] = b + sy + 1;
        o[4] = b + sz, o[5] = b + sz + 1, o[6] = b + sz + sy, o[7] = b + sz + sy + 1;
    }
    const auto n000 = ld4(nodes, o[0]), n100 = ld4(nodes, o[1]);
    const auto n010 = ld4(nodes, o[2]), n110 = ld4(nodes, o[3]);
    const auto n001 = ld4(nodes, o[4]), n101 = ld4(nodes, o[5]);
    const auto n011 = ld4(nodes, o[6]), n111 = ld4(nodes, o[7]);
#define QSQ_COMP(F, k)                                                                              \
    lerp_tree<T>((T)n000.F, (T)n100.F, (T)n010.F, (T)n110.F, (T)n001.F, (T)n101.F, (T)n011.F,       \
                 (T)n111.F, t[0], t[1], t[2], val[k], dx[k], dy[k], dz[k])
    QSQ_COMP(x, 0);
    QSQ_COMP(y, 1);
    QSQ_COMP(z, 2);
#undef QSQ_COMP
    if (MAG && normalize_first<MODE>())
        val[3] = lerp_val<T>((T)n000.w, (T)n100.w, (T)n010.w, (T)n110.w, (T)n001.w, (T)n101.w, (T)n011.w,
                             (T)n111.w, t[0], t[1], t[2]);
    field_finish<T, MODE, MAG>(g.ih, val, dx, dy, dz, u, G, mag);
}

// The interpolated direction u alone (no gradient): the same operations as
// the value part of field_at, so both give the same u bit for bit.
template <typename T, typename S, int MODE>
__device__ __forceinline__ void field_u(const S *__restrict__ nodes, const Geom &g, const int ib[3], const T q[3],
                                        T u[3])
{
    int c[3];
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(ib[d], q[d], g.n[d], c[d], t[d]);
    T val[3];
    if constexpr (interp_order<MODE>() > 1) {
        // the same stencil sums as field_at (the derivative sums are not used)
        constexpr int K = interp_order<MODE>() + 1;
        int s0[3];
        T w[3][K], dw[3][K], dx[3], dy[3], dz[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) axis_stencil<K, T>(c[d], t[d], g.n[d], s0[d], w[d], dw[d]);
        stencil_sum<K, 3, T, S>(nodes, g, s0, w, dw, val, dx, dy, dz);
    } else {
        const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
        const int64_t b = (int64_t)c[2] * sz + (int64_t)c[1] * sy + c[0];
        const auto n000 = ld4(nodes, b), n100 = ld4(nodes, b + 1);
        const auto n010 = ld4(nodes, b + sy), n110 = ld4(nodes, b + sy + 1);
        const auto n001 = ld4(nodes, b + sz), n101 = ld4(nodes, b + sz + 1);
        const auto n011 = ld4(nodes, b + sz + sy), n111 = ld4(nodes, b + sz + sy + 1);
#define QSQ_COMPV(F, k)                                                                                  \
    val[k] = lerp_val<T>((T)n000.F, (T)n100.F, (T)n010.F, (T)n110.F, (T)n001.F, (T)n101.F, (T)n011.F,    \
                         (T)n111.F, t[0], t[1], t[2])
        QSQ_COMPV(x, 0);
        QSQ_COMPV(y, 1);
        QSQ_COMPV(z, 2);
#undef QSQ_COMPV
    }
    if (normalize_first<MODE>()) {
#pragma unroll
        for (int i = 0; i < 3; ++i) u[i] = val[i];
    } else {
        const T bb = val[0] * val[0] + val[1] * val[1] + val[2] * val[2];
        const T bn = sqrt(bb);
        const T inv = bn > (T)1e-300 ? (T)1 / bn : (T)0;
#pragma unroll
        for (int i = 0; i < 3; ++i) u[i] = val[i] * inv;
    }
}

// a0 b0 + a1 b1 + a2 b2 with the fused operations spelled out, so that the
// rounding does not depend on how the compiler contracts the expression
template <typename T>
__device__ __forceinline__ T jdot(T a0, T a1, T a2, T b0, T b1, T b2)
{
    return fma(a2, b2, fma(a1, b1, a0 * b0));
}

// Right-hand side f(y) = sigma * (u, J dx1, J dx2), J_ij = d u_i / d x_j
// (eq. 1 and eq. 5).  Returns |u|^2 for the null test.
template <typename T>
__device__ __forceinline__ T rhs_from(T sigma, const T u[3], const T G[3][3], const T d1[3], const T d2[3],
                                      T kx[3], T k1[3], T k2[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        kx[i] = sigma * u[i];
        k1[i] = sigma * jdot(G[0][i], G[1][i], G[2][i], d1[0], d1[1], d1[2]);
        k2[i] = sigma * jdot(G[0][i], G[1][i], G[2][i], d2[0], d2[1], d2[2]);
    }
    return jdot(u[0], u[1], u[2], u[0], u[1], u[2]);
}

template <typename T, typename S, int MODE, bool CELLS = false>
__device__ __forceinline__ T rhs(const S *__restrict__ nodes, const Geom &g, const int ib[3],
                                 const T q[3], T sigma, const T d1[3], const T d2[3], T kx[3],
                                 T k1[3], T k2[3])
{
    T u[3], G[3][3], mag;
    field_at<T, S, MODE, false, CELLS>(nodes, g, ib, q, u, G, mag);
    return rhs_from(sigma, u, G, d1, d2, kx, k1, k2);
}

// Raw buffer load of 16 bytes.  Lanes whose byte offset lies at or beyond the
// buffer's record count get zeros back without any memory access, which lets a
// wave gather only for the lanes that need new data, with no divergent branch.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ f32x4 qsq_buffer_load16(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.load.v4f32");

// Raw buffer load of 8 bytes (one BF16 node record), same out-of-range rule.
typedef int i32x2 __attribute__((ext_vector_type(2)));
__device__ i32x2 qsq_buffer_load8(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.load.v2i32");

// Buffer resource over the node records (gfx9 descriptor word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t node_rsrc(const void *nodes, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(nodes), (short)0, bytes, 0x00020000);
}

// bytes of one node record: 4 x FP32 or 4 x BF16
template <typename S>
constexpr int node_bytes() { return std::is_same<S, float>::value ? 16 : 8; }

// direction part (3 values, widened to FP32 exactly) of the node record at a
// byte offset
template <typename S>
__device__ __forceinline__ void load_dir(__amdgpu_buffer_rsrc_t rsrc, int off, float &x, float &y, float &z)
{
    if constexpr (std::is_same<S, float>::value) {
        const f32x4 v = qsq_buffer_load16(rsrc, off, 0, 0);
        x = v.x;
        y = v.y;
        z = v.z;
    } else {
        const i32x2 v = qsq_buffer_load8(rsrc, off, 0, 0);
        x = __uint_as_float((uint32_t)v.x << 16);
        y = __uint_as_float((uint32_t)v.x & 0xffff0000u);
        z = __uint_as_float((uint32_t)v.y << 16);
    }
}

// Per-lane cache of the 8 corner records (direction part, 24 floats) of the
// cell a lane evaluated last, kept in LDS (6 float4 planes of one workgroup's
// lanes, lane-consecutive, conflict-free 16-byte accesses).  Consecutive Runge-Kutta
// stages mostly fall in the same cell: only lanes whose stage point moved to
// another cell fetch from memory (the others issue out-of-range offsets, see
// above) and store the new corners into their slot; every lane then reads its
// slot (a wave's LDS operations complete in order).  Keyed by cell index
// alone, so it stays valid across the lines a lane traces.
constexpr int kCachePlanes = 6;

template <typename T, typename S, int MODE>
__device__ __forceinline__ T rhs_cached(__amdgpu_buffer_rsrc_t rsrc, int bytes, const Geom &g, const int ib[3],
                                        const T q[3], T sigma, const T d1[3], const T d2[3], T kx[3], T k1[3],
                                        T k2[3], int cc[3], float4 *slot, int stride)
{
    int c[3];
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(ib[d], q[d], g.n[d], c[d], t[d]);
    const bool miss = c[0] != cc[0] || c[1] != cc[1] || c[2] != cc[2];
    const int sy = g.n[0], sz = g.n[0] * g.n[1];
    constexpr int NB = node_bytes<S>();
    const int base = miss ? NB * (c[2] * sz + c[1] * sy + c[0]) : bytes;
    float w[24];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int o = NB * (((k & 1) ? 1 : 0) + ((k & 2) ? sy : 0) + ((k & 4) ? sz : 0));
        load_dir<S>(rsrc, base + o, w[3 * k], w[3 * k + 1], w[3 * k + 2]);
    }
    if (miss) {
#pragma unroll
        for (int j = 0; j < kCachePlanes; ++j) slot[j * stride] = make_float4(w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]);
    }
    cc[0] = c[0];
    cc[1] = c[1];
    cc[2] = c[2];
    float v[24];
#pragma unroll
    for (int j = 0; j < kCachePlanes; ++j) {
        const float4 x = slot[j * stride];
        v[4 * j] = x.x;
        v[4 * j + 1] = x.y;
        v[4 * j + 2] = x.z;
        v[4 * j + 3] = x.w;
    }
    T val[3], dx[3], dy[3], dz[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        lerp_tree<T>((T)v[i], (T)v[3 + i], (T)v[6 + i], (T)v[9 + i], (T)v[12 + i], (T)v[15 + i],
                     (T)v[18 + i], (T)v[21 + i], t[0], t[1], t[2], val[i], dx[i], dy[i], dz[i]);
    const T ihx = (T)g.ih[0], ihy = (T)g.ih[1], ihz = (T)g.ih[2];
    T u[3], G[3][3];
    if (normalize_first<MODE>()) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i];
            G[0][i] = dx[i] * ihx;
            G[1][i] = dy[i] * ihy;
            G[2][i] = dz[i] * ihz;
        }
    } else {
        const T bb = val[0] * val[0] + val[1] * val[1] + val[2] * val[2];
        const T bn = sqrt(bb);
        const T inv = bn > (T)1e-300 ? (T)1 / bn : (T)0;
        T Gb[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i] * inv;
            Gb[0][i] = dx[i] * ihx;
            Gb[1][i] = dy[i] * ihy;
            Gb[2][i] = dz[i] * ihz;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T ug = u[0] * Gb[j][0] + u[1] * Gb[j][1] + u[2] * Gb[j][2];
#pragma unroll
            for (int i = 0; i < 3; ++i) G[j][i] = (Gb[j][i] - u[i] * ug) * inv;
        }
    }
    return rhs_from(sigma, u, G, d1, d2, kx, k1, k2);
}

// Per-lane cache of the 8 corner records (direction part, 24 floats) of the
// cell a lane evaluated last, kept in registers.  A wave in which some lane's
// stage point moved to another cell issues one gather (a branch taken by the
// whole wave): the lanes that moved load their new corners, the others pass
// out-of-range offsets (no memory access) and keep their registers by a
// select.  A wave whose lanes all stayed in their cells issues no load and
// waits for none.  No branch under the lane mask, so the 24 values keep their
// registers from stage to stage without copies.  The node values and the
// arithmetic are those of the direct gather: the results are the same bit for
// bit.  The key is the cell's node index within the field (below 2 GiB).
// Named scalars (not an array) so that they live in plain registers.
struct Corner {
    float x, y, z;
};
struct Brick {
    Corner c000, c100, c010, c110, c001, c101, c011, c111;
};

#ifndef QSQ_SECOND_CELL
#define QSQ_SECOND_CELL 1
#endif

typedef uint32_t u32x3_t __attribute__((ext_vector_type(3)));

// the direction part of a node record, loaded straight into a corner
template <typename S>
__device__ __forceinline__ void load_corner(__amdgpu_buffer_rsrc_t rsrc, int off, Corner &c)
{
    if constexpr (std::is_same<S, float>::value) {
        const u32x3_t v = __builtin_amdgcn_raw_buffer_load_b96(rsrc, off, 0, 0);
        c.x = __uint_as_float(v.x);
        c.y = __uint_as_float(v.y);
        c.z = __uint_as_float(v.z);
    } else {
        load_dir<S>(rsrc, off, c.x, c.y, c.z);
    }
}


// the 24 direction values of a cell's corners packed in six float4 (corner
// order a + 2b + 4c, 3 values each): the parked cell's LDS slot and the
// direction records share this packing
__device__ __forceinline__ void unpack_cell(const float4 v[6], Brick &br)
{
    br.c000 = Corner{v[0].x, v[0].y, v[0].z};
    br.c100 = Corner{v[0].w, v[1].x, v[1].y};
    br.c010 = Corner{v[1].z, v[1].w, v[2].x};
    br.c110 = Corner{v[2].y, v[2].z, v[2].w};
    br.c001 = Corner{v[3].x, v[3].y, v[3].z};
    br.c101 = Corner{v[3].w, v[4].x, v[4].y};
    br.c011 = Corner{v[4].z, v[4].w, v[5].x};
    br.c111 = Corner{v[5].y, v[5].z, v[5].w};
}

// record layouts of the register cache
constexpr int kLayoutNodes = 0, kLayoutBricks = 1, kLayoutDirs = 2;

// BRICKS: the records are the field's brick records (2 x 2 x 2 node bricks,
// bricks x fastest): node (i, j, k) sits at ((k/2 nby + j/2) nbx + i/2) 8 +
// 4 (k & 1) + 2 (j & 1) + (i & 1), so the step from a corner to its neighbour
// along an axis is 1, 2, 4 records from an even index and 7, 8 nbx - 2,
// 8 nbx nby - 4 from an odd one.  DIRS: `dirs` holds the field's direction
// records, the cell's 24 values in six 16-byte loads (global addresses: the
// records may exceed 2 GiB), keyed by the cell's index.
template <typename T, typename S, int MODE, int LAYOUT = kLayoutNodes>
__device__ __forceinline__ T rhs_regs(__amdgpu_buffer_rsrc_t rsrc, int bytes, const float4 *__restrict__ dirs,
                                      const Geom &g, const int ib[3], const T q[3], T sigma, const T d1[3],
                                      const T d2[3], T kx[3], T k1[3], T k2[3], int &cell, Brick &br, float4 *slot,
                                      int stride, int &cell2)
{
    int c[3];
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(ib[d], q[d], g.n[d], c[d], t[d]);
    int b, sx, sy, sz;
    if constexpr (LAYOUT == kLayoutDirs) {
        b = (c[2] * (g.n[1] - 1) + c[1]) * (g.n[0] - 1) + c[0];
        sx = sy = sz = 0;
    } else if constexpr (LAYOUT == kLayoutBricks) {
        const int nbx = (g.n[0] + 1) >> 1, nby = (g.n[1] + 1) >> 1;
        b = (((c[2] >> 1) * nby + (c[1] >> 1)) * nbx + (c[0] >> 1)) * 8 + ((c[2] & 1) << 2) + ((c[1] & 1) << 1) +
            (c[0] & 1);
        sx = (c[0] & 1) ? 7 : 1;
        sy = (c[1] & 1) ? 8 * nbx - 2 : 2;
        sz = (c[2] & 1) ? 8 * nbx * nby - 4 : 4;
    } else {
        sx = 1;
        sy = g.n[0];
        sz = g.n[0] * g.n[1];
        b = c[2] * sz + c[1] * sy + c[0];
    }
    const bool miss = b != cell;
    if (miss) {
        // only the lanes that moved load (the memory pipeline returns data for
        // active lanes alone), the direction part only (12 bytes of FP32)
        constexpr int NB = node_bytes<S>();
#if QSQ_SECOND_CELL
        // the cell left behind is parked in the lane's LDS slot; a lane that
        // moves back into it takes its corners from there instead of memory
        const bool back = b == cell2;
        float4 keep[kCachePlanes];
        if (back) {
#pragma unroll
            for (int j = 0; j < kCachePlanes; ++j) keep[j] = slot[j * stride];
        }
        slot[0 * stride] = make_float4(br.c000.x, br.c000.y, br.c000.z, br.c100.x);
        slot[1 * stride] = make_float4(br.c100.y, br.c100.z, br.c010.x, br.c010.y);
        slot[2 * stride] = make_float4(br.c010.z, br.c110.x, br.c110.y, br.c110.z);
        slot[3 * stride] = make_float4(br.c001.x, br.c001.y, br.c001.z, br.c101.x);
        slot[4 * stride] = make_float4(br.c101.y, br.c101.z, br.c011.x, br.c011.y);
        slot[5 * stride] = make_float4(br.c011.z, br.c111.x, br.c111.y, br.c111.z);
        cell2 = cell;
        if (back) {
            unpack_cell(keep, br);
        } else
#endif
        if constexpr (LAYOUT == kLayoutDirs) {
            const float4 *p = dirs + 6 * (int64_t)b;
            float4 v[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) v[j] = p[j];
            unpack_cell(v, br);
        } else {
            const int o = NB * b;
            const int ox = NB * sx, oy = NB * sy, oz = NB * sz;
            load_corner<S>(rsrc, o, br.c000);
            load_corner<S>(rsrc, o + ox, br.c100);
            load_corner<S>(rsrc, o + oy, br.c010);
            load_corner<S>(rsrc, o + oy + ox, br.c110);
            load_corner<S>(rsrc, o + oz, br.c001);
            load_corner<S>(rsrc, o + oz + ox, br.c101);
            load_corner<S>(rsrc, o + oz + oy, br.c011);
            load_corner<S>(rsrc, o + oz + oy + ox, br.c111);
        }
        cell = b;
    }
    T val[3], dx[3], dy[3], dz[3];
#define QSQ_COMPB(F, k)                                                                               \
    lerp_tree<T>((T)br.c000.F, (T)br.c100.F, (T)br.c010.F, (T)br.c110.F, (T)br.c001.F, (T)br.c101.F,  \
                 (T)br.c011.F, (T)br.c111.F, t[0], t[1], t[2], val[k], dx[k], dy[k], dz[k])
    QSQ_COMPB(x, 0);
    QSQ_COMPB(y, 1);
    QSQ_COMPB(z, 2);
#undef QSQ_COMPB
    const T ihx = (T)g.ih[0], ihy = (T)g.ih[1], ihz = (T)g.ih[2];
    T u[3], G[3][3];
    if (normalize_first<MODE>()) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i];
            G[0][i] = dx[i] * ihx;
            G[1][i] = dy[i] * ihy;
            G[2][i] = dz[i] * ihz;
        }
    } else {
        const T bb = val[0] * val[0] + val[1] * val[1] + val[2] * val[2];
        const T bn = sqrt(bb);
        const T inv = bn > (T)1e-300 ? (T)1 / bn : (T)0;
        T Gb[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i] * inv;
            Gb[0][i] = dx[i] * ihx;
            Gb[1][i] = dy[i] * ihy;
            Gb[2][i] = dz[i] * ihz;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T ug = u[0] * Gb[j][0] + u[1] * Gb[j][1] + u[2] * Gb[j][2];
#pragma unroll
            for (int i = 0; i < 3; ++i) G[j][i] = (Gb[j][i] - u[i] * ug) * inv;
        }
    }
    return rhs_from(sigma, u, G, d1, d2, kx, k1, k2);
}

// 5th-order combination and the 5th-minus-4th error combination of the
// stage slopes, fused operations spelled out
template <typename T>
__device__ __forceinline__ T ck_b5(T k0, T k2, T k3, T k5)
{
    return fma((T)ck::b6, k5, fma((T)ck::b4, k3, fma((T)ck::b3, k2, (T)ck::b1 * k0)));
}

template <typename T>
__device__ __forceinline__ T ck_e(T k0, T k2, T k3, T k4, T k5)
{
    return fma((T)ck::e6, k5, fma((T)ck::e5, k4, fma((T)ck::e4, k3, fma((T)ck::e3, k2, (T)ck::e1 * k0))));
}

// atol + rtol max(|old|, |new|)
template <typename T>
__device__ __forceinline__ T err_scale(T atol, T rtol, T a, T b)
{
    return fma(rtol, fmax(fabs(a), fabs(b)), atol);
}

// a / b of the error norm: FP32 stepping multiplies by the hardware
// reciprocal (within 1 ulp; the norm only steers accept/reject and the step
// factor), FP64 stepping divides exactly
__device__ __forceinline__ float err_ratio(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double err_ratio(double a, double b) { return a / b; }

// gather variants of the stepping kernel: direct corner loads, the LDS cell
// cache and the register cell cache (the caches: FP32 or BF16 storage, FP32
// stepping, one field below 2 GiB)
constexpr int kGatherDirect = 0, kGatherLds = 1, kGatherRegs = 2, kGatherCells = 3, kGatherBricks = 4,
              kGatherDirs = 5;

// one RHS evaluation of the stepping kernel
template <typename T, typename S, int MODE, int GATHER>
__device__ __forceinline__ T rhs_step(const S *__restrict__ nodes, __amdgpu_buffer_rsrc_t rsrc, int bytes,
                                      const Geom &g, const int ib[3], const T q[3], T sigma, const T d1[3],
                                      const T d2[3], T kx[3], T k1[3], T k2[3], int cc[3], float4 *slot,
                                      int stride, int &cell, Brick &br)
{
    if constexpr (GATHER == kGatherLds)
        return rhs_cached<T, S, MODE>(rsrc, bytes, g, ib, q, sigma, d1, d2, kx, k1, k2, cc, slot, stride);
    else if constexpr (GATHER == kGatherRegs || GATHER == kGatherBricks || GATHER == kGatherDirs)
        // (cc[0], the LDS variant's cell key, keys the register cache's parked
        // cell; the direction records' variant gets them as `nodes`)
        return rhs_regs<T, S, MODE,
                        GATHER == kGatherBricks ? kLayoutBricks : GATHER == kGatherDirs ? kLayoutDirs : kLayoutNodes>(
            rsrc, bytes, reinterpret_cast<const float4 *>(nodes), g, ib, q, sigma, d1, d2, kx, k1, k2, cell, br, slot,
            stride, cc[0]);
    else
        return rhs<T, S, MODE, GATHER == kGatherCells>(nodes, g, ib, q, sigma, d1, d2, kx, k1, k2);
}

// ---------------------------------------------------------------------------
// General geometry (Sect. 3.1-3.2): spherical coordinates (longitude phi,
// latitude theta, radius r; field components in the local orthonormal basis)
// and rectilinear axes whose cells have spans of their own.  MODE bit 3.
// These fields are stepped in physical coordinates by k_trace_geo and landed
// by k_land_geo; the seed pass and the Q assembly are shared.
// ---------------------------------------------------------------------------
template <int MODE>
constexpr bool geo_mode() { return (MODE & 8) != 0; }

// cell, fraction of the cell and the cell's span per axis at a physical point;
// a rectilinear axis is searched by bisection for the last cell whose lower
// node lies at or below the point (clamped to the grid's cells)
__device__ __forceinline__ void geo_cell(const Geom &g, const double x[3], int c[3], double t[3], double h[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *X = g.coord[d];
        const int n = g.n[d];
        if (X) {
            const double xv = fmax(x[d], -1e300);   // NaN -> the lowest cell
            int lo = 0, hi = n - 2;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (X[mid] <= xv)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            c[d] = lo;
            h[d] = X[lo + 1] - X[lo];
            t[d] = (x[d] - X[lo]) / h[d];
        } else {
            const double sg = fmin(fmax((x[d] - g.o[d]) * g.ih[d], -1e9), 1e9);
            double fl = floor(sg);
            fl = fl < 0.0 ? 0.0 : (fl > (double)(n - 2) ? (double)(n - 2) : fl);
            c[d] = (int)fl;
            t[d] = sg - fl;
            h[d] = g.h[d];
        }
    }
}

// trilinear value and physical gradient at a physical point
template <typename T, typename S, int MODE, bool MAG>
__device__ __forceinline__ void field_at_geo(const S *__restrict__ nodes, const Geom &g, const double x[3], T u[3],
                                             T G[3][3], T &mag)
{
    int c[3];
    double t64[3], h[3];
    geo_cell(g, x, c, t64, h);
    const T t[3] = {(T)t64[0], (T)t64[1], (T)t64[2]};
    const double ih[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t b = (int64_t)c[2] * sz + (int64_t)c[1] * sy + c[0];
    const auto n000 = ld4(nodes, b), n100 = ld4(nodes, b + 1);
    const auto n010 = ld4(nodes, b + sy), n110 = ld4(nodes, b + sy + 1);
    const auto n001 = ld4(nodes, b + sz), n101 = ld4(nodes, b + sz + 1);
    const auto n011 = ld4(nodes, b + sz + sy), n111 = ld4(nodes, b + sz + sy + 1);
    T val[4], dx[4], dy[4], dz[4];
#define QSQ_COMPG(F, k)                                                                             \
    lerp_tree<T>((T)n000.F, (T)n100.F, (T)n010.F, (T)n110.F, (T)n001.F, (T)n101.F, (T)n011.F,       \
                 (T)n111.F, t[0], t[1], t[2], val[k], dx[k], dy[k], dz[k])
    QSQ_COMPG(x, 0);
    QSQ_COMPG(y, 1);
    QSQ_COMPG(z, 2);
#undef QSQ_COMPG
    if (MAG && normalize_first<MODE>())
        val[3] = lerp_val<T>((T)n000.w, (T)n100.w, (T)n010.w, (T)n110.w, (T)n001.w, (T)n101.w, (T)n011.w,
                             (T)n111.w, t[0], t[1], t[2]);
    field_finish<T, MODE, MAG>(ih, val, dx, dy, dz, u, G, mag);
}

// metric factors of eq. (2) and (8) at a physical point: (r cos theta, r, 1)
// in spherical geometry, ones otherwise
__device__ __forceinline__ void geo_scale(const Geom &g, const double x[3], double sc[3])
{
    if (g.geometry == QSQ_GEOMETRY_SPHERICAL) {
        sc[0] = x[2] * cos(x[1]);
        sc[1] = x[2];
        sc[2] = 1.0;
    } else {
        sc[0] = sc[1] = sc[2] = 1.0;
    }
}

// FP64 evaluation at a physical point (landing, assembly, seed frame)
template <typename S, int MODE, bool MAG>
__device__ __forceinline__ void field_at_x(const S *__restrict__ nodes, const Geom &g, const double x[3],
                                           double u[3], double G[3][3], double &mag)
{
    if constexpr (geo_mode<MODE>()) {
        field_at_geo<double, S, MODE, MAG>(nodes, g, x, u, G, mag);
        return;
    }
    int ib[3];
    double q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double s = (x[d] - g.o[d]) * g.ih[d];
        s = fmin(fmax(s, -1e9), 1e9);
        const double fl = floor(s);
        ib[d] = (int)fl;
        q[d] = s - fl;
    }
    field_at<double, S, MODE, MAG>(nodes, g, ib, q, u, G, mag);
}

// not a point of the closed box (a non-finite coordinate is outside)
__device__ __forceinline__ bool outside_box(const Geom &g, double x0, double x1, double x2)
{
    return !(x0 >= g.lo[0] && x0 <= g.hi[0] && x1 >= g.lo[1] && x1 <= g.hi[1] && x2 >= g.lo[2] && x2 <= g.hi[2]);
}

// orthonormal (a, b) completing the unit vector n, branch-free
// (Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin 2017, JCGT 6(1))
__device__ __forceinline__ void frame_of(const double n[3], double a[3], double b[3])
{
    const double sg = copysign(1.0, n[2]);
    const double p = -1.0 / (sg + n[2]);
    const double q = n[0] * n[1] * p;
    a[0] = 1.0 + sg * n[0] * n[0] * p;
    a[1] = sg * q;
    a[2] = -sg * n[0];
    b[0] = q;
    b[1] = sg + n[1] * n[1] * p;
    b[2] = -n[1];
}

// ---------------------------------------------------------------------------
// end records
// ---------------------------------------------------------------------------
__device__ __forceinline__ void put_rec(const Records &r, int64_t i, const double y[9], double s,
                                        double h, int status, int attempts)
{
    const int64_t P = 2 * r.cap;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.y[k * P + i] = y[k];
    r.s[i] = s;
    r.h[i] = h;
    r.status[i] = status;
    r.attempts[i] = attempts;
}

__device__ __forceinline__ void get_rec(const Records &r, int64_t i, double y[9], double &s, double &h)
{
    const int64_t P = 2 * r.cap;
#pragma unroll
    for (int k = 0; k < 9; ++k) y[k] = r.y[k * P + i];
    s = r.s[i];
    h = r.h[i];
}

__device__ __forceinline__ int64_t seed_count(const TraceJob &j)
{
    return j.n_dev ? *j.n_dev : j.n_host;
}

// ---------------------------------------------------------------------------
// seed pass (FP64, one thread per seed): frame of eq. (9), and the half-lines
// that end at once -- seed outside the box, a null at the seed, or a seed on a
// face with its (signed) field pointing out (zero length, lowest such face).
// The others are flagged for stepping.
// ---------------------------------------------------------------------------
// set holding global seed i: the last set whose first seed is <= i (empty
// sets share their offset with the next set and are skipped)
__device__ __forceinline__ int find_set(const SetDesc *sets, int nsets, int64_t i)
{
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sets[mid].off <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename S, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_seed_pass(TraceJob job)
{
    const int64_t n = seed_count(job);
    if (blockIdx.x == 0 && threadIdx.x == 0) *job.rec.n_items = 2 * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        Geom gl = job.g;
        const double *sp = job.seeds;
        int64_t ss = job.seed_stride, li = i;
        if constexpr (BATCH) {
            const int set = find_set(job.sets, job.nsets, i);
            job.set_of[i] = set;
            const SetDesc &sd = job.sets[set];
            gl = sd.g;
            nodes = static_cast<const S *>(sd.nodes);
            sp = sd.seeds;
            ss = sd.n;
            li = i - sd.off;
        }
        const Geom &g = gl;
        const double x0[3] = {sp[li], sp[ss + li], sp[2 * ss + li]};
        double y0[9] = {x0[0], x0[1], x0[2], 0, 0, 0, 0, 0, 0};
        int st[2] = {-1, -1};
        if (outside_box(g, x0[0], x0[1], x0[2])) {
            st[0] = st[1] = QSQ_END_SEED_OUTSIDE;
        } else {
            double u[3], G[3][3], mag;
            field_at_x<S, MODE, false>(nodes, g, x0, u, G, mag);
            const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (un < 1e-6) {
                st[0] = st[1] = QSQ_END_NULL;
            } else {
                const double nn[3] = {u[0] / un, u[1] / un, u[2] / un};
                double a[3], b[3];
                frame_of(nn, a, b);
                double sc[3] = {1.0, 1.0, 1.0};
                if constexpr (geo_mode<MODE>()) geo_scale(g, x0, sc);   // eq. (8) inverted
                for (int k = 0; k < 3; ++k) {
                    y0[3 + k] = a[k] / sc[k];
                    y0[6 + k] = b[k] / sc[k];
                }
                for (int dir = 0; dir < 2; ++dir) {
                    const double sg = dir ? -1.0 : 1.0;
                    int face = -1;
                    for (int f = 0; f < 6 && face < 0; ++f) {
                        const int d = f >> 1;
                        const bool on = (f & 1) ? x0[d] == g.hi[d] : x0[d] == g.lo[d];
                        const double out = (f & 1) ? sg * nn[d] : -sg * nn[d];
                        if (on && out > 0.0) face = f;
                    }
                    st[dir] = face >= 0 ? face : kPendingStep;
                }
            }
        }
        for (int dir = 0; dir < 2; ++dir) {
            put_rec(job.rec, dir * job.rec.cap + i, y0, 0.0, 0.0, st[dir], 0);
            job.rec.flag[dir * n + i] = st[dir] == kPendingStep ? 1 : 0;
        }
    }
}

// work list: record indices of the flagged half-lines, forward ones first,
// each in seed order
static __global__ void k_compact(TraceJob job)
{
    const int64_t n2 = *job.rec.n_items, n = n2 / 2;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n2; it += (int64_t)gridDim.x * blockDim.x)
        if (job.rec.flag[it]) job.rec.work[job.rec.wpos[it]] = (int32_t)(it >= n ? job.rec.cap + (it - n) : it);
}

// ---------------------------------------------------------------------------
// spatial order of the work list: sort keys (set, Morton index of the seed's
// cell at `bits` bits per axis of the set's box) for the compacted list; the
// sort itself is a stable radix sort.  No line's arithmetic depends on where
// it runs, so results do not change.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread3(uint32_t v)   // bit k of v -> bit 3k
{
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 10; ++k) r |= ((v >> k) & 1u) << (3 * k);
    return r;
}

template <bool BATCH>
__global__ void k_sort_keys(TraceJob job, int bits)
{
    const int64_t nw = *job.rec.n_work;
    const int64_t P = 2 * job.rec.cap;
    const int side = 1 << bits;
    uint32_t *keys = reinterpret_cast<uint32_t *>(job.rec.flag);
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = job.rec.work[w];
        const int64_t i = r >= job.rec.cap ? r - job.rec.cap : r;
        const Geom &g = BATCH ? job.sets[job.set_of[i]].g : job.g;
        uint32_t c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double u = (job.rec.y[d * P + r] - g.lo[d]) / (g.hi[d] - g.lo[d]);
            int k = (int)(u * side);
            k = k < 0 ? 0 : (k > side - 1 ? side - 1 : k);
            c[d] = (uint32_t)k;
        }
        const uint32_t set = BATCH ? (uint32_t)job.set_of[i] : 0u;
        keys[w] = (set << (3 * bits)) | spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    }
}

// The landing list: the half-lines that the stepping pass left outside the
// box, in record order (forward halves, then backward ones, each in seed
// order), so that the landing kernels read and write the record planes in
// runs rather than in the work list's (spatial) order.  Flags over the half-
// line records, then a compaction into work2.
__device__ __forceinline__ int64_t half_record(const TraceJob &job, int64_t it, int64_t n)
{
    return it >= n ? job.rec.cap + (it - n) : it;
}

static __global__ void k_land_flags(TraceJob job)
{
    const int64_t n2 = *job.rec.n_items, n = n2 / 2;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n2; it += (int64_t)gridDim.x * blockDim.x)
        job.rec.flag[it] = job.rec.status[half_record(job, it, n)] == kPendingLand ? 1 : 0;
}

static __global__ void k_land_compact(TraceJob job)
{
    const int64_t n2 = *job.rec.n_items, n = n2 / 2;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n2; it += (int64_t)gridDim.x * blockDim.x)
        if (job.rec.flag[it]) job.rec.work2[job.rec.wpos[it]] = (int32_t)half_record(job, it, n);
}

// ---------------------------------------------------------------------------
// k_trace: persistent stepping kernel
// ---------------------------------------------------------------------------
// (the Euler variants fit 3 waves per SIMD: one evaluation's state per step)
template <typename T, typename S, int MODE, int GATHER, bool BATCH, bool EULER = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EULER ? 3 : 1))) k_trace(TraceJob job)
{
    static_assert(GATHER == kGatherDirect || (!BATCH && sizeof(T) == 4),
                  "cell caches: one field per launch, FP32 corner values");
    static_assert(GATHER != kGatherDirs || std::is_same<S, float>::value, "direction records: FP32 storage");
    constexpr bool CACHED =
        GATHER == kGatherLds || GATHER == kGatherRegs || GATHER == kGatherBricks || GATHER == kGatherDirs;
    // field and step limits of the lane's line: launch constants for one
    // field, reloaded from the set table at each refill in a batch (the cell
    // records' variant reads them in place of the node records)
    const S *__restrict__ nodes = static_cast<const S *>(
        GATHER == kGatherCells ? job.cells : GATHER == kGatherDirs ? static_cast<const void *>(job.dirs) : job.nodes);
    Geom gl = job.g;
    const Geom &g = gl;
    const StepOpts &o = job.o;
    double h_init = o.h_init, hmin = o.hmin;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t total = *job.rec.n_work;

    // lane state
    double X[3] = {0, 0, 0}, s = 0.0;
    T D1[3] = {0, 0, 0}, D2[3] = {0, 0, 0};
    T h = 0, sigma = 1;
    int attempts = 0;
    int64_t rec = 0;
    bool active = false, done = false, have_k1 = false;
    T Kx[6][3], K1[6][3], K2[6][3];

    const T rtol = (T)o.rtol, atol = (T)o.atol;
    T hmax = (T)o.h_max;
    T ih[3] = {(T)g.ih[0], (T)g.ih[1], (T)g.ih[2]};
    unsigned long long c_att = 0, c_ev = 0, c_act = 0, c_land = 0;   // work counters
    // cached-gather state
    const uint64_t nrec = GATHER == kGatherBricks
                              ? 8 * (uint64_t)((g.n[0] + 1) / 2) * ((g.n[1] + 1) / 2) * ((g.n[2] + 1) / 2)
                              : (uint64_t)g.n[0] * g.n[1] * g.n[2];
    const int cbytes = CACHED ? (int)(node_bytes<S>() * nrec) : 0;
    const __amdgpu_buffer_rsrc_t rsrc = node_rsrc(GATHER == kGatherBricks ? job.bricks : job.nodes, cbytes);
    int cache_cell[3] = {-1, -1, -1};
    // LDS cell cache: kCachePlanes planes of blockDim.x float4 (dynamic size)
    extern __shared__ float4 lds_cache[];
    const int stride = (int)blockDim.x;
    float4 *slot = lds_cache + threadIdx.x;
    // register cell cache: the corners of the cell a lane evaluated last
    int reg_cell = -1;
    Brick reg_brick = {};

    // Work distribution.  The work list is split into nparts contiguous parts
    // (one, or kParts with the partition bit of the launch word), each with
    // its own counter.  Workgroup b starts in part b mod nparts -- the XCD
    // the hardware dispatches it to, so that the lanes of one XCD trace lines
    // whose seeds lie together along the curve and share that XCD's L2 -- and
    // the first item of each of its lanes is the lane's index within the
    // part's workgroups (the launcher starts each counter past those).  After
    // that each wave takes chunks of kChunk items of its part with one atomic
    // and hands them to its idle lanes itself; a wave whose part is used up
    // moves on to the following parts, and its lanes are done when every
    // part is.  Which lane traces which line never changes a result.
    constexpr int64_t kChunk = 64;
    const int nparts = (o.launch >> 9) & 1 ? kParts : 1;
    const int home = (int)(blockIdx.x % (unsigned)nparts);
    unsigned long long *pcount = job.counter + kPartCounter;
    auto pbeg = [&](int p) { return total * p / nparts; };
    int part = home, spent = 0;    // the wave's part; parts found used up
    int64_t cnext = 0, cend = 0;   // the wave's unassigned items [cnext, cend)
    bool first_fill = true;
    for (;;) {
        // ---- refill idle lanes
        const uint64_t need = __ballot(!active && !done);
        if (need) {
            const int j = __popcll(need & ((1ull << lane) - 1ull));   // rank among idle lanes
            int64_t item = -1;
            if (first_fill) {
                item = pbeg(home) + (int64_t)(blockIdx.x / (unsigned)nparts) * blockDim.x + (threadIdx.x & ~63u) + j;
                if (item >= pbeg(home + 1)) item = -1;
            } else {
                const int k = __popcll(need);
                const int64_t avail = cend - cnext;
                if (avail < k && spent < nparts) {
                    // one more chunk: from the wave's part, or the next part not used up
                    unsigned long long b = 0;
                    int p = part, t = spent;
                    const int leader = __ffsll((unsigned long long)need) - 1;
                    if (lane == leader) {
                        for (;;) {
                            b = atomicAdd(pcount + p, (unsigned long long)kChunk);
                            if ((int64_t)b < pbeg(p + 1)) break;
                            if (++t >= nparts) break;
                            p = p + 1 < nparts ? p + 1 : 0;
                        }
                    }
                    b = __shfl(b, leader);
                    part = __shfl(p, leader);
                    spent = __shfl(t, leader);
                    const int64_t fresh = (int64_t)b;
                    const int64_t fend = spent < nparts ? min(fresh + kChunk, pbeg(part + 1)) : fresh;
                    const int64_t got = fend - fresh;
                    if (j < avail)
                        item = cnext + j;
                    else if (j - avail < got)
                        item = fresh + (j - avail);
                    const int64_t used = k - avail < got ? k - avail : got;
                    cnext = fresh + used;
                    cend = fend;
                } else {
                    if (j < avail) item = cnext + j;
                    cnext += k < avail ? k : avail;
                }
            }
            first_fill = false;
            if (!active && !done) {
                if (item < 0) {
                    // no item this round; done once every part is used up
                    done = spent >= nparts;
                } else {
                    // the seed pass left x0 and the frame (eq. 9) in the record
                    rec = job.rec.work[item];
                    const int dir = rec >= job.rec.cap ? 1 : 0;
                    if constexpr (BATCH) {
                        const SetDesc &sd = job.sets[job.set_of[dir ? rec - job.rec.cap : rec]];
                        gl = sd.g;
                        nodes = static_cast<const S *>(sd.nodes);
                        h_init = sd.h_init;
                        hmin = sd.hmin;
                        hmax = (T)sd.h_max;
#pragma unroll
                        for (int d = 0; d < 3; ++d) ih[d] = (T)gl.ih[d];
                    }
                    sigma = dir ? (T)-1 : (T)1;
                    const int64_t P = 2 * job.rec.cap;
                    X[0] = job.rec.y[rec];
                    X[1] = job.rec.y[P + rec];
                    X[2] = job.rec.y[2 * P + rec];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        D1[k] = (T)job.rec.y[(3 + k) * P + rec];
                        D2[k] = (T)job.rec.y[(6 + k) * P + rec];
                    }
                    s = 0.0;
                    h = (T)h_init;
                    attempts = 0;
                    have_k1 = false;
                    active = true;
                    ++c_act;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        // issue priority among the waves of a SIMD: waves holding a line that
        // has run many attempts go first, so the long lines that end a launch
        // are slowed less by the short ones beside them (scheduling only)
        if (__ballot(active && attempts >= 512)) __builtin_amdgcn_s_setprio(3);
        else if (__ballot(active && attempts >= 256)) __builtin_amdgcn_s_setprio(2);
        else if (__ballot(active && attempts >= 128)) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        if (!active) continue;

        // ---- one step attempt (oracle order: step cap, null, trial, accept/reject, exit)
        int stop = -1;
        if (attempts >= o.max_steps) stop = QSQ_END_MAX_STEPS;

        int ib[3];
        T fb[3];
        if (stop < 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double xg = (X[d] - g.o[d]) * g.ih[d];
                const double fl = floor(xg);
                ib[d] = (int)fl;
                fb[d] = (T)(xg - fl);
            }
            if (!EULER && !have_k1) {
                const T un2 = rhs_step<T, S, MODE, GATHER>(nodes, rsrc, cbytes, g, ib, fb, (T)1, D1, D2, Kx[0], K1[0],
                                                           K2[0], cache_cell, slot, stride, reg_cell, reg_brick);
                ++c_ev;
                if (un2 < (T)1e-12) stop = QSQ_END_NULL;   // NaN: not a null (the step reports it)
                have_k1 = true;
            }
        }
        if constexpr (EULER) {
            // explicit Euler (Sect. 3.4): one evaluation at the current point
            // per fixed step h, the whole state advanced along it
            if (stop < 0) {
                const T un2 = rhs_step<T, S, MODE, GATHER>(nodes, rsrc, cbytes, g, ib, fb, (T)1, D1, D2, Kx[0],
                                                           K1[0], K2[0], cache_cell, slot, stride, reg_cell,
                                                           reg_brick);
                ++c_ev;
                if (un2 < (T)1e-12) stop = QSQ_END_NULL;   // NaN: not a null (the step reports it)
            }
            if (stop < 0) {
                T hs = h;
                bool last = false;
                if (o.max_length > 0.0 && (double)hs >= o.max_length - s) {
                    hs = (T)(o.max_length - s);
                    last = true;
                }
                const T hsig = sigma * hs;
                double Xn[3];
                T D1n[3], D2n[3], fsum = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    Xn[i] = X[i] + (double)(hsig * Kx[0][i]);
                    D1n[i] = fma(hsig, K1[0][i], D1[i]);
                    D2n[i] = fma(hsig, K2[0][i], D2[i]);
                    fsum += ((T)Xn[i] + D1n[i]) + D2n[i];
                }
                ++attempts;
                ++c_att;
                if (!isfinite(fsum)) {
                    stop = QSQ_END_NONFINITE;
                } else if (outside_box(g, Xn[0], Xn[1], Xn[2])) {
                    // the step that leaves the box: cut at the face in FP64
                    const double y[9] = {X[0], X[1], X[2], (double)D1[0], (double)D1[1], (double)D1[2],
                                         (double)D2[0], (double)D2[1], (double)D2[2]};
                    put_rec(job.rec, rec, y, s, (double)hs, kPendingLand, attempts);
                    active = false;
                    ++c_land;
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        X[i] = Xn[i];
                        D1[i] = D1n[i];
                        D2[i] = D2n[i];
                    }
                    if (last) {
                        s = o.max_length;
                        stop = QSQ_END_MAX_LENGTH;
                    } else {
                        s += (double)hs;
                    }
                }
            }
        }
        if (!EULER && stop < 0) {
            T hs = h < hmax ? h : hmax;
            bool last = false;
            if (o.max_length > 0.0 && (double)hs >= o.max_length - s) {
                hs = (T)(o.max_length - s);
                last = true;
            }
            // The stage slopes K hold the unsigned right-hand side F; the
            // direction sign rides on the step: sigma F h = F (sigma h), and
            // both products are exact sign flips, so the arithmetic is that of
            // f = sigma F bit for bit.
            const T hsig = sigma * hs;
            // stages 2..6
#define QSQ_STAGE(ST, ...)                                                                          \
    {                                                                                               \
        const T c_[] = {__VA_ARGS__};                                                               \
        T q[3], d1[3], d2[3];                                                                       \
        _Pragma("unroll") for (int i = 0; i < 3; ++i)                                               \
        {                                                                                           \
            T ax = 0, a1 = 0, a2 = 0;                                                               \
            _Pragma("unroll") for (int j = 0; j < ST; ++j)                                          \
            {                                                                                       \
                ax = fma(c_[j], Kx[j][i], ax);                                                      \
                a1 = fma(c_[j], K1[j][i], a1);                                                      \
                a2 = fma(c_[j], K2[j][i], a2);                                                      \
            }                                                                                       \
            q[i] = fma(hsig * ax, ih[i], fb[i]);                                                    \
            d1[i] = fma(hsig, a1, D1[i]);                                                           \
            d2[i] = fma(hsig, a2, D2[i]);                                                           \
        }                                                                                           \
        rhs_step<T, S, MODE, GATHER>(nodes, rsrc, cbytes, g, ib, q, (T)1, d1, d2, Kx[ST], K1[ST], K2[ST], \
                                     cache_cell, slot, stride, reg_cell, reg_brick);               \
    }
            QSQ_STAGE(1, (T)ck::a21)
            QSQ_STAGE(2, (T)ck::a31, (T)ck::a32)
            QSQ_STAGE(3, (T)ck::a41, (T)ck::a42, (T)ck::a43)
            QSQ_STAGE(4, (T)ck::a51, (T)ck::a52, (T)ck::a53, (T)ck::a54)
            QSQ_STAGE(5, (T)ck::a61, (T)ck::a62, (T)ck::a63, (T)ck::a64, (T)ck::a65)
#undef QSQ_STAGE
            // 5th-order solution (propagated) and the error estimate y5 - y4
            double Xn[3];
            T D1n[3], D2n[3];
            T err = 0, fsum = 0;
            bool finite;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T bx = ck_b5(Kx[0][i], Kx[2][i], Kx[3][i], Kx[5][i]);
                const T b1 = ck_b5(K1[0][i], K1[2][i], K1[3][i], K1[5][i]);
                const T b2 = ck_b5(K2[0][i], K2[2][i], K2[3][i], K2[5][i]);
                const T ex = ck_e(Kx[0][i], Kx[2][i], Kx[3][i], Kx[4][i], Kx[5][i]);
                const T e1 = ck_e(K1[0][i], K1[2][i], K1[3][i], K1[4][i], K1[5][i]);
                const T e2 = ck_e(K2[0][i], K2[2][i], K2[3][i], K2[4][i], K2[5][i]);
                Xn[i] = X[i] + (double)(hsig * bx);
                D1n[i] = fma(hsig, b1, D1[i]);
                D2n[i] = fma(hsig, b2, D2[i]);
                const T xo = (T)X[i], xn = (T)Xn[i];
                err = fmax(err, err_ratio(fabs(hs * ex), err_scale(atol, rtol, xo, xn)));
                err = fmax(err, err_ratio(fabs(hs * e1), err_scale(atol, rtol, D1[i], D1n[i])));
                err = fmax(err, err_ratio(fabs(hs * e2), err_scale(atol, rtol, D2[i], D2n[i])));
                // one test for the whole state: an infinity or NaN anywhere
                // makes the sum non-finite
                fsum += (xn + D1n[i]) + (D2n[i] + ex) + (e1 + e2);
            }
            finite = isfinite(fsum);
            ++attempts;
            ++c_att;
            c_ev += 5;
            if (!finite) {
                stop = QSQ_END_NONFINITE;
            } else if (err > (T)1) {
                // reject: shrink, keep k1 (y is unchanged)
                const T f = (T)0.9 * (T)exp2((T)-0.25 * (T)log2(err));
                h = hs * (f > (T)0.2 ? f : (T)0.2);
                if ((double)h < hmin) stop = QSQ_END_UNDERFLOW;
            } else if (outside_box(g, Xn[0], Xn[1], Xn[2])) {
                // accepted trial step leaves the box: hand over to FP64 landing
                const double y[9] = {X[0], X[1], X[2], (double)D1[0], (double)D1[1], (double)D1[2],
                                     (double)D2[0], (double)D2[1], (double)D2[2]};
                put_rec(job.rec, rec, y, s, (double)hs, kPendingLand, attempts);
                active = false;
                ++c_land;
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    X[i] = Xn[i];
                    D1[i] = D1n[i];
                    D2[i] = D2n[i];
                }
                have_k1 = false;
                if (last) {
                    s = o.max_length;
                    stop = QSQ_END_MAX_LENGTH;
                } else {
                    s += (double)hs;
                    const T f = err > (T)0 ? (T)0.9 * (T)exp2((T)-0.2 * (T)log2(err)) : (T)5;
                    h = hs * (f < (T)5 ? f : (T)5);
                }
            }
        }
        if (stop >= 0) {
            const double y[9] = {X[0], X[1], X[2], (double)D1[0], (double)D1[1], (double)D1[2],
                                 (double)D2[0], (double)D2[1], (double)D2[2]};
            put_rec(job.rec, rec, y, s, 0.0, stop, attempts);
            active = false;
        }
    }
    if (job.work) {
        // wave-level sums, one atomic per counter per wave
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) {
            c_att += __shfl_xor(c_att, o2);
            c_ev += __shfl_xor(c_ev, o2);
            c_act += __shfl_xor(c_act, o2);
            c_land += __shfl_xor(c_land, o2);
        }
        if (lane == 0 && (c_att | c_ev | c_act | c_land)) {   // waves that stepped nothing add nothing
            atomicAdd(&job.work[0], c_att);
            atomicAdd(&job.work[1], c_ev);
            atomicAdd(&job.work[2], c_act);
            atomicAdd(&job.work[3], c_land);
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 Cash-Karp step used by the landing pass (5th-order end only)
// ---------------------------------------------------------------------------
template <typename S, int MODE>
__device__ void ck54_fp64(const S *__restrict__ nodes, const Geom &g, double sigma, const double y[9],
                          double hs, double yo[9])
{
    double K[6][9];
    const double A[6][5] = {{0, 0, 0, 0, 0},
                            {ck::a21, 0, 0, 0, 0},
                            {ck::a31, ck::a32, 0, 0, 0},
                            {ck::a41, ck::a42, ck::a43, 0, 0},
                            {ck::a51, ck::a52, ck::a53, ck::a54, 0},
                            {ck::a61, ck::a62, ck::a63, ck::a64, ck::a65}};
    int ib[3];
    double fb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xg = (y[d] - g.o[d]) * g.ih[d];
        const double fl = floor(fmin(fmax(xg, -1e9), 1e9));
        ib[d] = (int)fl;
        fb[d] = xg - fl;
    }
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        double q[3], d1[3], d2[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ax = 0, a1 = 0, a2 = 0;
#pragma unroll
            for (int j = 0; j < st; ++j) {
                ax = fma(A[st][j], K[j][i], ax);
                a1 = fma(A[st][j], K[j][3 + i], a1);
                a2 = fma(A[st][j], K[j][6 + i], a2);
            }
            q[i] = fma(hs * ax, g.ih[i], fb[i]);
            d1[i] = fma(hs, a1, y[3 + i]);
            d2[i] = fma(hs, a2, y[6 + i]);
        }
        double kx[3], k1[3], k2[3];
        rhs<double, S, MODE>(nodes, g, ib, q, sigma, d1, d2, kx, k1, k2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            K[st][i] = kx[i];
            K[st][3 + i] = k1[i];
            K[st][6 + i] = k2[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        yo[i] = y[i] + hs * (ck::b1 * K[0][i] + ck::b3 * K[2][i] + ck::b4 * K[3][i] + ck::b6 * K[5][i]);
}

// The position part of one FP64 Cash-Karp step (eq. (1) alone: the position
// does not depend on the deviation vectors), the same operations as the
// position components of ck54_fp64.
template <typename S, int MODE>
__device__ void ck54_pos(const S *__restrict__ nodes, const Geom &g, double sigma, const double y[3], double hs,
                         double yo[3], double *slope0 = nullptr, const double *k1 = nullptr)
{
    double K[6][3];
    const double A[6][5] = {{0, 0, 0, 0, 0},
                            {ck::a21, 0, 0, 0, 0},
                            {ck::a31, ck::a32, 0, 0, 0},
                            {ck::a41, ck::a42, ck::a43, 0, 0},
                            {ck::a51, ck::a52, ck::a53, ck::a54, 0},
                            {ck::a61, ck::a62, ck::a63, ck::a64, ck::a65}};
    int ib[3];
    double fb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xg = (y[d] - g.o[d]) * g.ih[d];
        const double fl = floor(fmin(fmax(xg, -1e9), 1e9));
        ib[d] = (int)fl;
        fb[d] = xg - fl;
    }
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        if (st == 0 && k1) {
            // the first stage sits at y whatever the step length: a caller
            // that took a step from y already has it
#pragma unroll
            for (int i = 0; i < 3; ++i) K[0][i] = k1[i];
            continue;
        }
        double q[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ax = 0;
#pragma unroll
            for (int j = 0; j < st; ++j) ax = fma(A[st][j], K[j][i], ax);
            q[i] = fma(hs * ax, g.ih[i], fb[i]);
        }
        double u[3];
        field_u<double, S, MODE>(nodes, g, ib, q, u);
#pragma unroll
        for (int i = 0; i < 3; ++i) K[st][i] = sigma * u[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        yo[i] = y[i] + hs * (ck::b1 * K[0][i] + ck::b3 * K[2][i] + ck::b4 * K[3][i] + ck::b6 * K[5][i]);
    if (slope0) {
        // dx/dlambda at the start of the step (the first stage)
#pragma unroll
        for (int i = 0; i < 3; ++i) slope0[i] = K[0][i];
    }
}

// First trial step length of the landing: the root in (0, hs) of the
// quadratic with gap g0 < 0 and slope s0 at 0 and gap g1 > 0 at hs, or the
// secant point if that root is not strictly inside.
__device__ __forceinline__ double landing_guess(double g0, double s0, double g1, double hs)
{
    const double sec = -g0 * hs / (g1 - g0);
    const double cq = (g1 - g0 - s0 * hs) / (hs * hs);
    const double disc = s0 * s0 - 4.0 * cq * g0;
    const double den = s0 + sqrt(fmax(disc, 0.0));
    const double h = den > 0.0 ? -2.0 * g0 / den : -1.0;
    return (h > 0.0 && h < hs) ? h : sec;
}

// v[d] for a run-time d in 0..2 as selects (a dynamic index would put the
// array in scratch memory)
__device__ __forceinline__ double pick3(const double *v, int d)
{
    return d == 0 ? v[0] : (d == 1 ? v[1] : v[2]);
}

// signed distance of x beyond face f (0..5 = x lo, x hi, y lo, ...): > 0 outside
__device__ __forceinline__ double beyond_face(const Geom &g, const double *x, int f)
{
    const int d = f >> 1;
    return (f & 1) ? pick3(x, d) - pick3(g.hi, d) : pick3(g.lo, d) - pick3(x, d);
}

template <typename S, int MODE>
__device__ double face_gap(const S *nodes, const Geom &g, double sigma, const double y[3], double hs,
                           int f, double yo[3], const double k1[3])
{
    if (hs == 0.0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) yo[i] = y[i];
    } else {
        ck54_pos<S, MODE>(nodes, g, sigma, y, hs, yo, nullptr, k1);
    }
    return beyond_face(g, yo, f);
}

// ---------------------------------------------------------------------------
// k_land: FP64 landing of pending half-lines on the first face crossed, in
// two passes.  The step length that ends on the face needs the position only
// (eq. (1) does not involve the deviation vectors), so the root find steps
// three components (few registers, many waves); k_land_final then takes the
// one full nine-component step to the root and snaps onto the face.
// ---------------------------------------------------------------------------
template <typename S, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_land(TraceJob job)
{
    // the list of half-lines to land (compacted after the stepping pass), so
    // that every lane of a wave has one
    const int64_t total = *job.rec.n_land;
    const int64_t P = 2 * job.rec.cap;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = job.rec.work2[it];
        const int dir = r >= job.rec.cap ? 1 : 0;
        const int64_t i = dir ? r - job.rec.cap : r;
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        Geom gl = job.g;
        double gtol = job.o.gtol;
        if constexpr (BATCH) {
            const SetDesc &sd = job.sets[job.set_of[i]];
            gl = sd.g;
            nodes = static_cast<const S *>(sd.nodes);
            gtol = sd.gtol;
        }
        const Geom &g = gl;
        const double sigma = dir ? -1.0 : 1.0;
        const double y[3] = {job.rec.y[r], job.rec.y[P + r], job.rec.y[2 * P + r]};
        const double hs = job.rec.h[r];
        double y5[3], v0[3];
        ck54_pos<S, MODE>(nodes, g, sigma, y, hs, y5, v0);
        double best = INFINITY;
        int face = -1;
        double gmax = -INFINITY;
        int fmax_ = 0;
        for (int f = 0; f < 6; ++f) {
            const double gend = beyond_face(g, y5, f);
            if (gend > gmax) {
                gmax = gend;
                fmax_ = f;
            }
            if (!(gend > 0.0)) continue;
            // regula falsi (Anderson-Bjorck) for the step length ending on face f
            double yo[3];
            double a = 0.0, b = hs;
            double ga = face_gap<S, MODE>(nodes, g, sigma, y, a, f, yo, v0);
            double hf;
            if (ga >= 0.0) {
                hf = 0.0;
            } else {
                double gb = gend;
                int side = 0;
                hf = -1.0;
                // the first trial uses the gap's slope at the start of the step
                // (a quadratic model); regula falsi from there on
                const int dd = f >> 1;
                const double s0 = (f & 1) ? pick3(v0, dd) : -pick3(v0, dd);
                const double c0 = landing_guess(ga, s0, gb, hs);
                for (int k = 0; k < 200; ++k) {
                    const double c = k == 0 ? c0 : (a * gb - b * ga) / (gb - ga);
                    const double gc = face_gap<S, MODE>(nodes, g, sigma, y, c, f, yo, v0);
                    if (fabs(gc) <= gtol) {
                        hf = c;
                        break;
                    }
                    // the same end replaced twice in a row: scale the kept
                    // end's gap (Anderson-Bjorck factor 1 - gc/g_old, 1/2
                    // when that is not positive, which is Illinois)
                    if (gc > 0.0) {
                        if (side == 1) {
                            const double m = 1.0 - gc / gb;
                            ga *= m > 0.0 ? m : 0.5;
                        }
                        b = c;
                        gb = gc;
                        side = 1;
                    } else {
                        if (side == -1) {
                            const double m = 1.0 - gc / ga;
                            gb *= m > 0.0 ? m : 0.5;
                        }
                        a = c;
                        ga = gc;
                        side = -1;
                    }
                    if (b - a <= 1e-15 * hs) break;
                }
                if (hf < 0.0) hf = ga > -gb ? a : b;
            }
            if (hf < best) {
                best = hf;
                face = f;
            }
        }
        if (face < 0) {
            // the FP64 re-solve ends inside (the trial end was within rounding
            // of a face): land on the nearest face at the full step
            face = fmax_;
            best = hs;
        }
        job.rec.h[r] = best;
        job.rec.status[r] = kLandFace + face;
    }
}

template <typename S, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_land_final(TraceJob job)
{
    const int64_t total = *job.rec.n_land;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = job.rec.work2[it];
        const int dir = r >= job.rec.cap ? 1 : 0;
        const int64_t i = dir ? r - job.rec.cap : r;
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        Geom gl = job.g;
        if constexpr (BATCH) {
            const SetDesc &sd = job.sets[job.set_of[i]];
            gl = sd.g;
            nodes = static_cast<const S *>(sd.nodes);
        }
        const Geom &g = gl;
        const double sigma = dir ? -1.0 : 1.0;
        double y[9], s, best, yl[9];
        get_rec(job.rec, r, y, s, best);
        const int face = job.rec.status[r] - kLandFace;
        if (best > 0.0) {
            ck54_fp64<S, MODE>(nodes, g, sigma, y, best, yl);
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) yl[k] = y[k];
        }
        const int d = face >> 1;
        const double snap = (face & 1) ? pick3(g.hi, d) : pick3(g.lo, d);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k == d) yl[k] = snap;
        const int att = job.rec.attempts[r];
        put_rec(job.rec, r, yl, s + best, 0.0, face, att);
    }
}

// ---------------------------------------------------------------------------
// k_land_euler: FP64 landing of an explicit Euler step.  The end of an Euler
// step moves linearly with its length, so the length that ends on face f is
// the distance to the face over the step's rate towards it; the first face
// crossed (the shortest such length; exact ties keep the lower face) takes
// the line, the whole state is advanced by that length and the position
// snapped to the face.
// ---------------------------------------------------------------------------
template <typename S, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_land_euler(TraceJob job)
{
    const int64_t total = *job.rec.n_land;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = job.rec.work2[it];
        const int dir = r >= job.rec.cap ? 1 : 0;
        const int64_t i = dir ? r - job.rec.cap : r;
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        Geom gl = job.g;
        if constexpr (BATCH) {
            const SetDesc &sd = job.sets[job.set_of[i]];
            gl = sd.g;
            nodes = static_cast<const S *>(sd.nodes);
        }
        const Geom &g = gl;
        const double sigma = dir ? -1.0 : 1.0;
        double y[9], s, hs;
        get_rec(job.rec, r, y, s, hs);
        double u[3], G[3][3], mag;
        field_at_x<S, MODE, false>(nodes, g, y, u, G, mag);
        double dy[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dy[k] = sigma * u[k];
            dy[3 + k] = sigma * (G[0][k] * y[3] + G[1][k] * y[4] + G[2][k] * y[5]);
            dy[6 + k] = sigma * (G[0][k] * y[6] + G[1][k] * y[7] + G[2][k] * y[8]);
        }
        double best = INFINITY;
        int face = -1;
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1;
            const double wall = (f & 1) ? pick3(g.hi, d) : pick3(g.lo, d);
            const double yd = pick3(y, d), vd = pick3(dy, d);
            const double end = yd + hs * vd;
            const double gap = (f & 1) ? end - wall : wall - end;
            if (!(gap > 0.0)) continue;
            double hf = (wall - yd) / vd;
            hf = hf < 0.0 ? 0.0 : (hf > hs ? hs : hf);
            if (hf < best) {
                best = hf;
                face = f;
            }
        }
        double yl[9];
        if (face < 0) {
            // the FP32 step left the box but the FP64 one does not: end on
            // the face nearest the FP64 end point of the full step
            best = hs;
            double gmax = -INFINITY;
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1;
                const double end = pick3(y, d) + hs * pick3(dy, d);
                const double gap = (f & 1) ? end - pick3(g.hi, d) : pick3(g.lo, d) - end;
                if (gap > gmax) {
                    gmax = gap;
                    face = f;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) yl[k] = y[k] + best * dy[k];
        const int d = face >> 1;
        const double snap = (face & 1) ? pick3(g.hi, d) : pick3(g.lo, d);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k == d) yl[k] = snap;
        put_rec(job.rec, r, yl, s + best, 0.0, face, job.rec.attempts[r]);
    }
}

// ---------------------------------------------------------------------------
// k_assemble: FP64 Q and length per seed (eq. 10-11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ double cross_len(const double *a, const double *b)
{
    const double c0 = a[1] * b[2] - a[2] * b[1];
    const double c1 = a[2] * b[0] - a[0] * b[2];
    const double c2 = a[0] * b[1] - a[1] * b[0];
    return sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

// a_F^2 b_B^2 + a_B^2 b_F^2 - 2 (a_B . b_B)(a_F . b_F)
__device__ __forceinline__ double q_bracket(const double *aF, const double *bF, const double *aB,
                                            const double *bB)
{
    return dot3(aF, aF) * dot3(bB, bB) + dot3(aB, aB) * dot3(bF, bF) - 2.0 * dot3(aB, bB) * dot3(aF, bF);
}

template <typename S, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_assemble(TraceJob job)
{
    const int64_t n = seed_count(job);
    const int64_t P = 2 * job.rec.cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rF = i, rB = job.rec.cap + i;
        // field, seeds and outputs of the seed (its set's in a batch)
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        Geom gl = job.g;
        const double *seeds = job.seeds;
        int64_t ss = job.seed_stride, os = job.out_stride, li = i;
        double *o_fpf = job.fp_fwd, *o_fpb = job.fp_bwd, *o_fll = job.fll;
        double *o_qp = job.q_perp, *o_qd = job.q_det, *o_qf = job.q_fp;
        int32_t *o_st = job.status, *o_steps = job.steps;
        if constexpr (BATCH) {
            const SetDesc &sd = job.sets[job.set_of[i]];
            gl = sd.g;
            nodes = static_cast<const S *>(sd.nodes);
            seeds = sd.seeds;
            ss = os = sd.n;
            li = i - sd.off;
            o_fpf = sd.fp_fwd;
            o_fpb = sd.fp_bwd;
            o_fll = sd.fll;
            o_qp = sd.q_perp;
            o_qd = sd.q_det;
            o_qf = sd.q_fp;
            o_st = sd.status;
            o_steps = sd.steps;
        }
        const Geom &g = gl;
        const int stF = job.rec.status[rF], stB = job.rec.status[rB];
        double yF[9], yB[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            yF[k] = job.rec.y[k * P + rF];
            yB[k] = job.rec.y[k * P + rB];
        }
        const double sF = job.rec.s[rF], sB = job.rec.s[rB];
        const bool open = !(stF == QSQ_END_ZLO && stB == QSQ_END_ZLO);
        const int word = (stF & 0xff) | ((stB & 0xff) << 8) | (open ? QSQ_STATUS_OPEN : 0);
        o_st[li] = word;
        if (o_fll) o_fll[li] = sF + sB;
        if (o_fpf)
            for (int k = 0; k < 3; ++k) o_fpf[k * os + li] = yF[k];
        if (o_fpb)
            for (int k = 0; k < 3; ++k) o_fpb[k * os + li] = yB[k];
        if (o_steps) {
            if (job.steps_sum) {
                o_steps[li] = job.rec.attempts[rF] + job.rec.attempts[rB];
            } else {
                o_steps[li] = job.rec.attempts[rF];
                o_steps[os + li] = job.rec.attempts[rB];
            }
        }
        double qp = NAN, qd = NAN, qf = NAN;
        const bool defF = stF >= QSQ_END_XLO && stF <= QSQ_END_MAX_STEPS;
        const bool defB = stB >= QSQ_END_XLO && stB <= QSQ_END_MAX_STEPS;
        const bool skip = (job.o.flags & QSQ_FLAG_SKIP_OPEN) && open;
        if (defF && defB && !skip) {
            const double x0[3] = {seeds[li], seeds[ss + li], seeds[2 * ss + li]};
            double G[3][3], uF[3], uB[3], u0[3], BF, BB, B0;
            field_at_x<S, MODE, true>(nodes, g, yF, uF, G, BF);
            field_at_x<S, MODE, true>(nodes, g, yB, uB, G, BB);
            field_at_x<S, MODE, true>(nodes, g, x0, u0, G, B0);
            const double vF[3] = {uF[0], uF[1], uF[2]}, vB[3] = {uB[0], uB[1], uB[2]};
            const double nF = sqrt(dot3(uF, uF)), nB = sqrt(dot3(uB, uB));
            for (int k = 0; k < 3; ++k) {
                uF[k] /= nF;
                uB[k] /= nB;
            }
            if constexpr (geo_mode<MODE>()) {
                // the deviations as lengths at each end, eq. (8)
                double scF[3], scB[3];
                geo_scale(g, yF, scF);
                geo_scale(g, yB, scB);
                for (int k = 0; k < 3; ++k) {
                    yF[3 + k] *= scF[k];
                    yF[6 + k] *= scF[k];
                    yB[3 + k] *= scB[k];
                    yB[6 + k] *= scB[k];
                }
            }
            // perpendicular parts of the deviations at both ends (Sect. 3.5)
            double aF[3], bF[3], aB[3], bB[3];
            const double pa = dot3(uF, yF + 3), pb = dot3(uF, yF + 6);
            const double qa = dot3(uB, yB + 3), qb = dot3(uB, yB + 6);
            for (int k = 0; k < 3; ++k) {
                aF[k] = yF[3 + k] - uF[k] * pa;
                bF[k] = yF[6 + k] - uF[k] * pb;
                aB[k] = yB[3 + k] - uB[k] * qa;
                bB[k] = yB[6 + k] - uB[k] * qb;
            }
            const double br = q_bracket(aF, bF, aB, bB);
            qp = BF * BB / (B0 * B0) * br;                                  // eq. (11)
            qd = br / (cross_len(aF, bF) * cross_len(aB, bB));
            if (stF <= QSQ_END_ZHI && stB <= QSQ_END_ZHI) {
                // slide the deviations along the line into the exit-face planes
                const int dF = stF >> 1, dB = stB >> 1;
                const double rF1 = yF[3 + dF] / vF[dF], rF2 = yF[6 + dF] / vF[dF];
                const double rB1 = yB[3 + dB] / vB[dB], rB2 = yB[6 + dB] / vB[dB];
                double pF1[3], pF2[3], pB1[3], pB2[3];
                for (int k = 0; k < 3; ++k) {
                    pF1[k] = yF[3 + k] - vF[k] * rF1;
                    pF2[k] = yF[6 + k] - vF[k] * rF2;
                    pB1[k] = yB[3 + k] - vB[k] * rB1;
                    pB2[k] = yB[6 + k] - vB[k] * rB2;
                }
                qf = q_bracket(pF1, pF2, pB1, pB2) / (cross_len(pF1, pF2) * cross_len(pB1, pB2));
            }
        }
        if (o_qp) o_qp[li] = qp;
        if (o_qd) o_qd[li] = qd;
        if (o_qf) o_qf[li] = qf;
    }
}

// ---------------------------------------------------------------------------
// General geometry: stepping and landing in physical coordinates
// ---------------------------------------------------------------------------
// f(y) of eq. (1)+(5) (Cartesian) or eq. (2)+(6) (spherical: the metric factors
// divide each component) at the physical point x; returns |u|^2
template <typename T, typename S, int MODE>
__device__ __forceinline__ T rhs_geo(const S *__restrict__ nodes, const Geom &g, const double x[3], T sigma,
                                     const T d1[3], const T d2[3], T kx[3], T k1[3], T k2[3])
{
    T u[3], G[3][3], mag;
    field_at_geo<T, S, MODE, false>(nodes, g, x, u, G, mag);
    const T un2 = rhs_from(sigma, u, G, d1, d2, kx, k1, k2);
    if (g.geometry == QSQ_GEOMETRY_SPHERICAL) {
        double sc[3];
        geo_scale(g, x, sc);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T m = (T)(1.0 / sc[i]);
            kx[i] *= m;
            k1[i] *= m;
            k2[i] *= m;
        }
    }
    return un2;
}

// one FP64 Cash-Karp step of the whole state in physical coordinates (5th-order end)
template <typename S, int MODE>
__device__ void ck54_geo(const S *__restrict__ nodes, const Geom &g, double sigma, const double y[9], double hs,
                         double yo[9])
{
    double K[6][9];
    const double A[6][5] = {{0, 0, 0, 0, 0},
                            {ck::a21, 0, 0, 0, 0},
                            {ck::a31, ck::a32, 0, 0, 0},
                            {ck::a41, ck::a42, ck::a43, 0, 0},
                            {ck::a51, ck::a52, ck::a53, ck::a54, 0},
                            {ck::a61, ck::a62, ck::a63, ck::a64, ck::a65}};
#pragma unroll 1
    for (int st = 0; st < 6; ++st) {
        double yt[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            double a = 0;
            for (int j = 0; j < st; ++j) a = fma(A[st][j], K[j][i], a);
            yt[i] = fma(hs, a, y[i]);
        }
        double kx[3], k1[3], k2[3];
        rhs_geo<double, S, MODE>(nodes, g, yt, sigma, yt + 3, yt + 6, kx, k1, k2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            K[st][i] = kx[i];
            K[st][3 + i] = k1[i];
            K[st][6 + i] = k2[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        yo[i] = y[i] + hs * (ck::b1 * K[0][i] + ck::b3 * K[2][i] + ck::b4 * K[3][i] + ck::b6 * K[5][i]);
}

// Adaptive Cash-Karp 5(4) stepping of general-geometry half-lines: one lane
// per half-line, items taken one at a time from the work counter; the same
// error norm, controller, limits and statuses as the uniform-grid kernel,
// positions held in FP64, stage arithmetic in T.
template <typename T, typename S, int MODE>
__global__ void __launch_bounds__(256) k_trace_geo(TraceJob job)
{
    const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
    const Geom g = job.g;
    const StepOpts &o = job.o;
    const int64_t total = *job.rec.n_work;
    const int64_t P = 2 * job.rec.cap;
    const T rtol = (T)o.rtol, atol = (T)o.atol;
    unsigned long long c_att = 0, c_ev = 0, c_act = 0, c_land = 0;
    for (;;) {
        const int64_t it = (int64_t)atomicAdd(job.counter, 1ull);
        if (it >= total) break;
        const int64_t rec = job.rec.work[it];
        const T sigma = rec >= job.rec.cap ? (T)-1 : (T)1;
        double X[3];
        T D1[3], D2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            X[k] = job.rec.y[k * P + rec];
            D1[k] = (T)job.rec.y[(3 + k) * P + rec];
            D2[k] = (T)job.rec.y[(6 + k) * P + rec];
        }
        double s = 0.0;
        T h = (T)o.h_init;
        int attempts = 0, stop = -1;
        ++c_act;
        for (;;) {
            if (attempts >= o.max_steps) {
                stop = QSQ_END_MAX_STEPS;
                break;
            }
            T K[6][9];
            // first stage (also the null test at the current point)
            {
                T kx[3], k1[3], k2[3];
                const T un2 = rhs_geo<T, S, MODE>(nodes, g, X, sigma, D1, D2, kx, k1, k2);
                ++c_ev;
                if (un2 < (T)1e-12) {
                    stop = QSQ_END_NULL;
                    break;
                }
                for (int i = 0; i < 3; ++i) {
                    K[0][i] = kx[i];
                    K[0][3 + i] = k1[i];
                    K[0][6 + i] = k2[i];
                }
            }
            T hs = h < (T)o.h_max ? h : (T)o.h_max;
            bool last = false;
            if (o.max_length > 0.0 && (double)hs >= o.max_length - s) {
                hs = (T)(o.max_length - s);
                last = true;
            }
            const double A[6][5] = {{0, 0, 0, 0, 0},
                                    {ck::a21, 0, 0, 0, 0},
                                    {ck::a31, ck::a32, 0, 0, 0},
                                    {ck::a41, ck::a42, ck::a43, 0, 0},
                                    {ck::a51, ck::a52, ck::a53, ck::a54, 0},
                                    {ck::a61, ck::a62, ck::a63, ck::a64, ck::a65}};
#pragma unroll 1
            for (int st = 1; st < 6; ++st) {
                double xs[3];
                T d1[3], d2[3];
                for (int i = 0; i < 3; ++i) {
                    T ax = 0, a1 = 0, a2 = 0;
                    for (int j = 0; j < st; ++j) {
                        ax = fma((T)A[st][j], K[j][i], ax);
                        a1 = fma((T)A[st][j], K[j][3 + i], a1);
                        a2 = fma((T)A[st][j], K[j][6 + i], a2);
                    }
                    xs[i] = X[i] + (double)(hs * ax);
                    d1[i] = fma(hs, a1, D1[i]);
                    d2[i] = fma(hs, a2, D2[i]);
                }
                T kx[3], k1[3], k2[3];
                rhs_geo<T, S, MODE>(nodes, g, xs, sigma, d1, d2, kx, k1, k2);
                ++c_ev;
                for (int i = 0; i < 3; ++i) {
                    K[st][i] = kx[i];
                    K[st][3 + i] = k1[i];
                    K[st][6 + i] = k2[i];
                }
            }
            double Xn[3];
            T D1n[3], D2n[3], err = 0, fsum = 0;
            for (int i = 0; i < 9; ++i) {
                const T b5 = ck_b5(K[0][i], K[2][i], K[3][i], K[5][i]);
                const T e = ck_e(K[0][i], K[2][i], K[3][i], K[4][i], K[5][i]);
                T yo, yn;
                if (i < 3) {
                    Xn[i] = X[i] + (double)(hs * b5);
                    yo = (T)X[i];
                    yn = (T)Xn[i];
                } else if (i < 6) {
                    D1n[i - 3] = fma(hs, b5, D1[i - 3]);
                    yo = D1[i - 3];
                    yn = D1n[i - 3];
                } else {
                    D2n[i - 6] = fma(hs, b5, D2[i - 6]);
                    yo = D2[i - 6];
                    yn = D2n[i - 6];
                }
                err = fmax(err, fabs(hs * e) / err_scale(atol, rtol, yo, yn));
                fsum += yn + e;
            }
            ++attempts;
            ++c_att;
            if (!isfinite(fsum)) {
                stop = QSQ_END_NONFINITE;
                break;
            }
            if (err > (T)1) {
                const T f = (T)0.9 * (T)pow((double)err, -0.25);
                h = hs * (f > (T)0.2 ? f : (T)0.2);
                if ((double)h < o.hmin) {
                    stop = QSQ_END_UNDERFLOW;
                    break;
                }
                continue;
            }
            if (outside_box(g, Xn[0], Xn[1], Xn[2])) {
                const double y[9] = {X[0], X[1], X[2], (double)D1[0], (double)D1[1], (double)D1[2],
                                     (double)D2[0], (double)D2[1], (double)D2[2]};
                put_rec(job.rec, rec, y, s, (double)hs, kPendingLand, attempts);
                ++c_land;
                break;
            }
            for (int i = 0; i < 3; ++i) {
                X[i] = Xn[i];
                D1[i] = D1n[i];
                D2[i] = D2n[i];
            }
            if (last) {
                s = o.max_length;
                stop = QSQ_END_MAX_LENGTH;
                break;
            }
            s += (double)hs;
            const T f = err > (T)0 ? (T)0.9 * (T)pow((double)err, -0.2) : (T)5;
            h = hs * (f < (T)5 ? f : (T)5);
        }
        if (stop >= 0) {
            const double y[9] = {X[0], X[1], X[2], (double)D1[0], (double)D1[1], (double)D1[2],
                                 (double)D2[0], (double)D2[1], (double)D2[2]};
            put_rec(job.rec, rec, y, s, 0.0, stop, attempts);
        }
    }
    if (job.work) {
        atomicAdd(&job.work[0], c_att);
        atomicAdd(&job.work[1], c_ev);
        atomicAdd(&job.work[2], c_act);
        atomicAdd(&job.work[3], c_land);
    }
}

// signed distance past face f of the FP64 step's end from y over length h
template <typename S, int MODE>
__device__ double face_gap_geo(const S *nodes, const Geom &g, double sigma, const double y[9], double h, int f,
                               double yo[9])
{
    if (h > 0.0) {
        ck54_geo<S, MODE>(nodes, g, sigma, y, h, yo);
    } else {
        for (int k = 0; k < 9; ++k) yo[k] = y[k];
    }
    return beyond_face(g, yo, f);
}

// FP64 landing of general-geometry half-lines: for every face the trial step
// crosses, Illinois regula falsi from the secant point on the face gap of the
// FP64 step's end over its length (|gap| <= gtol); the face reached first (the
// shortest length; exact ties keep the lower face) takes the line, the state
// is stepped there and snapped onto the face
template <typename S, int MODE>
__global__ void __launch_bounds__(256) k_land_geo(TraceJob job)
{
    const int64_t total = *job.rec.n_land;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = job.rec.work2[it];
        const S *__restrict__ nodes = static_cast<const S *>(job.nodes);
        const Geom &g = job.g;
        const double gtol = job.o.gtol;
        const double sigma = r >= job.rec.cap ? -1.0 : 1.0;
        double y[9], s, hs, yo[9];
        get_rec(job.rec, r, y, s, hs);
        ck54_geo<S, MODE>(nodes, g, sigma, y, hs, yo);
        double best = INFINITY;
        int face = -1;
        for (int f = 0; f < 6; ++f) {
            if (!(beyond_face(g, yo, f) > 0.0)) continue;
            double a = 0.0, b = hs, ga = face_gap_geo<S, MODE>(nodes, g, sigma, y, a, f, yo), gb, root;
            if (ga >= 0.0) {
                root = 0.0;
            } else {
                gb = face_gap_geo<S, MODE>(nodes, g, sigma, y, b, f, yo);
                int side = 0;
                root = -1.0;
                for (int k = 0; k < 200 && root < 0.0; ++k) {
                    const double c = (a * gb - b * ga) / (gb - ga);
                    const double gc = face_gap_geo<S, MODE>(nodes, g, sigma, y, c, f, yo);
                    if (fabs(gc) <= gtol) {
                        root = c;
                    } else if (gc > 0.0) {
                        b = c;
                        gb = gc;
                        if (side == +1) ga *= 0.5;
                        side = +1;
                    } else {
                        a = c;
                        ga = gc;
                        if (side == -1) gb *= 0.5;
                        side = -1;
                    }
                    if (root < 0.0 && b - a <= 1e-15 * hs) root = ga > -gb ? a : b;
                }
                if (root < 0.0) root = ga > -gb ? a : b;
            }
            if (root < best) {
                best = root;
                face = f;
            }
        }
        if (face < 0) {
            // the trial step left the box in FP32 but the FP64 step does not:
            // end on the face nearest the FP64 end
            best = hs;
            double gmax = -INFINITY;
            for (int f = 0; f < 6; ++f) {
                const double gp = beyond_face(g, yo, f);
                if (gp > gmax) {
                    gmax = gp;
                    face = f;
                }
            }
        }
        double yl[9];
        if (best > 0.0) {
            ck54_geo<S, MODE>(nodes, g, sigma, y, best, yl);
        } else {
            for (int k = 0; k < 9; ++k) yl[k] = y[k];
        }
        const int d = face >> 1;
        const double snap = (face & 1) ? pick3(g.hi, d) : pick3(g.lo, d);
        for (int k = 0; k < 3; ++k)
            if (k == d) yl[k] = snap;
        put_rec(job.rec, r, yl, s + best, 0.0, face, job.rec.attempts[r]);
    }
}

static __global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// counters of the stepping launch's work-list parts: part p starts past the
// first items of its workgroups (blocks b with b mod nparts = p, wg lanes each)
static __global__ void k_part_counters(TraceJob job, int blocks, int wg, int nparts)
{
    const int p = (int)threadIdx.x;
    if (p >= nparts) return;
    const int64_t total = *job.rec.n_work;
    const int64_t nb = p < blocks ? (blocks - p + nparts - 1) / nparts : 0;
    job.counter[kPartCounter + p] = (unsigned long long)(total * p / nparts + nb * wg);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#ifndef QSQ_TRACE_HIGH_TU
int set_bits_for(int nsets)
{
    int b = 0;
    while (b < 16 && ((int64_t)1 << b) < (int64_t)nsets) ++b;
    return b;
}

int spatial_bits_for(int nsets)
{
    const int b = (32 - set_bits_for(nsets)) / 3;
    return b < 8 ? b : 8;
}

uint64_t records_bytes(int64_t cap)
{
    const uint64_t P = 2 * (uint64_t)cap, NC = (uint64_t)sort_count_words((int64_t)P);
    const uint64_t scan_n = P > NC ? P : NC;
    return P * (11 * sizeof(double) + 6 * sizeof(int32_t)) + NC * sizeof(int32_t) + 8 +
           (uint64_t)scan_tmp_words((int64_t)scan_n) * 8;
}

void carve_records(void *scratch, int64_t cap, Records *rec, unsigned long long **counter)
{
    char *p = static_cast<char *>(scratch);
    *counter = reinterpret_cast<unsigned long long *>(p);
    p += 256;
    const uint64_t P = 2 * (uint64_t)cap;
    // the scan's block sums need 8-byte alignment; planes below keep it
    rec->y = reinterpret_cast<double *>(p);
    p += 9 * P * sizeof(double);
    rec->s = reinterpret_cast<double *>(p);
    p += P * sizeof(double);
    rec->h = reinterpret_cast<double *>(p);
    p += P * sizeof(double);
    rec->status = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    rec->attempts = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    rec->flag = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    rec->wpos = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    rec->work = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    rec->work2 = reinterpret_cast<int32_t *>(p);
    p += P * sizeof(int32_t);
    const uint64_t NC = (uint64_t)sort_count_words((int64_t)P);
    rec->scnt = reinterpret_cast<int32_t *>(p);
    p += NC * sizeof(int32_t);
    p += (8 - ((uintptr_t)p & 7)) & 7;
    rec->scan_tmp = reinterpret_cast<int64_t *>(p);
    rec->cap = cap;
    // device scalars share the 256-byte block with the work counter
    rec->n_work = reinterpret_cast<int64_t *>(static_cast<char *>(scratch) + 8);
    rec->n_items = reinterpret_cast<int64_t *>(static_cast<char *>(scratch) + 16);
    rec->n_land = reinterpret_cast<int64_t *>(static_cast<char *>(scratch) + 24);
    rec->n_sort = reinterpret_cast<int64_t *>(static_cast<char *>(scratch) + 32);
}

int device_cu_count()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// Workgroups of `kern` (wg lanes, lds bytes of dynamic LDS) that stay resident
// on one CU together, from the runtime's occupancy calculator (cached).
#endif  // QSQ_TRACE_HIGH_TU

static int resident_blocks(const void *kern, int wg, size_t lds)
{
    struct Entry {
        const void *k;
        int wg;
        size_t lds;
        int n;
    };
    static Entry cache[64];
    static int used = 0;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].k == kern && cache[i].wg == wg && cache[i].lds == lds) return cache[i].n;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, wg, lds) != hipSuccess || n < 1) n = 1;
    if (used < 64) cache[used++] = Entry{kern, wg, lds, n};
    return n;
}

// the stepping kernel of a gather variant for the job's stepper
template <typename T, typename S, int MODE, int GATHER, bool BATCH>
static const void *trace_kernel(bool euler)
{
    return euler ? reinterpret_cast<const void *>(&k_trace<T, S, MODE, GATHER, BATCH, true>)
                 : reinterpret_cast<const void *>(&k_trace<T, S, MODE, GATHER, BATCH, false>);
}

template <typename T, typename S, int MODE, bool BATCH>
static hipError_t launch_typed(const TraceJob &job, hipStream_t st)
{
    const bool euler = job.o.stepper == QSQ_STEPPER_EULER;
    const int cus = device_cu_count();
    const int64_t n_max = job.n_dev ? job.rec.cap : job.n_host;
    if (n_max <= 0) return hipSuccess;
    int64_t sb = (n_max + 255) / 256;
    const int sblocks = (int)(sb < (int64_t)cus * 16 ? sb : (int64_t)cus * 16);
    hipLaunchKernelGGL((k_seed_pass<S, MODE, BATCH>), dim3(sblocks), dim3(256), 0, st, job);
    int64_t cb = (2 * n_max + 255) / 256;
    const int cblocks = (int)(cb < (int64_t)cus * 16 ? cb : (int64_t)cus * 16);
    launch_scan_i32(job.rec.flag, job.rec.n_items, 2 * n_max, job.rec.scan_tmp, job.rec.wpos, job.rec.n_work, st);
    hipLaunchKernelGGL(k_compact, dim3(cblocks), dim3(256), 0, st, job);
    if (job.spatial_bits > 0) {
        // work list in spatial order: keys (in the flag array, free now),
        // then the stable sort with the work list as values
        const int bits = job.spatial_bits;
        hipLaunchKernelGGL((k_sort_keys<BATCH>), dim3(cblocks), dim3(256), 0, st, job, bits);
        const int key_bits = 3 * bits + (BATCH ? set_bits_for(job.nsets) : 0);
        launch_sort_pairs(reinterpret_cast<uint32_t *>(job.rec.flag), job.rec.work,
                          reinterpret_cast<uint32_t *>(job.rec.wpos), job.rec.work2, job.rec.scnt, job.rec.scan_tmp,
                          job.rec.n_sort, job.rec.n_work, 2 * n_max, key_bits, st);
    }
    // launch shape (QSQ_LAUNCH word): workgroup size and a resident-lane
    // target per CU, capped by what the kernel's registers and LDS let stay
    // resident, so that every workgroup of the persistent launch runs from the
    // start (the first item of each lane is its global index)
    const int lanes = (job.o.launch & 15) ? (job.o.launch & 15) : 8;
    const int wg_code = (job.o.launch >> 4) & 3, gather = (job.o.launch >> 6) & 7;
    const int wg = wg_code == 1 ? 64 : wg_code == 2 ? 128 : 256;
    const void *kern;
    size_t lds = 0;
    constexpr bool cacheable = sizeof(T) == 4 && interp_order<MODE>() == 1 &&
                               (std::is_same<S, float>::value || std::is_same<S, Bf16>::value);
    if constexpr (cacheable && !BATCH) {
        // the cell caches address the node records with 32-bit byte offsets
        const uint64_t field_bytes = (uint64_t)node_bytes<S>() * job.g.n[0] * job.g.n[1] * job.g.n[2];
        const uint64_t brick_bytes = (uint64_t)node_bytes<S>() * 8 * ((job.g.n[0] + 1) / 2) *
                                     ((job.g.n[1] + 1) / 2) * ((job.g.n[2] + 1) / 2);
        const uint64_t limit = ((uint64_t)1 << 31) - ((uint64_t)1 << 26);
        const bool fits = field_bytes < limit;
        // the direction records' variant keys cells by a 32-bit cell index
        const uint64_t ncells =
            (uint64_t)(job.g.n[0] - 1) * (uint64_t)(job.g.n[1] - 1) * (uint64_t)(job.g.n[2] - 1);
        const void *dirs_kern = nullptr;
        if constexpr (std::is_same<S, float>::value)
            if (gather == 6 && job.dirs && ncells < ((uint64_t)1 << 31))
                dirs_kern = trace_kernel<T, S, MODE, kGatherDirs, false>(euler);
        if (dirs_kern) {
            kern = dirs_kern;
            lds = QSQ_SECOND_CELL ? kCachePlanes * wg * sizeof(float4) : 0;
        } else if (gather == 5 && job.bricks && brick_bytes < limit) {
            kern = trace_kernel<T, S, MODE, kGatherBricks, false>(euler);
            lds = QSQ_SECOND_CELL ? kCachePlanes * wg * sizeof(float4) : 0;
        } else if (gather == 4 && job.cells) {
            kern = trace_kernel<T, S, MODE, kGatherCells, false>(euler);
        } else if ((gather == 3 || gather == 5 || gather == 6 || gather == 0) && fits) {
            kern = trace_kernel<T, S, MODE, kGatherRegs, false>(euler);
            lds = QSQ_SECOND_CELL ? kCachePlanes * wg * sizeof(float4) : 0;
        } else if (gather == 2 && fits) {
            kern = trace_kernel<T, S, MODE, kGatherLds, false>(euler);
            lds = kCachePlanes * wg * sizeof(float4);
        } else {
            kern = trace_kernel<T, S, MODE, kGatherDirect, false>(euler);
        }
    } else {
        (void)gather;
        kern = trace_kernel<T, S, MODE, kGatherDirect, BATCH>(euler);
    }
    const int64_t resident = (int64_t)cus * resident_blocks(kern, wg, lds);
    int64_t cap_blocks = (int64_t)cus * lanes * (256 / wg);
    if (cap_blocks > resident) cap_blocks = resident;
    const int64_t want = (2 * n_max + wg - 1) / wg;
    const int blocks = (int)(want < cap_blocks ? want : cap_blocks);
    const int nparts = (job.o.launch >> 9) & 1 ? kParts : 1;
    hipLaunchKernelGGL(k_part_counters, dim3(1), dim3(64), 0, st, job, blocks, wg, nparts);
    const bool prof = profiling();
    void *tok = nullptr;
    if (prof) prof_begin(kProfStep, st, &tok);
    void *args[] = {const_cast<TraceJob *>(&job)};
    const hipError_t le = hipLaunchKernel(kern, dim3(blocks), dim3(wg), args, lds, st);
    if (prof) prof_end(tok, st);
    if (le != hipSuccess) return le;
    int64_t lb = (2 * n_max + 255) / 256;
    int lblocks = (int)(lb < (int64_t)cus * 16 ? lb : (int64_t)cus * 16);
    if (prof) prof_begin(kProfLand, st, &tok);
    // list of the half-lines to land, in record order
    hipLaunchKernelGGL(k_land_flags, dim3(cblocks), dim3(256), 0, st, job);
    launch_scan_i32(job.rec.flag, job.rec.n_items, 2 * n_max, job.rec.scan_tmp, job.rec.wpos, job.rec.n_land, st);
    hipLaunchKernelGGL(k_land_compact, dim3(cblocks), dim3(256), 0, st, job);
    if (euler) {
        hipLaunchKernelGGL((k_land_euler<S, MODE, BATCH>), dim3(lblocks), dim3(256), 0, st, job);
    } else {
        hipLaunchKernelGGL((k_land<S, MODE, BATCH>), dim3(lblocks), dim3(256), 0, st, job);
        hipLaunchKernelGGL((k_land_final<S, MODE, BATCH>), dim3(lblocks), dim3(256), 0, st, job);
    }
    if (prof) prof_end(tok, st);
    int64_t ab = (n_max + 255) / 256;
    int ablocks = (int)(ab < (int64_t)cus * 16 ? ab : (int64_t)cus * 16);
    if (prof) prof_begin(kProfAssemble, st, &tok);
    hipLaunchKernelGGL((k_assemble<S, MODE, BATCH>), dim3(ablocks), dim3(256), 0, st, job);
    if (prof) prof_end(tok, st);
    return hipGetLastError();
}

#ifdef QSQ_TRACE_HIGH_TU
// higher interpolation orders: one field per call, FP32 or FP64 node records;
// each (order, mode) pair is instantiated in a translation unit of its own,
// so that the build compiles them side by side
// general geometry: seed pass, stepping in physical coordinates, FP64
// landing, the shared Q assembly
template <typename T, typename S, int MODE>
static hipError_t launch_geo(const TraceJob &job, hipStream_t st)
{
    const int cus = device_cu_count();
    const int64_t n_max = job.n_dev ? job.rec.cap : job.n_host;
    if (n_max <= 0) return hipSuccess;
    auto blocks_of = [&](int64_t items) {
        const int64_t b = (items + 255) / 256;
        return (int)(b < (int64_t)cus * 16 ? b : (int64_t)cus * 16);
    };
    hipLaunchKernelGGL((k_seed_pass<S, MODE, false>), dim3(blocks_of(n_max)), dim3(256), 0, st, job);
    launch_scan_i32(job.rec.flag, job.rec.n_items, 2 * n_max, job.rec.scan_tmp, job.rec.wpos, job.rec.n_work, st);
    hipLaunchKernelGGL(k_compact, dim3(blocks_of(2 * n_max)), dim3(256), 0, st, job);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, job.counter, 0ull);
    const bool prof = profiling();
    void *tok = nullptr;
    if (prof) prof_begin(kProfStep, st, &tok);
    hipLaunchKernelGGL((k_trace_geo<T, S, MODE>), dim3(cus * 8), dim3(256), 0, st, job);
    if (prof) prof_end(tok, st);
    if (prof) prof_begin(kProfLand, st, &tok);
    hipLaunchKernelGGL(k_land_flags, dim3(blocks_of(2 * n_max)), dim3(256), 0, st, job);
    launch_scan_i32(job.rec.flag, job.rec.n_items, 2 * n_max, job.rec.scan_tmp, job.rec.wpos, job.rec.n_land, st);
    hipLaunchKernelGGL(k_land_compact, dim3(blocks_of(2 * n_max)), dim3(256), 0, st, job);
    hipLaunchKernelGGL((k_land_geo<S, MODE>), dim3(blocks_of(2 * n_max)), dim3(256), 0, st, job);
    if (prof) prof_end(tok, st);
    if (prof) prof_begin(kProfAssemble, st, &tok);
    hipLaunchKernelGGL((k_assemble<S, MODE, false>), dim3(blocks_of(n_max)), dim3(256), 0, st, job);
    if (prof) prof_end(tok, st);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_trace_mode(const TraceJob &job, int step_dtype, hipStream_t st)
{
    const bool f32 = step_dtype == QSQ_F32;
    if constexpr (geo_mode<MODE>()) {
        if (job.storage == QSQ_F32)
            return f32 ? launch_geo<float, float, MODE>(job, st) : launch_geo<double, float, MODE>(job, st);
        if (job.storage == QSQ_F64)
            return f32 ? launch_geo<float, double, MODE>(job, st) : launch_geo<double, double, MODE>(job, st);
        return hipErrorNotSupported;
    } else {
        if (job.storage == QSQ_F32)
            return f32 ? launch_typed<float, float, MODE, false>(job, st)
                       : launch_typed<double, float, MODE, false>(job, st);
        if (job.storage == QSQ_F64)
            return f32 ? launch_typed<float, double, MODE, false>(job, st)
                       : launch_typed<double, double, MODE, false>(job, st);
        return hipErrorNotSupported;
    }
}

template hipError_t launch_trace_mode<QSQ_TRACE_HIGH_MODE>(const TraceJob &job, int step_dtype, hipStream_t st);
#else

template <bool BATCH>
static hipError_t dispatch(const TraceJob &job, int step_dtype, hipStream_t st)
{
    const bool f32 = step_dtype == QSQ_F32;
    const bool paper = (job.mode & 1) == QSQ_INTERP_PAPER;
    constexpr int P = QSQ_INTERP_PAPER, N = QSQ_INTERP_NORMALIZE;
    if (job.mode > 1) {
        // higher interpolation orders: one field per call
        if constexpr (BATCH) {
            return hipErrorNotSupported;
        } else {
            // job.mode = interpolation mode | (order - 1) << 1
            switch (job.mode) {
            case 2: return launch_trace_mode<2>(job, step_dtype, st);
            case 3: return launch_trace_mode<3>(job, step_dtype, st);
            case 4: return launch_trace_mode<4>(job, step_dtype, st);
            case 5: return launch_trace_mode<5>(job, step_dtype, st);
            case 8: return launch_trace_mode<8>(job, step_dtype, st);
            case 9: return launch_trace_mode<9>(job, step_dtype, st);
            default: return hipErrorNotSupported;
            }
        }
    }
    if (job.storage == QSQ_BF16) {
        if (f32) return paper ? launch_typed<float, Bf16, P, BATCH>(job, st) : launch_typed<float, Bf16, N, BATCH>(job, st);
        return paper ? launch_typed<double, Bf16, P, BATCH>(job, st) : launch_typed<double, Bf16, N, BATCH>(job, st);
    }
    if (job.storage == QSQ_F32) {
        if (f32) return paper ? launch_typed<float, float, P, BATCH>(job, st) : launch_typed<float, float, N, BATCH>(job, st);
        return paper ? launch_typed<double, float, P, BATCH>(job, st) : launch_typed<double, float, N, BATCH>(job, st);
    }
    if (f32) return paper ? launch_typed<float, double, P, BATCH>(job, st) : launch_typed<float, double, N, BATCH>(job, st);
    return paper ? launch_typed<double, double, P, BATCH>(job, st) : launch_typed<double, double, N, BATCH>(job, st);
}

hipError_t launch_trace(const TraceJob &job, int step_dtype, hipStream_t st)
{
    return dispatch<false>(job, step_dtype, st);
}

// The set table travels in kernel arguments, a few entries per launch, so
// that the whole batched call is plain kernel launches (capturable in a graph,
// no host buffer that must outlive the call).
constexpr int kSetsPerPut = 6;
struct SetChunk {
    SetDesc d[kSetsPerPut];
    int first, count;
};

__global__ void k_put_sets(SetDesc *table, SetChunk c)
{
    const int k = (int)threadIdx.x;
    if (k < c.count) table[c.first + k] = c.d[k];
}

hipError_t launch_trace_batch(const TraceJob &job, const SetDesc *host_sets, int nsets, int step_dtype,
                              hipStream_t st)
{
    SetDesc *table = const_cast<SetDesc *>(job.sets);
    for (int first = 0; first < nsets; first += kSetsPerPut) {
        SetChunk c{};
        c.first = first;
        c.count = nsets - first < kSetsPerPut ? nsets - first : kSetsPerPut;
        for (int k = 0; k < c.count; ++k) c.d[k] = host_sets[first + k];
        hipLaunchKernelGGL(k_put_sets, dim3(1), dim3(64), 0, st, table, c);
    }
    return dispatch<true>(job, step_dtype, st);
}

#endif  // QSQ_TRACE_HIGH_TU

}  // namespace qsq
