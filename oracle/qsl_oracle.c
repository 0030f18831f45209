/*
 * qsl_oracle.c -- plain FP64 CPU oracle of the QSL Squasher field-line /
 * squashing-factor path (Tassev & Savcheva, "QSL Squasher: A Fast
 * Quasi-Separatrix Layer Map Calculator", ApJS 2017, arXiv:1609.00724).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library
 * against the paper.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no source, header, table or helper
 * with the HIP library, and the HIP library never loads it.
 *
 * Everything is computed in double precision, in the order the paper states,
 * with no blocking or fusion:
 *   Sect. 3.1  field-line ODE  d x / d lambda = Bhat(x)                 eq. (1)
 *   Sect. 3.2  trilinear interpolation of the node field                 eq. (3)-(4)
 *              triquadratic (Dodgson 1997) and tricubic (Keys 1981) stencils  eq. (3)
 *   Sect. 3.3  linearised deviation d dx / d lambda = (dx . grad) Bhat   eq. (5)
 *   Sect. 3.4  adaptive Cash-Karp 5(4) Runge-Kutta stepping
 *   Sect. 3.5  orthonormal initial frame eq. (9), end vectors eq. (10),
 *              squashing factor eq. (11); field normalised on the nodes first
 *              and renormalised only when projecting (footnote to Sect. 3.5)
 *   Sect. 3.6  Hilbert-curve ordering of a slice (keys used by refinement)
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - cell lookup c = clamp(floor(s), 0, n-2); the fraction s-c is NOT clamped,
 *     so stage points a little outside the box are linearly extrapolated from
 *     the boundary cell;
 *   - error norm = max over all 9 state components of
 *     |y5 - y4| / (atol + rtol * max(|y|, |y5|)); textbook step controller
 *     (grow by min(5, 0.9 err^-1/5), shrink by max(0.2, 0.9 err^-1/4));
 *   - boundary landing: the step that leaves the closed box is re-solved for
 *     the step length at which its 5th-order solution lies on the first face
 *     crossed (Illinois regula falsi on the signed distance), then snapped;
 *     an Euler step is cut in closed form where it meets that face;
 *   - the explicit Euler scheme (Sect. 3.4) takes fixed steps h_init on the
 *     whole state (x, dx1, dx2), one right-hand side per step;
 *   - the frame (a, b) completing Bhat(x0) is the branchless construction of
 *     Duff et al. 2017 (JCGT 6(1)); Q does not depend on this choice.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_VERSION 1

/* field kinds */
enum { OR_PAPER = 0, OR_INTERP_NORMALIZE = 1, OR_ANALYTIC = 2 };
/* analytic fields */
enum { OR_AN_LINEAR = 0, OR_AN_CHARGES = 1 };

/* per-half-line outcome codes: exit faces first, then the other stops */
enum {
    OR_XLO = 0, OR_XHI = 1, OR_YLO = 2, OR_YHI = 3, OR_ZLO = 4, OR_ZHI = 5,
    OR_MAX_LENGTH = 6, OR_MAX_STEPS = 7, OR_NULL = 8, OR_UNDERFLOW = 9,
    OR_SEED_OUTSIDE = 10, OR_NONFINITE = 11
};
#define OR_OPEN_BIT (1 << 16)

typedef struct {
    int32_t kind;          /* OR_PAPER, OR_INTERP_NORMALIZE or OR_ANALYTIC */
    int32_t analytic;      /* OR_AN_LINEAR or OR_AN_CHARGES (analytic kind) */
    int64_t n[3];          /* nodes per axis (grid kinds) */
    double origin[3];      /* position of node (0,0,0) */
    double spacing[3];     /* node spacing per axis */
    double lo[3], hi[3];   /* closed box; for grids the node hull */
    const double *bx, *by, *bz;   /* node field, x fastest (grid kinds) */
    double lin[12];        /* linear field B = lin[0..2] + M x, M row-major lin[3..11] */
    const double *charges; /* ncharges x (x, y, z, q) */
    int64_t ncharges;
    int32_t quantize;      /* 1: round the prepared node values to FP32, 2: to
                              BF16 (the stored form of an FP32 / BF16 node field) */
    int32_t order;         /* interpolation order (Sect. 3.2): 1 trilinear (also 0),
                              2 triquadratic (Dodgson 1997), 3 tricubic (Keys 1981) */
    int32_t geometry;      /* OR_CARTESIAN, or OR_SPHERICAL (Sect. 3.1): coordinates
                              (phi, theta, r) = (longitude, latitude, radius), field
                              components (B_phi, B_theta, B_r) in the orthonormal basis */
    int32_t pad;
    const double *coord[3]; /* NULL: uniform axis (origin + i spacing); else the n[d]
                              increasing node coordinates of a rectilinear axis (Sect. 3.2:
                              h_c is the span of the point's cell); trilinear only */
} or_field_desc;

enum { OR_CARTESIAN = 0, OR_SPHERICAL = 1 };

typedef struct {
    or_field_desc d;
    double *c[4];          /* prepared node arrays */
} or_field;

typedef struct {
    double rtol, atol;
    double h_init;         /* first trial step (affine units) */
    double h_max;          /* largest step */
    double max_length;     /* <= 0: unlimited */
    int64_t max_steps;     /* accepted + rejected attempts per half-line */
    double frame_angle;    /* rotate (a, b) about Bhat(x0) by this angle */
    int32_t nthreads;      /* <= 0: OpenMP default */
    int32_t stepper;       /* OR_CK54 (adaptive) or OR_EULER (fixed step h_init) */
    int32_t round_f32;     /* sensitivity instrument, 0 = off (plain FP64): 1 rounds
                              every CK54 stage point and every accepted state to
                              FP32, the roundings FP32 stepping cannot avoid */
    int32_t pad;
} or_opts;

/* steppers (Sect. 3.4) */
enum { OR_CK54 = 0, OR_EULER = 1 };

/* BF16 value of x: x rounded to FP32, then to the nearest BF16 (8-bit
 * significand), ties to even; finite inputs only */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* ------------------------------------------------------------------ */
/* field preparation (footnote to Sect. 3.5: normalise the node field  */
/* first, keep |B| for the prefactor of eq. (11))                      */
/* ------------------------------------------------------------------ */

void *or_field_new(const or_field_desc *desc)
{
    or_field *F = (or_field *)calloc(1, sizeof(or_field));
    if (!F) return NULL;
    F->d = *desc;
    if (desc->kind == OR_ANALYTIC) return F;
    int64_t N = desc->n[0] * desc->n[1] * desc->n[2];
    for (int k = 0; k < 4; ++k) {
        F->c[k] = (double *)malloc((size_t)N * sizeof(double));
        if (!F->c[k]) return NULL;
    }
    for (int64_t i = 0; i < N; ++i) {
        double bx = desc->bx[i], by = desc->by[i], bz = desc->bz[i];
        if (desc->kind == OR_PAPER) {
            double b = sqrt(bx * bx + by * by + bz * bz);
            if (b < 1e-30) {
                F->c[0][i] = F->c[1][i] = F->c[2][i] = 0.0;
            } else {
                F->c[0][i] = bx / b;
                F->c[1][i] = by / b;
                F->c[2][i] = bz / b;
            }
            F->c[3][i] = b;
        } else {
            F->c[0][i] = bx;
            F->c[1][i] = by;
            F->c[2][i] = bz;
            F->c[3][i] = 0.0;
        }
        if (desc->quantize == 1)
            for (int k = 0; k < 4; ++k) F->c[k][i] = (double)(float)F->c[k][i];
        if (desc->quantize == 2)
            for (int k = 0; k < 4; ++k) F->c[k][i] = to_bf16(F->c[k][i]);
    }
    return F;
}

void or_field_free(void *h)
{
    or_field *F = (or_field *)h;
    if (!F) return;
    for (int k = 0; k < 4; ++k) free(F->c[k]);
    free(F);
}

/* ------------------------------------------------------------------ */
/* interpolation, eq. (3)-(4), and its analytic gradient (Sect. 3.3)   */
/* ------------------------------------------------------------------ */

/* cell c = vertex of the containing cell closest to the array origin, the
 * point's fraction t of the cell and the cell's span h (uniform axes: the
 * spacing; rectilinear axes: coord[c+1] - coord[c], found by bisection) */
static void locate_h(const or_field *F, const double x[3], int64_t c[3], double t[3], double h[3])
{
    for (int d = 0; d < 3; ++d) {
        const int64_t n = F->d.n[d];
        const double *X = F->d.coord[d];
        if (X) {
            double xv = x[d];
            if (!(xv > -1e300)) xv = -1e300;      /* also catches NaN */
            int64_t lo = 0, hi = n - 2;           /* last cell whose lower node <= x, clamped */
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) / 2;
                if (X[mid] <= xv) lo = mid;
                else hi = mid - 1;
            }
            c[d] = lo;
            h[d] = X[lo + 1] - X[lo];
            t[d] = (x[d] - X[lo]) / h[d];
            continue;
        }
        double s = (x[d] - F->d.origin[d]) / F->d.spacing[d];
        if (!(s > -1e9)) s = -1e9;      /* also catches NaN */
        if (s > 1e9) s = 1e9;
        double fl = floor(s);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(n - 2)) fl = (double)(n - 2);
        c[d] = (int64_t)fl;
        t[d] = s - fl;
        h[d] = F->d.spacing[d];
    }
}

static void locate(const or_field *F, const double x[3], int64_t c[3], double t[3])
{
    double h[3];
    locate_h(F, x, c, t, h);
}

/* sum over the 8 stencil vertices of value * f_v and value * grad f_v */
static void trilinear(const or_field *F, int ncomp, const double x[3],
                      double val[4], double grad[4][3])
{
    int64_t c[3];
    double t[3], h[3];
    locate_h(F, x, c, t, h);
    for (int k = 0; k < ncomp; ++k) {
        val[k] = 0.0;
        grad[k][0] = grad[k][1] = grad[k][2] = 0.0;
    }
    const int64_t nx = F->d.n[0], ny = F->d.n[1];
    for (int v = 0; v < 8; ++v) {
        int vv[3] = { v & 1, (v >> 1) & 1, (v >> 2) & 1 };
        double w[3], dw[3];
        for (int d = 0; d < 3; ++d) {
            w[d] = vv[d] ? t[d] : 1.0 - t[d];
            dw[d] = (vv[d] ? 1.0 : -1.0) / h[d];
        }
        double f = w[0] * w[1] * w[2];
        double df[3] = { dw[0] * w[1] * w[2], w[0] * dw[1] * w[2], w[0] * w[1] * dw[2] };
        int64_t idx = ((c[2] + vv[2]) * ny + (c[1] + vv[1])) * nx + (c[0] + vv[0]);
        for (int k = 0; k < ncomp; ++k) {
            double q = F->c[k][idx];
            val[k] += f * q;
            for (int j = 0; j < 3; ++j) grad[k][j] += df[j] * q;
        }
    }
}

/* Sect. 3.2: the triquadratic and tricubic kernels f_v of eq. (3) are
 * products of one-dimensional kernels of the distance d (in grid spacings)
 * between the point and a stencil node.
 *   Keys (1981) cubic convolution, a = -1/2, nodes c-1 .. c+2 of the cell c:
 *     W(d) = 3/2 d^3 - 5/2 d^2 + 1            (the cell's own nodes, d <= 1)
 *     W(d) = -1/2 d^3 + 5/2 d^2 - 4 d + 2     (the outer nodes, 1 <= d <= 2)
 *   Dodgson (1997) interpolating quadratic, the node m nearest the point and
 *   its two neighbours:
 *     W(d) = 1 - 2 d^2                        (node m, d <= 1/2)
 *     W(d) = d^2 - 5/2 d + 3/2                (the neighbours, 1/2 <= d <= 3/2)
 * Each node's piece is the one its place in the stencil gives; d is measured
 * so that it grows away from the node into the cell, and outside the box the
 * boundary cell's pieces continue as polynomials (as trilinear interpolation
 * continues the boundary cell linearly).  A stencil node beyond the grid
 * takes Keys' boundary value f(-1) = 3 f(0) - 3 f(1) + f(2) (mirrored at the
 * top end), axis by axis.  The gradient is the kernels' analytic derivative. */
static double node_value(const or_field *F, int k, const int64_t idx[3])
{
    for (int d = 0; d < 3; ++d) {
        const int64_t n = F->d.n[d];
        if (idx[d] < 0 || idx[d] > n - 1) {
            int64_t a[3] = { idx[0], idx[1], idx[2] };
            const int low = idx[d] < 0;
            double v = 0.0;
            const double coef[3] = { 3.0, -3.0, 1.0 };
            for (int m = 0; m < 3; ++m) {
                a[d] = low ? m : n - 1 - m;
                v += coef[m] * node_value(F, k, a);
            }
            return v;
        }
    }
    const int64_t nx = F->d.n[0], ny = F->d.n[1];
    return F->c[k][(idx[2] * ny + idx[1]) * nx + idx[0]];
}

/* weight and d(weight)/d(position in grid units) of stencil node j (of K)
 * for the point at fraction t of cell c along one axis; *first = index of
 * node 0 of the stencil */
static void kernel_1d(int order, int64_t c, double t, int j, int64_t *first, double *w, double *dw)
{
    if (order == 3) {
        /* node c - 1 + j at signed offset t - (j - 1) from the point */
        *first = c - 1;
        const int k = j - 1;
        const double d = k <= 0 ? t - k : k - t;     /* grows away from the node into the cell */
        const double sgn = k <= 0 ? 1.0 : -1.0;       /* d d / d t */
        if (k == 0 || k == 1) {
            *w = 1.5 * d * d * d - 2.5 * d * d + 1.0;
            *dw = sgn * (4.5 * d * d - 5.0 * d);
        } else {
            *w = -0.5 * d * d * d + 2.5 * d * d - 4.0 * d + 2.0;
            *dw = sgn * (-1.5 * d * d + 5.0 * d - 4.0);
        }
        return;
    }
    /* quadratic: centre m = c (t < 1/2) or c + 1, offset u = t - (m - c) */
    const int up = !(t < 0.5);
    const double u = up ? t - 1.0 : t;
    *first = c + up - 1;
    if (j == 1) {
        *w = 1.0 - 2.0 * u * u;
        *dw = -4.0 * u;
    } else {
        const double d = j == 0 ? 1.0 + u : 1.0 - u;
        const double sgn = j == 0 ? 1.0 : -1.0;
        *w = d * d - 2.5 * d + 1.5;
        *dw = sgn * (2.0 * d - 2.5);
    }
}

/* sum over the 27 or 64 stencil vertices of value * f_v and value * grad f_v */
static void stencil_interp(const or_field *F, int ncomp, const double x[3], double val[4], double grad[4][3])
{
    const int order = F->d.order, K = order + 1;
    int64_t c[3];
    double t[3];
    locate(F, x, c, t);
    for (int k = 0; k < ncomp; ++k) {
        val[k] = 0.0;
        grad[k][0] = grad[k][1] = grad[k][2] = 0.0;
    }
    double w[3][4], dw[3][4];
    int64_t first[3];
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < K; ++j) {
            kernel_1d(order, c[d], t[d], j, &first[d], &w[d][j], &dw[d][j]);
            dw[d][j] /= F->d.spacing[d];
        }
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b)
            for (int e = 0; e < K; ++e) {
                const int64_t idx[3] = { first[0] + a, first[1] + b, first[2] + e };
                const double f = w[0][a] * w[1][b] * w[2][e];
                const double df[3] = { dw[0][a] * w[1][b] * w[2][e], w[0][a] * dw[1][b] * w[2][e],
                                       w[0][a] * w[1][b] * dw[2][e] };
                for (int k = 0; k < ncomp; ++k) {
                    const double q = node_value(F, k, idx);
                    val[k] += f * q;
                    for (int j = 0; j < 3; ++j) grad[k][j] += df[j] * q;
                }
            }
}

/* the node interpolant of the field's order */
static void interp(const or_field *F, int ncomp, const double x[3], double val[4], double grad[4][3])
{
    if (F->d.order >= 2)
        stencil_interp(F, ncomp, x, val, grad);
    else
        trilinear(F, ncomp, x, val, grad);
}

/* u = B/|B| and grad u = (I - u u^T) grad B / |B| */
static void normalise(const double B[3], double G[3][3], double u[3], double J[3][3], double *bmag)
{
    double b = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    *bmag = b;
    if (b < 1e-300) {
        for (int i = 0; i < 3; ++i) {
            u[i] = 0.0;
            J[i][0] = J[i][1] = J[i][2] = 0.0;
        }
        return;
    }
    for (int i = 0; i < 3; ++i) u[i] = B[i] / b;
    for (int j = 0; j < 3; ++j) {
        double ug = u[0] * G[0][j] + u[1] * G[1][j] + u[2] * G[2][j];
        for (int i = 0; i < 3; ++i) J[i][j] = (G[i][j] - u[i] * ug) / b;
    }
}

static void analytic_B(const or_field *F, const double x[3], double B[3], double G[3][3])
{
    if (F->d.analytic == OR_AN_LINEAR) {
        const double *L = F->d.lin;
        for (int i = 0; i < 3; ++i) {
            B[i] = L[i];
            for (int j = 0; j < 3; ++j) {
                B[i] += L[3 + 3 * i + j] * x[j];
                G[i][j] = L[3 + 3 * i + j];
            }
        }
        return;
    }
    /* point charges: B = sum q (r - r_i) / |r - r_i|^3 */
    for (int i = 0; i < 3; ++i) {
        B[i] = 0.0;
        G[i][0] = G[i][1] = G[i][2] = 0.0;
    }
    for (int64_t m = 0; m < F->d.ncharges; ++m) {
        const double *ch = F->d.charges + 4 * m;
        double r[3] = { x[0] - ch[0], x[1] - ch[1], x[2] - ch[2] };
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double rn = sqrt(r2);
        double r3 = r2 * rn, r5 = r3 * r2;
        for (int i = 0; i < 3; ++i) {
            B[i] += ch[3] * r[i] / r3;
            for (int j = 0; j < 3; ++j)
                G[i][j] += ch[3] * ((i == j ? 1.0 : 0.0) / r3 - 3.0 * r[i] * r[j] / r5);
        }
    }
}

static double dot3(const double *a, const double *b);

/* Spherical geometry (Sect. 3.1): longitude phi, latitude theta, radius r;
 * the orthonormal basis (phi_hat, theta_hat, r_hat) at (phi, theta) */
static void sph_basis(double ph, double th, double e[3][3])
{
    const double cp = cos(ph), sp = sin(ph), ct = cos(th), st = sin(th);
    e[0][0] = -sp, e[0][1] = cp, e[0][2] = 0.0;                 /* phi_hat */
    e[1][0] = -st * cp, e[1][1] = -st * sp, e[1][2] = ct;       /* theta_hat */
    e[2][0] = ct * cp, e[2][1] = ct * sp, e[2][2] = st;         /* r_hat */
}

/* Cartesian position of the spherical point q = (phi, theta, r) */
static void sph_to_cart(const double q[3], double x[3])
{
    x[0] = q[2] * cos(q[1]) * cos(q[0]);
    x[1] = q[2] * cos(q[1]) * sin(q[0]);
    x[2] = q[2] * sin(q[1]);
}

/* An analytic Cartesian field seen in spherical coordinates: the components
 * B_i(q) = e_i(q) . B(x(q)) and their coordinate derivatives
 * d_j B_i = e_i . (grad B  d_j x) + (d_j e_i) . B, with d_phi x = r cos(theta)
 * phi_hat, d_theta x = r theta_hat, d_r x = r_hat and the basis derivatives
 * written out from the basis vectors' components. */
static void analytic_B(const or_field *F, const double x[3], double B[3], double G[3][3]);

static void analytic_sph(const or_field *F, const double q[3], double Bs[3], double Gs[3][3])
{
    const double ph = q[0], th = q[1], r = q[2];
    double x[3], Bc[3], Gc[3][3], e[3][3];
    sph_to_cart(q, x);
    analytic_B(F, x, Bc, Gc);
    sph_basis(ph, th, e);
    const double cp = cos(ph), sp = sin(ph), ct = cos(th), st = sin(th);
    /* d e_i / d phi and d e_i / d theta (d / d r of the basis is zero) */
    double dphi[3][3] = { { -cp, -sp, 0.0 }, { st * sp, -st * cp, 0.0 }, { -ct * sp, ct * cp, 0.0 } };
    double dth[3][3] = { { 0.0, 0.0, 0.0 }, { -ct * cp, -ct * sp, -st }, { -st * cp, -st * sp, ct } };
    double dx[3][3];   /* d x / d q_j, one vector per j */
    for (int k = 0; k < 3; ++k) {
        dx[0][k] = r * ct * e[0][k];
        dx[1][k] = r * e[1][k];
        dx[2][k] = e[2][k];
    }
    for (int i = 0; i < 3; ++i) {
        Bs[i] = dot3(e[i], Bc);
        for (int j = 0; j < 3; ++j) {
            double gdx[3];
            for (int k = 0; k < 3; ++k) gdx[k] = Gc[k][0] * dx[j][0] + Gc[k][1] * dx[j][1] + Gc[k][2] * dx[j][2];
            double de = 0.0;
            if (j == 0) de = dot3(dphi[i], Bc);
            if (j == 1) de = dot3(dth[i], Bc);
            Gs[i][j] = dot3(e[i], gdx) + de;
        }
    }
}

/* metric factors of the field-line equation in spherical geometry, eq. (2):
 * d phi / d lambda = Bhat_phi / (r cos theta), d theta / d lambda = Bhat_theta
 * / r, d r / d lambda = Bhat_r; the deviations of eq. (6) carry the same
 * factors, and eq. (8) turns them back into lengths.  Cartesian: all 1. */
static void metric(const or_field *F, const double q[3], double scale[3])
{
    if (F->d.geometry == OR_SPHERICAL) {
        scale[0] = q[2] * cos(q[1]);
        scale[1] = q[2];
        scale[2] = 1.0;
    } else {
        scale[0] = scale[1] = scale[2] = 1.0;
    }
}

/* Bhat(x), its gradient J[i][j] = d Bhat_i / d x_j, and |B|(x).
 * PAPER mode: Bhat is the interpolant of the normalised node field (not a
 * unit vector in general); |B| is the interpolant of the node magnitudes. */
static void field_eval(const or_field *F, const double x[3], double u[3], double J[3][3], double *bmag)
{
    if (F->d.kind == OR_PAPER) {
        double val[4], grad[4][3];
        interp(F, 4, x, val, grad);
        for (int i = 0; i < 3; ++i) {
            u[i] = val[i];
            for (int j = 0; j < 3; ++j) J[i][j] = grad[i][j];
        }
        *bmag = val[3];
        return;
    }
    double B[3], G[3][3];
    if (F->d.kind == OR_INTERP_NORMALIZE) {
        double val[4], grad[4][3];
        interp(F, 3, x, val, grad);
        for (int i = 0; i < 3; ++i) {
            B[i] = val[i];
            for (int j = 0; j < 3; ++j) G[i][j] = grad[i][j];
        }
    } else if (F->d.geometry == OR_SPHERICAL) {
        analytic_sph(F, x, B, G);
    } else {
        analytic_B(F, x, B, G);
    }
    normalise(B, G, u, J, bmag);
}

void or_field_eval(const void *h, int64_t n, const double *x, double *u, double *J, double *bmag)
{
    const or_field *F = (const or_field *)h;
    for (int64_t i = 0; i < n; ++i) {
        double JJ[3][3];
        field_eval(F, x + 3 * i, u + 3 * i, JJ, bmag + i);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) J[9 * i + 3 * a + b] = JJ[a][b];
    }
}

/* ------------------------------------------------------------------ */
/* right-hand side: y = (x, dx1, dx2); eq. (1) and eq. (5)             */
/* ------------------------------------------------------------------ */

static void rhs(const or_field *F, double sigma, const double y[9], double dy[9])
{
    double u[3], J[3][3], bm, sc[3];
    field_eval(F, y, u, J, &bm);
    metric(F, y, sc);
    /* Cartesian: eq. (1) and (5); spherical: eq. (2) and (6), the deviations
     * held as coordinate differences (d phi, d theta, d r), J the coordinate
     * derivatives of the interpolated components */
    for (int i = 0; i < 3; ++i) {
        dy[i] = sigma * u[i] / sc[i];
        dy[3 + i] = sigma * (J[i][0] * y[3] + J[i][1] * y[4] + J[i][2] * y[5]) / sc[i];
        dy[6 + i] = sigma * (J[i][0] * y[6] + J[i][1] * y[7] + J[i][2] * y[8]) / sc[i];
    }
}

/* ------------------------------------------------------------------ */
/* Cash-Karp 5(4) (Cash & Karp 1990, cited in Sect. 3.4)               */
/* ------------------------------------------------------------------ */

static const double CK_C[6] = { 0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0 };
static const double CK_A[6][5] = {
    { 0.0, 0.0, 0.0, 0.0, 0.0 },
    { 1.0 / 5.0, 0.0, 0.0, 0.0, 0.0 },
    { 3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0 },
    { 3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0 },
    { -11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0 },
    { 1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0 },
};
static const double CK_B5[6] = { 37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0 };
static const double CK_B4[6] = { 2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                 277.0 / 14336.0, 1.0 / 4.0 };

void or_ck54_tableau(double *c, double *a, double *b5, double *b4)
{
    for (int i = 0; i < 6; ++i) {
        c[i] = CK_C[i];
        b5[i] = CK_B5[i];
        b4[i] = CK_B4[i];
        for (int j = 0; j < 5; ++j) a[5 * i + j] = CK_A[i][j];
    }
}

/* one trial step: 5th-order solution (propagated) and embedded 4th order */
static void ck54_step(const or_field *F, double sigma, const double y[9], double h,
                      double y5[9], double y4[9], int round_f32)
{
    double k[6][9], yt[9];
    for (int s = 0; s < 6; ++s) {
        for (int i = 0; i < 9; ++i) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += CK_A[s][j] * k[j][i];
            yt[i] = y[i] + h * acc;
            if (round_f32) yt[i] = (double)(float)yt[i];
        }
        rhs(F, sigma, yt, k[s]);
        if (round_f32)
            for (int i = 0; i < 9; ++i) k[s][i] = (double)(float)k[s][i];
    }
    for (int i = 0; i < 9; ++i) {
        double a5 = 0.0, a4 = 0.0;
        for (int s = 0; s < 6; ++s) {
            a5 += CK_B5[s] * k[s][i];
            a4 += CK_B4[s] * k[s][i];
        }
        y5[i] = y[i] + h * a5;
        y4[i] = y[i] + h * a4;
    }
}

/* ------------------------------------------------------------------ */
/* one half-line: integrate to the boundary (Sect. 3.5)                */
/* ------------------------------------------------------------------ */

typedef struct {
    double y[9];           /* end state: x, dx1, dx2 */
    double s;              /* path parameter |lambda| at the end */
    int32_t status;
    int64_t accepted, rejected, land_iters;
} or_half;

/* a point that is not in the closed box; a non-finite coordinate is outside */
static int outside(const or_field *F, const double x[3])
{
    for (int d = 0; d < 3; ++d)
        if (!(x[d] >= F->d.lo[d] && x[d] <= F->d.hi[d])) return 1;
    return 0;
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* signed distance of the end of a trial step of length h beyond face f */
static double face_gap(const or_field *F, double sigma, const double y[9], double h, int f, double yo[9])
{
    double y4[9];
    if (h == 0.0)
        memcpy(yo, y, sizeof(double) * 9);
    else
        ck54_step(F, sigma, y, h, yo, y4, 0);
    int d = f / 2;
    return (f & 1) ? yo[d] - F->d.hi[d] : F->d.lo[d] - yo[d];
}

/* Illinois regula falsi for the step length that ends on face f */
static double land_on_face(const or_field *F, double sigma, const double y[9], double hstep, int f,
                           double gtol, int64_t *iters)
{
    double yo[9];
    double a = 0.0, b = hstep;
    double ga = face_gap(F, sigma, y, a, f, yo);
    if (ga >= 0.0) return 0.0;
    double gb = face_gap(F, sigma, y, b, f, yo);
    int side = 0;   /* which end was replaced last: +1 outside end, -1 inside end */
    for (int it = 0; it < 200; ++it) {
        double c = (a * gb - b * ga) / (gb - ga);
        double gc = face_gap(F, sigma, y, c, f, yo);
        ++*iters;
        if (fabs(gc) <= gtol) return c;
        if (gc > 0.0) {
            b = c;
            gb = gc;
            if (side == +1) ga *= 0.5;   /* Illinois: same end replaced twice */
            side = +1;
        } else {
            a = c;
            ga = gc;
            if (side == -1) gb *= 0.5;
            side = -1;
        }
        if (b - a <= 1e-15 * hstep) break;
    }
    return ga > -gb ? a : b;  /* smaller |g| of the bracket ends */
}

/* Explicit Euler with a fixed step h_init (Sect. 3.4): y <- y + h f(y) on the
 * whole state (x, dx1, dx2).  There is no error control.  The step whose end
 * leaves the box is cut where it meets the first face it crosses: the end of
 * an Euler step moves linearly with the step length, so that length is the
 * distance to the face divided by the step's rate towards it; the state is
 * taken there and the position snapped to the face. */
static void trace_half_euler(const or_field *F, const or_opts *O, double sigma, const double y0[9],
                             or_half *out)
{
    double y[9], dy[9], y1[9];
    memcpy(y, y0, sizeof y);
    double s = 0.0;
    const double h = O->h_init;
    out->accepted = out->rejected = out->land_iters = 0;
    out->status = -1;
    for (;;) {
        if (out->accepted >= O->max_steps) {
            out->status = OR_MAX_STEPS;
            break;
        }
        {   /* null: the interpolated unit field has (nearly) vanished here */
            double u[3], J[3][3], bm;
            field_eval(F, y, u, J, &bm);
            if (sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) < 1e-6) {
                out->status = OR_NULL;
                break;
            }
        }
        double hs = h;
        int last = 0;
        if (O->max_length > 0.0 && hs >= O->max_length - s) {
            hs = O->max_length - s;
            last = 1;
        }
        rhs(F, sigma, y, dy);
        for (int i = 0; i < 9; ++i) y1[i] = y[i] + hs * dy[i];
        if (!all_finite(y1, 9)) {
            out->status = OR_NONFINITE;
            break;
        }
        ++out->accepted;
        if (outside(F, y1)) {
            double best = INFINITY;
            int face = -1;
            for (int f = 0; f < 6; ++f) {
                int d = f / 2;
                double wall = (f & 1) ? F->d.hi[d] : F->d.lo[d];
                double g = (f & 1) ? y1[d] - wall : wall - y1[d];
                if (!(g > 0.0)) continue;
                double hf = (wall - y[d]) / dy[d];
                hf = hf < 0.0 ? 0.0 : (hf > hs ? hs : hf);
                if (hf < best) {
                    best = hf;
                    face = f;
                }
            }
            for (int i = 0; i < 9; ++i) y[i] = y[i] + best * dy[i];
            int d = face / 2;
            y[d] = (face & 1) ? F->d.hi[d] : F->d.lo[d];
            s += best;
            out->status = face;
            break;
        }
        memcpy(y, y1, sizeof y);
        if (last) {
            s = O->max_length;
            out->status = OR_MAX_LENGTH;
            break;
        }
        s += hs;
    }
    memcpy(out->y, y, sizeof y);
    out->s = s;
}

static void trace_half(const or_field *F, const or_opts *O, double sigma, const double y0[9], or_half *out)
{
    if (O->stepper == OR_EULER) {
        trace_half_euler(F, O, sigma, y0, out);
        return;
    }
    double y[9], y5[9], y4[9];
    memcpy(y, y0, sizeof y);
    double s = 0.0, h = O->h_init;
    double extent = 0.0;
    for (int d = 0; d < 3; ++d) extent = fmax(extent, F->d.hi[d] - F->d.lo[d]);
    const double hmin = 1e-12 * extent, gtol = 1e-12 * extent;
    out->accepted = out->rejected = out->land_iters = 0;
    out->status = -1;

    for (;;) {
        if (out->accepted + out->rejected >= O->max_steps) {
            out->status = OR_MAX_STEPS;
            break;
        }
        {   /* null: the interpolated unit field has (nearly) vanished here */
            double u[3], J[3][3], bm;
            field_eval(F, y, u, J, &bm);
            if (sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) < 1e-6) {
                out->status = OR_NULL;
                break;
            }
        }
        double hs = h < O->h_max ? h : O->h_max;
        int last = 0;
        if (O->max_length > 0.0 && hs >= O->max_length - s) {
            hs = O->max_length - s;
            last = 1;
        }
        ck54_step(F, sigma, y, hs, y5, y4, O->round_f32);
        if (!all_finite(y5, 9) || !all_finite(y4, 9)) {
            out->status = OR_NONFINITE;
            break;
        }
        double err = 0.0;
        for (int i = 0; i < 9; ++i) {
            double sc = O->atol + O->rtol * fmax(fabs(y[i]), fabs(y5[i]));
            err = fmax(err, fabs(y5[i] - y4[i]) / sc);
        }
        if (err > 1.0) {
            ++out->rejected;
            h = hs * fmax(0.2, 0.9 * pow(err, -0.25));
            if (h < hmin) {
                out->status = OR_UNDERFLOW;
                break;
            }
            continue;
        }
        ++out->accepted;
        if (outside(F, y5)) {
            /* land on the first face crossed; exact ties keep the lower face */
            double best = INFINITY;
            int face = -1;
            for (int f = 0; f < 6; ++f) {
                int d = f / 2;
                double g = (f & 1) ? y5[d] - F->d.hi[d] : F->d.lo[d] - y5[d];
                if (!(g > 0.0)) continue;
                double hf = land_on_face(F, sigma, y, hs, f, gtol, &out->land_iters);
                if (hf < best) {
                    best = hf;
                    face = f;
                }
            }
            double yl[9];
            if (best > 0.0)
                ck54_step(F, sigma, y, best, yl, y4, 0);
            else
                memcpy(yl, y, sizeof yl);
            int d = face / 2;
            yl[d] = (face & 1) ? F->d.hi[d] : F->d.lo[d];
            memcpy(y, yl, sizeof y);
            s += best;
            out->status = face;
            break;
        }
        memcpy(y, y5, sizeof y);
        if (O->round_f32)
            for (int i = 0; i < 9; ++i) y[i] = (double)(float)y[i];
        if (last) {
            s = O->max_length;
            out->status = OR_MAX_LENGTH;
            break;
        }
        s += hs;
        h = hs * (err > 0.0 ? fmin(5.0, 0.9 * pow(err, -0.2)) : 5.0);
    }
    memcpy(out->y, y, sizeof y);
    out->s = s;
}

/* ------------------------------------------------------------------ */
/* frame (eq. 9) and squashing factor (eq. 10-11)                      */
/* ------------------------------------------------------------------ */

/* orthonormal (a, b) completing the unit vector n (Duff et al. 2017) */
static void onb(const double n[3], double a[3], double b[3])
{
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double p = -1.0 / (sg + n[2]);
    double q = n[0] * n[1] * p;
    a[0] = 1.0 + sg * n[0] * n[0] * p;
    a[1] = sg * q;
    a[2] = -sg * n[0];
    b[0] = q;
    b[1] = sg + n[1] * n[1] * p;
    b[2] = -n[1];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double cross_norm(const double *a, const double *b)
{
    double c0 = a[1] * b[2] - a[2] * b[1];
    double c1 = a[2] * b[0] - a[0] * b[2];
    double c2 = a[0] * b[1] - a[1] * b[0];
    return sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

/* [aF^2 bB^2 + aB^2 bF^2 - 2 (aB.bB)(aF.bF)]: bracket of eq. (11) */
static double bracket(const double *aF, const double *bF, const double *aB, const double *bB)
{
    return dot3(aF, aF) * dot3(bB, bB) + dot3(aB, aB) * dot3(bF, bF) - 2.0 * dot3(aB, bB) * dot3(aF, bF);
}

/* remove the component along the renormalised field (Sect. 3.5) */
static void perp(const double *dx, const double *u, double *out)
{
    double p = dot3(u, dx);
    for (int i = 0; i < 3; ++i) out[i] = dx[i] - u[i] * p;
}

/* project along the field line onto the plane of exit face f */
static void along_to_face(const double *dx, const double *v, int f, double *out)
{
    int d = f / 2;
    double r = dx[d] / v[d];
    for (int i = 0; i < 3; ++i) out[i] = dx[i] - v[i] * r;
}

static int is_face(int st) { return st >= OR_XLO && st <= OR_ZHI; }
static int q_defined(int st) { return st >= OR_XLO && st <= OR_MAX_STEPS; }

/*
 * Trace n seeds (AoS, 3 per seed) forward and backward and assemble
 * per seed: footpoints, lengths, Q (eq. 11), Q from the determinant form,
 * Q in the exit-face planes, status; per half-line: step counters and the
 * end state.  Any output pointer except status may be NULL.
 */
void or_trace(const void *hf, const or_opts *O, int64_t n, const double *seeds,
              double *fp_fwd, double *fp_bwd, double *fll, double *q_perp, double *q_det,
              double *q_fp, double *lam_fwd, double *lam_bwd, int32_t *status,
              int64_t *counts, double *ends)
{
    const or_field *F = (const or_field *)hf;
#ifdef _OPENMP
    int nt = O->nthreads > 0 ? O->nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const double *x0 = seeds + 3 * i;
        or_half H[2];
        const double qnan = NAN;
        int stF, stB;
        double u0[3], J0[3][3], B0 = 0.0;
        memset(H, 0, sizeof H);

        if (outside(F, x0)) {
            stF = stB = OR_SEED_OUTSIDE;
            for (int k = 0; k < 2; ++k) {
                memcpy(H[k].y, x0, 3 * sizeof(double));
                H[k].status = OR_SEED_OUTSIDE;
            }
        } else {
            field_eval(F, x0, u0, J0, &B0);
            double un = sqrt(dot3(u0, u0));
            if (un < 1e-6) {
                stF = stB = OR_NULL;
                for (int k = 0; k < 2; ++k) {
                    memcpy(H[k].y, x0, 3 * sizeof(double));
                    H[k].status = OR_NULL;
                }
            } else {
                double nrm[3] = { u0[0] / un, u0[1] / un, u0[2] / un };
                double a[3], b[3], y0[9];
                onb(nrm, a, b);
                double ca = cos(O->frame_angle), sa = sin(O->frame_angle);
                double sc0[3];
                metric(F, x0, sc0);
                for (int j = 0; j < 3; ++j) {
                    y0[j] = x0[j];
                    y0[3 + j] = (ca * a[j] + sa * b[j]) / sc0[j];      /* eq. (9): dx1(0) = a */
                    y0[6 + j] = (-sa * a[j] + ca * b[j]) / sc0[j];     /* eq. (9): dx2(0) = b */
                }
                trace_half(F, O, +1.0, y0, &H[0]);
                trace_half(F, O, -1.0, y0, &H[1]);
                stF = H[0].status;
                stB = H[1].status;
            }
        }

        double lf = H[0].s, lb = -H[1].s;
        if (lam_fwd) lam_fwd[i] = lf;
        if (lam_bwd) lam_bwd[i] = lb;
        if (fll) fll[i] = lf - lb;
        for (int j = 0; j < 3; ++j) {
            if (fp_fwd) fp_fwd[3 * i + j] = H[0].y[j];
            if (fp_bwd) fp_bwd[3 * i + j] = H[1].y[j];
        }
        int open = !(stF == OR_ZLO && stB == OR_ZLO);
        status[i] = (stF & 0xff) | ((stB & 0xff) << 8) | (open ? OR_OPEN_BIT : 0);
        if (counts) {
            for (int k = 0; k < 2; ++k) {
                counts[6 * i + 3 * k + 0] = H[k].accepted;
                counts[6 * i + 3 * k + 1] = H[k].rejected;
                counts[6 * i + 3 * k + 2] = H[k].land_iters;
            }
        }
        if (ends) {
            for (int k = 0; k < 2; ++k) {
                for (int j = 0; j < 9; ++j) ends[20 * i + 10 * k + j] = H[k].y[j];
                ends[20 * i + 10 * k + 9] = k == 0 ? lf : lb;
            }
        }

        double qp = qnan, qd = qnan, qf = qnan;
        if (q_defined(stF) && q_defined(stB)) {
            double uF[3], uB[3], JF[3][3], JB[3][3], BF, BB;
            field_eval(F, H[0].y, uF, JF, &BF);
            field_eval(F, H[1].y, uB, JB, &BB);
            double vF[3] = { uF[0], uF[1], uF[2] }, vB[3] = { uB[0], uB[1], uB[2] };
            double nF = sqrt(dot3(uF, uF)), nB = sqrt(dot3(uB, uB));
            for (int j = 0; j < 3; ++j) {
                uF[j] /= nF;
                uB[j] /= nB;
            }
            /* the deviations as lengths at each end, eq. (8) (Cartesian: as held) */
            double scF[3], scB[3], dF1[3], dF2[3], dB1[3], dB2[3];
            metric(F, H[0].y, scF);
            metric(F, H[1].y, scB);
            for (int j = 0; j < 3; ++j) {
                dF1[j] = scF[j] * H[0].y[3 + j];
                dF2[j] = scF[j] * H[0].y[6 + j];
                dB1[j] = scB[j] * H[1].y[3 + j];
                dB2[j] = scB[j] * H[1].y[6 + j];
            }
            double aF[3], bF[3], aB[3], bB[3];
            perp(dF1, uF, aF);
            perp(dF2, uF, bF);
            perp(dB1, uB, aB);
            perp(dB2, uB, bB);
            double br = bracket(aF, bF, aB, bB);
            qp = BF * BB / (B0 * B0) * br;                               /* eq. (11) */
            qd = br / (cross_norm(aF, bF) * cross_norm(aB, bB));
            if (is_face(stF) && is_face(stB)) {
                double pF1[3], pF2[3], pB1[3], pB2[3];
                along_to_face(dF1, vF, stF, pF1);
                along_to_face(dF2, vF, stF, pF2);
                along_to_face(dB1, vB, stB, pB1);
                along_to_face(dB2, vB, stB, pB2);
                qf = bracket(pF1, pF2, pB1, pB2) / (cross_norm(pF1, pF2) * cross_norm(pB1, pB2));
            }
        }
        if (q_perp) q_perp[i] = qp;
        if (q_det) q_det[i] = qd;
        if (q_fp) q_fp[i] = qf;
    }
}

/* ------------------------------------------------------------------ */
/* Hilbert curve on a 2^L x 2^L slice (Sect. 3.6), from its recursive  */
/* definition: the curve of order L starts at (0,0) and ends at        */
/* (2^L-1, 0); it visits the lower-left, upper-left, upper-right and   */
/* lower-right quadrants in that order; the first quadrant holds the   */
/* order L-1 curve reflected in the diagonal, the middle two hold it   */
/* translated, the last holds it reflected in the anti-diagonal.       */
/* ------------------------------------------------------------------ */

static uint64_t h2_xy2d(int L, uint64_t x, uint64_t y)
{
    if (L == 0) return 0;
    uint64_t s = (uint64_t)1 << (L - 1);
    int rx = x >= s, ry = y >= s;
    uint64_t lx = x - (rx ? s : 0), ly = y - (ry ? s : 0);
    uint64_t q, cx, cy;
    if (!rx && !ry) { q = 0; cx = ly; cy = lx; }
    else if (!rx && ry) { q = 1; cx = lx; cy = ly; }
    else if (rx && ry) { q = 2; cx = lx; cy = ly; }
    else { q = 3; cx = s - 1 - ly; cy = s - 1 - lx; }
    return q * s * s + h2_xy2d(L - 1, cx, cy);
}

static void h2_d2xy(int L, uint64_t d, uint64_t *x, uint64_t *y)
{
    if (L == 0) { *x = *y = 0; return; }
    uint64_t s = (uint64_t)1 << (L - 1);
    uint64_t q = d / (s * s), cx, cy;
    h2_d2xy(L - 1, d % (s * s), &cx, &cy);
    switch (q) {
    case 0: *x = cy; *y = cx; break;
    case 1: *x = cx; *y = cy + s; break;
    case 2: *x = cx + s; *y = cy + s; break;
    default: *x = s + (s - 1 - cy); *y = s - 1 - cx; break;
    }
}

void or_hilbert2_xy2d(int L, int64_t n, const int64_t *x, const int64_t *y, int64_t *d)
{
    for (int64_t i = 0; i < n; ++i) d[i] = (int64_t)h2_xy2d(L, (uint64_t)x[i], (uint64_t)y[i]);
}

void or_hilbert2_d2xy(int L, int64_t n, const int64_t *d, int64_t *x, int64_t *y)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t xx, yy;
        h2_d2xy(L, (uint64_t)d[i], &xx, &yy);
        x[i] = (int64_t)xx;
        y[i] = (int64_t)yy;
    }
}

/* ------------------------------------------------------------------ */
/* Hilbert curve in 3D (Sect. 3.6, volumes): the transpose algorithm of */
/* Skilling 2004 ("Programming the Hilbert curve", AIP Conf. Proc. 707) */
/* for n = 3 axes of b bits.  The index H has 3b bits; its bits, most   */
/* significant first, are bit b-1 of X[0], X[1], X[2], then bit b-2 of  */
/* X[0], X[1], X[2], and so on (the "transpose" of H).                  */
/* ------------------------------------------------------------------ */

static void sk_transpose_to_axes(uint32_t X[3], int b)
{
    const int n = 3;
    uint32_t N = 2u << (b - 1), P, Q, t;
    /* Gray decode by H ^ (H / 2) */
    t = X[n - 1] >> 1;
    for (int i = n - 1; i > 0; --i) X[i] ^= X[i - 1];
    X[0] ^= t;
    /* undo excess work */
    for (Q = 2; Q != N; Q <<= 1) {
        P = Q - 1;
        for (int i = n - 1; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;                 /* invert */
            } else {
                t = (X[0] ^ X[i]) & P;     /* exchange */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
}

static void sk_axes_to_transpose(uint32_t X[3], int b)
{
    const int n = 3;
    uint32_t M = 1u << (b - 1), P, Q, t;
    /* inverse undo */
    for (Q = M; Q > 1; Q >>= 1) {
        P = Q - 1;
        for (int i = 0; i < n; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    /* Gray encode */
    for (int i = 1; i < n; ++i) X[i] ^= X[i - 1];
    t = 0;
    for (Q = M; Q > 1; Q >>= 1)
        if (X[n - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < n; ++i) X[i] ^= t;
}

void or_hilbert3_d2xyz(int b, int64_t n, const int64_t *d, int64_t *x, int64_t *y, int64_t *z)
{
    for (int64_t k = 0; k < n; ++k) {
        uint64_t h = (uint64_t)d[k];
        uint32_t X[3] = { 0, 0, 0 };
        for (int j = 0; j < b; ++j)          /* bit j of X[i] is bit 3j + 2 - i of h */
            for (int i = 0; i < 3; ++i)
                X[i] |= (uint32_t)((h >> (3 * j + 2 - i)) & 1u) << j;
        sk_transpose_to_axes(X, b);
        x[k] = X[0];
        y[k] = X[1];
        z[k] = X[2];
    }
}

void or_hilbert3_xyz2d(int b, int64_t n, const int64_t *x, const int64_t *y, const int64_t *z, int64_t *d)
{
    for (int64_t k = 0; k < n; ++k) {
        uint32_t X[3] = { (uint32_t)x[k], (uint32_t)y[k], (uint32_t)z[k] };
        sk_axes_to_transpose(X, b);
        uint64_t h = 0;
        for (int j = 0; j < b; ++j)
            for (int i = 0; i < 3; ++i)
                h |= (uint64_t)((X[i] >> j) & 1u) << (3 * j + 2 - i);
        d[k] = (int64_t)h;
    }
}

int or_version(void) { return OR_VERSION; }
