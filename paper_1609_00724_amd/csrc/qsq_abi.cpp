// C-ABI entry points of libqsq: argument validation, scratch carving and
// launches.  Every check happens before anything is enqueued.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "qsq_cnn.h"
#include "qsq_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int ok()
{
    g_err[0] = '\0';
    return QSQ_OK;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(QSQ_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_grid(const qsq_grid *g)
{
    if (!g) return fail(QSQ_ERR_INVALID_ARG, "grid is NULL");
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 2) return fail(QSQ_ERR_INVALID_ARG, "grid n[%d] = %lld < 2", d, (long long)g->n[d]);
        if (g->n[d] > (1 << 20)) return fail(QSQ_ERR_UNSUPPORTED, "grid n[%d] too large", d);
        if (!(g->spacing[d] > 0.0) || !isfinite(g->spacing[d]))
            return fail(QSQ_ERR_INVALID_ARG, "grid spacing[%d] must be finite and > 0", d);
        if (!isfinite(g->origin[d])) return fail(QSQ_ERR_INVALID_ARG, "grid origin[%d] not finite", d);
    }
    const double N = (double)g->n[0] * (double)g->n[1] * (double)g->n[2];
    if (N > 2147483647.0) return fail(QSQ_ERR_UNSUPPORTED, "grid has more than 2^31-1 nodes");
    return QSQ_OK;
}

int check_field(const qsq_field *f)
{
    if (!f) return fail(QSQ_ERR_INVALID_ARG, "field is NULL");
    int rc = check_grid(&f->grid);
    if (rc) return rc;
    if (f->storage != QSQ_F32 && f->storage != QSQ_F64 && f->storage != QSQ_BF16)
        return fail(QSQ_ERR_UNSUPPORTED, "field storage %d not supported", f->storage);
    if (f->mode != QSQ_INTERP_PAPER && f->mode != QSQ_INTERP_NORMALIZE)
        return fail(QSQ_ERR_INVALID_ARG, "field mode %d unknown", f->mode);
    if (!f->nodes) return fail(QSQ_ERR_INVALID_ARG, "field nodes is NULL");
    if (f->bytes < qsq_field_bytes(&f->grid, f->storage))
        return fail(QSQ_ERR_INVALID_ARG, "field bytes smaller than the grid needs");
    if (f->cells && f->cell_bytes < qsq::cell_record_bytes(&f->grid, f->storage))
        return fail(QSQ_ERR_INVALID_ARG, "field cell_bytes smaller than the grid's cell records");
    if (f->bricks && f->brick_bytes < qsq::brick_record_bytes(&f->grid, f->storage))
        return fail(QSQ_ERR_INVALID_ARG, "brick bytes smaller than the grid needs");
    if (f->dirs && (f->storage != QSQ_F32 || f->dir_bytes < qsq::cell_dir_bytes(&f->grid)))
        return fail(QSQ_ERR_INVALID_ARG, "direction records need FP32 storage and dir_bytes for every cell");
    if (f->order < 0 || f->order > QSQ_ORDER_CUBIC) return fail(QSQ_ERR_INVALID_ARG, "field order %d", f->order);
    if (f->geometry != QSQ_GEOMETRY_CARTESIAN && f->geometry != QSQ_GEOMETRY_SPHERICAL)
        return fail(QSQ_ERR_INVALID_ARG, "field geometry %d", f->geometry);
    const bool rect = f->coords[0] || f->coords[1] || f->coords[2];
    if (f->geometry == QSQ_GEOMETRY_SPHERICAL || rect) {
        if (f->order > QSQ_ORDER_LINEAR)
            return fail(QSQ_ERR_UNSUPPORTED, "spherical or rectilinear fields take the trilinear kernel");
        if (f->storage == QSQ_BF16)
            return fail(QSQ_ERR_UNSUPPORTED, "spherical or rectilinear fields need FP32 or FP64 node records");
    }
    if (f->geometry == QSQ_GEOMETRY_SPHERICAL) {
        const double th0 = f->grid.origin[1], th1 = th0 + (double)(f->grid.n[1] - 1) * f->grid.spacing[1];
        const double r0 = f->grid.origin[2];
        if (!(th0 > -1.5707963267948966) || !(th1 < 1.5707963267948966) || !(r0 > 0.0))
            return fail(QSQ_ERR_INVALID_ARG, "spherical grid needs latitudes inside (-pi/2, pi/2) and radii > 0");
    }
    if (f->order > QSQ_ORDER_LINEAR) {
        if (f->storage == QSQ_BF16)
            return fail(QSQ_ERR_UNSUPPORTED, "interpolation order %d needs FP32 or FP64 node records", f->order);
        for (int d = 0; d < 3; ++d)
            if (f->grid.n[d] < 4)
                return fail(QSQ_ERR_UNSUPPORTED, "interpolation order %d needs >= 4 nodes per axis", f->order);
    }
    return QSQ_OK;
}

int make_geom_opts(const qsq_field *f, const qsq_trace_opts *o, qsq::Geom *g, qsq::StepOpts *so)
{
    if (!o) return fail(QSQ_ERR_INVALID_ARG, "opts is NULL");
    if (o->stepper != QSQ_STEPPER_CK54 && o->stepper != QSQ_STEPPER_EULER)
        return fail(QSQ_ERR_UNSUPPORTED, "stepper %d not supported", o->stepper);
    if (o->step_dtype != QSQ_F32 && o->step_dtype != QSQ_F64)
        return fail(QSQ_ERR_UNSUPPORTED, "step dtype %d not supported", o->step_dtype);
    if (!(o->rtol > 0.0) || !(o->atol > 0.0) || !isfinite(o->rtol) || !isfinite(o->atol))
        return fail(QSQ_ERR_INVALID_ARG, "rtol and atol must be finite and > 0");
    if (!isfinite(o->h_init) || !isfinite(o->h_max) || !isfinite(o->max_length))
        return fail(QSQ_ERR_INVALID_ARG, "h_init, h_max and max_length must be finite");
    if (o->flags & ~QSQ_FLAG_SKIP_OPEN) return fail(QSQ_ERR_INVALID_ARG, "unknown flags 0x%x", o->flags);
    if ((o->launch & ~0x1fff) || ((o->launch >> 4) & 3) == 3 || ((o->launch >> 6) & 7) > 6 ||
        ((o->launch >> 10) & 7) > 6)
        return fail(QSQ_ERR_INVALID_ARG,
                    "launch word 0x%x outside QSQ_LAUNCH(0..15, 0..2, 0..6) | QSQ_LAUNCH_PARTS | "
                    "QSQ_LAUNCH_REFINE_GATHER(0..6)",
                    o->launch);
    double hmin_grid = f->grid.spacing[0];
    double extent = 0.0;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = (int)f->grid.n[d];
        g->o[d] = f->grid.origin[d];
        g->h[d] = f->grid.spacing[d];
        g->ih[d] = 1.0 / f->grid.spacing[d];
        g->lo[d] = f->grid.origin[d];
        g->hi[d] = f->grid.origin[d] + (double)(f->grid.n[d] - 1) * f->grid.spacing[d];
        hmin_grid = fmin(hmin_grid, f->grid.spacing[d]);
        extent = fmax(extent, g->hi[d] - g->lo[d]);
    }
    g->geometry = f->geometry;
    for (int d = 0; d < 3; ++d) g->coord[d] = f->coords[d];
    if (qsq::job_mode(f) & 8) {
        if (o->stepper != QSQ_STEPPER_CK54)
            return fail(QSQ_ERR_UNSUPPORTED, "spherical or rectilinear fields take the CK54 stepper");
    }
    so->rtol = o->rtol;
    so->atol = o->atol;
    so->h_max = o->h_max > 0.0 ? o->h_max : hmin_grid;
    so->h_init = o->h_init > 0.0 ? o->h_init : 0.1 * hmin_grid;
    if (so->h_init > so->h_max) so->h_init = so->h_max;
    if (o->stepper == QSQ_STEPPER_EULER) {
        // fixed step: about five samplings per grid spacing unless given
        so->h_init = o->h_init > 0.0 ? o->h_init : 0.2 * hmin_grid;
        so->h_max = so->h_init;
    }
    so->max_length = o->max_length > 0.0 ? o->max_length : 0.0;
    so->hmin = 1e-12 * extent;
    so->gtol = 1e-12 * extent;
    so->max_steps = o->max_steps > 0 ? o->max_steps : (int64_t)1 << 22;
    so->flags = o->flags;
    so->launch = o->launch;
    so->stepper = o->stepper;
    so->pad = 0;
    return QSQ_OK;
}

// ---- event-based kernel timing ----------------------------------------------
struct ProfPair {
    int kernel;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::vector<ProfPair> g_prof;
bool g_prof_on = false;

}  // namespace

namespace qsq {

bool profiling() { return g_prof_on; }

void prof_begin(int kernel, hipStream_t s, void **token)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfPair p{kernel, nullptr, nullptr};
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
        *token = nullptr;
        return;
    }
    hipEventRecord(p.a, s);
    g_prof.push_back(p);
    *token = reinterpret_cast<void *>(g_prof.size());   // 1-based slot
}

void prof_end(void *token, hipStream_t s)
{
    if (!token) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    const size_t i = reinterpret_cast<size_t>(token) - 1;
    if (i < g_prof.size()) hipEventRecord(g_prof[i].b, s);
}

}  // namespace qsq

extern "C" {

int qsq_profile_enable(int on)
{
    g_prof_on = on != 0;
    return ok();
}

int qsq_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : g_prof) {
        hipEventSynchronize(p.b);
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    g_prof.clear();
    return ok();
}

int qsq_profile_read(int kernel, int64_t *launches, double *total_ms)
{
    if (!launches || !total_ms) return fail(QSQ_ERR_INVALID_ARG, "NULL output pointer");
    if (kernel < QSQ_KERNEL_STEP || kernel > QSQ_KERNEL_ASSEMBLE) return fail(QSQ_ERR_INVALID_ARG, "kernel id");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int64_t n = 0;
    double tot = 0.0;
    for (auto &p : g_prof) {
        if (p.kernel != kernel) continue;
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return hip_fail(e, "qsq_profile_read");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return hip_fail(e, "qsq_profile_read");
        ++n;
        tot += ms;
    }
    *launches = n;
    *total_ms = tot;
    return ok();
}


int qsq_abi_version(void) { return QSQ_ABI_VERSION; }

const char *qsq_status_string(int code)
{
    switch (code) {
    case QSQ_END_XLO: return "left through the x = min face";
    case QSQ_END_XHI: return "left through the x = max face";
    case QSQ_END_YLO: return "left through the y = min face";
    case QSQ_END_YHI: return "left through the y = max face";
    case QSQ_END_ZLO: return "left through the z = min face";
    case QSQ_END_ZHI: return "left through the z = max face";
    case QSQ_END_MAX_LENGTH: return "reached max_length";
    case QSQ_END_MAX_STEPS: return "reached max_steps";
    case QSQ_END_NULL: return "field null (|Bhat| < 1e-6)";
    case QSQ_END_UNDERFLOW: return "step size underflow";
    case QSQ_END_SEED_OUTSIDE: return "seed outside the box";
    case QSQ_END_NONFINITE: return "state became non-finite";
    case QSQ_ERR_INVALID_ARG: return "invalid argument";
    case QSQ_ERR_UNSUPPORTED: return "unsupported";
    case QSQ_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case QSQ_ERR_HIP: return "HIP runtime error";
    case QSQ_ERR_COUNT_OVERFLOW: return "count overflow";
    default: return "unknown code";
    }
}

const char *qsq_last_error(void) { return g_err; }

uint64_t qsq_field_bytes(const qsq_grid *g, int storage)
{
    if (!g) return 0;
    const uint64_t N = (uint64_t)g->n[0] * (uint64_t)g->n[1] * (uint64_t)g->n[2];
    const uint64_t per = storage == QSQ_F64 ? 32 : storage == QSQ_F32 ? 16 : storage == QSQ_BF16 ? 8 : 0;
    return N * per;
}

int qsq_field_init(const qsq_grid *g, const void *bx, const void *by, const void *bz, int in_dtype,
                   int storage, int mode, void *ws, uint64_t ws_bytes, void *stream, qsq_field *out)
{
    int rc = check_grid(g);
    if (rc) return rc;
    if (!bx || !by || !bz || !ws || !out) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    if (in_dtype != QSQ_F32 && in_dtype != QSQ_F64) return fail(QSQ_ERR_INVALID_ARG, "in_dtype %d", in_dtype);
    if (storage != QSQ_F32 && storage != QSQ_F64 && storage != QSQ_BF16)
        return fail(QSQ_ERR_UNSUPPORTED, "storage %d not supported", storage);
    if (mode != QSQ_INTERP_PAPER && mode != QSQ_INTERP_NORMALIZE)
        return fail(QSQ_ERR_INVALID_ARG, "mode %d unknown", mode);
    if (!aligned(ws, 16)) return fail(QSQ_ERR_INVALID_ARG, "workspace must be 16-byte aligned");
    const uint64_t need = qsq_field_bytes(g, storage);
    if (ws_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "field workspace %llu < %llu bytes",
                    (unsigned long long)ws_bytes, (unsigned long long)need);
    hipError_t e = qsq::launch_field_init(g, bx, by, bz, in_dtype, storage, mode, ws,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_field_init");
    out->grid = *g;
    out->storage = storage;
    out->mode = mode;
    out->nodes = ws;
    out->bytes = need;
    out->cells = nullptr;
    out->cell_bytes = 0;
    out->bricks = nullptr;
    out->brick_bytes = 0;
    out->dirs = nullptr;
    out->dir_bytes = 0;
    out->order = QSQ_ORDER_LINEAR;
    out->geometry = QSQ_GEOMETRY_CARTESIAN;
    out->coords[0] = out->coords[1] = out->coords[2] = nullptr;
    return ok();
}

uint64_t qsq_field_cell_bytes(const qsq_grid *g, int storage)
{
    if (!g || g->n[0] < 2 || g->n[1] < 2 || g->n[2] < 2) return 0;
    if (storage != QSQ_F64 && storage != QSQ_F32 && storage != QSQ_BF16) return 0;
    return qsq::cell_record_bytes(g, storage);
}

int qsq_field_add_cells(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    if (!ws || !aligned(ws, 256)) return fail(QSQ_ERR_INVALID_ARG, "cell workspace NULL or not 256-byte aligned");
    const uint64_t need = qsq_field_cell_bytes(&f->grid, f->storage);
    if (ws_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "cell workspace %llu < %llu bytes", (unsigned long long)ws_bytes,
                    (unsigned long long)need);
    hipError_t e = qsq::launch_cell_records(f, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_field_add_cells");
    f->cells = ws;
    f->cell_bytes = need;
    return ok();
}

uint64_t qsq_field_brick_bytes(const qsq_grid *g, int storage)
{
    if (!g || g->n[0] < 2 || g->n[1] < 2 || g->n[2] < 2) return 0;
    if (storage != QSQ_F64 && storage != QSQ_F32 && storage != QSQ_BF16) return 0;
    return qsq::brick_record_bytes(g, storage);
}

int qsq_field_add_bricks(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    if (qsq::job_mode(f) > 1)
        return fail(QSQ_ERR_UNSUPPORTED, "brick records take trilinear Cartesian fields with uniform axes");
    if (!ws || !aligned(ws, 256)) return fail(QSQ_ERR_INVALID_ARG, "brick workspace NULL or not 256-byte aligned");
    const uint64_t need = qsq_field_brick_bytes(&f->grid, f->storage);
    if (ws_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "brick workspace %llu < %llu bytes", (unsigned long long)ws_bytes,
                    (unsigned long long)need);
    hipError_t e = qsq::launch_brick_records(f, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_field_add_bricks");
    f->bricks = ws;
    f->brick_bytes = need;
    return ok();
}

uint64_t qsq_field_cell_dir_bytes(const qsq_grid *g, int storage)
{
    if (!g || g->n[0] < 2 || g->n[1] < 2 || g->n[2] < 2 || storage != QSQ_F32) return 0;
    return qsq::cell_dir_bytes(g);
}

int qsq_field_add_cell_dirs(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    if (f->storage != QSQ_F32 || qsq::job_mode(f) > 1)
        return fail(QSQ_ERR_UNSUPPORTED, "direction records take FP32 trilinear Cartesian fields with uniform axes");
    if (!ws || !aligned(ws, 256)) return fail(QSQ_ERR_INVALID_ARG, "direction workspace NULL or not 256-byte aligned");
    const uint64_t need = qsq_field_cell_dir_bytes(&f->grid, f->storage);
    if (ws_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "direction workspace %llu < %llu bytes",
                    (unsigned long long)ws_bytes, (unsigned long long)need);
    hipError_t e = qsq::launch_cell_dirs(f, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_field_add_cell_dirs");
    f->dirs = ws;
    f->dir_bytes = need;
    return ok();
}

uint64_t qsq_trace_scratch_bytes(int64_t n)
{
    if (n < 0) return 0;
    return 256 + qsq::records_bytes(n);
}

int qsq_trace(const qsq_field *f, const double *seeds, int64_t n, const qsq_trace_opts *opts,
              const qsq_trace_out *out, void *scratch, uint64_t scratch_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    qsq::Geom g;
    qsq::StepOpts so;
    rc = make_geom_opts(f, opts, &g, &so);
    if (rc) return rc;
    if (n < 0) return fail(QSQ_ERR_INVALID_ARG, "n < 0");
    if (n > ((int64_t)1 << 30)) return fail(QSQ_ERR_COUNT_OVERFLOW, "n > 2^30 seeds");
    if (n == 0) return ok();   // nothing to enqueue; output pointers may be NULL
    if (!out || !out->status) return fail(QSQ_ERR_INVALID_ARG, "out or out->status is NULL");
    if (!seeds || !scratch) return fail(QSQ_ERR_INVALID_ARG, "NULL seeds or scratch");
    if (!aligned(scratch, 256)) return fail(QSQ_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    const uint64_t need = qsq_trace_scratch_bytes(n);
    if (scratch_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "trace scratch %llu < %llu bytes",
                    (unsigned long long)scratch_bytes, (unsigned long long)need);
    qsq::TraceJob job{};
    job.nodes = f->nodes;
    job.cells = f->cells;
    job.bricks = f->bricks;
    job.dirs = static_cast<const float *>(f->dirs);
    job.storage = f->storage;
    job.mode = qsq::job_mode(f);
    job.g = g;
    job.o = so;
    job.seeds = seeds;
    job.seed_stride = n;
    job.n_host = n;
    job.n_dev = nullptr;
    qsq::carve_records(scratch, n, &job.rec, &job.counter);
    job.spatial_bits = qsq::spatial_bits_for(1);
    job.fp_fwd = out->fp_fwd;
    job.fp_bwd = out->fp_bwd;
    job.fll = out->fll;
    job.q_perp = out->q_perp;
    job.q_det = out->q_det;
    job.q_fp = out->q_fp;
    job.status = out->status;
    job.steps = out->steps;
    job.out_stride = n;
    job.work = reinterpret_cast<unsigned long long *>(out->work);
    hipError_t e = qsq::launch_trace(job, opts->step_dtype, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_trace");
    return ok();
}

}  // extern "C"

// Scratch of qsq_trace_noalloc: a fixed device array, one copy per device,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
#define QSQ_NOALLOC_SCRATCH_BYTES (64ull << 20)
static __device__ __align__(256) unsigned char scratch[QSQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (set up on the first call
// made with that device current)
int noalloc_scratch(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "qsq_trace_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(QSQ_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "qsq_trace_noalloc: hipGetSymbolAddress");
        if (!p || !aligned(p, 256)) return fail(QSQ_ERR_HIP, "qsq_trace_noalloc: bad scratch address");
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return QSQ_OK;
}
}  // namespace

extern "C" {

int qsq_trace_noalloc(const qsq_field *f, const double *seeds, int64_t n, const qsq_trace_opts *opts,
                      const qsq_trace_out *out, void *stream)
{
    if (n > QSQ_TRACE_NOALLOC_MAX_SEEDS)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "qsq_trace_noalloc: n = %lld > %d seeds", (long long)n,
                    QSQ_TRACE_NOALLOC_MAX_SEEDS);
    if (qsq_trace_scratch_bytes(n) > QSQ_NOALLOC_SCRATCH_BYTES)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "qsq_trace_noalloc: scratch of %lld seeds exceeds %llu bytes",
                    (long long)n, (unsigned long long)QSQ_NOALLOC_SCRATCH_BYTES);
    void *ptr = nullptr;
    if (n > 0) {
        // the other arguments are checked by qsq_trace before anything is enqueued
        const int rc = noalloc_scratch(&ptr);
        if (rc) return rc;
    }
    return qsq_trace(f, seeds, n, opts, out, ptr, QSQ_NOALLOC_SCRATCH_BYTES, stream);
}

static uint64_t round256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

// prefix the last error message with the set that caused it
static int set_fail(int rc, int k)
{
    char msg[sizeof g_err];
    memcpy(msg, g_err, sizeof msg);
    return fail(rc, "set %d: %s", k, msg);
}

uint64_t qsq_trace_batch_scratch_bytes(int32_t nsets, int64_t total)
{
    if (nsets < 0 || total < 0) return 0;
    return round256(256 + qsq::records_bytes(total)) + round256((uint64_t)total * sizeof(int32_t)) +
           round256((uint64_t)nsets * sizeof(qsq::SetDesc));
}

int qsq_trace_batch(const qsq_trace_set *sets, int32_t nsets, const qsq_trace_opts *opts, uint64_t *work,
                    void *scratch, uint64_t scratch_bytes, void *stream)
{
    if (!sets) return fail(QSQ_ERR_INVALID_ARG, "sets is NULL");
    if (nsets < 1 || nsets > QSQ_MAX_TRACE_SETS)
        return fail(QSQ_ERR_INVALID_ARG, "nsets = %d outside [1, %d]", nsets, QSQ_MAX_TRACE_SETS);
    std::vector<qsq::SetDesc> table((size_t)nsets);
    int64_t total = 0;
    qsq::StepOpts so0{};
    for (int k = 0; k < nsets; ++k) {
        const qsq_trace_set &t = sets[k];
        int rc = check_field(&t.field);
        if (rc) return set_fail(rc, k);
        if (t.field.order > QSQ_ORDER_LINEAR || (qsq::job_mode(&t.field) & 8)) return set_fail(QSQ_ERR_UNSUPPORTED, k);
        if (t.field.storage != sets[0].field.storage || t.field.mode != sets[0].field.mode)
            return fail(QSQ_ERR_INVALID_ARG, "set %d: storage and mode must match set 0", k);
        qsq::Geom g;
        qsq::StepOpts so;
        rc = make_geom_opts(&t.field, opts, &g, &so);
        if (rc) return set_fail(rc, k);
        if (t.n < 0) return fail(QSQ_ERR_INVALID_ARG, "set %d: n < 0", k);
        if (t.n > 0 && (!t.seeds || !t.out.status))
            return fail(QSQ_ERR_INVALID_ARG, "set %d: NULL seeds or out.status", k);
        if (k == 0) so0 = so;
        qsq::SetDesc &d = table[k];
        d = qsq::SetDesc{};
        d.g = g;
        d.nodes = t.field.nodes;
        d.seeds = t.seeds;
        d.n = t.n;
        d.off = total;
        d.h_init = so.h_init;
        d.h_max = so.h_max;
        d.hmin = so.hmin;
        d.gtol = so.gtol;
        d.fp_fwd = t.out.fp_fwd;
        d.fp_bwd = t.out.fp_bwd;
        d.fll = t.out.fll;
        d.q_perp = t.out.q_perp;
        d.q_det = t.out.q_det;
        d.q_fp = t.out.q_fp;
        d.status = t.out.status;
        d.steps = t.out.steps;
        total += t.n;
        if (total > ((int64_t)1 << 30)) return fail(QSQ_ERR_COUNT_OVERFLOW, "more than 2^30 seeds in the batch");
    }
    if (total == 0) return ok();
    if (!scratch) return fail(QSQ_ERR_INVALID_ARG, "scratch is NULL");
    if (!aligned(scratch, 256)) return fail(QSQ_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    const uint64_t need = qsq_trace_batch_scratch_bytes(nsets, total);
    if (scratch_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "batch scratch %llu < %llu bytes",
                    (unsigned long long)scratch_bytes, (unsigned long long)need);
    qsq::TraceJob job{};
    job.storage = sets[0].field.storage;
    job.mode = qsq::job_mode(&sets[0].field);
    job.nodes = sets[0].field.nodes;
    job.g = table[0].g;
    job.o = so0;   // rtol, atol, max_length, max_steps, flags; per-set limits come from the table
    job.n_host = total;
    job.n_dev = nullptr;
    qsq::carve_records(scratch, total, &job.rec, &job.counter);
    char *p = static_cast<char *>(scratch) + round256(256 + qsq::records_bytes(total));
    job.set_of = reinterpret_cast<int32_t *>(p);
    p += round256((uint64_t)total * sizeof(int32_t));
    job.sets = reinterpret_cast<const qsq::SetDesc *>(p);
    job.nsets = nsets;
    job.spatial_bits = qsq::spatial_bits_for(nsets);
    job.work = reinterpret_cast<unsigned long long *>(work);
    hipError_t e = qsq::launch_trace_batch(job, table.data(), nsets, opts->step_dtype, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_trace_batch");
    return ok();
}

int qsq_fledge(const float *in, int ndim, const int64_t *shape, float *out, void *stream)
{
    if (!in || !out || !shape) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    if (ndim != 2 && ndim != 3) return fail(QSQ_ERR_INVALID_ARG, "ndim must be 2 or 3");
    uint64_t N = 1;
    for (int d = 0; d < ndim; ++d) {
        if (shape[d] < 1) return fail(QSQ_ERR_INVALID_ARG, "shape[%d] < 1", d);
        N *= (uint64_t)shape[d];
    }
    const char *a = reinterpret_cast<const char *>(in), *b = reinterpret_cast<const char *>(out);
    if (a < b + N * 4 && b < a + N * 4) return fail(QSQ_ERR_INVALID_ARG, "in and out overlap");
    hipError_t e = qsq::launch_fledge(in, ndim, shape, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_fledge");
    return ok();
}

int qsq_hilbert2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, void *stream)
{
    if (L < 1 || L > 31) return fail(QSQ_ERR_INVALID_ARG, "L must be in [1, 31]");
    if (n < 0) return fail(QSQ_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (!d || !x || !y) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    hipError_t e = qsq::launch_hilbert2_d2xy(L, d, n, x, y, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_hilbert2_d2xy");
    return ok();
}

int qsq_hilbert2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d, void *stream)
{
    if (L < 1 || L > 31) return fail(QSQ_ERR_INVALID_ARG, "L must be in [1, 31]");
    if (n < 0) return fail(QSQ_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (!d || !x || !y) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    hipError_t e = qsq::launch_hilbert2_xy2d(L, x, y, n, d, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_hilbert2_xy2d");
    return ok();
}

int qsq_hilbert3_d2xyz(int b, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, uint32_t *z, void *stream)
{
    if (b < 1 || b > 21) return fail(QSQ_ERR_INVALID_ARG, "b must be in [1, 21]");
    if (n < 0) return fail(QSQ_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (!d || !x || !y || !z) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    hipError_t e = qsq::launch_hilbert3_d2xyz(b, d, n, x, y, z, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_hilbert3_d2xyz");
    return ok();
}

int qsq_hilbert3_xyz2d(int b, const uint32_t *x, const uint32_t *y, const uint32_t *z, int64_t n, uint64_t *d,
                       void *stream)
{
    if (b < 1 || b > 21) return fail(QSQ_ERR_INVALID_ARG, "b must be in [1, 21]");
    if (n < 0) return fail(QSQ_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (!d || !x || !y || !z) return fail(QSQ_ERR_INVALID_ARG, "NULL pointer argument");
    hipError_t e = qsq::launch_hilbert3_xyz2d(b, x, y, z, n, d, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_hilbert3_xyz2d");
    return ok();
}

// the shifted-curve re-pass options shared by slices and volumes (L = m + r)
static int check_shift(int32_t shift, int32_t max_cycles, int L, bool propose)
{
    if (shift == 0) return QSQ_OK;
    if (shift < 0 || (int64_t)shift >= ((int64_t)1 << L))
        return fail(QSQ_ERR_INVALID_ARG, "shift must be 0 or in (0, 2^(base_level + refine_levels))");
    if (max_cycles > 48) return fail(QSQ_ERR_INVALID_ARG, "max_cycles must be <= 48");
    if (propose) return fail(QSQ_ERR_UNSUPPORTED, "proposals and the shifted re-pass cannot be combined");
    return QSQ_OK;
}

static int check_map(const qsq_map_desc *d)
{
    if (!d) return fail(QSQ_ERR_INVALID_ARG, "map desc is NULL");
    if (d->base_level < 1 || d->refine_levels < 0 || d->base_level + d->refine_levels > 16)
        return fail(QSQ_ERR_INVALID_ARG, "need base_level >= 1, refine_levels >= 0, sum <= 16");
    if (d->out_level < d->base_level || d->out_level > d->base_level + d->refine_levels)
        return fail(QSQ_ERR_INVALID_ARG, "out_level outside [base_level, base_level + refine_levels]");
    if (d->tilted) {
        double uu = 0.0, vv = 0.0, cr[3];
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(d->corner[a]) || !isfinite(d->edge_u[a]) || !isfinite(d->edge_v[a]))
                return fail(QSQ_ERR_INVALID_ARG, "tilted slice corner and edges must be finite");
            uu += d->edge_u[a] * d->edge_u[a];
            vv += d->edge_v[a] * d->edge_v[a];
        }
        cr[0] = d->edge_u[1] * d->edge_v[2] - d->edge_u[2] * d->edge_v[1];
        cr[1] = d->edge_u[2] * d->edge_v[0] - d->edge_u[0] * d->edge_v[2];
        cr[2] = d->edge_u[0] * d->edge_v[1] - d->edge_u[1] * d->edge_v[0];
        if (!(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] > 1e-24 * uu * vv))
            return fail(QSQ_ERR_INVALID_ARG, "tilted slice edges must span a plane");
    } else if (!(d->x1 > d->x0) || !(d->y1 > d->y0) || !isfinite(d->z0)) {
        return fail(QSQ_ERR_INVALID_ARG, "slice extent must satisfy x1 > x0, y1 > y0, finite z0");
    }
    if (!(d->threshold >= 0.0)) return fail(QSQ_ERR_INVALID_ARG, "threshold must be >= 0");
    if (d->base_given != 0 && d->base_given != 1) return fail(QSQ_ERR_INVALID_ARG, "base_given must be 0 or 1");
    return check_shift(d->shift, d->max_cycles, d->base_level + d->refine_levels, d->propose != nullptr);
}

static int check_volume(const qsq_volume_desc *d)
{
    if (!d) return fail(QSQ_ERR_INVALID_ARG, "volume desc is NULL");
    if (d->base_level < 1 || d->refine_levels < 0 || d->base_level + d->refine_levels > 21)
        return fail(QSQ_ERR_INVALID_ARG, "need base_level >= 1, refine_levels >= 0, sum <= 21");
    if (3 * d->base_level > 30) return fail(QSQ_ERR_UNSUPPORTED, "base_level > 10 (more than 2^30 base cells)");
    if (d->out_level < d->base_level || d->out_level > d->base_level + d->refine_levels)
        return fail(QSQ_ERR_INVALID_ARG, "out_level outside [base_level, base_level + refine_levels]");
    if (3 * d->out_level > 33) return fail(QSQ_ERR_UNSUPPORTED, "out_level > 11");
    if (!(d->x1 > d->x0) || !(d->y1 > d->y0) || !(d->z1 > d->z0))
        return fail(QSQ_ERR_INVALID_ARG, "volume extent must satisfy x1 > x0, y1 > y0, z1 > z0");
    if (!(d->threshold >= 0.0)) return fail(QSQ_ERR_INVALID_ARG, "threshold must be >= 0");
    if (d->shift > 0 && d->base_level + d->refine_levels > 20)
        return fail(QSQ_ERR_UNSUPPORTED, "shifted re-pass needs base_level + refine_levels <= 20 for volumes");
    return check_shift(d->shift, d->max_cycles, d->base_level + d->refine_levels, d->propose != nullptr);
}

uint64_t qsq_vmap_scratch_bytes(const qsq_volume_desc *d, int64_t capacity)
{
    if (!d || capacity <= 0) return 0;
    return qsq::vmap_scratch_bytes(d, capacity);
}

int qsq_vmap(const qsq_field *f, const qsq_volume_desc *d, const qsq_trace_opts *opts, const qsq_map_out *out,
             void *scratch, uint64_t scratch_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    rc = check_volume(d);
    if (rc) return rc;
    qsq::Geom g;
    qsq::StepOpts so;
    rc = make_geom_opts(f, opts, &g, &so);
    if (rc) return rc;
    if (!out) return fail(QSQ_ERR_INVALID_ARG, "out is NULL");
    const int64_t nb = (int64_t)1 << (3 * d->base_level);
    if (out->capacity < nb) return fail(QSQ_ERR_INVALID_ARG, "capacity < 8^base_level");
    // the trace records hold 2 x capacity half-lines addressed by int32 work
    // entries and scan offsets, as qsq_trace bounds its seed count
    if (out->capacity > ((int64_t)1 << 30)) return fail(QSQ_ERR_COUNT_OVERFLOW, "capacity > 2^30");
    if (!out->keys || !out->fll || !out->q_perp || !out->status || !out->count || !out->overflow)
        return fail(QSQ_ERR_INVALID_ARG, "sample arrays, count and overflow are required");
    if (!scratch || !aligned(scratch, 256)) return fail(QSQ_ERR_INVALID_ARG, "scratch NULL or not 256-byte aligned");
    const uint64_t need = qsq::vmap_scratch_bytes(d, out->capacity);
    if (scratch_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "vmap scratch %llu < %llu bytes",
                    (unsigned long long)scratch_bytes, (unsigned long long)need);
    hipError_t e = qsq::launch_vmap(f, g, so, opts->step_dtype, d, out, scratch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_vmap");
    return ok();
}

uint64_t qsq_qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity)
{
    if (!d || capacity <= 0) return 0;
    return qsq::qmap_scratch_bytes(d, capacity);
}

int qsq_qmap(const qsq_field *f, const qsq_map_desc *d, const qsq_trace_opts *opts, const qsq_map_out *out,
             void *scratch, uint64_t scratch_bytes, void *stream)
{
    int rc = check_field(f);
    if (rc) return rc;
    rc = check_map(d);
    if (rc) return rc;
    qsq::Geom g;
    qsq::StepOpts so;
    rc = make_geom_opts(f, opts, &g, &so);
    if (rc) return rc;
    if (!out) return fail(QSQ_ERR_INVALID_ARG, "out is NULL");
    const int64_t nb = (int64_t)1 << (2 * d->base_level);
    if (out->capacity < nb) return fail(QSQ_ERR_INVALID_ARG, "capacity < 4^base_level");
    // the trace records hold 2 x capacity half-lines addressed by int32 work
    // entries and scan offsets, as qsq_trace bounds its seed count
    if (out->capacity > ((int64_t)1 << 30)) return fail(QSQ_ERR_COUNT_OVERFLOW, "capacity > 2^30");
    if (!out->keys || !out->fll || !out->q_perp || !out->status || !out->count || !out->overflow)
        return fail(QSQ_ERR_INVALID_ARG, "sample arrays, count and overflow are required");
    if (!scratch || !aligned(scratch, 256)) return fail(QSQ_ERR_INVALID_ARG, "scratch NULL or not 256-byte aligned");
    const uint64_t need = qsq::qmap_scratch_bytes(d, out->capacity);
    if (scratch_bytes < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "qmap scratch %llu < %llu bytes",
                    (unsigned long long)scratch_bytes, (unsigned long long)need);
    hipError_t e = qsq::launch_qmap(f, g, so, opts->step_dtype, d, out, scratch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_qmap");
    return ok();
}

// ---- learned refinement proposer -------------------------------------------

static int check_tiles(int64_t n, int h, int w)
{
    if (n < 1 || h < 32 || w < 32 || h % 32 || w % 32)
        return fail(QSQ_ERR_INVALID_ARG, "need n >= 1 and h, w positive multiples of 32 (got %lld, %d, %d)",
                    (long long)n, h, w);
    if ((double)n * h * w >= 2147483648.0) return fail(QSQ_ERR_COUNT_OVERFLOW, "n h w >= 2^31 pixels");
    if ((int64_t)h * w > ((int64_t)1 << 24)) return fail(QSQ_ERR_COUNT_OVERFLOW, "h w > 2^24 pixels per tile");
    return QSQ_OK;
}

uint64_t qsq_cnn_prep_bytes(void) { return qsq::cnn_prep_bytes(); }

uint64_t qsq_cnn_workspace_bytes(int64_t n, int h, int w)
{
    if (n < 1 || h < 1 || w < 1) return 0;
    return qsq::cnn_workspace_bytes(n, h, w);
}

uint64_t qsq_cnn_layer_scratch_bytes(int64_t n, int h, int w)
{
    if (n < 1 || h < 1 || w < 1) return 0;
    return qsq::cnn_wgrad_scratch_bytes(n, h, w);
}

int qsq_cnn_prepare(const float *params, void *prep, void *stream)
{
    if (!params || !prep) return fail(QSQ_ERR_INVALID_ARG, "NULL params or prep");
    if (!aligned(prep, 16)) return fail(QSQ_ERR_INVALID_ARG, "prep must be 16-byte aligned");
    hipError_t e = qsq::cnn_prepare(params, prep, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_cnn_prepare");
    return ok();
}

static int check_ws(void *ws, uint64_t have, uint64_t need)
{
    if (!ws) return fail(QSQ_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(QSQ_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (have < need)
        return fail(QSQ_ERR_WORKSPACE_TOO_SMALL, "workspace %llu < %llu bytes", (unsigned long long)have,
                    (unsigned long long)need);
    return QSQ_OK;
}

int qsq_cnn_forward(const void *prep, const float *x, int64_t n, int h, int w, float *out, void *ws,
                    uint64_t ws_bytes, void *stream)
{
    int rc = check_tiles(n, h, w);
    if (rc) return rc;
    if (!prep || !x || !out) return fail(QSQ_ERR_INVALID_ARG, "NULL prep, x or out");
    rc = check_ws(ws, ws_bytes, qsq::cnn_workspace_bytes(n, h, w));
    if (rc) return rc;
    hipError_t e = qsq::cnn_forward(prep, x, n, h, w, out, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_cnn_forward");
    return ok();
}

int qsq_cnn_train_step(float *params, float *adam_m, float *adam_v, int64_t t, float lr, const float *x,
                       const float *mask, const float *logq, int64_t n, int h, int w, float lam, void *prep,
                       float *grad_out, double *loss_out, void *ws, uint64_t ws_bytes, void *stream)
{
    int rc = check_tiles(n, h, w);
    if (rc) return rc;
    if (!params || !adam_m || !adam_v || !x || !mask || !logq || !prep)
        return fail(QSQ_ERR_INVALID_ARG, "NULL params, Adam state, inputs, targets or prep");
    if (t < 1) return fail(QSQ_ERR_INVALID_ARG, "Adam step t must be >= 1");
    if (!(lr > 0.0f) || !isfinite(lr) || !(lam >= 0.0f) || !isfinite(lam))
        return fail(QSQ_ERR_INVALID_ARG, "lr must be > 0 and lam >= 0, both finite");
    rc = check_ws(ws, ws_bytes, qsq::cnn_workspace_bytes(n, h, w));
    if (rc) return rc;
    hipError_t e = qsq::cnn_train_step(params, adam_m, adam_v, t, lr, x, mask, logq, n, h, w, lam, prep, grad_out,
                                       loss_out, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_cnn_train_step");
    return ok();
}

int qsq_cnn_layer_forward(int layer, const void *prep, const void *in, int64_t n, int h, int w, float *out_f32,
                          void *stream)
{
    if (layer < 0 || layer > 3) return fail(QSQ_ERR_INVALID_ARG, "layer %d outside 0..3", layer);
    int rc = check_tiles(n, h, w);
    if (rc) return rc;
    if (!prep || !in || !out_f32) return fail(QSQ_ERR_INVALID_ARG, "NULL prep, in or out");
    hipError_t e = qsq::cnn_layer_forward(layer, prep, in, n, h, w, out_f32, nullptr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_cnn_layer_forward");
    return ok();
}

int qsq_cnn_layer_backward(int layer, const void *prep, const void *in, const uint16_t *dy, int64_t n, int h, int w,
                           float *dw, float *db, float *dx, void *scratch, uint64_t scratch_bytes, void *stream)
{
    if (layer < 0 || layer > 3) return fail(QSQ_ERR_INVALID_ARG, "layer %d outside 0..3", layer);
    int rc = check_tiles(n, h, w);
    if (rc) return rc;
    if (!prep || !in || !dy || !dw || !db) return fail(QSQ_ERR_INVALID_ARG, "NULL prep, in, dy, dw or db");
    if (layer == 0 && dx) return fail(QSQ_ERR_INVALID_ARG, "layer 0 has no input gradient");
    rc = check_ws(scratch, scratch_bytes, qsq::cnn_wgrad_scratch_bytes(n, h, w));
    if (rc) return rc;
    hipError_t e = qsq::cnn_layer_backward(layer, prep, in, dy, n, h, w, dw, db, dx, nullptr, nullptr, scratch,
                                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "qsq_cnn_layer_backward");
    return ok();
}

}  // extern "C"
