// Internal declarations shared by the HIP translation units of libqsq.
// Nothing here is part of the public C-ABI (include/qsq.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsq.h"

namespace qsq {

// end-record status of a half-line whose last trial step left the box and still
// has to be landed on the face (FP64 landing pass)
constexpr int kPendingLand = 0x7f;

// Grid geometry as the kernels see it.
struct Geom {
    int n[3];          // nodes per axis
    int pad;
    double o[3];       // origin
    double h[3];       // spacing
    double ih[3];      // 1 / spacing
    double lo[3];      // closed box
    double hi[3];
};

struct StepOpts {
    double rtol, atol;
    double h_init, h_max;
    double max_length;   // <= 0: unlimited
    double hmin;         // step underflow limit
    double gtol;         // landing tolerance on the face distance
    int64_t max_steps;
    int flags;
    int pad;
};

// Per half-line end records, SoA planes of length 2*cap; half-line (dir, seed)
// lives at dir*cap + seed (dir 0 = forward, 1 = backward).
struct Records {
    double *y;          // 9 planes: x0..2, dx1 0..2, dx2 0..2
    double *s;          // path length so far
    double *h;          // trial step that left the box (pending landing)
    int32_t *status;
    int32_t *attempts;
    int64_t cap;
};

struct TraceJob {
    const void *nodes;
    int storage;        // QSQ_F32 / QSQ_F64
    int mode;           // QSQ_INTERP_*
    Geom g;
    StepOpts o;
    const double *seeds;      // SoA planes with stride seed_stride
    int64_t seed_stride;
    int64_t n_host;           // seed count when n_dev is null
    const int64_t *n_dev;     // device seed count (overrides n_host)
    Records rec;
    unsigned long long *counter;   // device work counter (zeroed by the launcher)
    // per-seed outputs (stride out_stride for the fp planes); any may be null
    double *fp_fwd, *fp_bwd, *fll, *q_perp, *q_det, *q_fp;
    int32_t *status;
    int32_t *steps;           // 2 planes of out_stride
    int64_t out_stride;
    unsigned long long *work; // 4 device counters accumulated (nullable)
};

// kernels the profiler can time
constexpr int kProfStep = 0, kProfLand = 1, kProfAssemble = 2;
bool profiling();
void prof_begin(int kernel, hipStream_t s, void **token);
void prof_end(void *token, hipStream_t s);

// Bytes of the record block for cap seeds (without the 256-byte counter block).
uint64_t records_bytes(int64_t cap);
// Carve records + counter out of a scratch block (256-byte aligned).
void carve_records(void *scratch, int64_t cap, Records *rec, unsigned long long **counter);

// Enqueue the whole trace (work-counter reset, stepping, FP64 landing, FP64 Q assembly).
hipError_t launch_trace(const TraceJob &job, int step_dtype, hipStream_t stream);

// Field preparation.
hipError_t launch_field_init(const qsq_grid *g, const void *bx, const void *by, const void *bz,
                             int in_dtype, int storage, int mode, void *ws, hipStream_t stream);

// Maps.
hipError_t launch_fledge(const float *in, int ndim, const int64_t *shape, float *out, hipStream_t stream);
hipError_t launch_hilbert2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, hipStream_t s);
hipError_t launch_hilbert2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d, hipStream_t s);

uint64_t qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity);
hipError_t launch_qmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_map_desc *d, const qsq_map_out *out, void *scratch, hipStream_t stream);

int device_cu_count();

}  // namespace qsq
