// Internal declarations shared by the HIP translation units of libqsq.
// Nothing here is part of the public C-ABI (include/qsq.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsq.h"

namespace qsq {

// tag type of BF16 node records (4 x 16-bit values per node, 8 bytes)
struct Bf16 {
    uint16_t bits;
};

// end-record status of a half-line whose last trial step left the box and still
// has to be landed on the face (FP64 landing pass)
constexpr int kPendingLand = 0x7f;
// record status of a half-line the seed pass set up for stepping
constexpr int kPendingStep = 0x7e;
// record status of a half-line whose landing step length is found (face
// kLandFace + f, step length in the record's h) and whose landed state is not
// yet computed
constexpr int kLandFace = 0x70;

// Grid geometry as the kernels see it.
struct Geom {
    int n[3];          // nodes per axis
    int geometry;      // QSQ_GEOMETRY_*
    double o[3];       // origin
    double h[3];       // spacing
    double ih[3];      // 1 / spacing
    double lo[3];      // closed box
    double hi[3];
    const double *coord[3];   // rectilinear axes: node coordinates (device), else null
};

struct StepOpts {
    double rtol, atol;
    double h_init, h_max;
    double max_length;   // <= 0: unlimited
    double hmin;         // step underflow limit
    double gtol;         // landing tolerance on the face distance
    int64_t max_steps;
    int flags;
    int launch;          // QSQ_LAUNCH word (0: defaults)
    int stepper;         // QSQ_STEPPER_*
    int pad;
};

// Per half-line end records, SoA planes of length 2*cap; half-line (dir, seed)
// lives at dir*cap + seed (dir 0 = forward, 1 = backward).
// Work-list parts of the persistent stepping launch (one per XCD) and the
// index of their counters in the 256-byte counter block (u64 slots 8 .. 15).
constexpr int kParts = 8;
constexpr int kPartCounter = 8;

struct Records {
    double *y;          // 9 planes: x0..2, dx1 0..2, dx2 0..2
    double *s;          // path length so far
    double *h;          // trial step that left the box (pending landing)
    int32_t *status;
    int32_t *attempts;
    int64_t cap;
    // work list of the half-lines to step (record indices in seed order)
    int32_t *flag;      // 2*cap: 1 if the half-line needs stepping
    int32_t *wpos;      // 2*cap: exclusive scan of flag
    int32_t *work;      // 2*cap: record index of each work item
    int64_t *scan_tmp;  // block sums of the scan
    int64_t *n_work;    // device scalar: work items
    int64_t *n_items;   // device scalar: half-lines of the call (2 n)
    int64_t *n_land;    // device scalar: half-lines the landing pass takes (listed in work2)
    int32_t *work2;     // 2*cap: second buffer of the work-list sort
    int32_t *scnt;      // digit counts of the work-list sort (sort_count_words(2 cap))
    int64_t *n_sort;    // device scalars of the sort: count entries, item total
};

// One seed set of a batched trace: its own field, seeds, per-grid step
// limits and outputs.  Seeds of all sets are numbered globally; set s holds
// global seeds [off, off + n).
struct SetDesc {
    Geom g;
    const void *nodes;
    const double *seeds;      // SoA planes with stride n
    int64_t n, off;
    double h_init, h_max, hmin, gtol;
    double *fp_fwd, *fp_bwd, *fll, *q_perp, *q_det, *q_fp;   // stride n, nullable
    int32_t *status;
    int32_t *steps;           // 2 planes of stride n, nullable
};

struct TraceJob {
    const void *nodes;
    const void *cells;  // cell records (nullable): 8 corner records per cell
    const void *bricks; // brick records (nullable): the nodes in 2 x 2 x 2 bricks
    const float *dirs;  // direction records (nullable): 24 FP32 values per cell
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
    int32_t *steps;           // 2 planes of out_stride; with steps_sum one plane
    int steps_sum;            // 1: steps[i] = forward + backward attempts
    int64_t out_stride;
    unsigned long long *work; // 4 device counters accumulated (nullable)
    // batched traces: nsets > 0, the set table and the set of each global seed
    const SetDesc *sets;
    int32_t *set_of;
    int nsets;
    // > 0: the work list is sorted by (set, Morton index of the seed's cell at
    // this many bits per axis of the set's box) before stepping, so that the
    // lanes of a wave trace nearby lines; 0: seed order (maps, whose seeds
    // already follow a space-filling curve)
    int spatial_bits;
};

// kernels the profiler can time
constexpr int kProfStep = 0, kProfLand = 1, kProfAssemble = 2;
bool profiling();
void prof_begin(int kernel, hipStream_t s, void **token);
void prof_end(void *token, hipStream_t s);

// Bytes of the record block for cap seeds (without the 256-byte counter block).
uint64_t records_bytes(int64_t cap);
// Bits per axis of the spatial sort key for nsets sets (set index above a
// 3-axis Morton index, 32 bits in all).
int spatial_bits_for(int nsets);
int set_bits_for(int nsets);
// Stable LSD radix sort of n (*n_dev, at most n_max) uint32 keys with int32
// values, key_bits low bits, 8 per pass; cnt holds sort_count_words(n_max)
// words, scan_tmp scan_tmp_words(sort_count_words(n_max)), n_cnt two int64.
int64_t sort_count_words(int64_t n_max);
void launch_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int32_t *cnt,
                       int64_t *scan_tmp, int64_t *n_cnt, const int64_t *n_dev, int64_t n_max, int key_bits,
                       hipStream_t st);
// The same with uint64 keys.
void launch_sort_pairs64(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, int32_t *cnt,
                         int64_t *scan_tmp, int64_t *n_cnt, const int64_t *n_dev, int64_t n_max, int key_bits,
                         hipStream_t st);
// Exclusive scan of n int32 values (n from *n_dev, at most n_max) into off and
// the total into *total; tmp holds scan_tmp_words(n_max) int64 words.
int64_t scan_tmp_words(int64_t n_max);
void launch_scan_i32(const int32_t *v, const int64_t *n_dev, int64_t n_max, int64_t *tmp, int32_t *off,
                     int64_t *total, hipStream_t st);
// Carve records + counter out of a scratch block (256-byte aligned).
void carve_records(void *scratch, int64_t cap, Records *rec, unsigned long long **counter);

// The same for a higher interpolation order, one field: MODE = job.mode =
// interpolation mode | (order - 1) << 1, 2..5 (instantiated in trace_o*.hip).
template <int MODE>
hipError_t launch_trace_mode(const TraceJob &job, int step_dtype, hipStream_t stream);
// Enqueue the whole trace (work-counter reset, stepping, FP64 landing, FP64 Q assembly).
hipError_t launch_trace(const TraceJob &job, int step_dtype, hipStream_t stream);
// Batched trace: writes the host set table into job.sets (device) with small
// kernels, then the same passes over all sets' seeds with one stepping launch.
// job.n_host is the total seed count, job.rec.cap >= it.
hipError_t launch_trace_batch(const TraceJob &job, const SetDesc *host_sets, int nsets, int step_dtype,
                              hipStream_t stream);

// Field preparation.
// Internal mode of a trace job: the field's interpolation mode in bit 0, its
// interpolation order - 1 in bits 1-2, and bit 3 for the general geometry
// (spherical coordinates or rectilinear axes).
inline int job_mode(const qsq_field *f)
{
    const int order = f->order > 1 ? f->order : 1;
    const bool geo = f->geometry != QSQ_GEOMETRY_CARTESIAN || f->coords[0] || f->coords[1] || f->coords[2];
    return f->mode | ((order - 1) << 1) | (geo ? 8 : 0);
}
// Cell records (8 corner records per cell) copied from a prepared field's nodes.
uint64_t cell_record_bytes(const qsq_grid *g, int storage);
hipError_t launch_cell_records(const qsq_field *f, void *ws, hipStream_t st);
// Brick records (2 x 2 x 2 node bricks) copied from a prepared field's nodes.
uint64_t brick_record_bytes(const qsq_grid *g, int storage);
hipError_t launch_brick_records(const qsq_field *f, void *ws, hipStream_t st);
uint64_t cell_dir_bytes(const qsq_grid *g);
hipError_t launch_cell_dirs(const qsq_field *f, void *ws, hipStream_t st);
hipError_t launch_field_init(const qsq_grid *g, const void *bx, const void *by, const void *bz,
                             int in_dtype, int storage, int mode, void *ws, hipStream_t stream);

// Maps.
hipError_t launch_fledge(const float *in, int ndim, const int64_t *shape, float *out, hipStream_t stream);
hipError_t launch_hilbert2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, hipStream_t s);
hipError_t launch_hilbert2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d, hipStream_t s);

hipError_t launch_hilbert3_d2xyz(int b, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, uint32_t *z,
                                 hipStream_t s);
hipError_t launch_hilbert3_xyz2d(int b, const uint32_t *x, const uint32_t *y, const uint32_t *z, int64_t n,
                                 uint64_t *d, hipStream_t s);

uint64_t qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity);
uint64_t vmap_scratch_bytes(const qsq_volume_desc *d, int64_t capacity);
hipError_t launch_vmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_volume_desc *d, const qsq_map_out *out, void *scratch, hipStream_t stream);
hipError_t launch_qmap(const qsq_field *f, const Geom &g, const StepOpts &o, int step_dtype,
                       const qsq_map_desc *d, const qsq_map_out *out, void *scratch, hipStream_t stream);

int device_cu_count();

// Learned refinement proposer (cnn.hip).
uint64_t cnn_prep_bytes();
uint64_t cnn_workspace_bytes(int64_t n, int h, int w);
uint64_t cnn_wgrad_scratch_bytes(int64_t n, int h, int w);
hipError_t cnn_prepare(const float *params, void *prep, hipStream_t st);
hipError_t cnn_forward(const void *prep, const float *x, int64_t n, int h, int w, float *out, void *ws, hipStream_t st);
hipError_t cnn_train_step(float *params, float *adam_m, float *adam_v, int64_t t, float lr, const float *x,
                          const float *mask, const float *logq, int64_t n, int h, int w, float lam, void *prep,
                          float *grad_out, double *loss_out, void *ws, hipStream_t st);
hipError_t cnn_layer_forward(int l, const void *prep, const void *in, int64_t n, int h, int w, float *out_f32,
                             uint16_t *out_bf, hipStream_t st);
hipError_t cnn_layer_backward(int l, const void *prep, const void *in, const uint16_t *dy, int64_t n, int h, int w,
                              float *dw, float *db, float *dx_f32, uint16_t *dx_masked, const uint16_t *mask_cm,
                              void *scratch, hipStream_t st);

}  // namespace qsq
