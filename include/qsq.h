/*
 * qsq.h -- C-ABI of libqsq, an MI355X (gfx950) field-line tracer computing the
 * squashing factor Q, field-line lengths and FLEDGE maps of a gridded 3D
 * magnetic field (Tassev & Savcheva 2017, "QSL Squasher", arXiv:1609.00724).
 *
 * Conventions for every entry point
 *   - Plain C types only.  "device" pointers are HIP device memory on the
 *     current device; "host" pointers are ordinary host memory.
 *   - The library never allocates device memory.  The caller passes every
 *     buffer, including the field workspace (qsq_field_bytes) and scratch
 *     (qsq_*_scratch_bytes).  Descriptors such as qsq_field point into caller
 *     memory and stay valid while that memory lives.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls only enqueue work and return; results are valid once the stream
 *     has been synchronised.  No call synchronises the host.
 *   - Return value: QSQ_OK (0) or a negative QSQ_ERR_* code.  Arguments are
 *     validated before anything is enqueued; on error nothing is enqueued and
 *     qsq_last_error() holds a message (per host thread).  Per-line outcomes
 *     never appear in the return value: they go to status arrays.
 *   - Calls on distinct streams are independent.  Two calls that share a
 *     scratch buffer must be ordered (same stream).
 *
 * Geometry: uniform Cartesian node-centred grid, x fastest.  Node (i,j,k) sits
 * at origin + (i,j,k) * spacing; the box is the closed node hull (points on a
 * face are inside).  Seeds and footpoints are FP64 in domain units; lambda is
 * the affine parameter of the field-line equation (Sect. 3.1, eq. 1), i.e. the
 * arc length measured with the interpolated unit field.
 */
#ifndef QSQ_H
#define QSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSQ_ABI_VERSION 4

/* return codes */
#define QSQ_OK 0
#define QSQ_ERR_INVALID_ARG (-1)
#define QSQ_ERR_UNSUPPORTED (-2)
#define QSQ_ERR_WORKSPACE_TOO_SMALL (-3)
#define QSQ_ERR_HIP (-4)
#define QSQ_ERR_COUNT_OVERFLOW (-5)

/* element types */
#define QSQ_F64 0
#define QSQ_F32 1
#define QSQ_BF16 2

/* how the field between nodes is formed (Sect. 3.2 and the footnote to Sect. 3.5):
 * PAPER: B is normalised on the nodes, then Bhat and |B| are interpolated
 *        trilinearly (Bhat(x) is then not exactly a unit vector);
 * INTERP_NORMALIZE: B and grad B are interpolated, then normalised. */
#define QSQ_INTERP_PAPER 0
#define QSQ_INTERP_NORMALIZE 1

/* interpolation order (Sect. 3.2): the kernel f_v of eq. (3) over a stencil of
 * 8, 27 or 64 nodes around the point's cell.  Per axis: LINEAR, the two nodes
 * of the cell; QUADRATIC, Dodgson's (1997) interpolating quadratic kernel
 * (1 - 2d^2 for |d| <= 1/2, d^2 - 5|d|/2 + 3/2 for 1/2 < |d| <= 3/2, d in
 * spacings) over the node nearest the point and its two neighbours; CUBIC,
 * Keys' (1981) cubic convolution kernel with a = -1/2 over nodes c-1 .. c+2 of
 * the cell c.  Gradients are the analytic derivatives of the kernels.  A
 * stencil node beyond the grid takes Keys' boundary value 3 f(0) - 3 f(1) +
 * f(2) (mirrored at the top end).  QUADRATIC and CUBIC need >= 4 nodes per
 * axis and FP32 or FP64 node records, and are not available in batched
 * traces; the stepping kernel then reads the nodes directly (no cell caches). */
#define QSQ_ORDER_LINEAR 1
#define QSQ_ORDER_QUADRATIC 2
#define QSQ_ORDER_CUBIC 3

/* steppers (Sect. 3.4) */
#define QSQ_STEPPER_CK54 0   /* adaptive Cash-Karp 5(4) */
#define QSQ_STEPPER_EULER 1  /* explicit Euler, fixed step h_init */

/* outcome of one half-line: the exit face (the box is left through it) or why
 * tracing stopped elsewhere */
#define QSQ_END_XLO 0
#define QSQ_END_XHI 1
#define QSQ_END_YLO 2
#define QSQ_END_YHI 3
#define QSQ_END_ZLO 4
#define QSQ_END_ZHI 5
#define QSQ_END_MAX_LENGTH 6    /* reached opts.max_length ("local Q", Sect. 3.5) */
#define QSQ_END_MAX_STEPS 7     /* reached opts.max_steps step attempts */
#define QSQ_END_NULL 8          /* |Bhat| < 1e-6: a null of the field */
#define QSQ_END_UNDERFLOW 9     /* step size fell below 1e-12 of the box extent */
#define QSQ_END_SEED_OUTSIDE 10 /* seed lies outside the closed box (or is not finite) */
#define QSQ_END_NONFINITE 11    /* a trial step's state became NaN or Inf (e.g. a non-finite
                                   node value in its cells); the end state is the last
                                   finite one */

/* per-seed status word: forward | backward << 8 | QSQ_STATUS_OPEN; OPEN is set
 * unless both ends lie on the bottom (z = min) face (open lines, Sect. 3.5) */
#define QSQ_STATUS_FWD(s) ((s) & 0xff)
#define QSQ_STATUS_BWD(s) (((s) >> 8) & 0xff)
#define QSQ_STATUS_OPEN (1 << 16)

/* trace flags */
#define QSQ_FLAG_SKIP_OPEN 1    /* write NaN Q for open lines (Sect. 3.5 switch) */

typedef struct qsq_grid {
    int64_t n[3];          /* nodes per axis, each >= 2 */
    double origin[3];      /* position of node (0,0,0) */
    double spacing[3];     /* node spacing per axis, > 0 */
} qsq_grid;

/* A prepared field: POD descriptor of caller-owned device memory. */
typedef struct qsq_field {
    qsq_grid grid;
    int32_t storage;       /* QSQ_F64, QSQ_F32 or QSQ_BF16 */
    int32_t mode;          /* QSQ_INTERP_* */
    void *nodes;           /* device: n0*n1*n2 records of 4 storage values:
                              PAPER (Bx/|B|, By/|B|, Bz/|B|, |B|),
                              INTERP_NORMALIZE (Bx, By, Bz, 0); x fastest */
    uint64_t bytes;        /* size of the node records */
    void *cells;           /* NULL, or device cell records (qsq_field_add_cells): for
                              each of the (n0-1)(n1-1)(n2-1) cells, x fastest, the
                              node records of its 8 corners (i+a, j+b, k+c) in the
                              order a + 2b + 4c, contiguous */
    uint64_t cell_bytes;   /* size of the cell records (0 without) */
    int32_t order;         /* interpolation order (Sect. 3.2, eq. 3): QSQ_ORDER_*; 0 reads as
                              trilinear.  qsq_field_init sets trilinear; a caller may
                              set another order on the descriptor afterwards */
    int32_t geometry;      /* QSQ_GEOMETRY_*; qsq_field_init sets CARTESIAN */
    const double *coords[3]; /* NULL, or device: the n[d] increasing node coordinates of a
                              rectilinear axis d (Sect. 3.2: each cell has its own span
                              h_c); grid.origin[d] and grid.origin[d] + (n[d]-1)
                              grid.spacing[d] must be its first and last coordinates
                              (the box).  qsq_field_init sets NULL */
    void *bricks;          /* NULL, or device brick records (qsq_field_add_bricks): the
                              node records in 2 x 2 x 2 bricks, bricks x fastest, node
                              (i, j, k) at ((k/2 nby + j/2) nbx + i/2) 8 + 4 (k%2) +
                              2 (j%2) + i%2 with nbx = (n0+1)/2, nby = (n1+1)/2;
                              padding nodes zero.  Read by launch gather 5 only */
    uint64_t brick_bytes;  /* size of the brick records (0 without) */
    void *dirs;            /* NULL, or device direction records (qsq_field_add_cell_dirs,
                              FP32 storage only): for each of the (n0-1)(n1-1)(n2-1)
                              cells, x fastest, the first 3 values of its 8 corner
                              records in the order a + 2b + 4c, 24 floats (96 bytes)
                              contiguous.  Read by launch gather 6 only */
    uint64_t dir_bytes;    /* size of the direction records (0 without) */
} qsq_field;

/* Geometry of a field (Sect. 3.1).  SPHERICAL: the grid axes are longitude phi,
 * latitude theta (radians) and radius r, the input arrays (B_phi, B_theta,
 * B_r) in the local orthonormal basis; field lines follow eq. (2), deviations
 * eq. (6)-(7) held as coordinate differences (d phi, d theta, d r), turned into
 * lengths by eq. (8) for Q; footpoints are returned in (phi, theta, r).
 * SPHERICAL fields and fields with rectilinear axes take the trilinear
 * kernel, FP32 or FP64 node records and the CK54 stepper, one field per call;
 * they are stepped in physical coordinates by a kernel of their own.  h_init
 * and h_max (arc length) should be given explicitly for spherical grids. */
#define QSQ_GEOMETRY_CARTESIAN 0
#define QSQ_GEOMETRY_SPHERICAL 1

typedef struct qsq_trace_opts {
    int32_t stepper;       /* QSQ_STEPPER_CK54, or QSQ_STEPPER_EULER: fixed steps
                              h_init (0: one fifth of the smallest grid
                              spacing) of the line and both deviation
                              vectors, one field evaluation per step, no error
                              control (rtol and atol are validated but unused,
                              h_max unused); the step that leaves the box is
                              cut where it meets the first face it crosses */
    int32_t step_dtype;    /* QSQ_F32: stage arithmetic in FP32, position and
                              length accumulated in FP64; QSQ_F64: all FP64.
                              Boundary landing and Q assembly are always FP64. */
    double rtol, atol;     /* error control per state component (> 0) */
    double h_init;         /* first trial step; <= 0: 0.1 * min spacing */
    double h_max;          /* largest step; <= 0: min spacing */
    double max_length;     /* <= 0: unlimited; else stop each half-line there */
    int64_t max_steps;     /* step attempts per half-line; <= 0: 1 << 22 */
    int32_t flags;         /* QSQ_FLAG_* */
    int32_t launch;        /* launch shape of the stepping kernel, QSQ_LAUNCH(...);
                              0 = library defaults.  Results do not depend on it
                              (each line's arithmetic is the same in every shape). */
} qsq_trace_opts;

/* Launch-shape word of qsq_trace_opts.launch (what an autotuner varies):
 *   lanes  resident-lane target of the persistent stepping launch, in units of
 *          256 lanes per compute unit, 1..15 (0: 8)
 *   wg     workgroup size code: 0 = 256, 1 = 64, 2 = 128 lanes
 *   gather 0 = automatic (3 where it applies, otherwise 1),
 *          1 = direct corner loads, 2 = per-lane LDS cache of
 *          the last cell's corners (FP32 or BF16 records and FP32 stepping,
 *          one field per call, field below 2 GiB; otherwise direct),
 *          3 = per-lane register cache of the last cell's corners (same
 *          conditions as 2; results identical to direct loads bit for bit),
 *          4 = direct loads of the cell's corners from the field's cell
 *          records (FP32 or BF16 storage, FP32 stepping, one field per call,
 *          field with cell records; otherwise direct; identical results),
 *          5 = the register cache of 3 reading the field's brick records (same
 *          conditions as 3, field with brick records; otherwise as 3;
 *          identical results),
 *          6 = the register cache of 3 reading the field's direction records
 *          (FP32 storage and stepping, one field per call, field with
 *          direction records, fewer than 2^31 cells; otherwise as 3;
 *          identical results)
 * and the flag
 *   QSQ_LAUNCH_PARTS  split the work list of the persistent stepping launch
 *          into 8 contiguous parts with a counter each; workgroup b starts in
 *          part b mod 8 (the XCD it is dispatched to, so that one XCD's L2
 *          serves lines whose seeds lie together) and moves on to the other
 *          parts once its own is used up (scheduling only: identical results)
 * and, read by qsq_qmap and qsq_vmap only (other calls ignore it),
 *   QSQ_LAUNCH_REFINE_GATHER(g)  gather (1..6, as above) of every stepping
 *          launch after the base lattice (proposals, refinement rounds,
 *          shifted re-pass); 0 (default): the word's gather.  The base
 *          lattice and the sparser refinement lines differ in how often lines
 *          in flight share cells, so each may want its own record layout
 *          (identical results) */
#define QSQ_LAUNCH(lanes, wg, gather) (((lanes) & 15) | (((wg) & 3) << 4) | (((gather) & 7) << 6))
#define QSQ_LAUNCH_PARTS (1 << 9)
#define QSQ_LAUNCH_REFINE_GATHER(g) (((g) & 7) << 10)

/* Per-seed results (device arrays of n entries; fp_* are SoA planes 3 x n:
 * x at [0,n), y at [n,2n), z at [2n,3n)).  Any pointer except status may be
 * NULL to skip that output. */
typedef struct qsq_trace_out {
    double *fp_fwd;        /* forward end point x(lambda_F) */
    double *fp_bwd;        /* backward end point x(lambda_B) */
    double *fll;           /* field-line length lambda_F - lambda_B */
    double *q_perp;        /* Q of eq. (11) (perpendicular planes, |B| ratios) */
    double *q_det;         /* same planes, determinant form (flux ratios exact) */
    double *q_fp;          /* Q in the exit-face planes (NaN unless both ends are faces) */
    int32_t *status;       /* status word, see QSQ_STATUS_* (required) */
    int32_t *steps;        /* 2 x n: step attempts, forward at [0,n), backward at [n,2n) */
    uint64_t *work;        /* 4 device counters the call adds to (caller zeroes them):
                              step attempts, RHS evaluations and half-lines of the
                              stepping kernel, and half-lines handed to FP64 landing */
} qsq_trace_out;

/* ---- library ---------------------------------------------------------- */

/* QSQ_ABI_VERSION of the built library. */
int qsq_abi_version(void);

/* Static description of a QSQ_END_* code or a QSQ_ERR_* return code. */
const char *qsq_status_string(int code);

/* Message of the last failed call on this host thread ("" if none). */
const char *qsq_last_error(void);

/* ---- field preparation (Sect. 3.2; footnote to Sect. 3.5) ------------- */

/* Bytes of node records for grid g at the given storage type. */
uint64_t qsq_field_bytes(const qsq_grid *g, int storage);

/*
 * Prepare a field from three device arrays of node values (x fastest,
 * n0*n1*n2 each, type `in_dtype` = QSQ_F64 or QSQ_F32) into `ws` (device,
 * >= qsq_field_bytes, 16-byte aligned).  PAPER mode stores Bhat = B/|B| (0 where
 * |B| < 1e-30) and |B| per node; INTERP_NORMALIZE stores B.  Values are
 * formed in FP64 and rounded to the storage type (BF16: to FP32, then to the
 * nearest BF16, ties to even; 8 bytes per node).  Fills *out.
 * Errors: INVALID_ARG (null pointers, n < 2, spacing <= 0, bad enums),
 * WORKSPACE_TOO_SMALL, UNSUPPORTED (storage other than F64/F32/BF16), HIP.
 */
int qsq_field_init(const qsq_grid *g, const void *bx, const void *by, const void *bz,
                   int in_dtype, int storage, int mode, void *ws, uint64_t ws_bytes,
                   void *stream, qsq_field *out);

/* Bytes of cell records for grid g at the given storage type:
 * 8 node records per cell, (n0-1)(n1-1)(n2-1) cells. */
uint64_t qsq_field_cell_bytes(const qsq_grid *g, int storage);

/*
 * Add cell records to a prepared field (Sect. 3.2: the trilinear stencil of a
 * cell is its 8 corner nodes): for every cell the records of its 8 corners,
 * copied from f->nodes into `ws` (device, >= qsq_field_cell_bytes, 256-byte
 * aligned), so that one evaluation reads one contiguous block (128 bytes for
 * FP32 records) instead of four pairs of records in four node rows.  The
 * stepping kernel reads them with launch gather 4; the values, and so every
 * result, are those of the node records.  Sets f->cells and f->cell_bytes.
 * Errors: INVALID_ARG (f invalid, ws NULL or misaligned), WORKSPACE_TOO_SMALL,
 * HIP.
 */
int qsq_field_add_cells(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream);

/* Bytes of brick records for grid g at the given storage type: 8 node records
 * per brick, ((n0+1)/2)((n1+1)/2)((n2+1)/2) bricks. */
uint64_t qsq_field_brick_bytes(const qsq_grid *g, int storage);

/*
 * Add brick records to a prepared field: the node records reordered into
 * 2 x 2 x 2 bricks (layout at qsq_field.bricks) in `ws` (device, >=
 * qsq_field_brick_bytes, 256-byte aligned), so that the 8 corners of a cell
 * (Sect. 3.2) touch fewer cache lines (a brick of FP32 records is one
 * 128-byte line); the stepping kernel reads them with
 * launch gather 5, every other pass reads f->nodes; the values, and so every
 * result, are those of the node records.  Trilinear Cartesian fields with
 * uniform axes only.  Sets f->bricks and f->brick_bytes.  Errors: INVALID_ARG
 * (f invalid, ws NULL or misaligned), UNSUPPORTED (higher order, spherical or
 * rectilinear field), WORKSPACE_TOO_SMALL, HIP.
 */
int qsq_field_add_bricks(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream);

/* Bytes of direction records for grid g: 96 per cell for FP32 storage, 0 for
 * any other storage (not offered). */
uint64_t qsq_field_cell_dir_bytes(const qsq_grid *g, int storage);

/*
 * Add direction records to a prepared FP32 field: for each cell the direction
 * part (first 3 values) of its 8 corner records (Sect. 3.2), 96 contiguous
 * bytes (layout at qsq_field.dirs), in `ws` (device, >=
 * qsq_field_cell_dir_bytes, 256-byte aligned), so that the stepping kernel's
 * register cache (launch gather 6) loads a cell in six 16-byte loads from at
 * most two 128-byte lines; every other pass reads f->nodes, and the values,
 * so every result, are those of the node records.  FP32 trilinear Cartesian
 * fields with uniform axes only.  Sets f->dirs and f->dir_bytes.  Errors:
 * INVALID_ARG (f invalid, ws NULL or misaligned), UNSUPPORTED (other storage,
 * higher order, spherical or rectilinear field), WORKSPACE_TOO_SMALL, HIP.
 */
int qsq_field_add_cell_dirs(qsq_field *f, void *ws, uint64_t ws_bytes, void *stream);

/* ---- tracing (Sect. 3.1-3.5) ------------------------------------------ */

/* Scratch bytes qsq_trace needs for n seeds. */
uint64_t qsq_trace_scratch_bytes(int64_t n);

/*
 * Trace n seeds both ways to the boundary and assemble Q and lengths.
 * seeds: device FP64, SoA 3 x n.  For each seed x0: u0 = Bhat(x0)/|Bhat(x0)|,
 * an orthonormal (a, b) completing u0 (eq. 9); integrate x, dx1 = a, dx2 = b
 * with eq. (1) and eq. (5) forwards and backwards (Cash-Karp 5(4) with
 * adaptive steps) until the box is left (landing exactly on the face crossed
 * first), max_length, max_steps, a null or a non-finite state; then Q by
 * eq. (10)-(11).  The half-lines are stepped in spatial order (sorted by the
 * Morton index of their seed's cell; outputs stay in seed order and do not
 * depend on that order).  scratch: device, >= qsq_trace_scratch_bytes(n),
 * 256-byte aligned.  n = 0 enqueues nothing and succeeds.  Errors: INVALID_ARG,
 * UNSUPPORTED, WORKSPACE_TOO_SMALL, COUNT_OVERFLOW (n > 2^30), HIP.
 */
int qsq_trace(const qsq_field *f, const double *seeds, int64_t n, const qsq_trace_opts *opts,
              const qsq_trace_out *out, void *scratch, uint64_t scratch_bytes, void *stream);

/* ---- tracing without allocation ---------------------------------------- */

#define QSQ_TRACE_NOALLOC_MAX_SEEDS (1 << 18)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qsq_trace
 * with its scratch in a fixed 64 MiB device array owned by the library (one
 * copy per device, held until the process ends) instead of a caller buffer.
 * The caller still passes the field, seeds and outputs; the call allocates
 * nothing and computes exactly what qsq_trace computes.  At most
 * QSQ_TRACE_NOALLOC_MAX_SEEDS seeds per call (WORKSPACE_TOO_SMALL beyond).
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (different streams or host threads without ordering)
 * race and give undefined results; calls on one stream are ordered and safe.
 * The first call on a device looks up the array's address there.  Errors: as
 * qsq_trace, plus WORKSPACE_TOO_SMALL for n above the limit.
 */
int qsq_trace_noalloc(const qsq_field *f, const double *seeds, int64_t n, const qsq_trace_opts *opts,
                      const qsq_trace_out *out, void *stream);

/* ---- batched trace ------------------------------------------------------ */

/* One seed set of a batched trace: a prepared field, its seeds and outputs. */
typedef struct qsq_trace_set {
    qsq_field field;       /* prepared by qsq_field_init; every set of a call has
                              the same storage and mode (grids may differ) */
    const double *seeds;   /* device FP64, SoA 3 x n */
    int64_t n;             /* seeds of the set, >= 0 */
    qsq_trace_out out;     /* results of the set's seeds (n entries, as for
                              qsq_trace); out.work is ignored */
} qsq_trace_set;

#define QSQ_MAX_TRACE_SETS 65536

/* Scratch bytes qsq_trace_batch needs for nsets sets of `total` seeds in all. */
uint64_t qsq_trace_batch_scratch_bytes(int32_t nsets, int64_t total);

/*
 * Trace many seed sets, each in its own field, as one job: the same per-seed
 * computation as qsq_trace (Sect. 3.1-3.5, eq. (1), (5), (9)-(11)), with the
 * half-lines of all sets served from one work list to one persistent stepping
 * launch, so that sets of uneven size and line length share the device.
 * The work list is sorted by (set, Morton index of the seed's cell) so that
 * neighbouring lanes trace neighbouring lines; outputs stay in seed order.
 * sets: host array of nsets entries (1 <= nsets <= QSQ_MAX_TRACE_SETS), read
 * during the call only.  opts applies to every set, except that h_init <= 0
 * and h_max <= 0 select 0.1 and 1 times each set's own smallest spacing.
 * work: NULL or 4 device counters as in qsq_trace_out.work, summed over the
 * batch.  scratch: device, >= qsq_trace_batch_scratch_bytes(nsets, total),
 * 256-byte aligned.  The call enqueues kernel launches only (no memory
 * copies or fills), so it can be captured in a HIP graph and replayed while
 * sets, seeds, outputs and scratch stay at the same addresses.  Sets with
 * n = 0 are skipped; a batch with no seeds enqueues nothing.  Errors:
 * INVALID_ARG (naming the set), UNSUPPORTED, WORKSPACE_TOO_SMALL,
 * COUNT_OVERFLOW (more than 2^30 seeds in all), HIP.
 */
int qsq_trace_batch(const qsq_trace_set *sets, int32_t nsets, const qsq_trace_opts *opts, uint64_t *work,
                    void *scratch, uint64_t scratch_bytes, void *stream);

/* ---- FLEDGE (Sect. 3.6) ------------------------------------------------ */

/*
 * FLEDGE map: Sobel gradient magnitude sqrt(sum_d G_d^2) of a 2D or 3D FP32
 * map (device, C order, last axis fastest), derivative [-1, 0, 1] along axis d
 * convolved with [1, 2, 1] along the others, mirror boundary (d c b a | a b c
 * d), pixel units.  `in` and `out` must not overlap.  shape: host, ndim
 * entries, each >= 1.  Errors: INVALID_ARG, HIP.
 */
int qsq_fledge(const float *in, int ndim, const int64_t *shape, float *out, void *stream);

/* ---- Hilbert ordering (Sect. 3.6) -------------------------------------- */

/*
 * Order-L Hilbert curve on a 2^L x 2^L slice (1 <= L <= 31).  The curve starts
 * at cell (0,0) and ends at (2^L-1, 0); the order-1 curve visits (0,0), (0,1),
 * (1,1), (1,0), and the order-L curve visits the four quadrants in that order,
 * holding the order L-1 curve reflected in the diagonal, translated, translated,
 * and reflected in the anti-diagonal.  d2xy maps n curve indices to cells, xy2d
 * the reverse (device arrays).
 */
int qsq_hilbert2_d2xy(int L, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, void *stream);
int qsq_hilbert2_xy2d(int L, const uint32_t *x, const uint32_t *y, int64_t n, uint64_t *d, void *stream);

/*
 * Hilbert curve on a 2^b cube (1 <= b <= 21), Skilling's transpose algorithm
 * (AIP Conf. Proc. 707, 2004): the index holds, most significant first, bit
 * b-1 of x, y, z, then bit b-2 of x, y, z, and so on; the curve starts at
 * (0,0,0) and ends at (2^b-1, 0, 0).  Device arrays of n entries.
 */
int qsq_hilbert3_d2xyz(int b, const uint64_t *d, int64_t n, uint32_t *x, uint32_t *y, uint32_t *z, void *stream);
int qsq_hilbert3_xyz2d(int b, const uint32_t *x, const uint32_t *y, const uint32_t *z, int64_t n, uint64_t *d,
                       void *stream);

/* ---- adaptive map of a slice (Sect. 3.6) -------------------------------- */

typedef struct qsq_map_desc {
    double z0;             /* horizontal slice z = z0 ... */
    double x0, x1, y0, y1; /* ... over [x0, x1] x [y0, y1] */
    int32_t base_level;    /* m: 2^m x 2^m base pixels, sampled at centres */
    int32_t refine_levels; /* r: finest cells are 2^(m+r) per side (m + r <= 16) */
    int32_t out_level;     /* level of the output grids, m <= out_level <= m + r */
    int32_t refine_batch;  /* refinement levels decided per device round, 1..5 (see
                              qsq_qmap); <= 0: min(2r, 4) */
    double threshold;      /* FLL jump that triggers a new sample (length units) */
    const uint8_t *propose; /* NULL, or device bytes, one per base pixel in level-m
                              curve order: a nonzero byte adds every finest cell
                              of that pixel as a sample before the FLL-jump rule
                              runs (proposals of a learned or external model);
                              the rule then refines what is left (fallback) */
    int32_t shift;         /* 0, or the shifted-curve re-pass (Sect. 3.6, last paragraph):
                              after every pass of the rule along the curve, one pass
                              along the curve shifted by `shift` finest cells per
                              axis (0 < shift < 2^(m+r); see qsq_qmap) */
    int32_t max_cycles;    /* with shift: at most this many cycles (1..48; <= 0: 48) */
    int32_t tilted;        /* 0: the horizontal slice above; 1: the planar slice of any
                              orientation corner + s edge_u + t edge_v, s, t in [0, 1]
                              (Sect. 2), pixel (i, j) of level L at s = (i + 1/2) / 2^L,
                              t = (j + 1/2) / 2^L (z0, x0, x1, y0, y1 unused) */
    int32_t base_given;    /* 1: out->fll, q_perp and status (and steps) already hold the
                              base lattice's 4^m samples in level-m curve order -- e.g. a
                              map of the same slice with refine_levels 0 -- and are not
                              traced again; their keys are rewritten to q 4^r + 4^r/2 */
    double corner[3], edge_u[3], edge_v[3];
} qsq_map_desc;

/* Results of qsq_qmap (device memory).  Samples are kept in curve order. */
typedef struct qsq_map_out {
    int64_t capacity;      /* entries available in each sample array (>= 4^m; 8^m for volumes;
                              at most 2^30) */
    uint64_t *keys;        /* finest-level curve index of each sample */
    double *fll;           /* field-line length per sample */
    double *q_perp;        /* Q of eq. (11) per sample */
    int32_t *status;       /* status word per sample */
    int64_t *count;        /* device scalar: samples held (<= capacity) */
    int32_t *overflow;     /* device scalar: bit 0 set if refinement wanted more than
                              capacity; bit 1 set if the shifted re-pass was still
                              inserting samples in its last cycle */
    float *q_grid;         /* 2^out_level squared, row y: max Q per cell, gaps filled
                              by log Q interpolated along the curve; NULL: skip */
    float *fll_grid;       /* same for the length (linear gap fill); NULL: skip */
    float *fledge;         /* 2^m squared: Sobel FLEDGE of the base length map; NULL: skip */
    uint64_t *work;        /* as qsq_trace_out.work, summed over every pass; NULL: skip */
    int32_t *steps;        /* NULL, or capacity entries: step attempts of each kept
                              sample's line (forward + backward), in sample order;
                              lines traced and then dropped by the rule count in
                              `work` only */
} qsq_map_out;

/* Scratch bytes qsq_qmap needs for a map with `capacity` samples. */
uint64_t qsq_qmap_scratch_bytes(const qsq_map_desc *d, int64_t capacity);

/*
 * Q / length / FLEDGE map of a horizontal slice with FLL-jump refinement along
 * the Hilbert curve (Sect. 3.6).  Base samples: the 2^m x 2^m pixel centres,
 * in level-m curve order q, with key q*4^r + 4^r/2.  Each pass inserts, between
 * curve-successive samples whose keys differ by >= 2 and whose lengths differ
 * by more than `threshold`, a sample at key floor((k1+k2)/2), placed at the
 * centre of that finest cell; passes repeat (2r of them at most) until none
 * fires.  The samples kept are exactly those of that pass-by-pass rule; the
 * device decides `refine_batch` passes per round by tracing, for every gap
 * that fires, all 2^b - 1 keys the next b passes could insert into it and then
 * applying the rule to the traced values (fewer, larger launches; the keys
 * the rule rejects are traced but not kept).  All rounds run on the device
 * without host synchronisation.  With `propose`, the finest cells of the
 * proposed pixels are traced and merged in key order after the base lattice;
 * the rule then runs one pass per round on the (now irregular) gaps, the new
 * key of a firing gap always being floor((k1+k2)/2).  Samples beyond
 * `capacity`, or proposed or speculative keys beyond the trace slots
 * (`capacity`), are dropped and set *overflow.
 * With `shift` > 0 (the shifted-curve re-pass, Sect. 3.6, last paragraph)
 * refinement runs in cycles: one pass of the rule along the curve (one new key
 * floor((k1+k2)/2) per firing gap), then one pass along a shifted curve -- each
 * sample's finest cell moved by `shift` cells along every axis into the square
 * of side 2^(m+r+1) and ordered by that square's order-(m+r+1) Hilbert index;
 * successive samples of that order whose indices differ by >= 2 and whose
 * lengths differ by more than `threshold` add a sample in the cell of index
 * floor((k1'+k2')/2), moved back by `shift`, if it lies inside the map.
 * Cycles repeat until one inserts nothing (at most max_cycles; bit 1 of
 * *overflow if the last one still inserted).  refine_batch is ignored, and
 * `propose` must be NULL (UNSUPPORTED otherwise).
 * Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE_TOO_SMALL, COUNT_OVERFLOW
 * (capacity > 2^30), HIP.
 */
int qsq_qmap(const qsq_field *f, const qsq_map_desc *d, const qsq_trace_opts *opts,
             const qsq_map_out *out, void *scratch, uint64_t scratch_bytes, void *stream);

/* ---- adaptive map of a volume (Sect. 3.6, 3D maps) ---------------------- */

typedef struct qsq_volume_desc {
    double x0, x1, y0, y1, z0, z1; /* axis-aligned volume */
    int32_t base_level;    /* m: 2^m cells per axis, sampled at centres */
    int32_t refine_levels; /* r: finest cells are 2^(m+r) per axis (m + r <= 21) */
    int32_t out_level;     /* level of the output grids, m <= out_level <= m + r */
    int32_t refine_batch;  /* as in qsq_map_desc; <= 0: 1 */
    double threshold;      /* FLL jump that triggers a new sample (length units) */
    const uint8_t *propose; /* as in qsq_map_desc, one byte per base cell (8^m) */
    int32_t shift;         /* as in qsq_map_desc, on the 3D curve */
    int32_t max_cycles;    /* as in qsq_map_desc */
} qsq_volume_desc;

/* Scratch bytes qsq_vmap needs for a map with `capacity` samples. */
uint64_t qsq_vmap_scratch_bytes(const qsq_volume_desc *d, int64_t capacity);

/*
 * Q / length / FLEDGE map of a volume: qsq_qmap's rule on the 3D Hilbert curve
 * (qsq_hilbert3_*).  Base samples: the (2^m)^3 cell centres in level-m curve
 * order q with key q*8^r + 8^r/2; the key gap halves over 3r passes.  Output
 * grids are (2^out_level)^3 and the FLEDGE map (2^m)^3, C order [z][y][x];
 * capacity >= 8^m.  Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE_TOO_SMALL,
 * COUNT_OVERFLOW (capacity > 2^30), HIP.
 */
int qsq_vmap(const qsq_field *f, const qsq_volume_desc *d, const qsq_trace_opts *opts,
             const qsq_map_out *out, void *scratch, uint64_t scratch_bytes, void *stream);

/* ---- measurement -------------------------------------------------------- */

/* kernels the profiler times */
#define QSQ_KERNEL_STEP 0       /* adaptive stepping kernel */
#define QSQ_KERNEL_LAND 1       /* FP64 boundary landing */
#define QSQ_KERNEL_ASSEMBLE 2   /* FP64 Q assembly */

/*
 * Kernel timing for benchmarks.  While enabled (process-wide), every launch of
 * the kernels above is bracketed by two HIP events recorded on the launch's
 * own stream.  qsq_profile_read waits for the recorded events and returns the
 * number of launches of `kernel` since the last reset and their summed
 * duration in milliseconds; qsq_profile_reset releases the events.  Not for
 * use while another thread is launching.  Errors: INVALID_ARG, HIP.
 */
int qsq_profile_enable(int on);
int qsq_profile_reset(void);
int qsq_profile_read(int kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* QSQ_H */
