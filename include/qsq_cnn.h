/*
 * qsq_cnn.h -- C-ABI of libqsq's learned refinement proposer.
 *
 * An extension beyond the paper (QSL Squasher, arXiv:1609.00724): a small
 * convolutional network reads coarse tiles of three maps the method makes --
 * field-line length, its FLEDGE map (Sect. 3.6) and Bz on the slice -- and
 * proposes which coarse pixels the refinement of Sect. 3.6 should refine; the
 * FLL-jump rule stays the fallback and scores the proposals.
 *
 * Network: four 3x3 'same' convolutions (zero padding), 3 -> 32 -> 32 -> 32 ->
 * 2 channels, FP32 bias, ReLU after the first three; output channel 0 is the
 * refine-mask logit, channel 1 the predicted log10 Q.  Contractions run on
 * the matrix cores with BF16 operands and FP32 accumulation; hidden
 * activations are stored in BF16.
 *
 * Conventions as in qsq.h (plain pointers, caller-owned device buffers, calls
 * only enqueue on `stream`, QSQ_OK or a negative QSQ_ERR_* code).
 *
 * Layouts
 *   params  FP32 master parameters, QSQ_CNN_PARAMS floats: for each layer l,
 *           W_l as (3, 3, Ci, Co) row-major -- tap (dy, dx) multiplies the
 *           input at (y + dy - 1, x + dx - 1) -- followed by b_l (Co)
 *   prep    the device-side prepared weights (BF16 matrices in matrix-core
 *           order, FP32 biases), qsq_cnn_prep_bytes() bytes, filled by
 *           qsq_cnn_prepare from params
 *   x       input tiles, FP32 NHWC (n, h, w, 3)
 *   out     FP32 NHWC (n, h, w, 2)
 *   acts    BF16 (raw 16-bit) NHWC with 32 channels
 *   h, w    multiples of 32 (tiles of 64 x 64 in practice); n * h * w < 2^31
 *           and h * w <= 2^24 (a tile's tensors are addressed with 32-bit
 *           byte offsets); otherwise QSQ_ERR_COUNT_OVERFLOW
 */
#ifndef QSQ_CNN_H
#define QSQ_CNN_H

#include <stdint.h>

#include "qsq.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QSQ_CNN_PARAMS 19970

/* Bytes of the prepared weights. */
uint64_t qsq_cnn_prep_bytes(void);

/* Convert FP32 master params (device) into prepared weights (device). */
int qsq_cnn_prepare(const float *params, void *prep, void *stream);

/* Workspace bytes of qsq_cnn_forward / qsq_cnn_train_step for n tiles of h x w. */
uint64_t qsq_cnn_workspace_bytes(int64_t n, int h, int w);

/* Scratch bytes of qsq_cnn_layer_backward for n tiles of h x w. */
uint64_t qsq_cnn_layer_scratch_bytes(int64_t n, int h, int w);

/*
 * Whole network forward: out = net(x).  ws: >= qsq_cnn_workspace_bytes,
 * 256-byte aligned (holds the hidden activations).  Errors: INVALID_ARG,
 * WORKSPACE_TOO_SMALL, HIP.
 */
int qsq_cnn_forward(const void *prep, const float *x, int64_t n, int h, int w, float *out, void *ws,
                    uint64_t ws_bytes, void *stream);

/*
 * One training step on a batch: forward; loss = mean over pixels of the
 * logistic loss of the mask logit against mask (0 or 1) plus lam times the
 * mean squared error of the log10 Q output against logq over pixels whose
 * logq is finite; backward through all layers (the output gradient and the
 * hidden gradients rounded to BF16 as matrix-core operands); one Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, step t >= 1) of params with adam_m and
 * adam_v (FP32, QSQ_CNN_PARAMS each, zero before step 1).  prep must hold
 * qsq_cnn_prepare(params) on entry (the forward pass reads it); the update
 * rewrites the entries of prep that the changed params feed, so it again
 * equals qsq_cnn_prepare(params) on return.  mask, logq: FP32 (n, h, w).
 * grad_out: NULL or QSQ_CNN_PARAMS floats receiving the gradient (params
 * layout).  loss_out: NULL or one device double receiving the loss before
 * the update.
 */
int qsq_cnn_train_step(float *params, float *adam_m, float *adam_v, int64_t t, float lr, const float *x,
                       const float *mask, const float *logq, int64_t n, int h, int w, float lam, void *prep,
                       float *grad_out, double *loss_out, void *ws, uint64_t ws_bytes, void *stream);

/*
 * One layer (0..3) alone, for checking.  layer_forward: in is x (FP32, 3
 * channels) for layer 0, else BF16 activations (32 channels); out_f32 gets
 * ReLU(conv + b) (no ReLU for layer 3) in FP32 before any rounding, Co
 * channels.  layer_backward: given dy = dL/d(layer output) (BF16, Co
 * channels), writes dw (9 Ci Co floats, params layout), db (Co) and, for
 * layers 1..3 if dx is not NULL, dx = dL/d(layer input) in FP32 (32 channels,
 * no ReLU mask).  scratch: >= qsq_cnn_layer_scratch_bytes.
 */
int qsq_cnn_layer_forward(int layer, const void *prep, const void *in, int64_t n, int h, int w, float *out_f32,
                          void *stream);
int qsq_cnn_layer_backward(int layer, const void *prep, const void *in, const uint16_t *dy, int64_t n, int h, int w,
                           float *dw, float *db, float *dx, void *scratch, uint64_t scratch_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QSQ_CNN_H */
