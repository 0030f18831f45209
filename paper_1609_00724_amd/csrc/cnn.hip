// Learned refinement proposer on gfx950: a 4-layer 3x3 convolutional network
// (3 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the hidden layers) that reads
// coarse tiles of the field-line length, its FLEDGE map (Sect. 3.6) and Bz,
// and outputs a refine-mask logit and a log10 Q estimate per pixel.  The
// network is an extension beyond the paper; the FLL-jump rule of Sect. 3.6
// stays the fallback and the reference its proposals are scored against.
//
// Every contraction runs on the matrix cores: v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation), one wave per 16x16 output tile.
//   forward / input gradient: M = 16 pixels of a row, N = 16 output channels,
//     K = 32 (one tap's 32 input channels, or all 9 taps of a 2-3 channel
//     input packed into one chunk)
//   weight gradient: M = 16 input channels, N = 16 output channels, K = 32
//     pixels of a row; per-wave partial sums reduced in a fixed order
// Activations are BF16 NHWC with 32 channels; the network input is FP32 with
// 3 channels, the output FP32 with 2.
#include <math.h>

#include "qsq_cnn.h"
#include "qsq_internal.h"

namespace qsq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ __bf16 as_bf(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// network shape
constexpr int kCi[4] = {3, 32, 32, 32};
constexpr int kCo[4] = {32, 32, 32, 2};

__host__ __device__ constexpr int ntile(int c) { return (c + 15) / 16; }
__host__ __device__ constexpr int nchunk(int ci) { return ci >= 32 ? 9 : 1; }

// ---------------------------------------------------------------------------
// Prepared weights (BF16 matrices in MFMA-friendly order + FP32 biases)
//   fwd[l]: [nchunk(Ci)][16 ntile(Co)][32]: element (kc, co, kk) multiplies
//           input channel/tap (tap = kc, ci = kk) for Ci = 32, or
//           (tap = k / Ci, ci = k % Ci, k = kk < 9 Ci) for Ci < 32
//   bwd[l] (l >= 1): the transposed, tap-flipped kernel of the input
//           gradient, a convolution from Co channels to Ci = 32: element
//           (kc, ci, kk) = W[flip(tap)][ci][c] with (tap, c) taken from
//           (kc, kk) as above with Co in the role of Ci
// Master parameters (FP32): per layer W (3, 3, Ci, Co) row-major, then b (Co).
// ---------------------------------------------------------------------------
struct PrepLayout {
    int64_t fwd[4], bwd[4], bias[4], total_u16;
};

__host__ __device__ inline int64_t master_w(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += 9 * kCi[k] * kCo[k] + kCo[k];
    return o;
}

__host__ __device__ inline PrepLayout prep_layout()
{
    PrepLayout p{};
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
        p.fwd[l] = o;
        o += (int64_t)nchunk(kCi[l]) * 16 * ntile(kCo[l]) * 32;
    }
    for (int l = 0; l < 4; ++l) {
        p.bwd[l] = o;
        if (l >= 1) o += (int64_t)nchunk(kCo[l]) * 32 * 32;
    }
    o = (o + 127) & ~(int64_t)127;
    for (int l = 0; l < 4; ++l) {
        p.bias[l] = o;      // FP32 biases stored in u16 units (2 per float)
        o += 2 * 32;
    }
    p.total_u16 = o;
    return p;
}

__global__ void k_prepare(const float *params, uint16_t *prep)
{
    const PrepLayout P = prep_layout();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // forward matrices
    for (int l = 0; l < 4; ++l) {
        const int Ci = kCi[l], Co = kCo[l], COP = 16 * ntile(Co), NK = nchunk(Ci);
        const int64_t N = (int64_t)NK * COP * 32;
        const float *W = params + master_w(l);
        for (int64_t e = t; e < N; e += (int64_t)gridDim.x * blockDim.x) {
            const int kk = (int)(e % 32), co = (int)((e / 32) % COP), kc = (int)(e / (32 * COP));
            int tap, ci;
            if (Ci >= 32) {
                tap = kc;
                ci = kk;
            } else {
                tap = kk / Ci;
                ci = kk % Ci;
            }
            const bool ok = co < Co && tap < 9;
            prep[P.fwd[l] + e] = ok ? f2bf(W[((int64_t)tap * Ci + ci) * Co + co]) : (uint16_t)0;
        }
    }
    // transposed, flipped matrices of the input gradients
    for (int l = 1; l < 4; ++l) {
        const int Ci = kCi[l], Co = kCo[l], NK = nchunk(Co);
        const int64_t N = (int64_t)NK * 32 * 32;
        const float *W = params + master_w(l);
        for (int64_t e = t; e < N; e += (int64_t)gridDim.x * blockDim.x) {
            const int kk = (int)(e % 32), ci = (int)((e / 32) % 32), kc = (int)(e / (32 * 32));
            int tap, c;
            if (Co >= 32) {
                tap = kc;
                c = kk;
            } else {
                tap = kk / Co;
                c = kk % Co;
            }
            const bool ok = tap < 9 && ci < Ci;
            prep[P.bwd[l] + e] = ok ? f2bf(W[((int64_t)(8 - tap) * Ci + ci) * Co + c]) : (uint16_t)0;
        }
    }
    for (int l = 0; l < 4; ++l) {
        float *b = reinterpret_cast<float *>(prep + P.bias[l]);
        const float *src = params + master_w(l) + 9 * kCi[l] * kCo[l];
        for (int64_t e = t; e < 32; e += (int64_t)gridDim.x * blockDim.x) b[e] = e < kCo[l] ? src[e] : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// 3x3 'same' convolution, one wave per 16-pixel strip of kConvRows rows, all
// output channels.  The wave keeps the weight operands in registers for its
// rows and, for 32-channel inputs, a sliding window of the input operands
// (three rows x three pixel shifts: each new output row loads one new input
// row).  in: BF16 (32 channels) or, for CI < 32, FP32 / BF16 with CI
// channels.  Outputs (each nullable): BF16 activations (ReLU applied), FP32
// values, and a BF16 copy masked by act_mask > 0 (input gradients).
// ---------------------------------------------------------------------------
struct ConvDims {
    int64_t n;
    int h, w;
};

constexpr int kConvRows = 4;   // divides h (a multiple of 32)

template <int CI, int CO, bool SRC_F32>
__global__ void __launch_bounds__(256) k_conv(const void *in, ConvDims d, const uint16_t *wm, const float *bias,
                                              bool relu, uint16_t *out_bf, float *out_f32, uint16_t *out_masked,
                                              const uint16_t *act_mask)
{
    constexpr int NT = ntile(CO), COP = 16 * NT, NK = nchunk(CI), R = kConvRows;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int spr = d.w / 16, rb = d.h / R;
    if (wave >= d.n * rb * spr) return;   // the whole wave leaves together
    const int64_t blk = wave / spr;       // image * rb + row block
    const int x0 = (int)(wave % spr) * 16, y0 = (int)(blk % rb) * R;
    const int64_t img = blk / rb;
    const int i = lane & 15, kg = lane >> 4;
    bf16x8 bw[NK][NT];
#pragma unroll
    for (int kc = 0; kc < NK; ++kc)
#pragma unroll
        for (int t = 0; t < NT; ++t) bw[kc][t] = ld_bf16x8(wm + ((int64_t)(kc * COP + t * 16 + i) * 32 + 8 * kg));
    // A operand of one input row yy at pixel shift dx (32 channels: lane i
    // takes pixel x0 + i + dx, channels 8 kg .. 8 kg + 7)
    auto a32 = [&](int yy, int dx) {
        bf16x8 a;
        const int xx = x0 + i + dx;
        if (CI >= 32 && yy >= 0 && yy < d.h && xx >= 0 && xx < d.w) {
            a = ld_bf16x8(static_cast<const uint16_t *>(in) + (((img * d.h + yy) * d.w + xx) * 32 + 8 * kg));
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = as_bf(0);
        }
        return a;
    };
    bf16x8 win[3][3];   // [input row y-1, y, y+1][dx + 1]
    if constexpr (CI >= 32) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) win[r][dx] = a32(y0 - 1 + r, dx - 1);
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int y = y0 + rr;
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (CI >= 32) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) win[2][dx] = a32(y + 1, dx - 1);
#pragma unroll
            for (int kc = 0; kc < 9; ++kc)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma(win[kc / 3][kc % 3], bw[kc][t], acc[t]);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                win[0][dx] = win[1][dx];
                win[1][dx] = win[2][dx];
            }
        } else {
            // all 9 taps of the CI input channels packed into one K chunk
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * kg + j, tap = k / CI, c = k % CI;
                const int yy = y + tap / 3 - 1, xx = x0 + i + tap % 3 - 1;
                uint16_t v = 0;
                if (tap < 9 && yy >= 0 && yy < d.h && xx >= 0 && xx < d.w) {
                    const int64_t e = ((img * d.h + yy) * d.w + xx) * CI + c;
                    v = SRC_F32 ? f2bf(static_cast<const float *>(in)[e]) : static_cast<const uint16_t *>(in)[e];
                }
                a[j] = as_bf(v);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma(a, bw[0][t], acc[t]);
        }
        // lane holds D[pixel 4 kg + r][channel t 16 + i]
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + i;
            if (co >= CO) continue;
            const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[t][r] + bv;
                if (relu) v = fmaxf(v, 0.0f);
                const int64_t pix = (img * d.h + y) * d.w + x0 + 4 * kg + r;
                if (out_f32) out_f32[pix * CO + co] = v;
                if (out_bf) out_bf[pix * CO + co] = f2bf(v);
                if (out_masked)
                    out_masked[pix * CO + co] = bf2f(act_mask[pix * CO + co]) > 0.0f ? f2bf(v) : (uint16_t)0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of one layer: dW[tap][ci][co] = sum over pixels
// of x[p + tap - (1,1)][ci] dy[p][co], db[co] = sum of dy[p][co].  Each wave
// (one per block) takes whole rows, keeps all 9 x CI x CO partial sums in its
// accumulators and writes them to its own slot; k_wgrad_reduce1/2 add the slots
// in a fixed order (deterministic).  The contraction runs over pixels, which
// are strided in the NHWC activations, so each 32-pixel strip is first staged
// in LDS channel-major: the three input rows around the output row, each in
// three copies shifted by one pixel (every MFMA operand is then one aligned
// 16-byte LDS read), and the output-gradient strip.  A wave walks its rows
// strip by strip, so consecutive output rows share two of their input rows.
// ---------------------------------------------------------------------------
template <int CI, int CO, bool SRC_F32>
__global__ void __launch_bounds__(64) k_wgrad(const void *x, const uint16_t *dy, ConvDims d, int64_t rows_per_wave,
                                              float *part)
{
    constexpr int TI = ntile(CI), TO = ntile(CO), CIP = 16 * TI, COP = 16 * TO;
    constexpr int64_t SLOT = 9 * CIP * COP + COP;
    constexpr int GI = SRC_F32 ? 1 : CI / 8;   // loads per input pixel: 8 BF16 channels, or all CI floats
    constexpr int GO = CO >= 8 ? CO / 8 : 1;   // loads per output-gradient pixel
    static_assert(SRC_F32 ? CI <= 8 : CI % 8 == 0, "input channels per load");
    static_assert(CO >= 8 ? CO % 8 == 0 : true, "output channels per load");
    // xs[slot][shift][ci][k]: input row yy sits in slot yy mod 3, so moving to
    // the next output row of the same image loads one new input row
    __shared__ __attribute__((aligned(16))) uint16_t xs[3][3][CIP][32];
    __shared__ __attribute__((aligned(16))) uint16_t gs[COP][32];
    const int lane = (int)threadIdx.x, i = lane & 15, kg = lane >> 4;
    const int64_t rows = d.n * d.h;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wave;
    const int64_t r1 = r0 + rows_per_wave < rows ? r0 + rows_per_wave : rows;
    // padded channel rows stay zero; every real entry is rewritten when used
    for (int e = lane; e < 9 * CIP * 32; e += 64) (&xs[0][0][0][0])[e] = 0;
    for (int e = lane; e < COP * 32; e += 64) (&gs[0][0])[e] = 0;
    f32x4 acc[9][TI][TO];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
        for (int a = 0; a < TI; ++a)
#pragma unroll
            for (int b = 0; b < TO; ++b) acc[tp][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbs[TO];
#pragma unroll
    for (int b = 0; b < TO; ++b) dbs[b] = 0.0f;
    for (int p0 = 0; p0 < d.w; p0 += 32) {
        int64_t prev = -2;   // row whose input rows the slots hold
        for (int64_t row = r0; row < r1; ++row) {
            const int y = (int)(row % d.h);
            const int64_t img = row / d.h;
            // input rows to load: all three, or y+1 only after row - 1 of the same image
            const bool slide = row == prev + 1 && y > 0;
            const int first = slide ? 2 : 0;
            prev = row;
            __syncthreads();   // the previous row's reads are done
            for (int e = lane; e < (3 - first) * 34 * GI; e += 64) {
                const int r = first + e / (34 * GI), j = (e / GI) % 34, g = e % GI;
                const int yy = y + r - 1, xx = p0 - 1 + j;
                if (yy < 0 || yy >= d.h) continue;     // its taps are skipped
                const int sl = yy % 3;
                const bool in = xx >= 0 && xx < d.w;
                const int64_t pix = (img * d.h + yy) * d.w + xx;
                uint16_t v[8];
                if constexpr (SRC_F32) {
#pragma unroll
                    for (int c = 0; c < CI; ++c) v[c] = in ? f2bf(static_cast<const float *>(x)[pix * CI + c]) : 0;
                } else {
                    uint4 q = make_uint4(0, 0, 0, 0);
                    if (in) q = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(x) + pix * CI + 8 * g);
                    const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int c = 0; c < 8; ++c) v[c] = (uint16_t)(w4[c >> 1] >> (16 * (c & 1)));
                }
                constexpr int NC = SRC_F32 ? CI : 8;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int ci = SRC_F32 ? c : 8 * g + c;
#pragma unroll
                    for (int sft = 0; sft < 3; ++sft) {
                        const int k = j - sft;
                        if (k >= 0 && k < 32) xs[sl][sft][ci][k] = v[c];
                    }
                }
            }
            // output-gradient strip, pixels p0 .. p0+31
            for (int e = lane; e < 32 * GO; e += 64) {
                const int k = e / GO, g = e % GO;
                const int64_t pix = (img * d.h + y) * d.w + p0 + k;
                if constexpr (CO >= 8) {
                    const uint4 q = *reinterpret_cast<const uint4 *>(dy + pix * CO + 8 * g);
                    const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int c = 0; c < 8; ++c) gs[8 * g + c][k] = (uint16_t)(w4[c >> 1] >> (16 * (c & 1)));
                } else {
#pragma unroll
                    for (int c = 0; c < CO; ++c) gs[c][k] = dy[pix * CO + c];
                }
            }
            __syncthreads();
            bf16x8 bfr[TO];
#pragma unroll
            for (int b = 0; b < TO; ++b) {
                bfr[b] = ld_bf16x8(&gs[b * 16 + i][8 * kg]);
#pragma unroll
                for (int j = 0; j < 8; ++j) dbs[b] += (float)bfr[b][j];
            }
#pragma unroll
            for (int tp = 0; tp < 9; ++tp) {
                const int yy = y + tp / 3 - 1;
                if (yy < 0 || yy >= d.h) continue;            // uniform over the wave
                const int sl = yy % 3;
#pragma unroll
                for (int a = 0; a < TI; ++a) {
                    const bf16x8 afr = ld_bf16x8(&xs[sl][tp % 3][a * 16 + i][8 * kg]);
#pragma unroll
                    for (int b = 0; b < TO; ++b) acc[tp][a][b] = mfma(afr, bfr[b], acc[tp][a][b]);
                }
            }
        }
    }
    float *slot = part + (int64_t)blockIdx.x * SLOT;
    // lane holds D[ci = a 16 + 4 kg + r][co = b 16 + i]
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
        for (int a = 0; a < TI; ++a)
#pragma unroll
            for (int b = 0; b < TO; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    slot[((int64_t)tp * CIP + a * 16 + 4 * kg + r) * COP + b * 16 + i] = acc[tp][a][b][r];
#pragma unroll
    for (int b = 0; b < TO; ++b) {
        float sb = dbs[b];
        sb += __shfl_xor(sb, 16);
        sb += __shfl_xor(sb, 32);
        if (kg == 0) slot[9 * CIP * COP + b * 16 + i] = sb;
    }
}

// Slot sums in two fixed-order stages (deterministic for a given slot count):
// groups of kRedGroup consecutive slots, then the groups in order.
constexpr int kRedGroup = 32;

template <int CI, int CO>
__device__ __forceinline__ int64_t wgrad_src(int64_t e)
{
    constexpr int CIP = 16 * ntile(CI), COP = 16 * ntile(CO);
    if (e < 9 * CI * CO) {
        const int co = (int)(e % CO), ci = (int)((e / CO) % CI), tp = (int)(e / (CO * CI));
        return ((int64_t)tp * CIP + ci) * COP + co;
    }
    return (int64_t)9 * CIP * COP + (e - 9 * CI * CO);
}

// grid (outputs / 256, slot groups): tmp[group][e] = sum of its slots
template <int CI, int CO>
__global__ void k_wgrad_reduce1(const float *part, int64_t nslots, float *tmp)
{
    constexpr int CIP = 16 * ntile(CI), COP = 16 * ntile(CO);
    constexpr int64_t SLOT = 9 * CIP * COP + COP, NOUT = 9 * CI * CO + CO;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NOUT) return;
    const int64_t src = wgrad_src<CI, CO>(e);
    const int64_t w0 = (int64_t)blockIdx.y * kRedGroup;
    const int64_t w1 = w0 + kRedGroup < nslots ? w0 + kRedGroup : nslots;
    float acc = 0.0f;
    for (int64_t w = w0; w < w1; ++w) acc += part[w * SLOT + src];
    tmp[(int64_t)blockIdx.y * NOUT + e] = acc;
}

template <int CI, int CO>
__global__ void k_wgrad_reduce2(const float *tmp, int64_t ngroups, float *dw, float *db)
{
    constexpr int64_t NOUT = 9 * CI * CO + CO;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NOUT) return;
    float acc = 0.0f;
    for (int64_t k = 0; k < ngroups; ++k) acc += tmp[k * NOUT + e];
    if (e < 9 * CI * CO)
        dw[e] = acc;
    else
        db[e - 9 * CI * CO] = acc;
}

// ---------------------------------------------------------------------------
// loss: mean logistic loss of the mask logit + lam * mean squared error of
// log10 Q over pixels with a finite target; writes dL/d(out) as BF16 (the
// operand precision of the backward contractions) and per-block sums
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_loss(const float *out, const float *mask, const float *logq, int64_t P,
                                              float lam, uint16_t *g, double *part)
{
    __shared__ double red[256];
    double s = 0.0;
    const double invP = 1.0 / (double)P;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const float z = out[2 * p], qh = out[2 * p + 1], t = mask[p], tq = logq[p];
        const bool valid = isfinite(tq);
        const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
        const float dq = valid ? qh - tq : 0.0f;
        s += (double)(sp - t * z) + (double)lam * (double)dq * (double)dq;
        const float sig = 1.0f / (1.0f + expf(-z));
        g[2 * p] = f2bf((float)((sig - t) * invP));
        g[2 * p + 1] = f2bf((float)(2.0 * lam * dq * invP));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * invP;
}

// one block of 256 threads: strided partial sums, then a fixed-order tree
__global__ void __launch_bounds__(256) k_sum_parts(const double *part, int n, double *out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = (int)threadIdx.x; k < n; k += 256) acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters
// b1, b2 are the decay rates, ob1 = 1 - b1 and ob2 = 1 - b2 (formed in FP64
// on the host: 1 - b2 taken in FP32 from the rounded 0.999f is 1.3e-5 off),
// c1, c2 the bias corrections 1 - b^t.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float ob1,
                       float ob2, float eps, float c1, float c2)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + ob1 * ge;
        const float ve = b2 * v[e] + ob2 * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

uint64_t cnn_prep_bytes() { return (uint64_t)prep_layout().total_u16 * 2; }

static const uint16_t *fwd_mat(const void *prep, int l)
{
    return static_cast<const uint16_t *>(prep) + prep_layout().fwd[l];
}
static const uint16_t *bwd_mat(const void *prep, int l)
{
    return static_cast<const uint16_t *>(prep) + prep_layout().bwd[l];
}
static const float *bias_of(const void *prep, int l)
{
    return reinterpret_cast<const float *>(static_cast<const uint16_t *>(prep) + prep_layout().bias[l]);
}

hipError_t cnn_prepare(const float *params, void *prep, hipStream_t st)
{
    hipLaunchKernelGGL(k_prepare, dim3(64), dim3(256), 0, st, params, static_cast<uint16_t *>(prep));
    return hipGetLastError();
}

static void conv_launch(int l, bool transposed, const void *in, ConvDims d, const void *prep, bool relu, uint16_t *out_bf,
                        float *out_f32, uint16_t *out_masked, const uint16_t *act_mask, hipStream_t st)
{
    const int64_t waves = d.n * (d.h / kConvRows) * (d.w / 16);
    const dim3 grid(blocks_for(waves * 64, 256)), block(256);
    if (!transposed) {
        const uint16_t *wm = fwd_mat(prep, l);
        const float *b = bias_of(prep, l);
        if (l == 0)
            hipLaunchKernelGGL((k_conv<3, 32, true>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, act_mask);
        else if (l == 3)
            hipLaunchKernelGGL((k_conv<32, 2, false>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, act_mask);
        else
            hipLaunchKernelGGL((k_conv<32, 32, false>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, act_mask);
    } else {
        // input gradient of layer l: a convolution from Co(l) to Ci(l) = 32 channels
        const uint16_t *wm = bwd_mat(prep, l);
        if (l == 3)
            hipLaunchKernelGGL((k_conv<2, 32, false>), grid, block, 0, st, in, d, wm, (const float *)nullptr, false,
                               out_bf, out_f32, out_masked, act_mask);
        else
            hipLaunchKernelGGL((k_conv<32, 32, false>), grid, block, 0, st, in, d, wm, (const float *)nullptr, false,
                               out_bf, out_f32, out_masked, act_mask);
    }
}

// waves of the weight-gradient pass and its partial-sum slots
static int64_t wgrad_waves(ConvDims d) { return d.n * d.h < 1024 ? d.n * d.h : 1024; }

// per-wave partial slots, then the first-stage group sums
static int64_t wgrad_groups(ConvDims d) { return (wgrad_waves(d) + kRedGroup - 1) / kRedGroup; }

uint64_t cnn_wgrad_scratch_bytes(int64_t n, int h, int w)
{
    ConvDims d{n, h, w};
    const int64_t slot = 9 * 32 * 32 + 32;
    return (uint64_t)wgrad_waves(d) * slot * 4 + (uint64_t)wgrad_groups(d) * slot * 4;
}

template <int CI, int CO, bool SRC_F32>
static void wgrad_typed(const void *x, const uint16_t *dy, ConvDims d, float *part, float *dw, float *db,
                        hipStream_t st)
{
    const int64_t waves = wgrad_waves(d), rows = d.n * d.h;
    const int64_t rpw = (rows + waves - 1) / waves;
    const int64_t used = (rows + rpw - 1) / rpw;
    const int64_t nout = 9 * CI * CO + CO;
    const int64_t groups = (used + kRedGroup - 1) / kRedGroup;
    float *tmp = part + wgrad_waves(d) * (int64_t)(9 * 32 * 32 + 32);
    hipLaunchKernelGGL((k_wgrad<CI, CO, SRC_F32>), dim3(used), dim3(64), 0, st, x, dy, d, rpw, part);
    hipLaunchKernelGGL((k_wgrad_reduce1<CI, CO>), dim3(blocks_for(nout, 256), groups), dim3(256), 0, st, part, used,
                       tmp);
    hipLaunchKernelGGL((k_wgrad_reduce2<CI, CO>), dim3(blocks_for(nout, 256)), dim3(256), 0, st, tmp, groups, dw, db);
}

static void wgrad_launch(int l, const void *x, const uint16_t *dy, ConvDims d, float *part, float *dw, float *db,
                         hipStream_t st)
{
    if (l == 0)
        wgrad_typed<3, 32, true>(x, dy, d, part, dw, db, st);
    else if (l == 3)
        wgrad_typed<32, 2, false>(x, dy, d, part, dw, db, st);
    else
        wgrad_typed<32, 32, false>(x, dy, d, part, dw, db, st);
}

hipError_t cnn_layer_forward(int l, const void *prep, const void *in, int64_t n, int h, int w, float *out_f32,
                             uint16_t *out_bf, hipStream_t st)
{
    conv_launch(l, false, in, ConvDims{n, h, w}, prep, l < 3, out_bf, out_f32, nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t cnn_layer_backward(int l, const void *prep, const void *in, const uint16_t *dy, int64_t n, int h, int w,
                              float *dw, float *db, float *dx_f32, uint16_t *dx_masked, const uint16_t *act_mask,
                              void *scratch, hipStream_t st)
{
    const ConvDims d{n, h, w};
    wgrad_launch(l, in, dy, d, static_cast<float *>(scratch), dw, db, st);
    if (l > 0 && (dx_f32 || dx_masked))
        conv_launch(l, true, dy, d, prep, false, nullptr, dx_f32, dx_masked, act_mask, st);
    return hipGetLastError();
}

// Workspace of the whole-network calls: 3 hidden activations (BF16, 32 ch),
// output (FP32, 2 ch), output gradient (BF16, 2 ch), two hidden gradients
// (BF16, 32 ch), gradient vector, loss partials, weight-gradient slots.
struct CnnWs {
    uint16_t *act[3], *gout, *gh[2];
    float *out, *grad, *part;
    double *lpart, *loss;
    uint64_t total;
};

static uint64_t al256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }
constexpr int kLossBlocks = 512;

static CnnWs ws_layout(void *base, int64_t n, int h, int w)
{
    const uint64_t P = (uint64_t)n * h * w;
    CnnWs s{};
    char *p = static_cast<char *>(base);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        char *q = p ? p + o : nullptr;
        o += al256(bytes);
        return q;
    };
    for (int k = 0; k < 3; ++k) s.act[k] = reinterpret_cast<uint16_t *>(take(P * 32 * 2));
    s.out = reinterpret_cast<float *>(take(P * 2 * 4));
    s.gout = reinterpret_cast<uint16_t *>(take(P * 2 * 2));
    for (int k = 0; k < 2; ++k) s.gh[k] = reinterpret_cast<uint16_t *>(take(P * 32 * 2));
    s.grad = reinterpret_cast<float *>(take(QSQ_CNN_PARAMS * 4));
    s.lpart = reinterpret_cast<double *>(take(kLossBlocks * 8));
    s.loss = reinterpret_cast<double *>(take(8));
    s.part = reinterpret_cast<float *>(take(cnn_wgrad_scratch_bytes(n, h, w)));
    s.total = o;
    return s;
}

uint64_t cnn_workspace_bytes(int64_t n, int h, int w) { return ws_layout(nullptr, n, h, w).total; }

hipError_t cnn_forward(const void *prep, const float *x, int64_t n, int h, int w, float *out, void *ws, hipStream_t st)
{
    const CnnWs s = ws_layout(ws, n, h, w);
    const ConvDims d{n, h, w};
    conv_launch(0, false, x, d, prep, true, s.act[0], nullptr, nullptr, nullptr, st);
    conv_launch(1, false, s.act[0], d, prep, true, s.act[1], nullptr, nullptr, nullptr, st);
    conv_launch(2, false, s.act[1], d, prep, true, s.act[2], nullptr, nullptr, nullptr, st);
    conv_launch(3, false, s.act[2], d, prep, false, nullptr, out, nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t cnn_train_step(float *params, float *adam_m, float *adam_v, int64_t t, float lr, const float *x,
                          const float *mask, const float *logq, int64_t n, int h, int w, float lam, void *prep,
                          float *grad_out, double *loss_out, void *ws, hipStream_t st)
{
    const CnnWs s = ws_layout(ws, n, h, w);
    const int64_t P = n * h * w;
    hipError_t e = cnn_forward(prep, x, n, h, w, s.out, ws, st);
    if (e != hipSuccess) return e;
    const int lb = (int)(blocks_for(P, 256) < kLossBlocks ? blocks_for(P, 256) : kLossBlocks);
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, st, s.out, mask, logq, P, lam, s.gout, s.lpart);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, s.lpart, lb, loss_out ? loss_out : s.loss);
    float *g = grad_out ? grad_out : s.grad;
    // layer 4 .. 1: weight gradients, then the input gradient masked by the
    // ReLU of the layer below (its BF16 activation > 0)
    const uint16_t *gin = s.gout;
    for (int l = 3; l >= 0; --l) {
        const void *xin = l == 0 ? static_cast<const void *>(x) : static_cast<const void *>(s.act[l - 1]);
        float *dw = g + master_w(l), *db = dw + 9 * kCi[l] * kCo[l];
        uint16_t *gnext = l > 0 ? s.gh[l % 2] : nullptr;
        e = cnn_layer_backward(l, prep, xin, gin, n, h, w, dw, db, nullptr, gnext, l > 0 ? s.act[l - 1] : nullptr,
                               s.part, st);
        if (e != hipSuccess) return e;
        gin = gnext;
    }
    // Kingma & Ba's defaults; every constant is formed in FP64 and rounded once
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)t)), c2 = (float)(1.0 - pow(b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(QSQ_CNN_PARAMS, 256)), dim3(256), 0, st, params, g, adam_m, adam_v,
                       (int64_t)QSQ_CNN_PARAMS, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f,
                       c1, c2);
    return cnn_prepare(params, prep, st);
}

}  // namespace qsq
