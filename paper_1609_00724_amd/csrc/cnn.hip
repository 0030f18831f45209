// Learned refinement proposer on gfx950: a 4-layer 3x3 convolutional network
// (3 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the hidden layers) that reads
// coarse tiles of the field-line length, its FLEDGE map (Sect. 3.6) and Bz,
// and outputs a refine-mask logit and a log10 Q estimate per pixel.  The
// network is an extension beyond the paper; the FLL-jump rule of Sect. 3.6
// stays the fallback and the reference its proposals are scored against.
//
// Every contraction runs on the matrix cores: v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation), each wave accumulating one or more 16x16
// output tiles.
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
// channels per tap in the packed K layout of an input with fewer than 32
// channels (3 is padded to 4 so that a tap's channels fill whole dwords)
__host__ __device__ constexpr int cpad(int ci) { return ci == 3 ? 4 : ci; }
__host__ __device__ constexpr int nchunk(int ci) { return ci >= 32 ? 9 : (9 * cpad(ci) + 31) / 32; }

// ---------------------------------------------------------------------------
// Prepared weights (BF16 matrices in MFMA-friendly order + FP32 biases)
//   fwd[l]: [nchunk(Ci)][16 ntile(Co)][32]: element (kc, co, kk) multiplies
//           input channel/tap (tap = kc, ci = kk) for Ci = 32, or
//           (tap = k / cpad(Ci), ci = k % cpad(Ci), k = 32 kc + kk; zero
//           where ci >= Ci or tap >= 9) for Ci < 32
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
                tap = (32 * kc + kk) / cpad(Ci);
                ci = (32 * kc + kk) % cpad(Ci);
            }
            const bool ok = co < Co && tap < 9 && ci < Ci;
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
                tap = (32 * kc + kk) / cpad(Co);
                c = (32 * kc + kk) % cpad(Co);
            }
            const bool ok = tap < 9 && ci < Ci && c < Co;
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
// 3x3 'same' convolution.  A workgroup of 4 waves takes kConvRows rows of a
// 64-pixel column chunk of one image, a wave a 16-pixel strip of it, all
// output channels; the wave keeps the weight operands in registers.
// 32-channel inputs (BF16): the workgroup first stages its input rows
// (kConvRows + 2, pixels x - 1 .. x + 64, zeros outside the image) in LDS with
// all loads in flight at once; lane (i, kg) then reads pixels x0 + i - 1,
// x0 + i, x0 + i + 1, channels 8 kg .. 8 kg + 7, of each row from there, in a
// window of three rows sliding down the strip.  Inputs with CI < 32 channels
// (FP32 with 3, BF16 with 2) are staged the same way, as BF16 with cpad(CI)
// channels per pixel, and the 9 taps' channels packed along K (cpad(CI) per
// tap) are read from there.  Outputs (each
// nullable): BF16 activations (ReLU applied), FP32 values, a BF16 copy masked
// by mask_cm > 0 (input gradients; mask_cm is the channel-major copy of the
// layer's input activations), and the channel-major copy of the BF16 output
// (masked too when mask_cm is given).  A BF16 NHWC output of 32 channels goes
// through LDS so that each lane stores one pixel's 8 channels (16 bytes) and
// the wave a row's 1 KB with one store.  One tile's tensors are addressed
// with 32-bit byte offsets (h w <= 2^24).
// ---------------------------------------------------------------------------
struct ConvDims {
    int64_t n;
    int h, w;
};

constexpr int kConvRows = 8;   // divides h (a multiple of 32)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// buffer resource over `bytes` bytes at p (gfx9 descriptor word 3: 32-bit
// data format, untyped access); offsets at or past `bytes` read zeros and
// drop writes
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}

// two FP32 values to a BF16 pair (round to nearest even), a in the low half
__device__ __forceinline__ uint32_t pack_bf2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// BF16 pair with each half kept where the matching half of m (BF16) is > 0
__device__ __forceinline__ uint32_t mask_bf2(uint32_t v, uint32_t m)
{
    const bool lo = __uint_as_float(m << 16) > 0.0f, hi = __uint_as_float(m & 0xffff0000u) > 0.0f;
    return (lo ? v & 0xffffu : 0u) | (hi ? v & 0xffff0000u : 0u);
}

struct Row3 {
    bf16x8 m, z, p;   // the lane's pixel shifted by -1, 0, +1
};

template <int CI, int CO, bool SRC_F32>
__global__ void __launch_bounds__(256) k_conv(const void *__restrict__ in, ConvDims d,
                                              const uint16_t *__restrict__ wm, const float *__restrict__ bias,
                                              bool relu, uint16_t *__restrict__ out_bf, float *__restrict__ out_f32,
                                              uint16_t *__restrict__ out_masked,
                                              const uint16_t *__restrict__ mask_cm, uint16_t *__restrict__ out_cm)
{
    constexpr int NT = ntile(CO), COP = 16 * NT, NK = nchunk(CI), R = kConvRows;
    static_assert(CI >= 32 ? !SRC_F32 : (CI == 3) == SRC_F32, "FP32 input has 3 channels, BF16 input 2 or 32");
    const int lane = (int)(threadIdx.x & 63);
    // workgroup: R rows of a 64-pixel column chunk of one image; wave s (a
    // scalar, so that the buffer resources below are too) the 16-pixel strip
    // x0 = xc + 16 s
    const int cpr = (d.w + 63) / 64, rb = d.h / R;
    const int64_t blk = blockIdx.x / cpr;   // image * rb + row block
    const int xc = (int)(blockIdx.x % cpr) * 64, y0 = (int)(blk % rb) * R;
    const int64_t img = blk / rb;
    const int sw = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int x0 = xc + 16 * sw;
    const int i = lane & 15, kg = lane >> 4;
    const int64_t npix = (int64_t)d.h * d.w;   // pixels of one tile
    // 32-channel inputs: the workgroup's R + 2 input rows, pixels xc - 1 ..
    // xc + 64 (zeros outside the image), staged in LDS with all loads in
    // flight at once: [row][pixel][4 chunks of 8 channels]
    constexpr int PW = 66, NCH = (R + 2) * PW * 4, PER = (NCH + 255) / 256;
    uint4 *lrows = nullptr;
    if constexpr (CI >= 32) {
        __shared__ uint4 rows_lds[NCH];
        lrows = rows_lds;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(static_cast<const uint16_t *>(in) + img * npix * 32, (int)(npix * 64));
        u32x4 tmp[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = (int)threadIdx.x + 256 * k;
            const int r = c / (PW * 4), rem = c % (PW * 4), px = xc - 1 + (rem >> 2), q = rem & 3;
            // rows above and below the tile lie outside the buffer range (zeros), and so
            // do the pixels left and right of it
            const int off = px >= 0 && px < d.w ? (((y0 - 1 + r) * d.w + px) * 32 + 8 * q) * 2 : (int)(npix * 64);
            tmp[k] = c < NCH ? __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = (int)threadIdx.x + 256 * k;
            if (c < NCH) rows_lds[c] = make_uint4(tmp[k].x, tmp[k].y, tmp[k].z, tmp[k].w);
        }
        __syncthreads();
    }
    // inputs with CI < 32 channels: the same rows as BF16 with cpad(CI)
    // channels per pixel (the pad channel zero), WPT dwords per pixel
    constexpr int WPT = cpad(CI) / 2, NPX = (R + 2) * PW;
    uint32_t *lsmall = nullptr;
    if constexpr (CI < 32) {
        __shared__ uint32_t small_lds[NPX * WPT];
        lsmall = small_lds;
        constexpr int PERS = (NPX + 255) / 256;
        uint32_t tmp[PERS][WPT];
#pragma unroll
        for (int k = 0; k < PERS; ++k) {
            const int q = (int)threadIdx.x + 256 * k;
            const int yy = y0 - 1 + q / PW, px = xc - 1 + q % PW;
#pragma unroll
            for (int j = 0; j < WPT; ++j) tmp[k][j] = 0u;
            if (q < NPX && yy >= 0 && yy < d.h && px >= 0 && px < d.w) {
                const int64_t pix = (img * d.h + yy) * d.w + px;
                if constexpr (SRC_F32) {
                    const float *pf = static_cast<const float *>(in) + pix * 3;
                    tmp[k][0] = (uint32_t)f2bf(pf[0]) | ((uint32_t)f2bf(pf[1]) << 16);
                    tmp[k][1] = (uint32_t)f2bf(pf[2]);
                } else {
                    tmp[k][0] = *reinterpret_cast<const uint32_t *>(static_cast<const uint16_t *>(in) + pix * 2);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PERS; ++k) {
            const int q = (int)threadIdx.x + 256 * k;
            if (q < NPX) {
#pragma unroll
                for (int j = 0; j < WPT; ++j) small_lds[q * WPT + j] = tmp[k][j];
            }
        }
        __syncthreads();
    }
    if (x0 >= d.w) return;   // the whole wave leaves together (no barrier follows)
    bf16x8 bw[NK][NT];
#pragma unroll
    for (int kc = 0; kc < NK; ++kc)
#pragma unroll
        for (int t = 0; t < NT; ++t) bw[kc][t] = ld_bf16x8(wm + ((int64_t)(kc * COP + t * 16 + i) * 32 + 8 * kg));
    float bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bv[t] = bias && t * 16 + i < CO ? bias[t * 16 + i] : 0.0f;
    // the tile's channel-major tensors (mask, output copy): CO channels per row
    const int cm_bytes = (int)(npix * CO * 2);
    const __amdgpu_buffer_rsrc_t mask_rs = buf_rsrc(mask_cm ? mask_cm + img * npix * CO : nullptr, cm_bytes);
    const __amdgpu_buffer_rsrc_t cm_rs = buf_rsrc(out_cm ? out_cm + img * npix * CO : nullptr, cm_bytes);
    // byte offset of (row y, channel 16 t + i, pixel x0 + 4 kg) in them
    auto cm_off = [&](int y, int t) { return ((y * CO + t * 16 + i) * d.w + x0 + 4 * kg) * 2; };
    // BF16 NHWC output of 32 channels through the wave's LDS stage
    __shared__ uint16_t stage_all[4][16 * 32];
    uint16_t *stage = stage_all[threadIdx.x >> 6];
    auto store_nhwc = [&](uint16_t *dst, int y, const uint32_t (&hp)[NT][2]) {
        if constexpr (CO == 32) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    stage[(4 * kg + r) * 32 + 16 * t + i] = (uint16_t)(hp[t][r >> 1] >> (16 * (r & 1)));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const u32x4 q = reinterpret_cast<const u32x4 *>(stage)[lane];
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(dst + img * npix * 32, (int)(npix * 64));
            __builtin_amdgcn_raw_buffer_store_b128(q, rs, ((y * d.w + x0) * 32 + 8 * lane) * 2, 0, 0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int co = t * 16 + i;
                if (co >= CO) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    dst[((img * d.h + y) * d.w + x0 + 4 * kg + r) * CO + co] = (uint16_t)(hp[t][r >> 1] >> (16 * (r & 1)));
            }
        }
    };
    // the lane's three shifted operands of staged row r (input row y0 - 1 + r)
    auto lds3 = [&](int r) {
        const int base = (r * PW + 16 * sw + i) * 4 + kg;
        Row3 o;
        o.m = __builtin_bit_cast(bf16x8, lrows[base]);
        o.z = __builtin_bit_cast(bf16x8, lrows[base + 4]);
        o.p = __builtin_bit_cast(bf16x8, lrows[base + 8]);
        return o;
    };
    Row3 win[3];   // input rows y - 1, y, y + 1
    if constexpr (CI >= 32) {
        win[0] = lds3(0);
        win[1] = lds3(1);
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const int y = y0 + rr;
        // mask of this row's pixels 4 kg .. 4 kg + 3, fetched before the
        // products so that its latency overlaps them
        u32x2 mk[NT];
        if (mask_cm) {
#pragma unroll
            for (int t = 0; t < NT; ++t) mk[t] = __builtin_amdgcn_raw_buffer_load_b64(mask_rs, cm_off(y, t), 0, 0);
        }
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (CI >= 32) {
            win[2] = lds3(rr + 2);
#pragma unroll
            for (int ty = 0; ty < 3; ++ty)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[t] = mfma(win[ty].m, bw[3 * ty + 0][t], acc[t]);
                    acc[t] = mfma(win[ty].z, bw[3 * ty + 1][t], acc[t]);
                    acc[t] = mfma(win[ty].p, bw[3 * ty + 2][t], acc[t]);
                }
            win[0] = win[1];
            win[1] = win[2];
        } else {
            // the 9 taps' channels packed along K: lane kg takes taps
            // (32 kc + 8 kg) / cpad .. + 8 / cpad - 1 of chunk kc
            // (read from the staged rows: staged row rr + dy, pixel 16 s + i + dx)
            constexpr int CP = cpad(CI), TPL = 8 / CP;
#pragma unroll
            for (int kc = 0; kc < NK; ++kc) {
                uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int tt = 0; tt < TPL; ++tt) {
                    const int tap = (32 * kc + 8 * kg) / CP + tt;
                    if (tap < 9) {
                        const int q = (rr + tap / 3) * PW + 16 * sw + i + tap % 3;
#pragma unroll
                        for (int j = 0; j < WPT; ++j) wd[WPT * tt + j] = lsmall[q * WPT + j];
                    }
                }
                const bf16x8 a = __builtin_bit_cast(bf16x8, make_uint4(wd[0], wd[1], wd[2], wd[3]));
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma(a, bw[kc][t], acc[t]);
            }
        }
        // lane holds D[pixel 4 kg + r][channel t 16 + i]; BF16 pairs of
        // pixels (4 kg, 4 kg + 1) and (4 kg + 2, 4 kg + 3)
        float v[NT][4];
        uint32_t hp[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[t][r] = acc[t][r] + bv[t];
                if (relu) v[t][r] = fmaxf(v[t][r], 0.0f);
            }
            hp[t][0] = pack_bf2(v[t][0], v[t][1]);
            hp[t][1] = pack_bf2(v[t][2], v[t][3]);
        }
        if (out_f32) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int co = t * 16 + i;
                if (co >= CO) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) out_f32[((img * d.h + y) * d.w + x0 + 4 * kg + r) * CO + co] = v[t][r];
            }
        }
        if (out_bf) store_nhwc(out_bf, y, hp);
        if (mask_cm) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                hp[t][0] = mask_bf2(hp[t][0], mk[t].x);
                hp[t][1] = mask_bf2(hp[t][1], mk[t].y);
            }
            if (out_masked) store_nhwc(out_masked, y, hp);
        }
        if (out_cm) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (t * 16 + i < CO) __builtin_amdgcn_raw_buffer_store_b64(u32x2{hp[t][0], hp[t][1]}, cm_rs, cm_off(y, t), 0, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Channel-major row copies.  The weight gradient contracts over pixels, and a
// matrix-core operand takes 8 consecutive K values per lane, so its operands
// are read from copies of the activations and gradients laid out per image
// row as [channel][x] (BF16): cm[((img h + y) C + c) w + x].  The producing
// kernels (convolutions, loss) write them beside their NHWC outputs; k_to_cm
// makes them from NHWC data (the network input, the per-layer check calls).
// ---------------------------------------------------------------------------
template <int C, bool SRC_F32>
__global__ void k_to_cm(const void *in, int64_t rows, int w, uint16_t *out)
{
    if constexpr (C <= 4) {
        // one pixel per thread: its C values read together, one store per
        // channel row (consecutive threads write consecutive pixels)
        const int64_t total = rows * w;
        for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
             p += (int64_t)gridDim.x * blockDim.x) {
            const int64_t row = p / w, x = p % w;
#pragma unroll
            for (int c = 0; c < C; ++c)
                out[(row * C + c) * w + x] = SRC_F32 ? f2bf(static_cast<const float *>(in)[p * C + c])
                                                     : static_cast<const uint16_t *>(in)[p * C + c];
        }
    } else {
        const int64_t total = rows * C * w;
        for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
             o += (int64_t)gridDim.x * blockDim.x) {
            const int x = (int)(o % w), c = (int)((o / w) % C);
            const int64_t row = o / ((int64_t)w * C), e = (row * w + x) * C + c;
            out[o] = SRC_F32 ? f2bf(static_cast<const float *>(in)[e]) : static_cast<const uint16_t *>(in)[e];
        }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of one layer: dW[tap][ci][co] = sum over pixels
// of x[p + tap - (1,1)][ci] dy[p][co], db[co] = sum of dy[p][co], from the
// channel-major copies.  MFMA: M = 16 input channels, N = 16 output
// channels, K = 32 pixels of a row.  A workgroup takes R rows of one image
// and a 64-pixel column chunk, one wave per (input tile, output tile) pair;
// each wave covers the whole chunk as two K halves: lane (i, kg) reads
// pixels x0 + 8 kg .. + 7 and x0 + 32 + 8 kg .. + 7 of channel i (two aligned
// 16-byte buffer loads per row, zeros outside the tile).  The pixel pairs
// either side, for the operands shifted by one pixel (byte-align of adjacent
// dwords), come from the neighbouring lanes (kg - 1, kg + 1, and across the
// two halves) by ds_bpermute; only the chunk's outer edges are loaded, and
// only where the chunk does not end at the image edge.  Each wave slides a
// window of three input rows down its R rows, four at a time, and writes its
// sums to the workgroup's slot; k_wgrad_reduce1/2 add the slots in a fixed
// order (deterministic).
// ---------------------------------------------------------------------------
struct Shift3 {
    bf16x8 m, z, p;   // pixels shifted by -1, 0, +1
};

// one input row of a lane: the two 8-pixel chunks and the pixel pairs either
// side of each
struct XRow {
    uint32_t d[2][4], lft[2], rgt[2];
};

__device__ __forceinline__ Shift3 shift3(const uint32_t (&d)[4], uint32_t lft, uint32_t rgt)
{
    const uint32_t e12 = __builtin_amdgcn_alignbyte(d[1], d[0], 2), e34 = __builtin_amdgcn_alignbyte(d[2], d[1], 2),
                   e56 = __builtin_amdgcn_alignbyte(d[3], d[2], 2);
    Shift3 s;
    s.z = __builtin_bit_cast(bf16x8, make_uint4(d[0], d[1], d[2], d[3]));
    s.m = __builtin_bit_cast(bf16x8, make_uint4(__builtin_amdgcn_alignbyte(d[0], lft, 2), e12, e34, e56));
    s.p = __builtin_bit_cast(bf16x8, make_uint4(e12, e34, e56, __builtin_amdgcn_alignbyte(rgt, d[3], 2)));
    return s;
}

template <int CI, int CO>
__global__ void __launch_bounds__(256) k_wgrad(const uint16_t *__restrict__ xcm, const uint16_t *__restrict__ gcm,
                                               ConvDims d, int R, float *__restrict__ part)
{
    constexpr int TO = ntile(CO);
    constexpr int SLOT = 9 * CI * CO + CO;   // dW (tap, ci, co) then db (co): the parameter order
    const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
    const int a = wid / TO, b = wid % TO;
    const int i = lane & 15, kg = lane >> 4;
    const int cpr = (d.w + 63) / 64, rb = d.h / R;
    const int64_t unit = blockIdx.x;
    const int x0 = (int)(unit % cpr) * 64, y0 = (int)((unit / cpr) % rb) * R;
    const int64_t img = unit / ((int64_t)cpr * rb);
    const int c = a * 16 + i, co = b * 16 + i;
    const int64_t npix = (int64_t)d.h * d.w;
    const int xbytes = (int)(npix * CI * 2), gbytes = (int)(npix * CO * 2);
    const __amdgpu_buffer_rsrc_t xrs = buf_rsrc(xcm + img * npix * CI, xbytes);
    const __amdgpu_buffer_rsrc_t grs = buf_rsrc(gcm + img * npix * CO, gbytes);
    // byte offset of pixel x of row yy of channel ch (out of range: zeros)
    auto xoff = [&](int yy, int x) {
        return c < CI && yy >= 0 && yy < d.h && x >= 0 && x < d.w ? ((yy * CI + c) * d.w + x) * 2 : xbytes;
    };
    const bool edge_l = x0 > 0, edge_r = x0 + 64 < d.w;   // chunk edges inside the image
    const int up = ((lane + 48) & 63) << 2, dn = ((lane + 16) & 63) << 2;   // ds_bpermute addresses of kg - 1, kg + 1
    auto xrow = [&](int yy) {
        XRow r;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(xrs, xoff(yy, x0 + 32 * h + 8 * kg), 0, 0);
            r.d[h][0] = q.x;
            r.d[h][1] = q.y;
            r.d[h][2] = q.z;
            r.d[h][3] = q.w;
        }
        // pixel pairs left of each chunk: lane kg - 1's last dword (for kg = 0
        // of the second half: lane kg = 3 of the first half)
        const uint32_t l0 = (uint32_t)__builtin_amdgcn_ds_bpermute(up, (int)r.d[0][3]);
        const uint32_t l1 = (uint32_t)__builtin_amdgcn_ds_bpermute(up, (int)r.d[1][3]);
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_ds_bpermute(dn, (int)r.d[0][0]);
        const uint32_t r1 = (uint32_t)__builtin_amdgcn_ds_bpermute(dn, (int)r.d[1][0]);
        uint32_t el = 0, er = 0;
        if (edge_l) el = __builtin_amdgcn_raw_buffer_load_b32(xrs, kg == 0 ? xoff(yy, x0 - 2) : xbytes, 0, 0);
        if (edge_r) er = __builtin_amdgcn_raw_buffer_load_b32(xrs, kg == 3 ? xoff(yy, x0 + 64) : xbytes, 0, 0);
        r.lft[0] = kg > 0 ? l0 : el;
        r.lft[1] = kg > 0 ? l1 : l0;
        r.rgt[0] = kg < 3 ? r0 : r1;
        r.rgt[1] = kg < 3 ? r1 : er;
        return r;
    };
    auto grow = [&](int yy, int h) {
        const int x = x0 + 32 * h + 8 * kg;
        const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(
            grs, co < CO && yy < d.h && x < d.w ? ((yy * CO + co) * d.w + x) * 2 : gbytes, 0, 0);
        return __builtin_bit_cast(bf16x8, q);
    };
    f32x4 acc[9];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) acc[tp] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbs = 0.0f;   // bias gradient (waves of input tile 0 only)
    // rows go four at a time: all loads of a group are issued before its
    // products, so their latencies overlap (R is a multiple of 4)
    XRow win[6];   // input rows y - 1 .. y + 4
    win[0] = xrow(y0 - 1);
    win[1] = xrow(y0);
    for (int rr = 0; rr < R; rr += 4) {
        const int y = y0 + rr;
        bf16x8 gb[4][2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            win[2 + k] = xrow(y + 1 + k);
            gb[k][0] = grow(y + k, 0);
            gb[k][1] = grow(y + k, 1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (a == 0) {
#pragma unroll
                for (int j = 0; j < 8; ++j) dbs += (float)gb[k][0][j] + (float)gb[k][1][j];
            }
#pragma unroll
            for (int ty = 0; ty < 3; ++ty)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const XRow &xr = win[k + ty];
                    const Shift3 xs3 = shift3(xr.d[h], xr.lft[h], xr.rgt[h]);
                    acc[3 * ty + 0] = mfma(xs3.m, gb[k][h], acc[3 * ty + 0]);
                    acc[3 * ty + 1] = mfma(xs3.z, gb[k][h], acc[3 * ty + 1]);
                    acc[3 * ty + 2] = mfma(xs3.p, gb[k][h], acc[3 * ty + 2]);
                }
        }
        win[0] = win[4];
        win[1] = win[5];
    }
    // lane holds D[ci = a 16 + 4 kg + r][co = b 16 + i]; the slot keeps the
    // real channels only
    float *slot = part + unit * SLOT;
    if (co < CO) {
#pragma unroll
        for (int tp = 0; tp < 9; ++tp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = a * 16 + 4 * kg + r;
                if (ci < CI) slot[(tp * CI + ci) * CO + co] = acc[tp][r];
            }
    }
    if (a == 0) {
        dbs += __shfl_xor(dbs, 16);
        dbs += __shfl_xor(dbs, 32);
        if (kg == 0 && co < CO) slot[9 * CI * CO + co] = dbs;
    }
}

// Slot sums in two fixed-order stages (deterministic for a given slot count):
// groups of kRedGroup consecutive slots, then the groups in order.  One pair
// of launches reduces the slots of up to four layers (a training step's
// backward pass) at once.
constexpr int kRedGroup = 64;

struct RedSeg {
    const float *part;   // the layer's slots (each: dW (tap, ci, co), then db)
    float *dw, *db;
    int64_t nw;                   // weights (9 ci co); the slot holds nw + co floats
    int64_t nslots, nout, e0;     // slots, outputs (= slot floats), first output in the job
};

struct RedJob {
    RedSeg s[4];
    int nseg;
    int64_t total;
};

// output e of the job: its segment and the offset of its value within a slot
__device__ __forceinline__ const RedSeg &red_seg(const RedJob &J, int64_t e)
{
    int k = 0;
    while (k + 1 < J.nseg && e >= J.s[k + 1].e0) ++k;
    return J.s[k];
}

// grid (outputs / 256, slot groups): tmp[group][e] = sum of its slots
__global__ void k_wgrad_reduce1(RedJob J, float *__restrict__ tmp)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= J.total) return;
    const RedSeg &g = red_seg(J, e);
    const int64_t src = e - g.e0;
    const int64_t w0 = (int64_t)blockIdx.y * kRedGroup;
    const int64_t w1 = w0 + kRedGroup < g.nslots ? w0 + kRedGroup : g.nslots;
    float acc = 0.0f;
#pragma unroll 8
    for (int64_t w = w0; w < w1; ++w) acc += g.part[w * g.nout + src];
    tmp[(int64_t)blockIdx.y * J.total + e] = acc;
}

__global__ void k_wgrad_reduce2(RedJob J, const float *__restrict__ tmp, int64_t ngroups)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= J.total) return;
    const RedSeg &g = red_seg(J, e);
    float acc = 0.0f;
#pragma unroll 8
    for (int64_t k = 0; k < ngroups; ++k) acc += tmp[k * J.total + e];
    const int64_t le = e - g.e0;
    if (le < g.nw)
        g.dw[le] = acc;
    else
        g.db[le - g.nw] = acc;
}

// ---------------------------------------------------------------------------
// loss: mean logistic loss of the mask logit + lam * mean squared error of
// log10 Q over pixels with a finite target; writes dL/d(out) as BF16 (the
// operand precision of the backward contractions) and per-block sums
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_loss(const float *out, const float *mask, const float *logq, int64_t P,
                                              float lam, uint16_t *g, double *part, int w, uint16_t *g_cm)
{
    __shared__ double red[256];
    double s = 0.0;
    const double invP = 1.0 / (double)P;
    // (pixel indices fit 32 bits: n h w < 2^31)
    for (int p = (int)(blockIdx.x * blockDim.x + threadIdx.x); p < (int)P; p += (int)(gridDim.x * blockDim.x)) {
        const float2 zo = reinterpret_cast<const float2 *>(out)[p];
        const float z = zo.x, qh = zo.y, t = mask[p], tq = logq[p];
        const bool valid = isfinite(tq);
        const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
        const float dq = valid ? qh - tq : 0.0f;
        s += (double)(sp - t * z) + (double)lam * (double)dq * (double)dq;
        const float sig = 1.0f / (1.0f + expf(-z));
        const uint16_t g0 = f2bf((float)((sig - t) * invP)), g1 = f2bf((float)(2.0 * lam * dq * invP));
        reinterpret_cast<uint32_t *>(g)[p] = (uint32_t)g0 | ((uint32_t)g1 << 16);
        const int row = p / w, x = p - row * w;
        g_cm[(int64_t)(row * 2 + 0) * w + x] = g0;
        g_cm[(int64_t)(row * 2 + 1) * w + x] = g1;
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
// The updated parameter is also written where k_prepare would put it in the
// prepared weights (its forward matrix entry, its transposed and flipped
// input-gradient entry, or its bias), so no separate preparation pass runs;
// the zero padding of the prepared matrices is never touched.
__device__ __forceinline__ void prep_store(int64_t e, float val, uint16_t *prep)
{
    const PrepLayout P = prep_layout();
    int l = 0;
    while (l < 3 && e >= master_w(l + 1)) ++l;
    const int Ci = kCi[l], Co = kCo[l];
    const int64_t le = e - master_w(l);
    if (le >= 9LL * Ci * Co) {
        reinterpret_cast<float *>(prep + P.bias[l])[le - 9LL * Ci * Co] = val;
        return;
    }
    const int co = (int)(le % Co), ci = (int)((le / Co) % Ci), tap = (int)(le / ((int64_t)Co * Ci));
    const uint16_t hb = f2bf(val);
    {
        const int k = Ci >= 32 ? 32 * tap + ci : tap * cpad(Ci) + ci;   // K index (chunk kc = k / 32)
        prep[P.fwd[l] + ((int64_t)(k / 32) * 16 * ntile(Co) + co) * 32 + k % 32] = hb;
    }
    if (l >= 1) {
        const int tf = 8 - tap;
        const int k = Co >= 32 ? 32 * tf + co : tf * cpad(Co) + co;
        prep[P.bwd[l] + ((int64_t)(k / 32) * 32 + ci) * 32 + k % 32] = hb;
    }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float ob1,
                       float ob2, float eps, float c1, float c2, uint16_t *prep)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + ob1 * ge;
        const float ve = b2 * v[e] + ob2 * ge * ge;
        m[e] = me;
        v[e] = ve;
        const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
        p[e] = pe;
        prep_store(e, pe, prep);
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
                        float *out_f32, uint16_t *out_masked, const uint16_t *mask_cm, uint16_t *out_cm,
                        hipStream_t st)
{
    const dim3 grid((unsigned)(d.n * (d.h / kConvRows) * ((d.w + 63) / 64))), block(256);
    if (!transposed) {
        const uint16_t *wm = fwd_mat(prep, l);
        const float *b = bias_of(prep, l);
        if (l == 0)
            hipLaunchKernelGGL((k_conv<3, 32, true>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, mask_cm, out_cm);
        else if (l == 3)
            hipLaunchKernelGGL((k_conv<32, 2, false>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, mask_cm, out_cm);
        else
            hipLaunchKernelGGL((k_conv<32, 32, false>), grid, block, 0, st, in, d, wm, b, relu, out_bf, out_f32,
                               out_masked, mask_cm, out_cm);
    } else {
        // input gradient of layer l: a convolution from Co(l) to Ci(l) = 32 channels
        const uint16_t *wm = bwd_mat(prep, l);
        if (l == 3)
            hipLaunchKernelGGL((k_conv<2, 32, false>), grid, block, 0, st, in, d, wm, (const float *)nullptr, false,
                               out_bf, out_f32, out_masked, mask_cm, out_cm);
        else
            hipLaunchKernelGGL((k_conv<32, 32, false>), grid, block, 0, st, in, d, wm, (const float *)nullptr, false,
                               out_bf, out_f32, out_masked, mask_cm, out_cm);
    }
}

// Rows per workgroup of layer l's weight-gradient pass: the smallest power
// of two >= 4 dividing h that keeps its slots (one per workgroup: R rows of a
// 64-pixel column chunk) at 2048 / (waves per workgroup) or fewer, h at most
// -- about 2048 waves for the 32 x 32 layers and the narrow ones alike.
static int wgrad_rows(ConvDims d, int l)
{
    const int64_t cap = 2048 / (ntile(kCi[l]) * ntile(kCo[l]));
    int R = 4;
    while (R < d.h && d.h % (2 * R) == 0 && d.n * (d.h / R) * ((d.w + 63) / 64) > cap) R *= 2;
    return R;
}

static int64_t wgrad_slots(ConvDims d, int l) { return d.n * (d.h / wgrad_rows(d, l)) * ((d.w + 63) / 64); }

// first-stage groups of a reduction: enough for the layer with the most slots
static int64_t wgrad_groups(ConvDims d)
{
    int64_t m = 0;
    for (int l = 0; l < 4; ++l) m = wgrad_slots(d, l) > m ? wgrad_slots(d, l) : m;
    return (m + kRedGroup - 1) / kRedGroup;
}

static int64_t slot_floats(int l) { return 9LL * kCi[l] * kCo[l] + kCo[l]; }

static uint64_t al256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

static uint64_t slot_bytes(ConvDims d, int l) { return al256((uint64_t)wgrad_slots(d, l) * slot_floats(l) * 4); }

// slots of one layer (the largest layer's) and its group sums
static uint64_t wgrad_part_bytes(ConvDims d)
{
    uint64_t m = 0;
    for (int l = 0; l < 4; ++l) m = slot_bytes(d, l) > m ? slot_bytes(d, l) : m;
    return m + (uint64_t)wgrad_groups(d) * (9 * 32 * 32 + 32) * 4;
}

// slots of all four layers and the group sums of the whole parameter vector
static uint64_t train_part_bytes(ConvDims d)
{
    uint64_t b = 0;
    for (int l = 0; l < 4; ++l) b += slot_bytes(d, l);
    return b + (uint64_t)wgrad_groups(d) * QSQ_CNN_PARAMS * 4;
}

// per-layer backward: channel-major copies of the input and of dy, then the slots
uint64_t cnn_wgrad_scratch_bytes(int64_t n, int h, int w)
{
    const uint64_t cm = al256((uint64_t)n * h * w * 32 * 2);
    return 2 * cm + wgrad_part_bytes(ConvDims{n, h, w});
}

// the slots of layer l (written to `part`) as a segment of a reduction job
static void wgrad_slots_launch(int l, const uint16_t *xcm, const uint16_t *gcm, ConvDims d, float *part, float *dw,
                               float *db, RedJob &J, hipStream_t st)
{
    const int64_t slots = wgrad_slots(d, l);
    const int R = wgrad_rows(d, l);
    const dim3 grid(slots), block(64 * ntile(kCi[l]) * ntile(kCo[l]));
    if (l == 0)
        hipLaunchKernelGGL((k_wgrad<3, 32>), grid, block, 0, st, xcm, gcm, d, R, part);
    else if (l == 3)
        hipLaunchKernelGGL((k_wgrad<32, 2>), grid, block, 0, st, xcm, gcm, d, R, part);
    else
        hipLaunchKernelGGL((k_wgrad<32, 32>), grid, block, 0, st, xcm, gcm, d, R, part);
    RedSeg &g = J.s[J.nseg++];
    g.part = part;
    g.dw = dw;
    g.db = db;
    g.nw = 9LL * kCi[l] * kCo[l];
    g.nslots = slots;
    g.nout = slot_floats(l);
    g.e0 = J.total;
    J.total += g.nout;
}

static void wgrad_reduce(const RedJob &J, float *tmp, ConvDims d, hipStream_t st)
{
    const int64_t groups = wgrad_groups(d);
    hipLaunchKernelGGL(k_wgrad_reduce1, dim3(blocks_for(J.total, 256), groups), dim3(256), 0, st, J, tmp);
    hipLaunchKernelGGL(k_wgrad_reduce2, dim3(blocks_for(J.total, 256)), dim3(256), 0, st, J, (const float *)tmp,
                       groups);
}

static void wgrad_launch(int l, const uint16_t *xcm, const uint16_t *gcm, ConvDims d, float *part, float *dw,
                         float *db, hipStream_t st)
{
    RedJob J{};
    wgrad_slots_launch(l, xcm, gcm, d, part, dw, db, J, st);
    uint64_t m = 0;
    for (int k = 0; k < 4; ++k) m = slot_bytes(d, k) > m ? slot_bytes(d, k) : m;
    wgrad_reduce(J, part + m / 4, d, st);
}

template <int C, bool SRC_F32>
static void to_cm(const void *in, ConvDims d, uint16_t *out, hipStream_t st)
{
    const int64_t total = d.n * d.h * (int64_t)d.w * (C <= 4 ? 1 : C);
    const int blocks = (int)(blocks_for(total, 256) < 8192 ? blocks_for(total, 256) : 8192);
    hipLaunchKernelGGL((k_to_cm<C, SRC_F32>), dim3(blocks), dim3(256), 0, st, in, d.n * d.h, d.w, out);
}

hipError_t cnn_layer_forward(int l, const void *prep, const void *in, int64_t n, int h, int w, float *out_f32,
                             uint16_t *out_bf, hipStream_t st)
{
    conv_launch(l, false, in, ConvDims{n, h, w}, prep, l < 3, out_bf, out_f32, nullptr, nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t cnn_layer_backward(int l, const void *prep, const void *in, const uint16_t *dy, int64_t n, int h, int w,
                              float *dw, float *db, float *dx_f32, uint16_t *dx_masked, const uint16_t *mask_cm,
                              void *scratch, hipStream_t st)
{
    const ConvDims d{n, h, w};
    const uint64_t cm = al256((uint64_t)n * h * w * 32 * 2);
    uint16_t *xcm = static_cast<uint16_t *>(scratch);
    uint16_t *gcm = reinterpret_cast<uint16_t *>(static_cast<char *>(scratch) + cm);
    float *part = reinterpret_cast<float *>(static_cast<char *>(scratch) + 2 * cm);
    if (l == 0)
        to_cm<3, true>(in, d, xcm, st);
    else
        to_cm<32, false>(in, d, xcm, st);
    if (l == 3)
        to_cm<2, false>(dy, d, gcm, st);
    else
        to_cm<32, false>(dy, d, gcm, st);
    wgrad_launch(l, xcm, gcm, d, part, dw, db, st);
    if (l > 0 && (dx_f32 || dx_masked))
        conv_launch(l, true, dy, d, prep, false, nullptr, dx_f32, dx_masked, mask_cm, nullptr, st);
    return hipGetLastError();
}

// Workspace of the whole-network calls: 3 hidden activations (BF16, 32 ch),
// output (FP32, 2 ch), output gradient (BF16, 2 ch), two hidden gradients
// (BF16, 32 ch), channel-major copies of the input, the activations and the
// gradients, gradient vector, loss partials, weight-gradient slots.
struct CnnWs {
    uint16_t *act[3], *gout, *gh[2];
    uint16_t *x_cm, *act_cm[3], *gout_cm, *gh_cm[2];
    float *out, *grad, *part;
    double *lpart, *loss;
    uint64_t total;
};

constexpr int kLossBlocks = 2048;

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
    s.x_cm = reinterpret_cast<uint16_t *>(take(P * 3 * 2));
    for (int k = 0; k < 3; ++k) s.act_cm[k] = reinterpret_cast<uint16_t *>(take(P * 32 * 2));
    s.gout_cm = reinterpret_cast<uint16_t *>(take(P * 2 * 2));
    for (int k = 0; k < 2; ++k) s.gh_cm[k] = reinterpret_cast<uint16_t *>(take(P * 32 * 2));
    s.grad = reinterpret_cast<float *>(take(QSQ_CNN_PARAMS * 4));
    s.lpart = reinterpret_cast<double *>(take(kLossBlocks * 8));
    s.loss = reinterpret_cast<double *>(take(8));
    s.part = reinterpret_cast<float *>(take(train_part_bytes(ConvDims{n, h, w})));
    s.total = o;
    return s;
}

uint64_t cnn_workspace_bytes(int64_t n, int h, int w) { return ws_layout(nullptr, n, h, w).total; }

// forward through the four layers; with cm, also the channel-major copies of
// the hidden activations (for the weight gradients of a training step)
static void forward_layers(const void *prep, const float *x, ConvDims d, float *out, const CnnWs &s, bool cm,
                           hipStream_t st)
{
    conv_launch(0, false, x, d, prep, true, s.act[0], nullptr, nullptr, nullptr, cm ? s.act_cm[0] : nullptr, st);
    conv_launch(1, false, s.act[0], d, prep, true, s.act[1], nullptr, nullptr, nullptr, cm ? s.act_cm[1] : nullptr,
                st);
    conv_launch(2, false, s.act[1], d, prep, true, s.act[2], nullptr, nullptr, nullptr, cm ? s.act_cm[2] : nullptr,
                st);
    conv_launch(3, false, s.act[2], d, prep, false, nullptr, out, nullptr, nullptr, nullptr, st);
}

hipError_t cnn_forward(const void *prep, const float *x, int64_t n, int h, int w, float *out, void *ws, hipStream_t st)
{
    forward_layers(prep, x, ConvDims{n, h, w}, out, ws_layout(ws, n, h, w), false, st);
    return hipGetLastError();
}

hipError_t cnn_train_step(float *params, float *adam_m, float *adam_v, int64_t t, float lr, const float *x,
                          const float *mask, const float *logq, int64_t n, int h, int w, float lam, void *prep,
                          float *grad_out, double *loss_out, void *ws, hipStream_t st)
{
    const CnnWs s = ws_layout(ws, n, h, w);
    const ConvDims d{n, h, w};
    const int64_t P = n * h * w;
    to_cm<3, true>(x, d, s.x_cm, st);
    forward_layers(prep, x, d, s.out, s, true, st);
    const int lb = (int)(blocks_for(P, 256) < kLossBlocks ? blocks_for(P, 256) : kLossBlocks);
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, st, s.out, mask, logq, P, lam, s.gout, s.lpart, w, s.gout_cm);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, s.lpart, lb, loss_out ? loss_out : s.loss);
    float *g = grad_out ? grad_out : s.grad;
    // layer 4 .. 1: weight gradients, then the input gradient masked by the
    // ReLU of the layer below (its BF16 activation > 0)
    // (each layer's weight-gradient slots in a region of their own; one
    // reduction of all four layers after the last)
    const uint16_t *gin = s.gout, *gin_cm = s.gout_cm;
    RedJob J{};
    float *part = s.part;
    for (int l = 3; l >= 0; --l) {
        const uint16_t *xcm = l == 0 ? s.x_cm : s.act_cm[l - 1];
        float *dw = g + master_w(l), *db = dw + 9 * kCi[l] * kCo[l];
        wgrad_slots_launch(l, xcm, gin_cm, d, part, dw, db, J, st);
        part += slot_bytes(d, l) / 4;
        if (l > 0) {
            // the input gradient of layer 1 feeds only layer 0's weight
            // gradient: its channel-major copy alone
            uint16_t *gnext = l > 1 ? s.gh[l % 2] : nullptr, *gnext_cm = s.gh_cm[l % 2];
            conv_launch(l, true, gin, d, prep, false, nullptr, nullptr, gnext, s.act_cm[l - 1], gnext_cm, st);
            gin = gnext;
            gin_cm = gnext_cm;
        }
    }
    wgrad_reduce(J, part, d, st);
    // Kingma & Ba's defaults; every constant is formed in FP64 and rounded once
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)t)), c2 = (float)(1.0 - pow(b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(QSQ_CNN_PARAMS, 256)), dim3(256), 0, st, params, g, adam_m, adam_v,
                       (int64_t)QSQ_CNN_PARAMS, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f,
                       c1, c2, static_cast<uint16_t *>(prep));
    return hipGetLastError();
}

}  // namespace qsq
