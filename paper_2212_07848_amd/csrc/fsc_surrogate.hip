// fsc_surrogate.hip -- learned coarse-grained surrogate of the phase-separating
// lattice: a small periodic convolutional network that maps the block-averaged
// density at time t to the one at t + k lattice steps.  Not part of the paper:
// it is the inference/training path next to the lattice, assessed against the
// lattice's own S(k, t) and L(t).
//
// Network (C = 32 hidden channels, L layers, K = 1 or 2 input channels):
//   x_0 = (rho_t - mean)/in_scale,  x_1 = (rho_t - rho_{t-k})/out_scale (K = 2)
//   a_0 = SiLU(conv(x));  a_l = SiLU(conv(a_{l-1}));  y = conv(a_{L-2})
//   rho_{t+k} = rho_t + out_scale (y - <y>_image)
// The second channel, the last increment, carries the flow that the density
// alone does not determine.
// conv = 3x3 cross-correlation with circular padding.  The C -> C layers run
// as implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation), forward, backward-data and backward-weight.  The C -> 1
// forward runs on the matrix cores too, with its FP32 weights split exactly
// into three BF16 parts; the 1 -> C layer, the other C -> 1 passes and the
// reductions are FP32 vector code.  Parameters are FP32 masters updated by
// Adam; BF16 copies feed the matrix cores.
//
// Activations are NHWC: pixel p = (n H + y) W + x, channel fastest.
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fsc.h"
#include "fsc_internal.h"

namespace fsc {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int SC = 32;          // hidden channels
constexpr int IMG_PARTS = 256;  // segments per image of the per-image FP64 sums

// SiLU and its derivative from the hardware exp2 and reciprocal (about one
// ulp each).  Their results are rounded to bfloat16 (2^-8 relative) or feed
// FP32 sums, so a correctly rounded exp and division would change nothing
// but the cost, which in the matrix-core layers is the epilogue's.
__device__ __forceinline__ float sigmoid(float z) {
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-1.44269504088896341f * z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigmoid(z);
    return s * (1.f + z * (1.f - s));
}
__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// Matrix-core operand layout of v_mfma_f32_16x16x32_bf16 as used here: lane l
// supplies row (l % 16) of A and column (l % 16) of B with the eight K values
// 8 (l / 16) .. 8 (l / 16) + 7; the result element D[4 (l / 16) + r][l % 16] is
// register r of lane l.  (Any K order that is the same for A and B gives the
// same product; the M/N/D placement is checked by fsc_mfma_probe.)
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Output channel of row m (0..15) of the A operand in MFMA tile nt (0, 1) of a
// C -> C layer: rows 4j .. 4j + 3 of tile nt hold channels 8j + 4nt .. 8j +
// 4nt + 3.  The result rows 4 (l/16) + r of lane l are then channels
// 8 (l/16) + 4nt + r: over both tiles, the eight consecutive channels
// 8 (l/16) .. 8 (l/16) + 7 of pixel l % 16, and one 16-byte store per lane
// writes whole 64-byte pixel records (a wave's store covers 1 KB).
__device__ __forceinline__ int mid_row_channel(int nt, int m) { return 8 * (m >> 2) + 4 * nt + (m & 3); }

// Epilogue of a C -> C layer tile computed as D = W (32 channels) x A (16
// pixels): lane l holds channels 8 (l/16) + 4nt + r, r = 0..3, of pixel l % 16
// in acc[nt] (mid_row_channel).  The forward pass starts its accumulators at
// the bias, so acc is already z.
//   forward:  z = acc (kept if ZOUT), a = bf16(SiLU(z))
//   backward: a = bf16(acc SiLU'(z_prev))
template <bool BWD, bool ZOUT>
__device__ __forceinline__ void mid_epilogue(const f32x4 (&acc)[2], size_t pix, int g,
                                             float *__restrict__ zout, bf16 *__restrict__ aout,
                                             const float *__restrict__ zprev) {
    const size_t o = pix * SC + 8 * g;
    bf16x8 out;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        if (BWD) {
            const f32x4 zp = *reinterpret_cast<const f32x4 *>(zprev + o + 4 * nt);
#pragma unroll
            for (int r = 0; r < 4; ++r) out[4 * nt + r] = bf16(acc[nt][r] * dsilu(zp[r]));
        } else {
            if (ZOUT) *reinterpret_cast<f32x4 *>(zout + o + 4 * nt) = acc[nt];
#pragma unroll
            for (int r = 0; r < 4; ++r) out[4 * nt + r] = bf16(silu(acc[nt][r]));
        }
    }
    // non-temporal: the next layer reads the records from memory anyway
    // (3% per rollout pass against the default policy)
    __builtin_nontemporal_store(out, reinterpret_cast<bf16x8 *>(aout + o));
}

__global__ void k_mfma_probe(const float *A, const float *B, float *Cm) {
    const int l = threadIdx.x, r16 = l & 15, g = l >> 4;
    bf16x8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = bf16(A[r16 * 32 + 8 * g + e]);
        b[e] = bf16(B[(8 * g + e) * 16 + r16]);
    }
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(a, b, c);
    for (int r = 0; r < 4; ++r) Cm[(4 * g + r) * 16 + r16] = c[r];
}

// ---------------------------------------------------------------------------
// Network input X[p][K] (FP32) from the current and previous fields.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_input(const float *__restrict__ cur,
                                               const float *__restrict__ prev, int P, int K,
                                               float mean, float inv_in, float inv_out,
                                               float *__restrict__ X) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const float c = cur[p];
    X[size_t(p) * K] = (c - mean) * inv_in;
    if (K == 2) X[size_t(p) * K + 1] = (c - prev[p]) * inv_out;
}

// ---------------------------------------------------------------------------
// Layer 0 (K -> C) forward, FP32: one lane per pixel computes all 32 output
// channels.  The weights and biases are the same for every lane, so they are
// read through the scalar cache and enter the FMAs as scalar operands.  ZOUT
// keeps the FP32 pre-activations for the backward pass (training); FUSED
// forms the network input from the fields on the fly (inference: no X buffer,
// one launch less).  A pixel's 32 BF16 activations go out as four 16-byte
// stores.
// ---------------------------------------------------------------------------
template <int K, bool ZOUT, bool FUSED>
__global__ void __launch_bounds__(256) k_first(const float *__restrict__ X, const float *__restrict__ cur,
                                               const float *__restrict__ prev, float mean, float inv_in,
                                               float inv_out, int B, int H, int W,
                                               const float *__restrict__ w,
                                               const float *__restrict__ b, float *__restrict__ z,
                                               bf16 *__restrict__ a) {
    const int P = B * H * W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int x = p % W, t = p / W, y = t % H, n = t / H;
    float xi[K][9];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const size_t q = size_t((n * H + wrapi(y + ky - 1, H)) * W + wrapi(x + kx - 1, W));
            if constexpr (FUSED) {
                const float c = cur[q];
                xi[0][ky * 3 + kx] = (c - mean) * inv_in;
                if constexpr (K == 2) xi[1][ky * 3 + kx] = (c - prev[q]) * inv_out;
            } else {
#pragma unroll
                for (int ci = 0; ci < K; ++ci) xi[ci][ky * 3 + kx] = X[q * K + ci];
            }
        }
#pragma unroll
    for (int c8 = 0; c8 < SC / 8; ++c8) {
        bf16x8 out;
        f32x4 zq[2];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int co = c8 * 8 + j;
            float acc = b[co];
#pragma unroll
            for (int ci = 0; ci < K; ++ci)
#pragma unroll
                for (int k = 0; k < 9; ++k) acc += w[(co * K + ci) * 9 + k] * xi[ci][k];
            zq[j >> 2][j & 3] = acc;
            out[j] = bf16(silu(acc));
        }
        if constexpr (ZOUT) {
            *reinterpret_cast<f32x4 *>(z + size_t(p) * SC + c8 * 8) = zq[0];
            *reinterpret_cast<f32x4 *>(z + size_t(p) * SC + c8 * 8 + 4) = zq[1];
        }
        *reinterpret_cast<bf16x8 *>(a + size_t(p) * SC + c8 * 8) = out;
    }
}

// ---------------------------------------------------------------------------
// C -> C layer on the matrix cores.  A wave computes 16 consecutive pixels of
// one image row for all 32 output channels: 9 taps x 2 tiles of 16x16x32
// MFMA, with the packed weights held in registers.  The weights are the A
// operand (16 output channels by 32 input channels) and the activations the B
// operand (32 input channels by 16 pixels); with the rows ordered by
// mid_row_channel, each lane's results over the two tiles are eight
// consecutive channels of one pixel (mid_epilogue).
//   forward:   out = conv(a_in; W) + bias -> z (FP32), SiLU(z) (BF16)
//   backward:  out = conv(dZ; W') (W' = tap-flipped transpose: the adjoint)
//              -> dZ_prev = out * SiLU'(z_prev) (BF16)
// ---------------------------------------------------------------------------
template <bool BWD, bool ZOUT = true>
__global__ void __launch_bounds__(256) k_mid(const bf16 *__restrict__ ain,
                                             const bf16 *__restrict__ wpk,
                                             const float *__restrict__ bias, int B, int H, int W,
                                             float *__restrict__ zout, bf16 *__restrict__ aout,
                                             const float *__restrict__ zprev) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * 4;
    const int r16 = lane & 15, g = lane >> 4;
    bf16x8 bop[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
            bop[t][nt] = *reinterpret_cast<const bf16x8 *>(
                wpk + (t * SC + mid_row_channel(nt, r16)) * SC + g * 8);
    f32x4 bv[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    if (!BWD) {
        bv[0] = *reinterpret_cast<const f32x4 *>(bias + 8 * g);
        bv[1] = *reinterpret_cast<const f32x4 *>(bias + 8 * g + 4);
    }
    const int tiles = (B * H * W) / 16;
    for (int tile = wave; tile < tiles; tile += nwaves) {
        const int p0 = tile * 16;
        const int x0 = p0 % W, t2 = p0 / W, y = t2 % H, n = t2 / H;
        f32x4 acc[2] = {bv[0], bv[1]};
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int rowbase = (n * H + wrapi(y + ky - 1, H)) * W;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int q = rowbase + wrapi(x0 + r16 + kx - 1, W);
                const bf16x8 aop = *reinterpret_cast<const bf16x8 *>(ain + size_t(q) * SC + g * 8);
                acc[0] = mfma16(bop[ky * 3 + kx][0], aop, acc[0]);
                acc[1] = mfma16(bop[ky * 3 + kx][1], aop, acc[1]);
            }
        }
        mid_epilogue<BWD, ZOUT>(acc, size_t(p0 + r16), g, zout, aout, zprev);
    }
}

// The same layer with the input staged in LDS: a block computes a tile of
// MR rows x MW pixels of one image (MR MW / 16 MFMA tiles of 16 pixels, dealt
// to the 4 waves in order), after loading the tile's (MR+2) x (MW+2) input
// pixels with their 32 channels once (coalesced 16-byte pieces) instead of
// reading each pixel for each of the 9 taps from L2.  Needs H % MR == 0 and
// W % MW == 0.  The tile shape is a build-time choice (FSC_SUR_MR, FSC_SUR_MW).
#ifndef FSC_SUR_MR
#define FSC_SUR_MR 4
#endif
#ifndef FSC_SUR_MW
#define FSC_SUR_MW 64
#endif
constexpr int MR = FSC_SUR_MR, MW = FSC_SUR_MW;
static_assert(MW % 16 == 0 && (MR * MW / 16) % 4 == 0, "whole MFMA tiles, the same count per wave");
template <bool BWD, bool ZOUT>
__global__ void __launch_bounds__(256) k_mid_lds(const bf16 *__restrict__ ain,
                                                 const bf16 *__restrict__ wpk,
                                                 const float *__restrict__ bias, int B, int H, int W,
                                                 float *__restrict__ zout, bf16 *__restrict__ aout,
                                                 const float *__restrict__ zprev) {
    constexpr int LW = MW + 2;
    __shared__ __attribute__((aligned(16))) bf16 tile_in[(MR + 2) * LW * SC];
#ifdef FSC_LDS_POISON
    lds_poison(tile_in, (MR + 2) * LW * SC);
    __syncthreads();
#endif
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int txs = W / MW, tys = H / MR;
    const int bx = blockIdx.x % txs, t1 = blockIdx.x / txs;
    const int by = t1 % tys, n = t1 / tys;
    const int x0 = bx * MW, y0 = by * MR;
    // stage the input window: pixel (r, c) of the window is image pixel
    // (y0 - 1 + r, x0 - 1 + c), periodic; 4 pieces of 8 channels per pixel
    for (int k = threadIdx.x; k < (MR + 2) * LW * 4; k += 256) {
        const int piece = k & 3, pc = k >> 2;
        const int r = pc / LW, c = pc % LW;
        const int yy = wrapi(y0 - 1 + r, H), xx = wrapi(x0 - 1 + c, W);
        const size_t q = size_t((n * H + yy) * W + xx);
        *reinterpret_cast<bf16x8 *>(tile_in + pc * SC + piece * 8) =
            *reinterpret_cast<const bf16x8 *>(ain + q * SC + piece * 8);
    }
    bf16x8 bop[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
            bop[t][nt] = *reinterpret_cast<const bf16x8 *>(
                wpk + (t * SC + mid_row_channel(nt, r16)) * SC + g * 8);
    f32x4 bv[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    if (!BWD) {
        bv[0] = *reinterpret_cast<const f32x4 *>(bias + 8 * g);
        bv[1] = *reinterpret_cast<const f32x4 *>(bias + 8 * g + 4);
    }
    __syncthreads();
    constexpr int TPW = MR * MW / 64;  // MFMA tiles per wave
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int k = wave * TPW + j;
        const int row = k / (MW / 16), tx = k % (MW / 16);
        const int y = y0 + row;
        f32x4 acc[2] = {bv[0], bv[1]};
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int pc = (row + ky) * LW + tx * 16 + r16 + kx;
                const bf16x8 aop = *reinterpret_cast<const bf16x8 *>(tile_in + pc * SC + g * 8);
                acc[0] = mfma16(bop[ky * 3 + kx][0], aop, acc[0]);
                acc[1] = mfma16(bop[ky * 3 + kx][1], aop, acc[1]);
            }
        const size_t p0 = size_t((n * H + y) * W + x0 + tx * 16);
        mid_epilogue<BWD, ZOUT>(acc, p0 + r16, g, zout, aout, zprev);
    }
}

// Two consecutive C -> C layers A and B of the forward pass (inference) in
// one launch.  A block stages the 8 x 68-pixel input window of its 4 x 64
// output tile, computes layer A on the 6 x 66-pixel window that layer B reads
// (the tile and a one-pixel ring: 24 row tiles of 16 pixels and one tile of
// the 12 ring pixels in the left and right columns) into LDS, then layer B on
// the tile, stored to memory.  Every activation is the same MFMA sequence on
// the same operands as in two k_mid_lds launches, so the results are bit for
// bit those of the unfused layers, without the round trip of layer A's
// activations through memory and one launch less.  Needs H % 4 == 0 and
// W % 64 == 0; without training (layer A's pre-activations are not kept).
constexpr int F2R = 4, F2W = 64;
constexpr int F2IR = F2R + 4, F2IW = F2W + 4;  // input window
constexpr int F2MR = F2R + 2, F2MW = F2W + 2;  // layer A window
__global__ void __launch_bounds__(256) k_mid2_lds(const bf16 *__restrict__ ain,
                                                  const bf16 *__restrict__ wA,
                                                  const float *__restrict__ bA,
                                                  const bf16 *__restrict__ wB,
                                                  const float *__restrict__ bB, int B, int H, int W,
                                                  bf16 *__restrict__ aout) {
    __shared__ __attribute__((aligned(16))) bf16 win[F2IR * F2IW * SC];
    __shared__ __attribute__((aligned(16))) bf16 mid[F2MR * F2MW * SC];
#ifdef FSC_LDS_POISON
    lds_poison(win, F2IR * F2IW * SC);
    lds_poison(mid, F2MR * F2MW * SC);
    __syncthreads();
#endif
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int txs = W / F2W, tys = H / F2R;
    const int bx = blockIdx.x % txs, t1 = blockIdx.x / txs;
    const int by = t1 % tys, n = t1 / tys;
    const int x0 = bx * F2W, y0 = by * F2R;
    // input window: pixel (r, c) is image pixel (y0 - 2 + r, x0 - 2 + c), periodic
    for (int k = threadIdx.x; k < F2IR * F2IW * 4; k += 256) {
        const int piece = k & 3, pc = k >> 2;
        const int r = pc / F2IW, c = pc % F2IW;
        const int yy = ((y0 - 2 + r) % H + H) % H, xx = ((x0 - 2 + c) % W + W) % W;
        const size_t q = size_t((n * H + yy) * W + xx);
        *reinterpret_cast<bf16x8 *>(win + pc * SC + piece * 8) =
            *reinterpret_cast<const bf16x8 *>(ain + q * SC + piece * 8);
    }
    bf16x8 bop[9][2];
    f32x4 bv[2];
    auto load_layer = [&](const bf16 *__restrict__ wpk, const float *__restrict__ bias) {
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                bop[t][nt] = *reinterpret_cast<const bf16x8 *>(
                    wpk + (t * SC + mid_row_channel(nt, r16)) * SC + g * 8);
        bv[0] = *reinterpret_cast<const f32x4 *>(bias + 8 * g);
        bv[1] = *reinterpret_cast<const f32x4 *>(bias + 8 * g + 4);
    };
    // acc = bias + sum over taps of W_tap x (32 channels of the tap pixel);
    // `src` is the window and (r, c) the window position of tap (0, 0)
    auto tile = [&](const bf16 *src, int sw, int r, int c, f32x4 (&acc)[2]) {
        acc[0] = bv[0];
        acc[1] = bv[1];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const bf16x8 aop =
                    *reinterpret_cast<const bf16x8 *>(src + ((r + ky) * sw + c + kx) * SC + g * 8);
                acc[0] = mfma16(bop[ky * 3 + kx][0], aop, acc[0]);
                acc[1] = mfma16(bop[ky * 3 + kx][1], aop, acc[1]);
            }
    };
    load_layer(wA, bA);
    __syncthreads();
    // layer A: window pixel (mr, mc) is image pixel (y0 - 1 + mr, x0 - 1 + mc);
    // its tap (0, 0) is input window pixel (mr, mc)
    for (int t = wave; t < F2MR * (F2W / 16) + 1; t += 4) {  // wave-uniform
        int mr, mc;
        bool keep = true;
        if (t < F2MR * (F2W / 16)) {
            mr = t / (F2W / 16);
            mc = 1 + 16 * (t % (F2W / 16)) + r16;
        } else {  // the ring columns 0 and F2MW - 1 of the F2MR rows; 4 lanes spare
            keep = r16 < 2 * F2MR;
            const int e = keep ? r16 : 0;
            mr = e >> 1;
            mc = (e & 1) ? F2MW - 1 : 0;
        }
        f32x4 acc[2];
        tile(win, F2IW, mr, mc, acc);
        bf16x8 out;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[4 * nt + r] = bf16(silu(acc[nt][r]));
        if (keep) *reinterpret_cast<bf16x8 *>(mid + (mr * F2MW + mc) * SC + 8 * g) = out;
    }
    __syncthreads();
    load_layer(wB, bB);
    // layer B: output pixel (y0 + row, x0 + cx), its tap (0, 0) is layer-A
    // window pixel (row, cx)
#pragma unroll
    for (int j = 0; j < F2R * F2W / 64; ++j) {
        const int k = wave * (F2R * F2W / 64) + j;
        const int row = k / (F2W / 16), cx = 16 * (k % (F2W / 16)) + r16;
        f32x4 acc[2];
        tile(mid, F2MW, row, cx, acc);
        const size_t p = size_t((n * H + y0 + row) * W + x0 + cx);
        mid_epilogue<false, false>(acc, p, g, nullptr, aout, nullptr);
    }
}

// ---------------------------------------------------------------------------
// Last layer (C -> 1) forward on the matrix cores.  Its FP32 weights enter as
// three BF16 parts each, w = hi + mid + lo (k_pack_last; exact for normal FP32
// values), in rows 0..2 of the A operand (rows 3..15 zero); B is 32 channels
// by 16 pixels for one tap, and the 9 taps accumulate.  Lane l < 16 ends with
// the three partial sums of pixel l in acc[0..2]: y = (hi + mid) + lo + bias.
// The products of BF16 activations with BF16 weight parts are exact and the
// sums FP32, so y is the FP32 evaluation of the layer up to the order of the
// sums.  Each wave takes one of the IMG_PARTS segments of an image: its
// pixels in tiles of 16, two tiles' loads in flight at a time (lanes past the
// segment repeat its last pixel), and the segment's FP64 sum of y (a fixed
// lane order).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_last(const bf16 *__restrict__ a, int B, int H, int W,
                                              const bf16 *__restrict__ wl3,
                                              const float *__restrict__ b, float *__restrict__ y,
                                              double *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const int sg = blockIdx.x * 4 + (threadIdx.x >> 6);  // segment over the batch
    bf16x8 wop[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        if (r16 < 3) {
            wop[t] = *reinterpret_cast<const bf16x8 *>(wl3 + (t * 3 + r16) * SC + g * 8);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) wop[t][e] = bf16(0.f);
        }
    }
    const float bias = b[0];
    const int HW = H * W;
    const int img = sg / IMG_PARTS, seg = sg % IMG_PARTS;
    const int len = (HW + IMG_PARTS - 1) / IMG_PARTS;
    const int lo = seg * len, hi = min(HW, lo + len);
    double s = 0.0;
    for (int i0 = lo; i0 < hi; i0 += 32) {  // wave-uniform: whole waves run the MFMAs
        bf16x8 bop[2][9];
        int pix[2];
        bool on[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = i0 + 16 * u + r16;
            on[u] = i < hi;
            pix[u] = img * HW + (on[u] ? i : hi - 1);
            const int p = pix[u];
            const int x = p % W, t = p / W, yy = t % H, n = t / H;
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int rowbase = (n * H + wrapi(yy + ky - 1, H)) * W;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int q = rowbase + wrapi(x + kx - 1, W);
                    bop[u][ky * 3 + kx] = *reinterpret_cast<const bf16x8 *>(a + size_t(q) * SC + g * 8);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) acc = mfma16(wop[t], bop[u][t], acc);
            if (g == 0 && on[u]) {
                const float v = (acc[0] + acc[1]) + acc[2] + bias;
                y[pix[u]] = v;
                s += double(v);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) part[sg] = s;
}

// Per-image sums of a field in FP64, in a fixed order: stage 1 sums each of
// IMG_PARTS contiguous segments of an image (one block each, a block-wide tree),
// stage 2 sums an image's segment sums (one block per image).
__global__ void __launch_bounds__(256) k_img_part(const float *__restrict__ v, int HW,
                                                  double *__restrict__ part) {
    __shared__ double sh[4];
    const int img = blockIdx.x / IMG_PARTS, seg = blockIdx.x % IMG_PARTS;
    const int len = (HW + IMG_PARTS - 1) / IMG_PARTS;
    const int lo = seg * len, hi = min(HW, lo + len);
    const float *row = v + size_t(img) * HW;
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += 256) s += double(row[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}
// sum of an image's IMG_PARTS segment sums by one wave, in a fixed order
__device__ inline double image_total(const double *__restrict__ part, int img) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < IMG_PARTS / 64; ++k) s += part[img * IMG_PARTS + k * 64 + lane];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}
__global__ void __launch_bounds__(64) k_img_total(const double *__restrict__ part,
                                                  double *__restrict__ out) {
    const double s = image_total(part, blockIdx.x);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}
static_assert(IMG_PARTS % 64 == 0, "a wave sums the segment sums (and k_last's blocks of four)");

// prediction rho_t + out_scale (y - <y>_image); block (image, segment), the
// image's mean from its IMG_PARTS segment sums (summed as k_img_total does)
__global__ void __launch_bounds__(256) k_pred(const float *__restrict__ in,
                                              const float *__restrict__ y,
                                              const double *__restrict__ part, int HW,
                                              float out_scale, float *__restrict__ out) {
    __shared__ float mean_sh;
    const int img = blockIdx.x / IMG_PARTS, seg = blockIdx.x % IMG_PARTS;
    if (threadIdx.x < 64) {
        const double t = image_total(part, img);
        if (threadIdx.x == 0) mean_sh = float(t / HW);
    }
    __syncthreads();
    const float mean = mean_sh;
    const int len = (HW + IMG_PARTS - 1) / IMG_PARTS;
    const int lo = seg * len, hi = min(HW, lo + len);
    for (int i = lo + threadIdx.x; i < hi; i += 256) {
        const size_t p = size_t(img) * HW + i;
        out[p] = in[p] + out_scale * (y[p] - mean);
    }
}

// loss terms and dL/dyhat; loss accumulated in FP64
__global__ void __launch_bounds__(256) k_loss(const float *__restrict__ in,
                                              const float *__restrict__ tgt,
                                              const float *__restrict__ y,
                                              const double *__restrict__ ysum, int P, int HW,
                                              float inv_out_scale, float invM,
                                              float *__restrict__ gout, double *__restrict__ loss) {
    __shared__ double sh[4];
    const int p = blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    if (p < P) {
        const float yhat = y[p] - float(ysum[p / HW] / HW);
        const float e = yhat - (tgt[p] - in[p]) * inv_out_scale;
        gout[p] = 2.f * e * invM;
        e2 = double(e) * double(e);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, sh[0] + sh[1] + sh[2] + sh[3]);
}

// Last layer backward-data: dZ_{L-2}[p][c] = SiLU'(z) sum_t dy[p - off(t)] W[c][t]
// with dy = g - <g>_image (the mean-free projection's adjoint).
__global__ void __launch_bounds__(256) k_last_bwd(const float *__restrict__ g,
                                                  const double *__restrict__ gsum, int B, int H,
                                                  int W, const float *__restrict__ w,
                                                  const float *__restrict__ zprev,
                                                  bf16 *__restrict__ dz) {
    const int P = B * H * W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int x = p % W, t = p / W, yy = t % H, n = t / H;
    const float gm = float(gsum[n] / (H * W));
    float dyv[9];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
            dyv[ky * 3 + kx] = g[(n * H + wrapi(yy - ky + 1, H)) * W + wrapi(x - kx + 1, W)] - gm;
#pragma unroll
    for (int c = 0; c < SC; ++c) {
        float da = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) da += dyv[k] * w[c * 9 + k];
        dz[size_t(p) * SC + c] = bf16(da * dsilu(zprev[size_t(p) * SC + c]));
    }
}

// Weight gradient of the last layer: dW[c][t] = sum_p dy[p] a[p + off(t)][c],
// db = sum_p dy[p].  Block: 32 channels x 8 pixel groups; FP32 atomics.
__global__ void __launch_bounds__(256) k_last_wgrad(const float *__restrict__ g,
                                                    const double *__restrict__ gsum, int B,
                                                    int H, int W, const bf16 *__restrict__ a,
                                                    float *__restrict__ dw, float *__restrict__ db,
                                                    int chunk) {
    __shared__ float red[8][SC][10];
    const int c = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int P = B * H * W;
    float acc[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int p_begin = blockIdx.x * chunk, p_end = min(P, p_begin + chunk);
    for (int p = p_begin + grp; p < p_end; p += 8) {
        const int x = p % W, t = p / W, yy = t % H, n = t / H;
        const float dy = g[p] - float(gsum[n] / (H * W));
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int q = (n * H + wrapi(yy + ky - 1, H)) * W + wrapi(x + kx - 1, W);
                acc[ky * 3 + kx] += dy * float(a[size_t(q) * SC + c]);
            }
        acc[9] += dy;
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) red[grp][c][k] = acc[k];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            float s = 0.f;
            for (int q = 0; q < 8; ++q) s += red[q][c][k];
            if (k < 9) atomicAdd(&dw[c * 9 + k], s);
            else if (c == 0) atomicAdd(db, s);
        }
    }
}

// Weight gradient of layer 0: dW[c][ci][t] = sum_p dZ0[p][c] X[p + off(t)][ci],
// db[c] = sum_p dZ0[p][c].  Block: 32 channels x 8 pixel groups; FP32 atomics.
template <int K>
__global__ void __launch_bounds__(256) k_first_wgrad(const bf16 *__restrict__ dz,
                                                     const float *__restrict__ X, int B, int H,
                                                     int W, float *__restrict__ dw,
                                                     float *__restrict__ db, int chunk) {
    constexpr int NT = 9 * K + 1;
    __shared__ float red[8][SC][NT];
    const int c = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int P = B * H * W;
    float acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = 0.f;
    const int p_begin = blockIdx.x * chunk, p_end = min(P, p_begin + chunk);
    for (int p = p_begin + grp; p < p_end; p += 8) {
        const int x = p % W, t = p / W, yy = t % H, n = t / H;
        const float d = float(dz[size_t(p) * SC + c]);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const size_t q = size_t((n * H + wrapi(yy + ky - 1, H)) * W + wrapi(x + kx - 1, W)) * K;
#pragma unroll
                for (int ci = 0; ci < K; ++ci) acc[ci * 9 + ky * 3 + kx] += d * X[q + ci];
            }
        acc[NT - 1] += d;
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) red[grp][c][k] = acc[k];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            float s = 0.f;
            for (int q = 0; q < 8; ++q) s += red[q][c][k];
            if (k < NT - 1) atomicAdd(&dw[c * 9 * K + k], s);
            else atomicAdd(&db[c], s);
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of a C -> C layer on the matrix cores:
//   dW[co][ci][t] = sum_p dZ[p][co] a[p + off(t)][ci],  db[co] = sum_p dZ[p][co]
// a GEMM over K = pixels.  A block stages 32 consecutive pixels of dZ and, for
// the nine taps, of the shifted activations in LDS, transposed to
// [channel][pixel] (one copy per horizontal shift keeps 16-byte reads aligned);
// wave w accumulates taps w, w + 4, w + 8 as 2 x 2 tiles of 16x16x32 MFMA.
// ---------------------------------------------------------------------------
constexpr int WSEG = 32;
constexpr int WPAD = 40;

__global__ void __launch_bounds__(256) k_mid_wgrad(const bf16 *__restrict__ dz,
                                                   const bf16 *__restrict__ ain, int B, int H,
                                                   int W, float *__restrict__ dw,
                                                   float *__restrict__ db) {
    __shared__ __attribute__((aligned(16))) bf16 sdz[SC][WPAD];
    __shared__ __attribute__((aligned(16))) bf16 sa[3][3][SC][WPAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    f32x4 acc[3][2][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[s][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const int nseg = (B * H * W) / WSEG;
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int p0 = seg * WSEG;
        const int x0 = p0 % W, t2 = p0 / W, y = t2 % H, n = t2 / H;
        __syncthreads();
        // dZ tile: 32 pixels x 32 channels, 4 values per thread
        {
            const int e = tid * 4;
            const int j = e / SC, c = e % SC;
#pragma unroll
            for (int k = 0; k < 4; ++k) sdz[c + k][j] = dz[size_t(p0 + j) * SC + c + k];
        }
        // shifted activation tiles
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int rowbase = (n * H + wrapi(y + ky - 1, H)) * W;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int e = tid * 4;
                const int j = e / SC, c = e % SC;
                const size_t q = size_t(rowbase + wrapi(x0 + j + kx - 1, W));
#pragma unroll
                for (int k = 0; k < 4; ++k) sa[kx][ky][c + k][j] = ain[q * SC + c + k];
            }
        }
        __syncthreads();
        if (tid < SC) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < WSEG; ++j) s += float(sdz[tid][j]);
            bacc += s;
        }
        bf16x8 aop[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
            aop[mt] = *reinterpret_cast<const bf16x8 *>(&sdz[mt * 16 + r16][8 * g]);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int t = wave + 4 * s;
            if (t < 9) {
                const int ky = t / 3, kx = t % 3;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const bf16x8 bop =
                        *reinterpret_cast<const bf16x8 *>(&sa[kx][ky][nt * 16 + r16][8 * g]);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) acc[s][mt][nt] = mfma16(aop[mt], bop, acc[s][mt][nt]);
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int t = wave + 4 * s;
        if (t < 9) {
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int co = mt * 16 + 4 * g + r, ci = nt * 16 + r16;
                        atomicAdd(&dw[(co * SC + ci) * 9 + t], acc[s][mt][nt][r]);
                    }
        }
    }
    if (tid < SC) atomicAdd(&db[tid], bacc);
}

// BF16 packings of a C -> C layer: forward wf[t][co][ci], adjoint wb[t][ci][co]
// = W[co][ci][8 - t] (tap flip).
__global__ void k_pack(const float *__restrict__ w, bf16 *__restrict__ wf, bf16 *__restrict__ wb) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= SC * SC * 9) return;
    const int t = k % 9, ci = (k / 9) % SC, co = k / (9 * SC);
    const bf16 v = bf16(w[k]);
    wf[(t * SC + co) * SC + ci] = v;
    wb[((8 - t) * SC + ci) * SC + co] = v;
}

// The last layer's FP32 weights w[c][t] (C -> 1) as three BF16 parts for the
// matrix cores, wl3[t][part][c]: hi = bf16(w), mid = bf16(w - hi), lo =
// bf16(w - hi - mid).  Each difference is exact in FP32, and what lo leaves
// is zero for normal FP32 weights, so hi + mid + lo = w.
__global__ void k_pack_last(const float *__restrict__ w, bf16 *__restrict__ wl3) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= SC * 9) return;
    const int t = k % 9, c = k / 9;
    const float v = w[k];
    const bf16 hi = bf16(v);
    const float r1 = v - float(hi);
    const bf16 mid = bf16(r1);
    const bf16 lo = bf16(r1 - float(mid));
    wl3[(t * 3 + 0) * SC + c] = hi;
    wl3[(t * 3 + 1) * SC + c] = mid;
    wl3[(t * 3 + 2) * SC + c] = lo;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
}

// ---------------------------------------------------------------------------
// Coarse-graining: mean density over f x f blocks of the streamed state.
// ---------------------------------------------------------------------------
template <class L, typename real>
__global__ void __launch_bounds__(256) k_coarsen(Geometry g, const real *__restrict__ src,
                                                 double rho0, int f, float *__restrict__ out) {
    const int cx = g.nx / f, cy = g.ny / f;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= cx * cy) return;
    const int X = k % cx, Y = k / cx;
    double s = 0.0;
    for (int dy = 0; dy < f; ++dy)
        for (int dx = 0; dx < f; ++dx) {
            const int x = X * f + dx, y = Y * f + dy;
            const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
            const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const int c0 = L::c(i, 0), c1 = L::c(i, 1);
                const int xs = c0 == 1 ? xm : (c0 == -1 ? xp : x);
                const int ys = c1 == 1 ? ym : (c1 == -1 ? yp : y);
                s += double(src[int64_t(i) * g.N + xs + int64_t(g.nx) * ys]);
            }
        }
    out[k] = float(rho0 + s / double(f * f));
}

hipError_t launch_coarsen(const Geometry &g, int precision, const void *buf, double rho0, int f,
                          float *out, hipStream_t s) {
    if (g.D != 2 || f < 1 || g.nx % f || g.ny % f) return hipErrorInvalidValue;
    const int n = (g.nx / f) * (g.ny / f);
    const unsigned nb = unsigned((n + 255) / 256);
    if (precision == 0)
        hipLaunchKernelGGL((k_coarsen<D2Q9, float>), dim3(nb), dim3(256), 0, s, g,
                           static_cast<const float *>(buf), rho0, f, out);
    else
        hipLaunchKernelGGL((k_coarsen<D2Q9, double>), dim3(nb), dim3(256), 0, s, g,
                           static_cast<const double *>(buf), rho0, f, out);
    return hipGetLastError();
}

// real field -> complex (for the S(k) pipeline on coarse fields)
__global__ void k_field_cplx(const float *__restrict__ f, int n, float *__restrict__ c) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    c[2 * k] = f[k];
    c[2 * k + 1] = 0.f;
}

hipError_t launch_field_cplx(const float *f, int n, void *c, hipStream_t s) {
    hipLaunchKernelGGL(k_field_cplx, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, f, n,
                       static_cast<float *>(c));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training batches from a snapshot stack S[K][R][H][W]: image b of the batch
// is snapshot t_b + dt of run r_b, moved by a periodic shift and optionally
// transposed (symmetries of the periodic square lattice):
//   out[b][y][x] = S[t_b + dt][r_b][(Y - sy) mod H][(X - sx) mod W],
//   (Y, X) = (x, y) if transposed, else (y, x).
// ---------------------------------------------------------------------------
constexpr int GATHER_MAX = 64;
struct GatherIdx {
    int t[GATHER_MAX], r[GATHER_MAX];
};

__global__ void __launch_bounds__(256) k_gather(const float *__restrict__ snaps, int R, int H,
                                                int W, GatherIdx idx, int dt, int sy, int sx,
                                                int transpose, float *__restrict__ out) {
    const int b = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= H * W) return;
    const int x = k % W, y = k / W;
    const int Y = transpose ? x : y, X = transpose ? y : x;
    int ys = (Y - sy) % H, xs = (X - sx) % W;
    ys += ys < 0 ? H : 0;
    xs += xs < 0 ? W : 0;
    const size_t img = size_t(idx.t[b] + dt) * R + idx.r[b];
    out[size_t(b) * H * W + k] = snaps[img * H * W + size_t(ys) * W + xs];
}

// Partial FP64 sums over a snapshot stack for the data scales: per block,
// sum (x - c) and (x - c)^2 over snapshots t_first.. K-1 and sum d, d^2 of the
// increments d = S[k+1] - S[k], k >= t_first (c: a centre close to the mean).
__global__ void __launch_bounds__(256) k_stack_moments(const float *__restrict__ S, int K,
                                                       int64_t per, int t_first, double c,
                                                       double *__restrict__ part) {
    __shared__ double sh[4][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t n = int64_t(K - t_first) * per;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const int64_t j = int64_t(t_first) * per + i;
        const double v = double(S[j]) - c;
        acc[0] += v;
        acc[1] += v * v;
        if (j + per < int64_t(K) * per) {
            const double d = double(S[j + per]) - double(S[j]);
            acc[2] += d;
            acc[3] += d * d;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        part[blockIdx.x * 4 + q] = sh[0][q] + sh[1][q] + sh[2][q] + sh[3][q];
    }
}

// Clears `words` 32-bit words (a fill kernel rather than a memset node, so the
// clearing can also sit inside a caller's captured graph).
__global__ void k_zero_words(uint32_t *p, int64_t words) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

hipError_t launch_zero_words(void *p, int64_t words, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3(unsigned((words + 255) / 256)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

}  // namespace fsc

// ===========================================================================
// Surrogate object and its C ABI.
// ===========================================================================
using namespace fsc;

struct fsc_sur {
    int layers = 5, in_ch = 1, H = 0, W = 0, maxB = 0;
    float mean = 1.f, in_scale = 1.f, out_scale = 1.f;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t nparams = 0;
    std::vector<int64_t> woff, boff;  // offsets of each layer's weights / biases
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    bf16 *wf = nullptr, *wb = nullptr;  // [mid layer][9][32][32]
    bf16 *wl3 = nullptr;                // last layer, [9][3][32] (k_pack_last)
    std::vector<float *> z;            // [layers - 1] of P x 32
    std::vector<bf16 *> a;             // [layers - 1] of P x 32
    bf16 *dzA = nullptr, *dzB = nullptr;
    float *y = nullptr, *gbuf = nullptr, *X = nullptr;
    double *ysum = nullptr, *gsum = nullptr, *loss = nullptr;
    double *part = nullptr;  // [maxB][IMG_PARTS] segment sums
    int64_t adam_t = 0;
    // captured rollouts: (prev, traj, batch, passes) -> graph, replayed on a
    // stream of the surrogate's own that is ordered after and before `stream`
    hipStream_t cap_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::map<std::tuple<const float *, float *, int, int>, hipGraphExec_t> rollouts;
    std::deque<std::tuple<const float *, float *, int, int>> rollout_order;  // oldest first
    int fuse = 2;  // pairs of C -> C layers as one k_mid2_lds: 0 never, 1 always, 2 small batches
    std::string err;
};

namespace {

thread_local std::string g_sur_error;

int sur_fail(fsc_sur *s, int code, const std::string &msg) {
    if (s) s->err = msg;
    else g_sur_error = msg;
    return code;
}

#define SCHK(s, expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return sur_fail((s), FSC_E_HIP, std::string(#expr) + ": " +   \
                                                                 hipGetErrorString(_e));    \
    } while (0)

int nmid(const fsc_sur *s) { return s->layers - 2; }

void sur_free(fsc_sur *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    void *ptrs[] = {s->params, s->grads, s->m,    s->v,    s->wf,   s->wb, s->wl3, s->dzA,
                    s->dzB,    s->y,     s->gbuf, s->ysum, s->gsum, s->loss, s->X, s->part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto p : s->z)
        if (p) (void)hipFree(p);
    for (auto p : s->a)
        if (p) (void)hipFree(p);
    for (auto &kv : s->rollouts) (void)hipGraphExecDestroy(kv.second);
    if (s->cap_stream) {
        (void)hipStreamSynchronize(s->cap_stream);
        (void)hipStreamDestroy(s->cap_stream);
    }
    if (s->ev_in) (void)hipEventDestroy(s->ev_in);
    if (s->ev_out) (void)hipEventDestroy(s->ev_out);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Fused pairs of C -> C layers (k_mid2_lds) hold 60 KB of LDS per block, so
// 2 blocks per CU instead of 4: measured on 9-layer passes over 128^2 images,
// they win up to 8 images (62.5 against 73.3 us for one, 87.0 against 100.3
// for eight) and lose from 16 (135.9 against 128.3).  Mode 2 fuses up to
// FUSE_MAX_PIXELS pixels per batch.
constexpr int64_t FUSE_MAX_PIXELS = 8 * 128 * 128;
bool fuse_pairs(const fsc_sur *s, int B) {
    return s->fuse == 1 || (s->fuse == 2 && int64_t(B) * s->H * s->W <= FUSE_MAX_PIXELS);
}

// Destroys the captured rollout graphs (after any replay still running), so
// that the next rollout captures the current settings.
int drop_rollouts(fsc_sur *s) {
    if (s->rollouts.empty()) return FSC_OK;
    if (s->cap_stream) SCHK(s, hipStreamSynchronize(s->cap_stream));
    for (auto &kv : s->rollouts) (void)hipGraphExecDestroy(kv.second);
    s->rollouts.clear();
    s->rollout_order.clear();
    return FSC_OK;
}

// Captured rollouts kept per surrogate; beyond that the oldest capture is
// dropped (a caller that hands over fresh buffers every time would otherwise
// grow the cache without bound).
constexpr size_t ROLLOUT_CACHE_MAX = 8;

int pack_weights(fsc_sur *s) {
    for (int l = 1; l <= nmid(s); ++l) {
        const size_t off = size_t(l - 1) * 9 * SC * SC;
        hipLaunchKernelGGL(k_pack, dim3((SC * SC * 9 + 255) / 256), dim3(256), 0, s->stream,
                           s->params + s->woff[l], s->wf + off, s->wb + off);
        SCHK(s, hipGetLastError());
    }
    hipLaunchKernelGGL(k_pack_last, dim3((SC * 9 + 255) / 256), dim3(256), 0, s->stream,
                       s->params + s->woff[s->layers - 1], s->wl3);
    SCHK(s, hipGetLastError());
    return FSC_OK;
}

int check_batch(fsc_sur *s, int batch) {
    if (batch < 1 || batch > s->maxB) return sur_fail(s, FSC_E_INVAL, "batch out of range");
    return FSC_OK;
}

// the LDS-staged C -> C layer applies when its tiles divide the image
bool lds_tiles(const fsc_sur *s) { return s->H % MR == 0 && s->W % MW == 0; }

int img_sums(fsc_sur *s, const float *v, int B, double *out) {
    hipLaunchKernelGGL(k_img_part, dim3(unsigned(B * IMG_PARTS)), dim3(256), 0, s->stream, v,
                       s->H * s->W, s->part);
    SCHK(s, hipGetLastError());
    hipLaunchKernelGGL(k_img_total, dim3(unsigned(B)), dim3(64), 0, s->stream, s->part, out);
    SCHK(s, hipGetLastError());
    return FSC_OK;
}

// forward pass up to y (and the per-image sums of y); `train` keeps what the
// backward pass needs (the FP32 pre-activations and the input X)
int sur_forward_core(fsc_sur *s, const float *prev, const float *cur, int B, bool train) {
    const int P = B * s->H * s->W;
    const unsigned nb = unsigned((P + 255) / 256);
    const float ii = 1.f / s->in_scale, io = 1.f / s->out_scale;
    const float *w0 = s->params + s->woff[0], *b0 = s->params + s->boff[0];
    if (train) {
        hipLaunchKernelGGL(k_input, dim3(nb), dim3(256), 0, s->stream, cur, prev, P, s->in_ch, s->mean,
                           ii, io, s->X);
        SCHK(s, hipGetLastError());
        if (s->in_ch == 2)
            hipLaunchKernelGGL((k_first<2, true, false>), dim3(nb), dim3(256), 0, s->stream, s->X, cur,
                               prev, s->mean, ii, io, B, s->H, s->W, w0, b0, s->z[0], s->a[0]);
        else
            hipLaunchKernelGGL((k_first<1, true, false>), dim3(nb), dim3(256), 0, s->stream, s->X, cur,
                               prev, s->mean, ii, io, B, s->H, s->W, w0, b0, s->z[0], s->a[0]);
    } else {
        if (s->in_ch == 2)
            hipLaunchKernelGGL((k_first<2, false, true>), dim3(nb), dim3(256), 0, s->stream, s->X, cur,
                               prev, s->mean, ii, io, B, s->H, s->W, w0, b0, s->z[0], s->a[0]);
        else
            hipLaunchKernelGGL((k_first<1, false, true>), dim3(nb), dim3(256), 0, s->stream, s->X, cur,
                               prev, s->mean, ii, io, B, s->H, s->W, w0, b0, s->z[0], s->a[0]);
    }
    SCHK(s, hipGetLastError());
    const int tiles = P / 16;
    const unsigned mb = unsigned(std::min(2048, std::max(1, tiles / 16)));
    for (int l = 1; l <= nmid(s); ++l) {
        const size_t off = size_t(l - 1) * 9 * SC * SC;
        const bf16 *ain = s->a[l - 1], *wl = s->wf + off;
        const float *bl = s->params + s->boff[l];
        if (!train && fuse_pairs(s, B) && l + 1 <= nmid(s) && s->H % F2R == 0 && s->W % F2W == 0) {
            // layers l and l + 1 in one launch; a[l] is not written
            const dim3 g(unsigned(B * (s->H / F2R) * (s->W / F2W)));
            hipLaunchKernelGGL(k_mid2_lds, g, dim3(256), 0, s->stream, ain, wl, bl,
                               s->wf + off + size_t(9) * SC * SC, s->params + s->boff[l + 1], B,
                               s->H, s->W, s->a[l + 1]);
            SCHK(s, hipGetLastError());
            ++l;
            continue;
        }
        if (lds_tiles(s)) {
            const dim3 g(unsigned(B * (s->H / MR) * (s->W / MW)));
            if (train)
                hipLaunchKernelGGL((k_mid_lds<false, true>), g, dim3(256), 0, s->stream, ain, wl, bl, B,
                                   s->H, s->W, s->z[l], s->a[l], nullptr);
            else
                hipLaunchKernelGGL((k_mid_lds<false, false>), g, dim3(256), 0, s->stream, ain, wl, bl, B,
                                   s->H, s->W, s->z[l], s->a[l], nullptr);
        } else if (train) {
            hipLaunchKernelGGL((k_mid<false, true>), dim3(mb), dim3(256), 0, s->stream, ain, wl, bl, B,
                               s->H, s->W, s->z[l], s->a[l], nullptr);
        } else {
            hipLaunchKernelGGL((k_mid<false, false>), dim3(mb), dim3(256), 0, s->stream, ain, wl, bl, B,
                               s->H, s->W, s->z[l], s->a[l], nullptr);
        }
        SCHK(s, hipGetLastError());
    }
    const int last = s->layers - 1;
    hipLaunchKernelGGL(k_last, dim3(unsigned(B * IMG_PARTS / 4)), dim3(256), 0, s->stream, s->a[last - 1], B,
                       s->H, s->W, s->wl3, s->params + s->boff[last], s->y, s->part);
    SCHK(s, hipGetLastError());
    if (train) {  // the loss needs the per-image sums of y
        hipLaunchKernelGGL(k_img_total, dim3(unsigned(B)), dim3(64), 0, s->stream, s->part, s->ysum);
        SCHK(s, hipGetLastError());
    }
    return FSC_OK;
}

int sur_backward(fsc_sur *s, const float *in, const float *tgt, int B) {
    const int H = s->H, W = s->W, P = B * H * W;
    const unsigned nb = unsigned((P + 255) / 256);
    SCHK(s, hipMemsetAsync(s->grads, 0, sizeof(float) * s->nparams, s->stream));
    SCHK(s, hipMemsetAsync(s->loss, 0, sizeof(double), s->stream));
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s->stream, in, tgt, s->y, s->ysum, P, H * W,
                       1.f / s->out_scale, 1.f / float(P), s->gbuf, s->loss);
    SCHK(s, hipGetLastError());
    {
        int rc = img_sums(s, s->gbuf, B, s->gsum);
        if (rc) return rc;
    }
    const int last = s->layers - 1;
    const int chunk = 2048;
    const unsigned cb = unsigned((P + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_last_wgrad, dim3(cb), dim3(256), 0, s->stream, s->gbuf, s->gsum, B, H, W,
                       s->a[last - 1], s->grads + s->woff[last], s->grads + s->boff[last], chunk);
    SCHK(s, hipGetLastError());
    bf16 *dz = s->dzA, *dzn = s->dzB;
    hipLaunchKernelGGL(k_last_bwd, dim3(nb), dim3(256), 0, s->stream, s->gbuf, s->gsum, B, H, W,
                       s->params + s->woff[last], s->z[last - 1], dz);
    SCHK(s, hipGetLastError());
    const int tiles = P / 16;
    const unsigned mb = unsigned(std::min(2048, std::max(1, tiles / 16)));
    const unsigned wgb = unsigned(std::min(1024, std::max(1, P / WSEG / 8)));
    for (int l = nmid(s); l >= 1; --l) {
        // dz holds dL/dz_l; weight gradient, then dL/dz_{l-1}
        hipLaunchKernelGGL(k_mid_wgrad, dim3(wgb), dim3(256), 0, s->stream, dz, s->a[l - 1], B, H,
                           W, s->grads + s->woff[l], s->grads + s->boff[l]);
        SCHK(s, hipGetLastError());
        const size_t off = size_t(l - 1) * 9 * SC * SC;
        if (lds_tiles(s))
            hipLaunchKernelGGL((k_mid_lds<true, true>), dim3(unsigned(B * (H / MR) * (W / MW))), dim3(256),
                               0, s->stream, dz, s->wb + off, nullptr, B, H, W, nullptr, dzn, s->z[l - 1]);
        else
            hipLaunchKernelGGL((k_mid<true, true>), dim3(mb), dim3(256), 0, s->stream, dz, s->wb + off,
                               nullptr, B, H, W, nullptr, dzn, s->z[l - 1]);
        SCHK(s, hipGetLastError());
        std::swap(dz, dzn);
    }
    if (s->in_ch == 2)
        hipLaunchKernelGGL(k_first_wgrad<2>, dim3(cb), dim3(256), 0, s->stream, dz, s->X, B, H, W,
                           s->grads + s->woff[0], s->grads + s->boff[0], chunk);
    else
        hipLaunchKernelGGL(k_first_wgrad<1>, dim3(cb), dim3(256), 0, s->stream, dz, s->X, B, H, W,
                           s->grads + s->woff[0], s->grads + s->boff[0], chunk);
    SCHK(s, hipGetLastError());
    return FSC_OK;
}

int check_inputs(fsc_sur *s, const float *prev, const float *cur) {
    if (!cur || (s->in_ch == 2 && !prev))
        return sur_fail(s, FSC_E_INVAL, "missing input field (two-channel networks need prev)");
    return FSC_OK;
}

}  // namespace

extern "C" {

int fsc_sur_create(int layers, int in_ch, int H, int W, int max_batch, uint64_t seed,
                   void *stream, fsc_sur **out) {
    if (!out) return FSC_E_INVAL;
    *out = nullptr;
    if (layers < 3 || layers > 16 || (in_ch != 1 && in_ch != 2) || H < 1 || W < 16 || (W % 32) ||
        max_batch < 1 || int64_t(max_batch) * H * W >= (int64_t(1) << 26))
        return sur_fail(nullptr, FSC_E_INVAL,
                        "need 3 <= layers <= 16, in_ch 1 or 2, W a multiple of 32, batch*H*W < 2^26");
    fsc_sur *s = new fsc_sur();
    s->layers = layers;
    s->in_ch = in_ch;
    s->H = H;
    s->W = W;
    s->maxB = max_batch;
    // NULL is the device's default (null) stream, so that calls are ordered
    // with other work on it (torch's default stream is the null stream)
    s->stream = static_cast<hipStream_t>(stream);
    // parameter layout: per layer W[co][ci][3][3] then b[co]
    int64_t o = 0;
    std::vector<float> host;
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
    auto rnd = [&]() {  // splitmix64 -> uniform in [-1, 1)
        st += 0x9E3779B97F4A7C15ull;
        uint64_t zz = st;
        zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
        zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
        zz ^= zz >> 31;
        return double(zz >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    for (int l = 0; l < layers; ++l) {
        const int ci = l == 0 ? in_ch : SC, co = l == layers - 1 ? 1 : SC;
        s->woff.push_back(o);
        // uniform in +-1/sqrt(fan_in) for weights and biases: a small initial
        // map keeps the rollouts of early training (used as inputs) tame
        const double bound = 1.0 / std::sqrt(double(ci * 9));
        for (int k = 0; k < co * ci * 9; ++k) host.push_back(float(bound * rnd()));
        o += co * ci * 9;
        s->boff.push_back(o);
        for (int k = 0; k < co; ++k) host.push_back(float(bound * rnd()));
        o += co;
    }
    s->nparams = o;
    const size_t P = size_t(max_batch) * H * W;
    bool ok = hipMalloc(&s->params, sizeof(float) * o) == hipSuccess &&
              hipMalloc(&s->grads, sizeof(float) * o) == hipSuccess &&
              hipMalloc(&s->m, sizeof(float) * o) == hipSuccess &&
              hipMalloc(&s->v, sizeof(float) * o) == hipSuccess &&
              hipMalloc(&s->wf, sizeof(bf16) * 9 * SC * SC * std::max(1, layers - 2)) == hipSuccess &&
              hipMalloc(&s->wb, sizeof(bf16) * 9 * SC * SC * std::max(1, layers - 2)) == hipSuccess &&
              hipMalloc(&s->wl3, sizeof(bf16) * 9 * 3 * SC) == hipSuccess &&
              hipMalloc(&s->dzA, sizeof(bf16) * P * SC) == hipSuccess &&
              hipMalloc(&s->dzB, sizeof(bf16) * P * SC) == hipSuccess &&
              hipMalloc(&s->y, sizeof(float) * P) == hipSuccess &&
              hipMalloc(&s->gbuf, sizeof(float) * P) == hipSuccess &&
              hipMalloc(&s->X, sizeof(float) * P * in_ch) == hipSuccess &&
              hipMalloc(&s->ysum, sizeof(double) * max_batch) == hipSuccess &&
              hipMalloc(&s->part, sizeof(double) * IMG_PARTS * max_batch) == hipSuccess &&
              hipMalloc(&s->gsum, sizeof(double) * max_batch) == hipSuccess &&
              hipMalloc(&s->loss, sizeof(double)) == hipSuccess;
    for (int l = 0; ok && l < layers - 1; ++l) {
        float *zz = nullptr;
        bf16 *aa = nullptr;
        ok = hipMalloc(&zz, sizeof(float) * P * SC) == hipSuccess &&
             hipMalloc(&aa, sizeof(bf16) * P * SC) == hipSuccess;
        s->z.push_back(zz);
        s->a.push_back(aa);
    }
    if (!ok) {
        (void)hipGetLastError();
        sur_free(s);
        return sur_fail(nullptr, FSC_E_OOM, "surrogate allocation failed");
    }
    if (hipMemcpy(s->params, host.data(), sizeof(float) * o, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->m, 0, sizeof(float) * o) != hipSuccess ||
        hipMemset(s->v, 0, sizeof(float) * o) != hipSuccess || pack_weights(s) != FSC_OK ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        sur_free(s);
        return sur_fail(nullptr, FSC_E_HIP, "surrogate initialisation failed");
    }
    *out = s;
    return FSC_OK;
}

int fsc_sur_destroy(fsc_sur *s) {
    if (!s) return FSC_E_INVAL;
    sur_free(s);
    return FSC_OK;
}

const char *fsc_sur_last_error(const fsc_sur *s) { return s ? s->err.c_str() : g_sur_error.c_str(); }

int fsc_sur_nparams(const fsc_sur *s, int64_t *n) {
    if (!s || !n) return FSC_E_INVAL;
    *n = s->nparams;
    return FSC_OK;
}

int fsc_sur_set_params(fsc_sur *s, const float *host, int64_t n) {
    if (!s || !host || n != s->nparams) return FSC_E_INVAL;
    SCHK(s, hipMemcpyAsync(s->params, host, sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    int rc = pack_weights(s);
    if (rc) return rc;
    SCHK(s, hipMemsetAsync(s->m, 0, sizeof(float) * n, s->stream));
    SCHK(s, hipMemsetAsync(s->v, 0, sizeof(float) * n, s->stream));
    s->adam_t = 0;
    SCHK(s, hipStreamSynchronize(s->stream));
    return FSC_OK;
}

int fsc_sur_get_params(fsc_sur *s, float *host, int64_t n) {
    if (!s || !host || n != s->nparams) return FSC_E_INVAL;
    SCHK(s, hipMemcpyAsync(host, s->params, sizeof(float) * n, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return FSC_OK;
}

int fsc_sur_set_norm(fsc_sur *s, float mean, float in_scale, float out_scale) {
    if (!s || !(in_scale > 0.f) || !(out_scale > 0.f)) return FSC_E_INVAL;
    if (mean != s->mean || in_scale != s->in_scale || out_scale != s->out_scale) {
        // the captured rollouts hold the old values as kernel arguments
        int rc = drop_rollouts(s);
        if (rc) return rc;
    }
    s->mean = mean;
    s->in_scale = in_scale;
    s->out_scale = out_scale;
    return FSC_OK;
}

int fsc_sur_set_fusion(fsc_sur *s, int mode) {
    if (!s || mode < 0 || mode > 2) return FSC_E_INVAL;
    if (mode != s->fuse) {
        int rc = drop_rollouts(s);  // captured with another kernel sequence
        if (rc) return rc;
    }
    s->fuse = mode;
    return FSC_OK;
}

int fsc_sur_forward(fsc_sur *s, const float *dev_prev, const float *dev_in, float *dev_out,
                    int batch) {
    TraceRange trace_("fsc sur_forward");
    if (!s || !dev_out) return FSC_E_INVAL;
    int rc = check_inputs(s, dev_prev, dev_in);
    if (rc) return rc;
    rc = check_batch(s, batch);
    if (rc) return rc;
    rc = sur_forward_core(s, dev_prev, dev_in, batch, false);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pred, dim3(unsigned(batch * IMG_PARTS)), dim3(256), 0, s->stream, dev_in,
                       s->y, s->part, s->H * s->W, s->out_scale, dev_out);
    SCHK(s, hipGetLastError());
    return FSC_OK;
}

int fsc_sur_grad(fsc_sur *s, const float *dev_prev, const float *dev_in, const float *dev_target,
                 int batch, float *host_grad, double *loss) {
    if (!s || !dev_target) return FSC_E_INVAL;
    int rc = check_inputs(s, dev_prev, dev_in);
    if (rc) return rc;
    rc = check_batch(s, batch);
    if (rc) return rc;
    rc = sur_forward_core(s, dev_prev, dev_in, batch, true);
    if (rc) return rc;
    rc = sur_backward(s, dev_in, dev_target, batch);
    if (rc) return rc;
    if (host_grad)
        SCHK(s, hipMemcpyAsync(host_grad, s->grads, sizeof(float) * s->nparams,
                               hipMemcpyDeviceToHost, s->stream));
    double l = 0.0;
    SCHK(s, hipMemcpyAsync(&l, s->loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    if (loss) *loss = l / double(batch * s->H * s->W);
    return FSC_OK;
}

int fsc_sur_train_step(fsc_sur *s, const float *dev_prev, const float *dev_in,
                       const float *dev_target, int batch, float lr, double *loss) {
    TraceRange trace_("fsc sur_train_step");
    if (!s || !dev_target || !(lr > 0.f)) return FSC_E_INVAL;
    int rc = check_inputs(s, dev_prev, dev_in);
    if (rc) return rc;
    rc = check_batch(s, batch);
    if (rc) return rc;
    rc = sur_forward_core(s, dev_prev, dev_in, batch, true);
    if (rc) return rc;
    rc = sur_backward(s, dev_in, dev_target, batch);
    if (rc) return rc;
    s->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - std::pow(b1, float(s->adam_t));
    const float bc2 = 1.f - std::pow(b2, float(s->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(unsigned((s->nparams + 255) / 256)), dim3(256), 0, s->stream,
                       s->params, s->grads, s->m, s->v, int(s->nparams), lr, b1, b2, 1e-8f, bc1,
                       bc2);
    SCHK(s, hipGetLastError());
    rc = pack_weights(s);
    if (rc) return rc;
    if (loss) {
        double l = 0.0;
        SCHK(s, hipMemcpyAsync(&l, s->loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        *loss = l / double(batch * s->H * s->W);
    }
    return FSC_OK;
}

int fsc_sur_rollout(fsc_sur *s, const float *dev_prev, float *dev_traj, int batch, int passes) {
    TraceRange trace_("fsc sur_rollout");
    if (!s || !dev_traj || passes < 1) return FSC_E_INVAL;
    int rc = check_batch(s, batch);
    if (rc) return rc;
    if (s->in_ch == 2 && !dev_prev)
        return sur_fail(s, FSC_E_INVAL, "missing input field (two-channel networks need prev)");
    if (!s->cap_stream) {
        SCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
        SCHK(s, hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
        SCHK(s, hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
    }
    const size_t img = size_t(batch) * s->H * s->W;
    auto key = std::make_tuple(dev_prev, dev_traj, batch, passes);
    auto it = s->rollouts.find(key);
    if (it == s->rollouts.end()) {
        // capture the passes on the private stream: the forward kernels use
        // no memset nodes, only launches
        hipStream_t user = s->stream;
        s->stream = s->cap_stream;
        hipGraph_t graph = nullptr;
        hipError_t ec = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
        int frc = FSC_OK;
        if (ec == hipSuccess) {
            for (int k = 0; k < passes && frc == FSC_OK; ++k) {
                const float *prev = k == 0 ? dev_prev : dev_traj + (k - 1) * img;
                frc = sur_forward_core(s, prev, dev_traj + k * img, batch, false);
                if (frc == FSC_OK) {
                    hipLaunchKernelGGL(k_pred, dim3(unsigned(batch * IMG_PARTS)), dim3(256), 0,
                                       s->stream, dev_traj + k * img, s->y, s->part, s->H * s->W,
                                       s->out_scale, dev_traj + (k + 1) * img);
                    if (hipGetLastError() != hipSuccess) frc = FSC_E_HIP;
                }
            }
            hipError_t ee = hipStreamEndCapture(s->cap_stream, &graph);
            if (ec == hipSuccess) ec = ee;
        }
        s->stream = user;
        if (frc != FSC_OK || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return frc != FSC_OK ? frc : sur_fail(s, FSC_E_HIP, std::string("rollout capture: ") +
                                                                      hipGetErrorString(ec));
        }
        hipGraphExec_t exec = nullptr;
        ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ec != hipSuccess)
            return sur_fail(s, FSC_E_HIP, std::string("rollout instantiate: ") + hipGetErrorString(ec));
        if (s->rollouts.size() >= ROLLOUT_CACHE_MAX) {
            SCHK(s, hipStreamSynchronize(s->cap_stream));  // no replay of it still running
            auto old = s->rollouts.find(s->rollout_order.front());
            (void)hipGraphExecDestroy(old->second);
            s->rollouts.erase(old);
            s->rollout_order.pop_front();
        }
        it = s->rollouts.emplace(key, exec).first;
        s->rollout_order.push_back(key);
    }
    // ordered after the caller's stream and before its later work
    SCHK(s, hipEventRecord(s->ev_in, s->stream));
    SCHK(s, hipStreamWaitEvent(s->cap_stream, s->ev_in, 0));
    SCHK(s, hipGraphLaunch(it->second, s->cap_stream));
    SCHK(s, hipEventRecord(s->ev_out, s->cap_stream));
    SCHK(s, hipStreamWaitEvent(s->stream, s->ev_out, 0));
    return FSC_OK;
}

int fsc_sur_gather(fsc_sur *s, const float *dev_snaps, int K, int R, const int *host_t,
                   const int *host_r, int batch, int dt, int sy, int sx, int transpose,
                   float *dev_out) {
    if (!s || !dev_snaps || !host_t || !host_r || !dev_out || K < 1 || R < 1) return FSC_E_INVAL;
    if (batch < 1 || batch > GATHER_MAX || batch > s->maxB)
        return sur_fail(s, FSC_E_INVAL, "gather batch out of range");
    if (transpose && s->H != s->W) return sur_fail(s, FSC_E_INVAL, "transpose needs H == W");
    GatherIdx idx{};
    for (int b = 0; b < batch; ++b) {
        if (host_t[b] + dt < 0 || host_t[b] + dt >= K || host_r[b] < 0 || host_r[b] >= R)
            return sur_fail(s, FSC_E_INVAL, "gather index out of the snapshot stack");
        idx.t[b] = host_t[b];
        idx.r[b] = host_r[b];
    }
    const int HW = s->H * s->W;
    const dim3 g(unsigned((HW + 255) / 256), unsigned(batch));
    hipLaunchKernelGGL(k_gather, g, dim3(256), 0, s->stream, dev_snaps, R, s->H, s->W, idx, dt,
                       ((sy % s->H) + s->H) % s->H, ((sx % s->W) + s->W) % s->W, transpose ? 1 : 0,
                       dev_out);
    SCHK(s, hipGetLastError());
    return FSC_OK;
}

int fsc_stack_scales(const float *dev_snaps, int K, int64_t per_snap, int t_first, double centre,
                     double *host_in_std, double *host_out_std, void *stream) {
    if (!dev_snaps || K < 2 || per_snap < 1 || t_first < 0 || t_first > K - 2 || !host_in_std ||
        !host_out_std)
        return FSC_E_INVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = 1024;
    double *part = nullptr;
    if (hipMalloc(&part, sizeof(double) * 4 * nb) != hipSuccess) return FSC_E_OOM;
    hipLaunchKernelGGL(k_stack_moments, dim3(nb), dim3(256), 0, st, dev_snaps, K, per_snap, t_first,
                       centre, part);
    std::vector<double> h(4 * nb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), part, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return FSC_E_HIP;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 4; ++q) a[q] += h[4 * b + q];
    const double n = double(K - t_first) * double(per_snap);
    const double nd = double(K - 1 - t_first) * double(per_snap);
    *host_in_std = std::sqrt((a[1] - a[0] * a[0] / n) / (n - 1.0));
    *host_out_std = std::sqrt((a[3] - a[2] * a[2] / nd) / (nd - 1.0));
    return FSC_OK;
}

int fsc_mfma_probe(const float *host_a, const float *host_b, float *host_c) {
    if (!host_a || !host_b || !host_c) return FSC_E_INVAL;
    float *d = nullptr;
    if (hipMalloc(&d, sizeof(float) * (16 * 32 + 32 * 16 + 16 * 16)) != hipSuccess) return FSC_E_OOM;
    hipError_t e = hipMemcpy(d, host_a, sizeof(float) * 512, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + 512, host_b, sizeof(float) * 512, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, nullptr, d, d + 512, d + 1024);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(host_c, d + 1024, sizeof(float) * 256, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? FSC_OK : FSC_E_HIP;
}

}  // extern "C"
