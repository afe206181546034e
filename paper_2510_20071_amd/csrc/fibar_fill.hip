// Learned stale fill on gfx950 (C ABI in include/fibar_fill.h).
//
// Activations are NHWC with 16 BF16 channels per pixel (32 bytes; the 3 input
// channels are zero-padded to 16, the 1 output channel is channel 0 of 16).
// A 3x3 layer is an implicit GEMM per 16-pixel row segment: the weights of
// two taps (output channels x 32) times the segment's shifted inputs (32 x 16
// pixels) in one v_mfma_f32_16x16x32_bf16, five per segment, FP32
// accumulation.  Operand lane layouts (checked on the device): for the
// 16x16x16 product lane l holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16]
// and D[4 (l / 16) + j][l % 16], j = 0..3; for 16x16x32, A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16], j = 0..7, with the same D.  Weights are stored
// per lane in operand order, so a lane loads an operand with one read.
//
// The input gradient of a layer is the same kernel with the tap-flipped,
// channel-transposed weights; the weight gradient is a GEMM over the columns
// of a row per tap (gradient x shifted input), summed per workgroup and then
// over workgroups in a fixed order, so training is deterministic.  Inference
// runs all four layers of a tile in one fused kernel.
#include "fibar.h"
#include "fibar_fill.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr int kC = 16;                          // channels of every activation
constexpr int kLayers = 4;
constexpr int kTaps = 9;
constexpr int kGradBlocks = 1024;               // workgroups of a weight gradient (256: 0.55 ms per training step, 1024: 0.37, 2048: 0.41)
constexpr int kWgEntries = kTaps * kC * kC + kC;   // one layer's (w, b) gradient, padded
constexpr int kLossBlocks = 256;
constexpr int kPairs = 5;                       // taps in pairs for the K = 32 products
constexpr int kPairs0 = 2;                      // K = 32 products of the first layer

__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 3 : 16; }
__host__ __device__ constexpr int cout_of(int l) { return l == 3 ? 1 : 16; }
__host__ __device__ constexpr int w_off(int l)
{
    return l == 0 ? 0 : l == 1 ? 448 : l == 2 ? 2768 : 5088;
}
__host__ __device__ constexpr int b_off(int l) { return w_off(l) + cout_of(l) * cin_of(l) * kTaps; }
static_assert(b_off(3) + 1 == FIBAR_FILL_PARAMS, "parameter layout");

typedef short bf16x4 __attribute__((__vector_size__(4 * sizeof(short))));
typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Weights: FP32 master parameters -> per-lane BF16 MFMA operands.
// wf[l][t][lane] = w[o = lane % 16][c = 4 (lane / 16) + j][t]        (forward)
// wb[l][t][lane] = w[o = 4 (lane / 16) + j][c = lane % 16][8 - t]   (input gradient)
// bias[l][o], zero beyond the layer's channels.  Grid: (4 layers x 9 taps), 64 threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_fill_pack_weights(const float* __restrict__ prm,
                                                          bf16x4* __restrict__ wf,
                                                          bf16x4* __restrict__ wb,
                                                          float* __restrict__ bias,
                                                          uint4* __restrict__ wk,
                                                          uint4* __restrict__ wpf,
                                                          uint4* __restrict__ wpb)
{
    const int l = blockIdx.x / kTaps, t = blockIdx.x % kTaps, lane = threadIdx.x;
    const int ci = cin_of(l), co = cout_of(l);
    const float* w = prm + w_off(l);
    bf16x4 f, b;
    for (int j = 0; j < 4; ++j) {
        const int fo = lane & 15, fc = 4 * (lane >> 4) + j;
        f[j] = (short)((fo < co && fc < ci) ? to_bf16(w[(fo * ci + fc) * kTaps + t]) : 0);
        const int bo = 4 * (lane >> 4) + j, bc = lane & 15;
        b[j] = (short)((bo < co && bc < ci) ? to_bf16(w[(bo * ci + bc) * kTaps + (kTaps - 1 - t)])
                                            : 0);
    }
    wf[(l * kTaps + t) * 64 + lane] = f;
    wb[(l * kTaps + t) * 64 + lane] = b;
    if (t == 0 && lane < kC) bias[l * kC + lane] = lane < co ? prm[b_off(l) + lane] : 0.f;
    // K = 32 operands of tap pairs for the layer-by-layer kernel, every layer:
    // pair q = t < 5, lane group g: tap 2q + g / 2 (a tenth tap is zero),
    // channels 8 (g % 2) + j of the operand's K side.
    //   wpf: A[m = o][k] = w[o][c = 8 (g % 2) + j][tap]                (forward)
    //   wpb: A[m = c][k] = w[o = 8 (g % 2) + j][c][8 - tap]            (input gradient)
    if (t < kPairs) {
        const int g = lane >> 4, m = lane & 15, tap = 2 * t + (g >> 1);
        uint16_t hf[8], hb[8];
        for (int j = 0; j < 8; ++j) {
            const int kc = 8 * (g & 1) + j;
            hf[j] = (tap < kTaps && m < co && kc < ci) ? to_bf16(w[(m * ci + kc) * kTaps + tap]) : 0;
            hb[j] = (tap < kTaps && kc < co && m < ci)
                        ? to_bf16(w[(kc * ci + m) * kTaps + (kTaps - 1 - tap)])
                        : 0;
        }
        wpf[(l * kPairs + t) * 64 + lane] =
            make_uint4(hf[0] | (uint32_t)hf[1] << 16, hf[2] | (uint32_t)hf[3] << 16,
                       hf[4] | (uint32_t)hf[5] << 16, hf[6] | (uint32_t)hf[7] << 16);
        wpb[(l * kPairs + t) * 64 + lane] =
            make_uint4(hb[0] | (uint32_t)hb[1] << 16, hb[2] | (uint32_t)hb[3] << 16,
                       hb[4] | (uint32_t)hb[5] << 16, hb[6] | (uint32_t)hb[7] << 16);
    }
    // K = 32 operands of tap pairs (2q, 2q + 1), q = t < 5: lane group g takes
    // tap 2q + g / 2, input channels 8 (g % 2) + j, j = 0..7; tap 9 is zero.
    // The first layer (3 input channels) instead packs 4 channels per tap:
    // operand q < 2, lane group g takes taps 8q + 2g + j / 4, channel j % 4.
    if (l == 0 && t < kPairs0) {
        const int g = lane >> 4, o = lane & 15;
        uint16_t h[8];
        for (int j = 0; j < 8; ++j) {
            const int tap = 8 * t + 2 * g + j / 4, c = j % 4;
            h[j] = (tap < kTaps && o < co && c < ci) ? to_bf16(w[(o * ci + c) * kTaps + tap]) : 0;
        }
        wk[t * 64 + lane] = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                                       h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
    } else if (l == kLayers - 1 && t == 0) {
        // the last layer (one output channel) in the fused kernel: B of a
        // 16x16x16 product, column n = tap, k = input channel 4 (lane / 16) + j
        const int tap = lane & 15;
        uint16_t h[4];
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * (lane >> 4) + j;
            h[j] = (tap < kTaps && co > 0 && c < ci) ? to_bf16(w[c * kTaps + tap]) : 0;
        }
        wk[l * kPairs * 64 + lane] = make_uint4(h[0] | (uint32_t)h[1] << 16,
                                                h[2] | (uint32_t)h[3] << 16, 0u, 0u);
    } else if (l > 0 && l < kLayers - 1 && t < kPairs) {
        const int g = lane >> 4, tap = 2 * t + (g >> 1), o = lane & 15;
        uint16_t h[8];
        for (int j = 0; j < 8; ++j) {
            const int c = 8 * (g & 1) + j;
            h[j] = (tap < kTaps && o < co && c < ci) ? to_bf16(w[(o * ci + c) * kTaps + tap]) : 0;
        }
        wk[(l * kPairs + t) * 64 + lane] =
            make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                       h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
    }
}

// Network input from readout planes: channels (L, stale, log(1 + age), 0 ...).
__global__ __launch_bounds__(256) void k_fill_pack_input(const float* __restrict__ L,
                                                         const uint8_t* __restrict__ stale,
                                                         const float* __restrict__ log_age,
                                                         size_t P, uint16_t* __restrict__ x)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint4 lo, hi = make_uint4(0u, 0u, 0u, 0u);
    lo.x = (uint32_t)to_bf16(L[p]) | ((uint32_t)(stale[p] ? to_bf16(1.f) : 0u) << 16);
    lo.y = (uint32_t)to_bf16(log_age[p]);
    lo.z = 0u;
    lo.w = 0u;
    uint4* dst = reinterpret_cast<uint4*>(x + p * kC);
    dst[0] = lo;
    dst[1] = hi;
}

// ---------------------------------------------------------------------------
// One 3x3 layer (or its input gradient).
// out[p][o] = bias[o] + sum_t sum_c in[p + off(t)][c] w_t[c][o], then ReLU if
// `relu`, then zero where gate[p][o] == 0 if `gate` (the ReLU of the layer
// below, for gradients).  Writes BF16 (out16) and/or channel 0 plus skip[p]
// as FP32 (out32: the prediction, L plus the network's correction).
//
// A workgroup takes units of kCvRowsPer rows of one image and a strip of
// kCvStrip columns; the input rows y - 1, y, y + 1 of the strip (plus one
// column each side) sit in LDS pixel-major, a ring of three, the next row's
// loads issued before the products.  Wave w takes the strip's 16-pixel
// segments 2w and 2w + 1: per segment five v_mfma_f32_16x16x32_bf16, the
// weights of a tap pair as A (output channels x 32) and the pixels' shifted
// inputs as B, a lane's eight channels of one pixel being one 16-byte LDS
// read; the result is channels x pixels, lane l holding output channels
// 4 (l / 16) .. + 3 of pixel l % 16 (one 8-byte gate load and store).  A tenth
// tap (zero weights) reads the ninth tap's input.  Outside the image the
// staged input is zero (the layer's zero padding).
// ---------------------------------------------------------------------------
constexpr int kCvStrip = 128;                   // output columns per unit (8 segments)
constexpr int kCvCols = kCvStrip + 2;           // staged columns x0 - 1 .. x0 + kCvStrip
constexpr int kCvRowsPer = 4;                   // output rows per unit
constexpr uint32_t kCvMaxGrid = 65535;

__host__ __device__ inline uint32_t conv_units(uint32_t n, uint32_t H, uint32_t W)
{
    return n * ((H + kCvRowsPer - 1) / kCvRowsPer) * ((W + kCvStrip - 1) / kCvStrip);
}

__global__ __launch_bounds__(256) void k_fill_conv(const uint16_t* __restrict__ in,
                                                   const uint4* __restrict__ w,
                                                   const float* __restrict__ bias, int relu,
                                                   const uint16_t* __restrict__ gate,
                                                   uint16_t* __restrict__ out16,
                                                   float* __restrict__ out32,
                                                   const float* __restrict__ skip, uint32_t n,
                                                   uint32_t H, uint32_t W)
{
    __shared__ __align__(16) uint16_t rowb[3][kCvCols][kC];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t g = lane >> 4, pxl = lane & 15;
    bf16x8 wa[kPairs];
    int dyq[kPairs], colq[kPairs];
#pragma unroll
    for (int q = 0; q < kPairs; ++q) {
        const uint4 v = w[q * 64 + lane];
        wa[q] = *reinterpret_cast<const bf16x8*>(&v);
        const int tap = min(2 * q + (int)(g >> 1), kTaps - 1);
        dyq[q] = tap / 3;                          // ring row: y - 1 + dy
        colq[q] = (int)pxl + tap % 3;              // staged column of segment column 0
    }
    float bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = bias ? bias[4 * g + j] : 0.f;
    const uint32_t ry = (H + kCvRowsPer - 1) / kCvRowsPer, sx = (W + kCvStrip - 1) / kCvStrip;
    const uint32_t units = n * ry * sx;

    // 16-byte chunk k (column k / 2, channel half k % 2) of a staged row
    auto ld = [&](size_t r0, int row, int x0, uint32_t k) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        const int x = x0 - 1 + (int)(k >> 1);
        if (k < 2u * kCvCols && row >= 0 && row < (int)H && x >= 0 && x < (int)W)
            v = *reinterpret_cast<const uint4*>(in + ((r0 + (size_t)row) * W + (size_t)x) * kC +
                                                8 * (k & 1));
        return v;
    };
    auto put = [&](int slot, uint32_t k, uint4 v) {
        if (k < 2u * kCvCols) *reinterpret_cast<uint4*>(&rowb[slot][k >> 1][8 * (k & 1)]) = v;
    };

    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const uint32_t img = u / (ry * sx), rem = u % (ry * sx);
        const int y0 = (int)((rem / sx) * kCvRowsPer);
        const int y1 = min(y0 + kCvRowsPer, (int)H);
        const int x0 = (int)((rem % sx) * kCvStrip);
        const size_t r0 = (size_t)img * H;
        // the ring holds row r at slot (r - y0 + 1) % 3
        put(0, t, ld(r0, y0 - 1, x0, t));
        put(0, t + 256, ld(r0, y0 - 1, x0, t + 256));
        put(1, t, ld(r0, y0, x0, t));
        put(1, t + 256, ld(r0, y0, x0, t + 256));
        uint4 n0 = ld(r0, y0 + 1, x0, t), n1 = ld(r0, y0 + 1, x0, t + 256);
        for (int y = y0; y < y1; ++y) {
            const int sl = (y - y0 + 2) % 3;
            put(sl, t, n0);
            put(sl, t + 256, n1);
            __syncthreads();
            if (y + 1 < y1) {
                n0 = ld(r0, y + 2, x0, t);
                n1 = ld(r0, y + 2, x0, t + 256);
            }
            // the gate and skip values of the row, loaded before the products
            uint2 gg2[2];
            float sk2[2];
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const int px = x0 + 16 * (2 * (int)wv + sg) + (int)pxl;
                const size_t p = (r0 + (size_t)y) * W + (size_t)(px < (int)W ? px : 0);
                gg2[sg] = make_uint2(0xffffffffu, 0xffffffffu);
                if (gate && px < (int)W) gg2[sg] = *reinterpret_cast<const uint2*>(gate + p * kC + 4 * g);
                sk2[sg] = (out32 && g == 0 && px < (int)W) ? skip[p] : 0.f;
            }
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const int seg = 2 * (int)wv + sg;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < kPairs; ++q) {
                    const bf16x8 bq = *reinterpret_cast<const bf16x8*>(
                        &rowb[(y - y0 + dyq[q]) % 3][16 * seg + colq[q]][8 * (g & 1)]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[q], bq, acc, 0, 0, 0);
                }
                const int px = x0 + 16 * seg + (int)pxl;
                if (px >= (int)W) continue;
                const size_t p = (r0 + (size_t)y) * W + (size_t)px;
                const uint2 gg = gg2[sg];
                const uint32_t gh[4] = {gg.x & 0xffffu, gg.x >> 16, gg.y & 0xffffu, gg.y >> 16};
                uint16_t hh[4];
                float v0 = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v = acc[j] + bv[j];
                    if (relu) v = v > 0.f ? v : 0.f;
                    if ((gh[j] & 0x7fffu) == 0) v = 0.f;
                    hh[j] = to_bf16(v);
                    if (j == 0) v0 = v;
                }
                if (out16)
                    *reinterpret_cast<uint2*>(out16 + p * kC + 4 * g) =
                        make_uint2(hh[0] | (uint32_t)hh[1] << 16, hh[2] | (uint32_t)hh[3] << 16);
                if (out32 && g == 0) out32[p] = v0 + sk2[sg];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of one layer: g[t][o][c] = sum_p gz[p][o] in[p + off(t)][c]
// and gb[o] = sum_p gz[p][o], as one partial sum per workgroup.
//
// With q = x + dx the input column, a tap (dy, dx) of output row y is
// sum_q gz[y][q - dx][o] in[y + dy][q][c]: a GEMM over the columns q of the
// row with both operands at q.  A workgroup takes units of kWgRowsPer rows of
// one image and one strip of kWgStrip columns; the three input rows y - 1,
// y, y + 1 (a ring) and the gradient row shifted by dx = -1, 0, +1 sit in LDS
// channel-major, so a lane's eight consecutive columns of one channel are
// one aligned 16-byte read.  Wave w takes columns 32 w .. + 31 of the strip:
// per row and tap one v_mfma_f32_16x16x32_bf16 with A = the shifted gradient
// (16 channels o x 32 columns) and B = the input row (32 columns x 16
// channels c).  The next row's loads are issued before the products.
// Zero padding: columns and rows outside the image are stored as zero.  The
// units a workgroup takes, and every sum's order, are fixed, so the result
// does not depend on timing.  Grid: min(units, kGradBlocks) x 256 threads.
// ---------------------------------------------------------------------------
constexpr int kWgStrip = 128;                   // columns per unit (4 waves x 32)
constexpr int kWgPitch = kWgStrip + 8;          // LDS row pitch, elements (spreads the 16 channels over banks)
constexpr int kWgRowsPer = 8;                   // output rows per unit

__host__ __device__ inline uint32_t wgrad_units(uint32_t n, uint32_t H, uint32_t W)
{
    return n * ((H + kWgRowsPer - 1) / kWgRowsPer) * ((W + kWgStrip - 1) / kWgStrip);
}

__global__ __launch_bounds__(256) void k_fill_wgrad(const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ gz, uint32_t n,
                                                    uint32_t H, uint32_t W,
                                                    float* __restrict__ partial)
{
    __shared__ __align__(16) uint16_t inb[3][kC][kWgPitch];    // input rows, a ring of three
    __shared__ __align__(16) uint16_t gzb[3][kC][kWgPitch];    // gradient row at q - dx, dx = -1, 0, 1
    __shared__ float red[4][kTaps * kC * kC];
    __shared__ float bsh[256][8];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t qq = t >> 1, h = t & 1;           // the column and channel half a thread stages
    const uint32_t ch = lane & 15, g = lane >> 4;
    const uint32_t ry = (H + kWgRowsPer - 1) / kWgRowsPer, sx = (W + kWgStrip - 1) / kWgStrip;
    const uint32_t units = n * ry * sx;
    f32x4 acc[kTaps];
#pragma unroll
    for (int k = 0; k < kTaps; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bs[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bs[j] = 0.f;

    // 16 bytes (8 channels) of pixel (row, x) of an image, zero outside it
    auto ld = [&](const uint16_t* a, size_t img_row0, int row, int x) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (row >= 0 && row < (int)H && x >= 0 && x < (int)W)
            v = *reinterpret_cast<const uint4*>(a + ((img_row0 + (size_t)row) * W + (size_t)x) * kC +
                                                8 * h);
        return v;
    };
    auto put = [&](uint16_t (*buf)[kWgPitch], uint4 v) {
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            buf[8 * h + 2 * j][qq] = (uint16_t)(w4[j] & 0xffffu);
            buf[8 * h + 2 * j + 1][qq] = (uint16_t)(w4[j] >> 16);
        }
    };

    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const uint32_t img = u / (ry * sx), rem = u % (ry * sx);
        const int y0 = (int)((rem / sx) * kWgRowsPer);
        const int y1 = min(y0 + kWgRowsPer, (int)H);
        const int x0 = (int)((rem % sx) * kWgStrip);
        const size_t r0 = (size_t)img * H;
        const int xq = x0 + (int)qq;
        // the ring holds row r at slot (r - y0 + 1) % 3
        put(inb[0], ld(in, r0, y0 - 1, xq));
        put(inb[1], ld(in, r0, y0, xq));
        uint4 vin = ld(in, r0, y0 + 1, xq);
        uint4 vg[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) vg[d] = ld(gz, r0, y0, xq - (d - 1));
        for (int y = y0; y < y1; ++y) {
            put(inb[(y - y0 + 2) % 3], vin);
#pragma unroll
            for (int d = 0; d < 3; ++d) put(gzb[d], vg[d]);
            {   // the bias: the unshifted gradient, each column of the strip once
                const uint32_t w4[4] = {vg[1].x, vg[1].y, vg[1].z, vg[1].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    bs[2 * j] += from_bf16((uint16_t)(w4[j] & 0xffffu));
                    bs[2 * j + 1] += from_bf16((uint16_t)(w4[j] >> 16));
                }
            }
            __syncthreads();
            if (y + 1 < y1) {
                vin = ld(in, r0, y + 2, xq);
#pragma unroll
                for (int d = 0; d < 3; ++d) vg[d] = ld(gz, r0, y + 1, xq - (d - 1));
            }
            const uint32_t q0 = 32 * wv + 8 * g;
            bf16x8 a3[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) a3[d] = *reinterpret_cast<const bf16x8*>(&gzb[d][ch][q0]);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                if (y + dy - 1 < 0 || y + dy - 1 >= (int)H) continue;   // a zero row
                const bf16x8 bv =
                    *reinterpret_cast<const bf16x8*>(&inb[(y - y0 + dy) % 3][ch][q0]);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    acc[dy * 3 + dx] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[dx], bv, acc[dy * 3 + dx], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    // D[m = o][n = c]: lane holds o = 4 (lane / 16) + j, c = lane % 16
#pragma unroll
    for (int k = 0; k < kTaps; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wv][k * kC * kC + (4 * g + j) * kC + ch] = acc[k][j];
#pragma unroll
    for (int j = 0; j < 8; ++j) bsh[t][j] = bs[j];
    __syncthreads();
    float* out = partial + (size_t)blockIdx.x * kWgEntries;
    for (int e = (int)t; e < kTaps * kC * kC; e += 256)
        out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    if (t < kC) {
        // channel t: the threads of its half, in thread order
        float sb = 0.f;
        for (uint32_t i = t >> 3; i < 256; i += 2) sb += bsh[i][t & 7];
        out[kTaps * kC * kC + t] = sb;
    }
}

// Sum the partials of layer l into the canonical gradient: one wave per
// entry, each lane adding every 64th partial in order, then a fixed butterfly
// over the lanes (deterministic).
__global__ __launch_bounds__(512) void k_fill_wgrad_reduce(const float* __restrict__ partial,
                                                           uint32_t blocks, int l,
                                                           float* __restrict__ grad)
{
    // 64 consecutive entries per workgroup (lane = entry), so each partial row
    // is read as 256 contiguous bytes; wave w sums rows w, w + 8, ... in order,
    // then the eight wave sums are added in wave order
    __shared__ float sh[8][64];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + (int)lane;
    const int ec = e < kWgEntries ? e : kWgEntries - 1;
    float s = 0.f;
#pragma unroll 8
    for (uint32_t b = wv; b < blocks; b += 8) s += partial[(size_t)b * kWgEntries + ec];
    sh[wv][lane] = s;
    __syncthreads();
    if (wv != 0 || e >= kWgEntries) return;
    s = sh[0][lane];
#pragma unroll
    for (int w = 1; w < 8; ++w) s += sh[w][lane];
    const int ci = cin_of(l), co = cout_of(l);
    if (e < kTaps * kC * kC) {
        const int t = e / (kC * kC), o = (e / kC) % kC, c = e % kC;
        if (o < co && c < ci) grad[w_off(l) + (o * ci + c) * kTaps + t] = s;
    } else {
        const int o = e - kTaps * kC * kC;
        if (o < co) grad[b_off(l) + o] = s;
    }
}

// ---------------------------------------------------------------------------
// Loss: mean of (pred - target)^2 over stale pixels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 block_sum_f2(float2 v, float2* sh)
{
    for (int m = 32; m > 0; m >>= 1) {
        v.x += __shfl_xor(v.x, m);
        v.y += __shfl_xor(v.y, m);
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float2 r = make_float2(0.f, 0.f);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        r.x += sh[w].x;
        r.y += sh[w].y;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_fill_loss_partial(const float* __restrict__ pred,
                                                           const float* __restrict__ target,
                                                           const uint8_t* __restrict__ stale, size_t P,
                                                           float2* __restrict__ part)
{
    __shared__ float2 sh[4];
    float2 v = make_float2(0.f, 0.f);
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (size_t)gridDim.x * blockDim.x)
        if (stale[p]) {
            const float d = pred[p] - target[p];
            v.x += d * d;
            v.y += 1.f;
        }
    v = block_sum_f2(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// loss2 = (loss, stale pixel count): one wave, lane l sums partials l, l + 64,
// ... in order, then a fixed butterfly (the same order every run).
__global__ __launch_bounds__(64) void k_fill_loss_final(const float2* __restrict__ part,
                                                        uint32_t blocks, float* __restrict__ loss2)
{
    const uint32_t lane = threadIdx.x;
    double s = 0.0, c = 0.0;
    for (uint32_t b = lane; b < blocks; b += 64) {
        s += part[b].x;
        c += part[b].y;
    }
    for (int m = 32; m > 0; m >>= 1) {
        s += __shfl_xor(s, m);
        c += __shfl_xor(c, m);
    }
    if (lane != 0) return;
    loss2[0] = c > 0 ? (float)(s / c) : 0.f;
    loss2[1] = (float)c;
}

// Gradient of the loss in the prediction, as channel 0 of a BF16 activation.
__global__ __launch_bounds__(256) void k_fill_loss_grad(const float* __restrict__ pred,
                                                        const float* __restrict__ target,
                                                        const uint8_t* __restrict__ stale, size_t P,
                                                        const float* __restrict__ loss2,
                                                        uint16_t* __restrict__ g)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float cnt = loss2[1];
    const float v = (stale[p] && cnt > 0.f) ? 2.f * (pred[p] - target[p]) / cnt : 0.f;
    uint4 lo = make_uint4((uint32_t)to_bf16(v), 0u, 0u, 0u), hi = make_uint4(0u, 0u, 0u, 0u);
    uint4* dst = reinterpret_cast<uint4*>(g + p * kC);
    dst[0] = lo;
    dst[1] = hi;
}

// Adam with bias correction; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void k_fill_adam(float* __restrict__ prm, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int n, float lr, float b1, float b2, float eps,
                                                   float bc1, float bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// Fused inference: the four layers of one output tile of kFuseH x kFuseW
// pixels in one workgroup, activations in LDS (two buffers used in turn), so
// a frame costs one read of its inputs and one write of the prediction.
//
// Region coordinates: region row r, column c is image pixel
// (y0 - 4 + r, x0 - 4 + c).  Layer k (1..4) computes rows [k, kFuseH + 8 - k)
// and the 16-pixel segments starting at columns k and k + 16; columns past
// what it needs (k + 32 > kFuseW + 8 - k) only ever feed other surplus
// columns.  Pixels outside the image are stored as zero at every layer (the
// layers' zero padding).  Layer 4 writes L + its channel 0 for the tile's
// pixels inside the image.
// ---------------------------------------------------------------------------
constexpr int kFuseH = 16, kFuseW = 26;
constexpr int kRegH = kFuseH + 8, kRegW = 37;      // widest read: layer 4, columns 3..36
constexpr int kFuseThreads = 512;
constexpr int kFuseWaves = kFuseThreads / 64;


// Raw inputs of the region pixels one thread stages (two at most); they are
// converted only when written to LDS, so their loads stay in flight while
// the previous tile's layers run.
struct RegionIn {
    float l[2], age[2];
    uint32_t st[2];
};

__device__ __forceinline__ void load_region(RegionIn& ri, const float* __restrict__ L,
                                            const uint8_t* __restrict__ stale,
                                            const float* __restrict__ log_age, int y0, int x0,
                                            uint32_t H, uint32_t W)
{
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = (int)threadIdx.x + q * kFuseThreads;
        const int r = k / kRegW, c = k % kRegW;
        const int y = y0 + r, x = x0 + c;
        float l = 0.f, a = 0.f;
        uint32_t st = 0u;
        if (k < kRegH * kRegW && y >= 0 && y < (int)H && x >= 0 && x < (int)W &&
            c < kFuseW + 8) {
            const size_t p = (size_t)y * W + x;
            l = L[p];
            a = log_age[p];
            st = stale[p];
        }
        ri.l[q] = l;
        ri.age[q] = a;
        ri.st[q] = st;
    }
}

// Operand addresses.  A lane's operands of a segment sit at fixed offsets
// from the segment's first pixel, so they are computed once per layer: the
// loop over segments then adds one wave-uniform base per segment instead of
// recomputing, and bounds-checking, every address.  No check is needed: layer
// k reads region rows [k - 1, kRegH - k] and columns [k - 1, k + 32], all
// inside the region.  A tap past the ninth (its weights are zero) reads the
// ninth tap's operand, finite data wherever the real tap's is.
//
// K = 32 operands (16 -> 16 layers): operand q takes tap 2q + (g >> 1) and
// channels 8 (g & 1) .. + 7 of pixel (lane & 15), g = lane / 16; element
// offsets in the 16-channel activation buffer.
__device__ __forceinline__ void tap_offsets(uint32_t lane, int (&off)[kPairs])
{
    const int g = (int)(lane >> 4), px = (int)(lane & 15);
#pragma unroll
    for (int q = 0; q < kPairs; ++q) {
        const int tap = min(2 * q + (g >> 1), kTaps - 1);
        off[q] = ((tap / 3 - 1) * kRegW + tap % 3 - 1 + px) * kC + 8 * (g & 1);
    }
}
// First layer (4 channels, 8 bytes per pixel): operand q takes taps
// 8q + 2g and 8q + 2g + 1 of pixel (lane & 15); offsets in pixels.
__device__ __forceinline__ void tap_offsets_first(uint32_t lane, int (&off)[kPairs0][2])
{
    const int g = (int)(lane >> 4), px = (int)(lane & 15);
#pragma unroll
    for (int q = 0; q < kPairs0; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int tap = min(8 * q + 2 * g + h, kTaps - 1);
            off[q][h] = (tap / 3 - 1) * kRegW + tap % 3 - 1 + px;
        }
}

// The 16x16x32 products of one or two 16-pixel segments (first pixels at
// element indices qa, qb), the two accumulation chains interleaved so that
// they overlap in the matrix pipeline.  The weights are the A operand and the
// activations the B operand, so the result is channels x pixels: lane l holds
// output channels 4 (l / 16) .. + 3 of pixel l % 16 (one 8-byte store of the
// four, instead of four 2-byte stores of one channel).
__device__ __forceinline__ void segment_pair(const uint16_t* __restrict__ in, int qa, int qb,
                                             bool two, const int (&off)[kPairs],
                                             const bf16x8* b, f32x4& acc0, f32x4& acc1)
{
    bf16x8 a0[kPairs], a1[kPairs];
#pragma unroll
    for (int q = 0; q < kPairs; ++q) a0[q] = *reinterpret_cast<const bf16x8*>(&in[qa + off[q]]);
    acc0 = f32x4{0.f, 0.f, 0.f, 0.f};
    acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
    if (two) {
#pragma unroll
        for (int q = 0; q < kPairs; ++q) a1[q] = *reinterpret_cast<const bf16x8*>(&in[qb + off[q]]);
#pragma unroll
        for (int q = 0; q < kPairs; ++q) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a0[q], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a1[q], acc1, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kPairs; ++q)
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a0[q], acc0, 0, 0, 0);
    }
}

// The first layer's two 16x16x32 products per segment: its input has 4
// channels per pixel (L, stale, log(1 + age), 0; 8 bytes), packed 4 per tap,
// so a lane's operand is two taps of one pixel; qa, qb index pixels.
__device__ __forceinline__ void segment_pair_first(const uint2* __restrict__ in4, int qa, int qb,
                                                   bool two, const int (&off)[kPairs0][2],
                                                   const bf16x8* b, f32x4& acc0, f32x4& acc1)
{
    bf16x8 a0[kPairs0], a1[kPairs0];
#pragma unroll
    for (int q = 0; q < kPairs0; ++q) {
        const uint2 u = in4[qa + off[q][0]], v = in4[qa + off[q][1]];
        const uint4 w = make_uint4(u.x, u.y, v.x, v.y);
        a0[q] = *reinterpret_cast<const bf16x8*>(&w);
    }
    acc0 = f32x4{0.f, 0.f, 0.f, 0.f};
    acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
    if (two) {
#pragma unroll
        for (int q = 0; q < kPairs0; ++q) {
            const uint2 u = in4[qb + off[q][0]], v = in4[qb + off[q][1]];
            const uint4 w = make_uint4(u.x, u.y, v.x, v.y);
            a1[q] = *reinterpret_cast<const bf16x8*>(&w);
        }
#pragma unroll
        for (int q = 0; q < kPairs0; ++q) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a0[q], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a1[q], acc1, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kPairs0; ++q)
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a0[q], acc0, 0, 0, 0);
    }
}

// One of the first three layers of a tile: 16-pixel segments of rows
// [k, kRegH - k), k = layer + 1, two per pass (independent product chains),
// bias, ReLU and zero padding, BF16 into the other buffer.  The first layer
// reads the 4-channel input in buf[1] and writes buf[0]; layer l > 0 reads
// buf[(l + 1) % 2] and writes buf[l % 2].  Ends with a barrier.
template <bool kFirst>
__device__ __forceinline__ void fused_layer(int layer, uint16_t (*buf)[kRegH * kRegW * kC],
                                            const uint4* wsh, const float* bsh, int y0, int x0,
                                            uint32_t H, uint32_t W, uint32_t lane, uint32_t wv)
{
    constexpr int nq = kFirst ? kPairs0 : kPairs;
    const int kk = layer + 1;
    const uint16_t* in = buf[(layer + 1) & 1];
    uint16_t* out = buf[layer & 1];
    bf16x8 b[nq];
#pragma unroll
    for (int q = 0; q < nq; ++q)
        b[q] = *reinterpret_cast<const bf16x8*>(&wsh[(layer * kPairs + q) * 64 + lane]);
    const uint32_t o4 = (lane >> 4) * 4;                 // this lane's four output channels
    int off[kPairs], off0[kPairs0][2];
    if (kFirst)
        tap_offsets_first(lane, off0);
    else
        tap_offsets(lane, off);
    const int nseg = (kRegH - 2 * kk) * 2;
    for (int s0 = (int)wv; s0 < nseg; s0 += 2 * kFuseWaves) {
        const int s1 = s0 + kFuseWaves;
        const bool two = s1 < nseg;
        const int ra = kk + s0 / 2, ca = kk + (s0 % 2) * 16;
        const int rb = kk + s1 / 2, cb = kk + (s1 % 2) * 16;
        f32x4 acc0, acc1;
        if (kFirst)
            segment_pair_first(reinterpret_cast<const uint2*>(buf[1]), ra * kRegW + ca,
                               rb * kRegW + cb, two, off0, b, acc0, acc1);
        else
            segment_pair(in, (ra * kRegW + ca) * kC, (rb * kRegW + cb) * kC, two, off, b, acc0,
                         acc1);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            if (half == 1 && !two) break;
            const int r = half ? rb : ra, c = (half ? cb : ca) + (int)(lane & 15);
            const f32x4 acc = half ? acc1 : acc0;
            // the biases are read here, not held (registers are short)
            const float4 bo = *reinterpret_cast<const float4*>(&bsh[layer * kC + o4]);
            const int y = y0 + r, x = x0 + c;
            const bool inside = y >= 0 && y < (int)H && x >= 0 && x < (int)W;
            // bias, ReLU, BF16 (round to nearest even, as to_bf16); pixels
            // outside the image are zero (the layers' zero padding)
            f32x2 v01, v23;
            v01.x = fmaxf(acc[0] + bo.x, 0.f);
            v01.y = fmaxf(acc[1] + bo.y, 0.f);
            v23.x = fmaxf(acc[2] + bo.z, 0.f);
            v23.y = fmaxf(acc[3] + bo.w, 0.f);
            const uint32_t w01 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v01, bf16x2));
            const uint32_t w23 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v23, bf16x2));
            const uint2 w = make_uint2(inside ? w01 : 0u, inside ? w23 : 0u);
            *reinterpret_cast<uint2*>(&out[(r * kRegW + c) * kC + o4]) = w;   // c < kRegW
        }
    }
    __syncthreads();
}

// The last layer (16 -> 1 channel) of a tile: phase A multiplies each input
// segment by all 9 taps at once (one 16x16x16 product, columns = taps):
// D[q][t] = sum_c act[q][c] w[t][c], stored per tap in buf[1] for input rows
// [3, 21) and columns [3, 35); phase B sums out(p) = b + sum_t D[p + off(t)][t]
// in tap order for the tile's pixels and writes L + out.  Ends with a barrier.
constexpr int kLastRows = kFuseH + 2, kLastCols = 32;

__device__ __forceinline__ void fused_last_layer(uint16_t (*buf)[kRegH * kRegW * kC],
                                                 const uint4* wsh, const float* bsh,
                                                 const float* Lsh, int y0, int x0, uint32_t H,
                                                 uint32_t W, uint32_t lane, uint32_t wv,
                                                 float* __restrict__ pred)
{
    const uint16_t* in = buf[0];
    float* D = reinterpret_cast<float*>(buf[1]);         // [tap][row][col]
    const uint4 wb = wsh[(kLayers - 1) * kPairs * 64 + lane];
    const bf16x4 b = __builtin_bit_cast(bf16x4, make_uint2(wb.x, wb.y));
    const uint32_t tap = lane & 15, cq = (lane >> 4) * 4;
    for (int s = (int)wv; s < kLastRows * 2; s += kFuseWaves) {
        const int rr = s / 2, cc0 = (s % 2) * 16;        // region row 3 + rr, column 3 + cc0
        const int q = (3 + rr) * kRegW + 3 + cc0 + (int)(lane & 15);
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(&in[q * kC + cq]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        if (tap < (uint32_t)kTaps)
            *reinterpret_cast<f32x4*>(&D[(tap * kLastRows + rr) * kLastCols + cc0 + cq]) = acc;
    }
    __syncthreads();
    const float bo = bsh[(kLayers - 1) * kC];
    // computed here, not hoisted out of the tile loop (registers are short)
    int t0 = (int)threadIdx.x;
    asm volatile("" : "+v"(t0));
    for (int t = t0; t < kFuseH * kFuseW; t += kFuseThreads) {
        const int r = 4 + t / kFuseW, c = 4 + t % kFuseW;  // region coordinates
        const int y = y0 + r, x = x0 + c;
        if (y >= (int)H || x >= (int)W) continue;
        float v = bo;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) {
            const int rr = r + k / 3 - 1 - 3, cc = c + k % 3 - 1 - 3;
            v += D[(k * kLastRows + rr) * kLastCols + cc];
        }
        pred[(size_t)y * W + x] = v + Lsh[r * kRegW + c];
    }
    __syncthreads();
}

// Persistent: workgroup w takes tiles w, w + grid, ...; the next tile's inputs
// are loaded into registers while the current tile's layers run.  The input
// region (4 channels per pixel) sits in buf[1], which the first layer does not
// write; the layers then go buf[0] -> buf[1] -> buf[0] -> prediction.
// Two workgroups per CU (LDS allows two): at most 128 registers per lane.
__global__ __launch_bounds__(kFuseThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_fill_fused(const float* __restrict__ L,
                                                             const uint8_t* __restrict__ stale,
                                                             const float* __restrict__ log_age,
                                                             const uint4* __restrict__ wk,
                                                             const float* __restrict__ bias,
                                                             uint32_t H, uint32_t W,
                                                             float* __restrict__ pred)
{
    __shared__ __align__(16) uint16_t buf[2][kRegH * kRegW * kC];
    __shared__ __align__(16) uint4 wsh[kLayers * kPairs * 64];
    __shared__ __align__(16) float bsh[kLayers * kC];
    __shared__ float Lsh[kRegH * kRegW];
    const uint32_t tiles_x = (W + kFuseW - 1) / kFuseW;
    const uint32_t tiles = tiles_x * ((H + kFuseH - 1) / kFuseH);
    // the wave index is uniform: in a scalar register, the segment loops'
    // index arithmetic runs on the scalar unit
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    for (int k = threadIdx.x; k < kLayers * kPairs * 64; k += kFuseThreads) wsh[k] = wk[k];
    if (threadIdx.x < kLayers * kC) bsh[threadIdx.x] = bias[threadIdx.x];
    uint32_t tile = blockIdx.x;
    RegionIn ri;
    if (tile < tiles)
        load_region(ri, L, stale, log_age, (int)(tile / tiles_x) * kFuseH - 4,
                    (int)(tile % tiles_x) * kFuseW - 4, H, W);
    for (; tile < tiles; tile += gridDim.x) {
        const int y0 = (int)(tile / tiles_x) * kFuseH - 4;
        const int x0 = (int)(tile % tiles_x) * kFuseW - 4;
        // input region: (L, stale, log(1 + age), 0), zero outside the image
        uint2* in4 = reinterpret_cast<uint2*>(buf[1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int k = (int)threadIdx.x + q * kFuseThreads;
            if (k >= kRegH * kRegW) continue;
            in4[k] = make_uint2((uint32_t)to_bf16(ri.l[q]) |
                                    ((uint32_t)(ri.st[q] ? to_bf16(1.f) : 0u) << 16),
                                (uint32_t)to_bf16(ri.age[q]));
            Lsh[k] = ri.l[q];
        }
        __syncthreads();
        const uint32_t next = tile + gridDim.x;
        if (next < tiles)
            load_region(ri, L, stale, log_age, (int)(next / tiles_x) * kFuseH - 4,
                        (int)(next % tiles_x) * kFuseW - 4, H, W);

        fused_layer<true>(0, buf, wsh, bsh, y0, x0, H, W, lane, wv);
        for (int layer = 1; layer < kLayers - 1; ++layer)
            fused_layer<false>(layer, buf, wsh, bsh, y0, x0, H, W, lane, wv);
        fused_last_layer(buf, wsh, bsh, Lsh, y0, x0, H, W, lane, wv, pred);
    }
}

// Filled image with the per-tile fallback; one workgroup per tile.  A tile
// takes the network's predictions at its stale pixels when more than a
// fraction theta of its pixels (inside the image) are stale and every one of
// those predictions is finite; otherwise it keeps L, the reconstruction's own
// blurred value.  `fallbacks` counts the tiles with stale pixels that keep L.
__global__ __launch_bounds__(256) void k_fill_apply(const float* __restrict__ L,
                                                    const uint8_t* __restrict__ stale,
                                                    const float* __restrict__ pred, uint32_t H,
                                                    uint32_t W, uint32_t tile, float theta,
                                                    float* __restrict__ out,
                                                    uint32_t* __restrict__ fallbacks)
{
    __shared__ uint32_t sh[2][4];
    const uint32_t tw = (W + tile - 1) / tile;
    const uint32_t ty0 = (blockIdx.x / tw) * tile, tx0 = (blockIdx.x % tw) * tile;
    const uint32_t th = min(tile, H - ty0), twd = min(tile, W - tx0);
    uint32_t nst = 0u, bad = 0u;
    for (uint32_t k = threadIdx.x; k < th * twd; k += blockDim.x) {
        const size_t p = (size_t)(ty0 + k / twd) * W + tx0 + k % twd;
        if (stale[p]) {
            ++nst;
            bad += isfinite(pred[p]) ? 0u : 1u;
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        nst += __shfl_xor(nst, m);
        bad += __shfl_xor(bad, m);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = nst;
        sh[1][threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    nst = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    bad = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    // stale fraction > theta, compared exactly: nst > theta * pixels
    const bool use = nst > 0u && bad == 0u && (double)nst > (double)theta * (double)(th * twd);
    if (nst > 0u && !use && threadIdx.x == 0) atomicAdd(fallbacks, 1u);
    for (uint32_t k = threadIdx.x; k < th * twd; k += blockDim.x) {
        const size_t p = (size_t)(ty0 + k / twd) * W + tx0 + k % twd;
        out[p] = (stale[p] && use) ? pred[p] : L[p];
    }
}

__global__ void k_fill_clear(uint32_t* __restrict__ c) { *c = 0u; }

// Scratch of fibar_fill_apply_noalloc: the prediction of one frame of up to
// kNoAllocPixels pixels, then the fallback counter.  One copy per device,
// held until the process ends; host code reaches it only through the address
// hipGetSymbolAddress gives on that device (noalloc_scratch below).
constexpr size_t kNoAllocPixels = 1u << 20;
constexpr size_t kNoAllocBytes = kNoAllocPixels * sizeof(float) + 256;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

}  // namespace

struct fibar_fill {
    hipStream_t st = nullptr;
    float* prm = nullptr;        // FP32 master parameters
    float* m = nullptr;          // Adam moments
    float* v = nullptr;
    float* grad = nullptr;       // canonical gradient
    bf16x4* wf = nullptr;        // [4][9][64]
    bf16x4* wb = nullptr;
    uint4* wk = nullptr;         // [4][5][64] K = 32 operands (8 BF16 each)
    uint4* wpf = nullptr;        // [4][5][64] tap-pair operands, forward
    uint4* wpb = nullptr;        // [4][5][64] tap-pair operands, input gradient
    float* bias = nullptr;       // [4][16]
    float* partial = nullptr;    // [kGradBlocks][kWgEntries]
    float2* lpart = nullptr;     // [kLossBlocks]
    float* loss2 = nullptr;      // loss, stale count
    uint32_t* fallbacks = nullptr;
    int step = 0;                // Adam steps since the parameters were set
    uint32_t cus = 256;          // compute units of the device
    uint8_t* noalloc = nullptr;  // this device's copy of `scratch`
    float* apply_pred = nullptr; // prediction buffer of fibar_fill_apply
    size_t apply_cap = 0;
    // workspace for up to cap pixels
    size_t cap = 0;
    uint16_t* act[4] = {};       // x0, a1, a2, a3 (BF16 x 16 channels)
    uint16_t* g[3] = {};         // gradient of the prediction, two ping-pong buffers
    float* pred = nullptr;
};

namespace {

int map_hip(hipError_t e)
{
    if (e == hipSuccess) return FIBAR_OK;
    if (e == hipErrorOutOfMemory) return FIBAR_E_NOMEM;
    return FIBAR_E_DEVICE;
}

#define FILL_TRY(x)                                  \
    do {                                             \
        const hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return map_hip(e_);    \
    } while (0)

void free_ws(fibar_fill* f)
{
    for (auto& a : f->act) (void)hipFree(a), a = nullptr;
    for (auto& a : f->g) (void)hipFree(a), a = nullptr;
    (void)hipFree(f->pred);
    f->pred = nullptr;
    f->cap = 0;
}

int ensure_apply_pred(fibar_fill* f, size_t P)
{
    if (P <= f->apply_cap) return FIBAR_OK;
    FILL_TRY(hipStreamSynchronize(f->st));
    (void)hipFree(f->apply_pred);
    f->apply_pred = nullptr;
    f->apply_cap = 0;
    FILL_TRY(hipMalloc((void**)&f->apply_pred, P * sizeof(float)));
    f->apply_cap = P;
    return FIBAR_OK;
}


int ensure_ws(fibar_fill* f, size_t P)
{
    if (P <= f->cap) return FIBAR_OK;
    FILL_TRY(hipStreamSynchronize(f->st));
    free_ws(f);
    hipError_t e = hipSuccess;
    for (auto& a : f->act)
        if (e == hipSuccess) e = hipMalloc((void**)&a, P * kC * sizeof(uint16_t));
    for (auto& a : f->g)
        if (e == hipSuccess) e = hipMalloc((void**)&a, P * kC * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc((void**)&f->pred, P * sizeof(float));
    if (e != hipSuccess) {
        free_ws(f);
        return map_hip(e);
    }
    f->cap = P;
    return FIBAR_OK;
}

// Device address of this device's `scratch` array, looked up once per
// device with that device current.
constexpr int kMaxDevices = 64;
uint8_t* g_noalloc[kMaxDevices] = {};
std::mutex g_noalloc_mu;

int noalloc_scratch(int dev, uint8_t** out)
{
    if (dev < 0 || dev >= kMaxDevices) return FIBAR_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return map_hip(e == hipSuccess ? hipErrorInvalidSymbol : e);
        g_noalloc[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_noalloc[dev];
    return FIBAR_OK;
}

int check_images(const fibar_fill* f, const void* L, const void* stale, const void* age,
                 uint32_t n, uint32_t H, uint32_t W)
{
    if (!f || !L || !stale || !age || n == 0 || H == 0 || W == 0) return FIBAR_E_INVALID_ARG;
    return FIBAR_OK;
}

hipError_t launch_conv(fibar_fill* f, const uint16_t* in, const uint4* w, const float* bias,
                       int relu, const uint16_t* gate, uint16_t* out16, float* out32,
                       const float* skip, uint32_t n, uint32_t H, uint32_t W)
{
    const uint32_t grid = std::min<uint32_t>(conv_units(n, H, W), kCvMaxGrid);
    hipLaunchKernelGGL(k_fill_conv, dim3(grid), dim3(256), 0, f->st, in, w, bias, relu, gate,
                       out16, out32, skip, n, H, W);
    return hipGetLastError();
}

// Fused inference of n images; the prediction lands in `pred`.
hipError_t forward_fused(fibar_fill* f, const float* L, const uint8_t* stale, const float* age,
                         uint32_t n, uint32_t H, uint32_t W, float* pred)
{
    const uint32_t tiles = ((H + kFuseH - 1) / kFuseH) * ((W + kFuseW - 1) / kFuseW);
    // two resident workgroups per CU (LDS), each looping over tiles
    const uint32_t grid = tiles < 2 * f->cus ? tiles : 2 * f->cus;
    const size_t P = (size_t)H * W;
    for (uint32_t i = 0; i < n; ++i)
        hipLaunchKernelGGL(k_fill_fused, dim3(grid), dim3(kFuseThreads), 0, f->st, L + i * P,
                           stale + i * P, age + i * P, f->wk, f->bias, H, W, pred + i * P);
    return hipGetLastError();
}

// The filled image of one frame (prediction into `pred`, fallback counter at
// `counter`); allocates nothing.
int apply_with(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
               uint32_t H, uint32_t W, uint32_t tile, float theta, float* out, float* pred,
               uint32_t* counter, uint32_t* fallback_tiles)
{
    FILL_TRY(forward_fused(f, L, stale, log_age, 1, H, W, pred));
    const uint32_t tiles = ((H + tile - 1) / tile) * ((W + tile - 1) / tile);
    // a kernel, not a memset: callers may capture this into a graph
    hipLaunchKernelGGL(k_fill_clear, dim3(1), dim3(1), 0, f->st, counter);
    hipLaunchKernelGGL(k_fill_apply, dim3(tiles), dim3(256), 0, f->st, L, stale, pred, H, W,
                       tile, theta, out, counter);
    FILL_TRY(hipGetLastError());
    if (fallback_tiles) {
        FILL_TRY(hipMemcpyAsync(fallback_tiles, counter, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, f->st));
        FILL_TRY(hipStreamSynchronize(f->st));
    }
    return FIBAR_OK;
}

// Pack the input and run the four layers one by one, keeping every layer's
// activations for the backward pass; the prediction lands in f->pred.
int forward(fibar_fill* f, const float* L, const uint8_t* stale, const float* age, uint32_t n,
            uint32_t H, uint32_t W)
{
    const size_t P = (size_t)n * H * W;
    int rc = ensure_ws(f, P);
    if (rc) return rc;
    hipLaunchKernelGGL(k_fill_pack_input, dim3((uint32_t)((P + 255) / 256)), dim3(256), 0, f->st, L,
                       stale, age, P, f->act[0]);
    FILL_TRY(hipGetLastError());
    for (int l = 0; l < kLayers; ++l) {
        const bool last = l == kLayers - 1;
        FILL_TRY(launch_conv(f, f->act[l], f->wpf + l * kPairs * 64, f->bias + l * kC, last ? 0 : 1,
                             nullptr, last ? nullptr : f->act[l + 1], last ? f->pred : nullptr,
                             last ? L : nullptr, n, H, W));
    }
    return FIBAR_OK;
}

// Loss and full gradient of a batch into f->loss2 and f->grad (device).
int loss_grad(fibar_fill* f, const float* L, const uint8_t* stale, const float* age,
              const float* target, uint32_t n, uint32_t H, uint32_t W)
{
    int rc = forward(f, L, stale, age, n, H, W);
    if (rc) return rc;
    const size_t P = (size_t)n * H * W;
    hipLaunchKernelGGL(k_fill_loss_partial, dim3(kLossBlocks), dim3(256), 0, f->st, f->pred, target,
                       stale, P, f->lpart);
    hipLaunchKernelGGL(k_fill_loss_final, dim3(1), dim3(64), 0, f->st, f->lpart, (uint32_t)kLossBlocks,
                       f->loss2);
    hipLaunchKernelGGL(k_fill_loss_grad, dim3((uint32_t)((P + 255) / 256)), dim3(256), 0, f->st,
                       f->pred, target, stale, P, f->loss2, f->g[0]);
    FILL_TRY(hipGetLastError());
    // layer by layer from the top: weight gradient, then the input gradient
    // gated by the ReLU of the layer below
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const uint32_t gblocks = std::min<uint32_t>(wgrad_units(n, H, W), kGradBlocks);
        hipLaunchKernelGGL(k_fill_wgrad, dim3(gblocks), dim3(256), 0, f->st, f->act[l], f->g[cur],
                           n, H, W, f->partial);
        hipLaunchKernelGGL(k_fill_wgrad_reduce, dim3((kWgEntries + 63) / 64), dim3(512), 0, f->st,
                           f->partial, gblocks, l, f->grad);
        FILL_TRY(hipGetLastError());
        if (l > 0) {
            const int nxt = cur == 1 ? 2 : 1;
            FILL_TRY(launch_conv(f, f->g[cur], f->wpb + l * kPairs * 64, nullptr, 0, f->act[l],
                                 f->g[nxt], nullptr, nullptr, n, H, W));
            cur = nxt;
        }
    }
    return FIBAR_OK;
}

hipError_t pack_weights(fibar_fill* f)
{
    hipLaunchKernelGGL(k_fill_pack_weights, dim3(kLayers * kTaps), dim3(64), 0, f->st, f->prm,
                       f->wf, f->wb, f->bias, f->wk, f->wpf, f->wpb);
    return hipGetLastError();
}

void free_fill(fibar_fill* f)
{
    if (!f) return;
    if (f->st) (void)hipStreamSynchronize(f->st);
    free_ws(f);
    (void)hipFree(f->apply_pred);
    void* p[] = {f->prm, f->m, f->v, f->grad, f->wf, f->wb, f->wk, f->wpf, f->wpb, f->bias,
                 f->partial, f->lpart, f->loss2, f->fallbacks};
    for (void* q : p) (void)hipFree(q);
    delete f;
}

}  // namespace

extern "C" {

int fibar_fill_create(void* stream, fibar_fill** out)
{
    if (!out) return FIBAR_E_INVALID_ARG;
    *out = nullptr;
    fibar_fill* f = new (std::nothrow) fibar_fill();
    if (!f) return FIBAR_E_NOMEM;
    f->st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t b) {
        if (e == hipSuccess) e = hipMalloc(p, b);
        if (e == hipSuccess) e = hipMemsetAsync(*p, 0, b, f->st);
    };
    alloc((void**)&f->prm, FIBAR_FILL_PARAMS * sizeof(float));
    alloc((void**)&f->m, FIBAR_FILL_PARAMS * sizeof(float));
    alloc((void**)&f->v, FIBAR_FILL_PARAMS * sizeof(float));
    alloc((void**)&f->grad, FIBAR_FILL_PARAMS * sizeof(float));
    alloc((void**)&f->wf, kLayers * kTaps * 64 * sizeof(bf16x4));
    alloc((void**)&f->wb, kLayers * kTaps * 64 * sizeof(bf16x4));
    alloc((void**)&f->wk, kLayers * kPairs * 64 * sizeof(uint4));
    alloc((void**)&f->wpf, kLayers * kPairs * 64 * sizeof(uint4));
    alloc((void**)&f->wpb, kLayers * kPairs * 64 * sizeof(uint4));
    alloc((void**)&f->bias, kLayers * kC * sizeof(float));
    alloc((void**)&f->partial, (size_t)kGradBlocks * kWgEntries * sizeof(float));
    alloc((void**)&f->lpart, kLossBlocks * sizeof(float2));
    alloc((void**)&f->loss2, 2 * sizeof(float));
    alloc((void**)&f->fallbacks, sizeof(uint32_t));
    int dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && cus > 0) f->cus = (uint32_t)cus;
    if (e == hipSuccess) {
        const int rc = noalloc_scratch(dev, &f->noalloc);
        if (rc) {
            free_fill(f);
            return rc;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(f->st);
    if (e != hipSuccess) {
        free_fill(f);
        return map_hip(e);
    }
    *out = f;
    return FIBAR_OK;
}

int fibar_fill_set_params(fibar_fill* f, const float* params)
{
    if (!f || !params) return FIBAR_E_INVALID_ARG;
    FILL_TRY(hipMemcpyAsync(f->prm, params, FIBAR_FILL_PARAMS * sizeof(float),
                            hipMemcpyHostToDevice, f->st));
    FILL_TRY(hipMemsetAsync(f->m, 0, FIBAR_FILL_PARAMS * sizeof(float), f->st));
    FILL_TRY(hipMemsetAsync(f->v, 0, FIBAR_FILL_PARAMS * sizeof(float), f->st));
    FILL_TRY(pack_weights(f));
    FILL_TRY(hipStreamSynchronize(f->st));
    f->step = 0;
    return FIBAR_OK;
}

int fibar_fill_get_params(fibar_fill* f, float* params)
{
    if (!f || !params) return FIBAR_E_INVALID_ARG;
    FILL_TRY(hipMemcpyAsync(params, f->prm, FIBAR_FILL_PARAMS * sizeof(float),
                            hipMemcpyDeviceToHost, f->st));
    FILL_TRY(hipStreamSynchronize(f->st));
    return FIBAR_OK;
}

int fibar_fill_predict(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                       uint32_t n, uint32_t H, uint32_t W, float* pred)
{
    int rc = check_images(f, L, stale, log_age, n, H, W);
    if (rc) return rc;
    if (!pred) return FIBAR_E_INVALID_ARG;
    FILL_TRY(forward_fused(f, L, stale, log_age, n, H, W, pred));
    return FIBAR_OK;
}

int fibar_fill_loss_grad(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                         const float* target, uint32_t n, uint32_t H, uint32_t W, float* loss,
                         float* grad)
{
    int rc = check_images(f, L, stale, log_age, n, H, W);
    if (rc) return rc;
    if (!target || !loss) return FIBAR_E_INVALID_ARG;
    rc = loss_grad(f, L, stale, log_age, target, n, H, W);
    if (rc) return rc;
    float l2[2];
    FILL_TRY(hipMemcpyAsync(l2, f->loss2, sizeof(l2), hipMemcpyDeviceToHost, f->st));
    if (grad)
        FILL_TRY(hipMemcpyAsync(grad, f->grad, FIBAR_FILL_PARAMS * sizeof(float),
                                hipMemcpyDeviceToHost, f->st));
    FILL_TRY(hipStreamSynchronize(f->st));
    *loss = l2[0];
    return FIBAR_OK;
}

int fibar_fill_train_step(fibar_fill* f, const float* L, const uint8_t* stale,
                          const float* log_age, const float* target, uint32_t n, uint32_t H,
                          uint32_t W, float lr, float* loss)
{
    int rc = check_images(f, L, stale, log_age, n, H, W);
    if (rc) return rc;
    if (!target || !(lr >= 0.f)) return FIBAR_E_INVALID_ARG;
    rc = loss_grad(f, L, stale, log_age, target, n, H, W);
    if (rc) return rc;
    const int t = ++f->step;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - pow(b1, t)), bc2 = (float)(1.0 - pow(b2, t));
    hipLaunchKernelGGL(k_fill_adam, dim3((FIBAR_FILL_PARAMS + 255) / 256), dim3(256), 0, f->st, f->prm,
                       f->grad, f->m, f->v, (int)FIBAR_FILL_PARAMS, lr, (float)b1, (float)b2,
                       1e-8f, bc1, bc2);
    FILL_TRY(hipGetLastError());
    FILL_TRY(pack_weights(f));
    if (loss) {
        float l2[2];
        FILL_TRY(hipMemcpyAsync(l2, f->loss2, sizeof(l2), hipMemcpyDeviceToHost, f->st));
        FILL_TRY(hipStreamSynchronize(f->st));
        *loss = l2[0];
    }
    return FIBAR_OK;
}

int fibar_fill_apply(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                     uint32_t H, uint32_t W, uint32_t tile, float theta, float* out,
                     uint32_t* fallback_tiles)
{
    int rc = check_images(f, L, stale, log_age, 1, H, W);
    if (rc) return rc;
    if (!out || tile < 4 || tile > 64 || !(theta >= 0.f)) return FIBAR_E_INVALID_ARG;
    rc = ensure_apply_pred(f, (size_t)H * W);
    if (rc) return rc;
    return apply_with(f, L, stale, log_age, H, W, tile, theta, out, f->apply_pred, f->fallbacks,
                      fallback_tiles);
}

int fibar_fill_apply_noalloc(fibar_fill* f, const float* L, const uint8_t* stale,
                             const float* log_age, uint32_t H, uint32_t W, uint32_t tile,
                             float theta, float* out, uint32_t* fallback_tiles)
{
    int rc = check_images(f, L, stale, log_age, 1, H, W);
    if (rc) return rc;
    if (!out || tile < 4 || tile > 64 || !(theta >= 0.f)) return FIBAR_E_INVALID_ARG;
    if ((size_t)H * W > kNoAllocPixels) return FIBAR_E_INVALID_ARG;
    if (!f->noalloc) return FIBAR_E_DEVICE;
    float* pred = reinterpret_cast<float*>(f->noalloc);
    uint32_t* counter = reinterpret_cast<uint32_t*>(f->noalloc + kNoAllocPixels * sizeof(float));
    return apply_with(f, L, stale, log_age, H, W, tile, theta, out, pred, counter,
                      fallback_tiles);
}

void fibar_fill_destroy(fibar_fill* f) { free_fill(f); }

}  // extern "C"
