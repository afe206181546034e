// Relative contrast thresholds (Experiments, "Inter-pixel threshold
// variation"; the threshold appendix, Eq. (21)-(30)): per-pixel ON/OFF event
// counts of a calibration recording, the relative thresholds formed from
// them, and the per-pixel multiplier of Eq. (6) that a context applies.
#include <new>

#include "fibar_ctx.h"
#include "fibar_internal.h"

namespace fibar {
namespace {

constexpr int kThrBlock = 256;

// bit 0: a coordinate out of range, bit 1: a polarity byte above 1
__global__ __launch_bounds__(kThrBlock) void k_check_events(const uint16_t* __restrict__ x,
                                                            const uint16_t* __restrict__ y,
                                                            const uint8_t* __restrict__ p,
                                                            uint64_t n, uint32_t W, uint32_t H,
                                                            uint32_t* bad)
{
    uint32_t b = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * kThrBlock + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * kThrBlock) {
        if (x[e] >= W || y[e] >= H) b |= 1u;
        if (p[e] > 1) b |= 2u;
    }
    if (b) atomicOr(bad, b);
}

__global__ __launch_bounds__(kThrBlock) void k_count_polarities(const uint16_t* __restrict__ x,
                                                                const uint16_t* __restrict__ y,
                                                                const uint8_t* __restrict__ p,
                                                                uint64_t n, uint32_t W,
                                                                uint32_t* n_on, uint32_t* n_off)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kThrBlock + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * kThrBlock) {
        const uint32_t i = (uint32_t)y[e] * W + x[e];
        atomicAdd(p[e] ? &n_on[i] : &n_off[i], 1u);
    }
}

// Sum of n_on + n_off over all pixels, one 64-bit atomic per workgroup.
__global__ __launch_bounds__(kThrBlock) void k_sum_counts(const uint32_t* __restrict__ n_on,
                                                          const uint32_t* __restrict__ n_off,
                                                          uint64_t npx, unsigned long long* sum)
{
    __shared__ unsigned long long part[kThrBlock / 64];
    unsigned long long v = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThrBlock + threadIdx.x; i < npx;
         i += (uint64_t)gridDim.x * kThrBlock)
        v += (unsigned long long)n_on[i] + n_off[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThrBlock / 64; ++w) t += part[w];
        atomicAdd(sum, t);
    }
}

// C'_i = N / (N_on_i + N_off_i), C'_on_i = N / (2 N_on_i), C'_off_i = N /
// (2 N_off_i) with N the mean count per pixel; 1 where a count is zero.  In
// double precision, rounded once.
__global__ __launch_bounds__(kThrBlock) void k_relative_thresholds(
    const uint32_t* __restrict__ n_on, const uint32_t* __restrict__ n_off, uint64_t npx,
    const unsigned long long* __restrict__ sum, float* c_rel, float* c_on, float* c_off)
{
    const double mean = (double)*sum / (double)npx;
    for (uint64_t i = (uint64_t)blockIdx.x * kThrBlock + threadIdx.x; i < npx;
         i += (uint64_t)gridDim.x * kThrBlock) {
        const uint32_t a = n_on[i], b = n_off[i];
        const uint64_t t = (uint64_t)a + b;
        c_rel[i] = t ? (float)(mean / (double)t) : 1.0f;
        if (c_on) c_on[i] = a ? (float)(0.5 * mean / (double)a) : 1.0f;
        if (c_off) c_off[i] = b ? (float)(0.5 * mean / (double)b) : 1.0f;
    }
}

inline uint32_t grid_for(uint64_t n)
{
    const uint64_t b = (n + kThrBlock - 1) / kThrBlock;
    return (uint32_t)(b < 2048 ? (b ? b : 1) : 2048);
}

}  // namespace
}  // namespace fibar

using namespace fibar;

extern "C" {

int fibar_count_polarities(const uint16_t* x, const uint16_t* y, const uint8_t* p, size_t n,
                           uint32_t width, uint32_t height, uint32_t* n_on, uint32_t* n_off,
                           void* stream)
{
    if (width == 0 || height == 0 || !n_on || !n_off) return FIBAR_E_INVALID_ARG;
    if (n == 0) return FIBAR_OK;
    if (!x || !y || !p) return FIBAR_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    uint32_t* bad = nullptr;
    uint32_t h_bad = 0;
    HIP_TRY(hipMallocAsync((void**)&bad, sizeof(uint32_t), st));
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(uint32_t), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_check_events, dim3(grid_for(n)), dim3(kThrBlock), 0, st, x, y, p,
                           (uint64_t)n, width, height, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    const hipError_t e2 = hipFreeAsync(bad, st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return map_err(e);
    if (h_bad & 1u) return FIBAR_E_RANGE;
    if (h_bad & 2u) return FIBAR_E_POLARITY;
    hipLaunchKernelGGL(k_count_polarities, dim3(grid_for(n)), dim3(kThrBlock), 0, st, x, y, p,
                       (uint64_t)n, width, n_on, n_off);
    return map_err(hipGetLastError());
}

int fibar_relative_thresholds(const uint32_t* n_on, const uint32_t* n_off, uint32_t width,
                              uint32_t height, float* c_rel, float* c_on_rel, float* c_off_rel,
                              void* stream)
{
    if (width == 0 || height == 0 || !n_on || !n_off || !c_rel) return FIBAR_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t npx = (uint64_t)width * height;
    unsigned long long* sum = nullptr;
    HIP_TRY(hipMallocAsync((void**)&sum, sizeof(*sum), st));
    hipError_t e = hipMemsetAsync(sum, 0, sizeof(*sum), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sum_counts, dim3(grid_for(npx)), dim3(kThrBlock), 0, st, n_on, n_off,
                           npx, sum);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_relative_thresholds, dim3(grid_for(npx)), dim3(kThrBlock), 0, st,
                           n_on, n_off, npx, (const unsigned long long*)sum, c_rel, c_on_rel,
                           c_off_rel);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipFreeAsync(sum, st);
    if (e == hipSuccess) e = e2;
    return map_err(e);
}

int fibar_set_pixel_gain(fibar_ctx* c, const float* gain)
{
    if (!c) return FIBAR_E_INVALID_ARG;
    if (!gain) {
        // launches already queued keep the multipliers they were given
        c->s.gain = nullptr;
        return FIBAR_OK;
    }
    if (!c->gain) HIP_TRY(hipMalloc((void**)&c->gain, c->npx * sizeof(float)));
    HIP_TRY(hipMemcpyAsync(c->gain, gain, c->npx * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    c->s.gain = c->gain;
    return FIBAR_OK;
}

}  // extern "C"
