// HIP kernels of libfibar for gfx950 (MI355X).
//
// Per pushed packet the work splits into a part that does not depend on the
// reconstruction state (grouping the packet's events by pixel and composing
// each pixel's temporal-filter updates) and an in-order part (applying the
// compositions to the state, moving the active-event window, detecting and
// blurring stale pixels).  The first part runs for many packets in one bulk
// launch (k_sort_compose, one 1024-thread workgroup per <=16384-event chunk);
// the second runs packet by packet (k_apply, then k_pop_blur).
//
// Blurred values of stale pixels live in a second image Lb (stored next to
// L, as Lp[i] = (L, Lb)): a pixel's current brightness is Lb[i] when it is
// stale (its newest event has left the window, last[i] < h) and L[i]
// otherwise.  The pop kernel of a step
// writes only Lb of the pixels that go stale in that step and reads
// neighbours with the window head h of the previous step, so every blur of
// the step sees the pre-blur image (the blurs of one step are simultaneous)
// without a separate write pass.
//
// Paper references: temporal filter Eq. (6), (7), (10); active event queue
// and its regulation Eq. (19), (20) (Method, "Spatial filtering"); one-time
// 3x3 Gaussian blur of stale pixels (same section).
#include "fibar_tile.h"

namespace fibar {
namespace {

using namespace tile;

// ---------------------------------------------------------------------------
// Bulk kernel: validate, stable LDS radix sort by pixel, segmented scan of
// the per-event affine maps.  One workgroup per chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_sort_compose(
    const ChunkDesc* __restrict__ chunks, SegRec* __restrict__ seg, uint32_t* __restrict__ seg_count,
    StepScratch* __restrict__ scratch, uint32_t W, uint32_t H, int key_bits, Coef coef)
{
    __shared__ uint32_t keypol[kChunk];                 // (pixel << 1) | polarity, arrival order
    __shared__ __align__(16) uint16_t idxA[kChunk];     // permutation ping
    __shared__ __align__(16) uint16_t idxB[kChunk];     // permutation pong
    __shared__ uint64_t scan4[kWaves + 1][4];
    __shared__ SegPair scanp[kWaves];
    __shared__ uint32_t scan1[kWaves + 1];
    __shared__ uint32_t bad_sh;

    const ChunkDesc cd = chunks[blockIdx.x];
    const uint32_t cn = cd.n;
    const int tid = threadIdx.x;
    if (tid == 0) bad_sh = 0u;
    __syncthreads();

    uint32_t bad = 0u;
    for (uint32_t e = tid; e < cn; e += kSortThreads) {
        const uint32_t x = cd.x[e], y = cd.y[e], p = cd.p[e];
        const bool inr = x < W && y < H;
        bad |= inr ? 0u : 1u;
        bad |= p > 1u ? 2u : 0u;
        keypol[e] = ((inr ? y * W + x : 0u) << 1) | (p & 1u);
        idxA[e] = (uint16_t)e;
    }
    if (bad) atomicOr(&bad_sh, bad);
    __syncthreads();
    if (tid == 0 && bad_sh) atomicOr(&scratch[cd.pkt].status, bad_sh);

    const uint16_t* sorted = tile_sort(keypol, idxA, idxB, cn, key_bits, scan4);
    SegRec* out = seg + (size_t)blockIdx.x * kChunk;
    const uint32_t total = tile_compose(keypol, sorted, cn, coef, scanp, scan1,
        [&](uint32_t key, const Aff& acc, uint32_t oid, uint32_t rank) {
            SegRec r;
            r.pix = key;
            r.n_last = (acc.n << 16) | oid;
            r.a = acc.a;
            r.g = acc.g;
            r.b = acc.b;
            r.u1 = acc.u1;
            r.u2 = acc.u2;
            r.pad = 0u;
            out[rank] = r;
        });
    if (tid == 0) seg_count[blockIdx.x] = total;
}

__device__ __forceinline__ uint32_t tile_of(const State& s, uint32_t pix)
{
    const uint32_t y = pix / s.W, x = pix - y * s.W;
    return (y >> 1) * s.TW + (x >> 1);
}

// ---------------------------------------------------------------------------
// Window scalars without completion tickets.
//
// Kernels of step b add their activation / deactivation counts to the step's
// scratch (one atomic per workgroup, spread over kSpread addresses).  Nobody
// waits for the last workgroup: the *next* kernel that needs the scalars
// after step b derives them from the last committed scalars plus step b's
// counters (every workgroup computes the same values), and its workgroup 0
// stores them into the other of two slots.  So no kernel reads a slot that a
// kernel running at the same time writes.
// ---------------------------------------------------------------------------
// min(floor(num / den), cap) with num = q * fill_num * 4 * T, exact.  A
// double quotient is within a relative 2^-51 of the true one; exact 128-bit
// products then fix the last unit (no 128-bit division, which is slow here).
__device__ uint64_t target_div(uint64_t q, uint64_t fill_num, uint64_t T, uint64_t den,
                               uint64_t cap)
{
    const unsigned __int128 num = (unsigned __int128)q * fill_num * 4u * T;
    const double est = (double)num / (double)den;
    if (est > (double)cap + 4096.0) return cap;
    uint64_t v = (uint64_t)est;
    while (v > 0 && (unsigned __int128)v * den > num) --v;
    while ((unsigned __int128)(v + 1) * den <= num) ++v;
    return v < cap ? v : cap;
}

// Window head and newest index after the pending step (cheap part of a
// commit: what every thread of the next kernel needs).
__device__ __forceinline__ void step_head(const DevScalars& c, const StepScratch* st, uint32_t n,
                                          int spatial, int64_t* k, uint64_t* h)
{
    *k = c.k;
    *h = c.h;
    if (st->status) return;
    const uint64_t k_end = (uint64_t)(c.k + (int64_t)n);
    *k = (int64_t)k_end;
    if (spatial && k_end + 1 > c.Q && k_end + 1 - c.Q > c.h) *h = k_end + 1 - c.Q;
}

// Full commit of the pending step: counts, Eq. (20), statistics.
__device__ DevScalars commit_step(const DevScalars& c, const StepScratch* st, uint32_t n,
                                  const State& s, int spatial)
{
    DevScalars r = c;
    const uint32_t status = st->status;
    if (status) {
        if (r.err == 0) r.err = (status & 1u) ? -2 : -3;   // FIBAR_E_RANGE / FIBAR_E_POLARITY
        return r;
    }
    int64_t k;
    uint64_t h_new;
    step_head(c, st, n, spatial, &k, &h_new);
    r.k = k;
    if (!spatial) return r;
    uint32_t act = 0, tact = 0, stale = 0, toff = 0;
#pragma unroll
    for (int i = 0; i < kSpread; ++i) {
        act += st->part[i][0];
        tact += st->part[i][1];
        stale += st->part[i][2];
        toff += st->part[i][3];
    }
    r.h = h_new;
    r.P = c.P + act - stale;
    r.T = c.T + tact - toff;
    const uint64_t q = (uint64_t)k + 1 - h_new;
    if (r.P > 0) {
        // Eq. (20) in integers: floor(q * r_fill / (P / (A T))), A = 4
        uint64_t Qn = target_div(q, s.fill_num, r.T, (uint64_t)s.fill_den * r.P, s.q_max);
        if (Qn < s.q_min) Qn = s.q_min;
        r.Q = Qn;
    }
    r.n_reg += 1;
    r.last_stale = stale;
    r.total_stale += stale;
    return r;
}

// (k, h) after the pending step, for every thread of a kernel.
__device__ __forceinline__ void current_head(const State& s, int slot_in, const StepScratch* prev,
                                             uint32_t prev_events, int spatial, int64_t* k,
                                             uint64_t* h)
{
    const DevScalars c = s.sc[slot_in];
    if (prev) {
        step_head(c, prev, prev_events, spatial, k, h);
    } else {
        *k = c.k;
        *h = c.h;
    }
}

// ---------------------------------------------------------------------------
// In-order kernels
// ---------------------------------------------------------------------------

// Apply one chunk's compositions to the state; push the chunk's events to
// the back of the window (spatial filter); count activations.
__global__ __launch_bounds__(128) void k_apply(State s, ChunkDesc cd, const SegRec* __restrict__ seg,
                                               const uint32_t* __restrict__ seg_count,
                                               uint32_t chunk_offset, StepScratch* step,
                                               const StepScratch* prev, uint32_t prev_events,
                                               int slot_in, int slot_out, int spatial)
{
    // the last workgroup only commits the previous step
    if (blockIdx.x == gridDim.x - 1) {
        if (prev && slot_out >= 0 && threadIdx.x == 0)
            s.sc[slot_out] = commit_step(s.sc[slot_in], prev, prev_events, s, spatial);
        return;
    }
    int64_t k0;
    uint64_t h0;
    current_head(s, slot_in, prev, prev_events, spatial, &k0, &h0);
    if (step->status) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t first = (uint64_t)(k0 + 1) + chunk_offset;
    if (spatial && i < cd.n) {
        const uint32_t x = cd.x[i], y = cd.y[i];
        s.ring[(first + i) & s.ring_mask] = y * s.W + x;
    }
    uint32_t dP = 0u, dT = 0u;
    if (i < *seg_count) {
        const SegRec r = seg[i];
        const uint32_t pix = r.pix;
        const float pb = s.pbar[pix];
        float2 lp = s.Lp[pix];
        float l = lp.x;
        if (spatial) {
            // a stale (or never seen) pixel's current value is its blurred one
            const int64_t last_old = s.last[pix];
            l = last_old < (int64_t)h0 ? lp.y : lp.x;
        }
        s.pbar[pix] = fmaf(r.a, pb, r.u1);
        lp.x = fmaf(r.g, pb, fmaf(r.b, l, r.u2));
        s.Lp[pix] = lp;
        s.last[pix] = (int64_t)(first + (r.n_last & 0xffffu));
        if (spatial) {
            const uint32_t old = s.cnt[pix];
            s.cnt[pix] = old + (r.n_last >> 16);
            if (old == 0u) {
                dP = 1u;
                if (atomicAdd(&s.tcnt[tile_of(s, pix)], 1u) == 0u) dT = 1u;
            }
        }
    }
    if (spatial) {
        block_sum2(dP, dT);
        if (threadIdx.x == 0 && (dP | dT)) {
            uint32_t* part = step->part[blockIdx.x % kSpread];
            atomicAdd(&part[0], dP);
            atomicAdd(&part[1], dT);
        }
    }
}

// Current brightness of pixel i while the pops of a step run: the blurred
// value for pixels that were already stale before the step, L otherwise.
__device__ __forceinline__ float cur_L(const State& s, size_t i, int64_t h_old)
{
    const float2 lp = s.Lp[i];
    return s.last[i] < h_old ? lp.y : lp.x;
}

// 3x3 binomial blur of the current image at `pix`, clamp-to-edge, fixed
// summation order.
__device__ __forceinline__ float blur_at(const State& s, uint32_t pix, int64_t h_old)
{
    const uint32_t y = pix / s.W, x = pix - y * s.W;
    const uint32_t xm = x > 0 ? x - 1 : 0, xp = x + 1 < s.W ? x + 1 : s.W - 1;
    const uint32_t ym = y > 0 ? y - 1 : 0, yp = y + 1 < s.H ? y + 1 : s.H - 1;
    const size_t r0 = (size_t)ym * s.W, r1 = (size_t)y * s.W, r2 = (size_t)yp * s.W;
    const float h0 = cur_L(s, r0 + xm, h_old) + 2.f * cur_L(s, r0 + x, h_old) + cur_L(s, r0 + xp, h_old);
    const float h1 = cur_L(s, r1 + xm, h_old) + 2.f * cur_L(s, r1 + x, h_old) + cur_L(s, r1 + xp, h_old);
    const float h2 = cur_L(s, r2 + xm, h_old) + 2.f * cur_L(s, r2 + x, h_old) + cur_L(s, r2 + xp, h_old);
    return (h0 + 2.f * h1 + h2) * 0.0625f;
}

// Move the window head by the target of the previous step (Eq. (20)),
// detect pixels whose last queued event leaves the window, and write their
// blurred values to Lb, reading the image as it was before this step's
// blurs.  `slot` holds the scalars after the previous step.
__global__ __launch_bounds__(128) void k_pop_blur(State s, uint32_t pkt_events, StepScratch* step,
                                                  int slot)
{
    if (step->status) return;
    const DevScalars c = s.sc[slot];
    const uint64_t k_end = (uint64_t)(c.k + (int64_t)pkt_events);
    const uint64_t h_old = c.h, Q = c.Q;
    uint64_t h_new = h_old;
    if (k_end + 1 > Q && k_end + 1 - Q > h_old) h_new = k_end + 1 - Q;

    uint32_t dP = 0u, dT = 0u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = h_old + blockIdx.x * blockDim.x + threadIdx.x; j < h_new; j += stride) {
        const uint32_t pix = s.ring[j & s.ring_mask];
        if (atomicSub(&s.cnt[pix], 1u) == 1u) {
            ++dP;
            // the tile update and the neighbourhood reads are independent:
            // issue both before waiting on either
            const uint32_t told = atomicSub(&s.tcnt[tile_of(s, pix)], 1u);
            const float b = blur_at(s, pix, (int64_t)h_old);
            s.Lp[pix].y = b;
            if (told == 1u) ++dT;
        }
    }
    block_sum2(dP, dT);
    if (threadIdx.x == 0 && (dP | dT)) {
        uint32_t* part = step->part[blockIdx.x % kSpread];
        atomicAdd(&part[2], dP);
        atomicAdd(&part[3], dT);
    }
}

// Commit a pending step into the other slot (one thread).
__global__ void k_commit(State s, const StepScratch* prev, uint32_t prev_events, int slot_in,
                         int slot_out, int spatial)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        s.sc[slot_out] = commit_step(s.sc[slot_in], prev, prev_events, s, spatial);
}

__global__ __launch_bounds__(256) void k_readout(State s, int spatial, const StepScratch* prev,
                                                 uint32_t prev_events, int slot, float* L,
                                                 float* pbar, uint8_t* stale, uint32_t* cnt,
                                                 int64_t* last, float* log_age, uint32_t* tcnt)
{
    int64_t k;
    uint64_t hu;
    current_head(s, slot, prev, prev_events, spatial, &k, &hu);
    const uint64_t npx = (uint64_t)s.W * s.H;
    const int64_t h = (int64_t)hu;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += stride) {
        int64_t li = 0;
        if (spatial || last || log_age) li = s.last[i];
        const float2 lp = s.Lp[i];
        L[i] = (spatial && li < h) ? lp.y : lp.x;
        if (pbar) pbar[i] = s.pbar[i];
        if (last) last[i] = li;
        if (log_age) log_age[i] = log1pf((float)(k - li));
        if (spatial) {
            const uint32_t cn = s.cnt[i];
            if (cnt) cnt[i] = cn;
            if (stale) stale[i] = (li >= 0 && cn == 0u) ? 1u : 0u;
        }
    }
    if (spatial && tcnt) {
        const uint64_t nt = (uint64_t)s.TW * ((s.H + 1) / 2);
        for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) tcnt[i] = s.tcnt[i];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sort_compose(const ChunkDesc* d_chunks, uint32_t n_chunks, SegRec* seg,
                               uint32_t* seg_count, StepScratch* scratch, uint32_t W,
                               uint32_t H, int key_bits, Coef coef, hipStream_t st)
{
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_compose, dim3(n_chunks), dim3(kSortThreads), 0, st, d_chunks, seg,
                       seg_count, scratch, W, H, key_bits, coef);
    return hipGetLastError();
}

hipError_t launch_apply(const State& s, const ChunkDesc* d_chunk, const SegRec* seg,
                        const uint32_t* seg_count, uint32_t chunk_events, uint32_t chunk_offset,
                        StepScratch* step, const StepScratch* prev, uint32_t prev_events,
                        int slot_in, int slot_out, int spatial, hipStream_t st)
{
    // one extra workgroup commits the previous step's scalars
    const uint32_t blocks = (chunk_events + 127) / 128 + 1;
    hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(128), 0, st, s, *d_chunk, seg,
                       seg_count, chunk_offset, step, prev, prev_events, slot_in, slot_out,
                       spatial);
    return hipGetLastError();
}

hipError_t launch_pop_blur(const State& s, uint32_t pkt_events, StepScratch* step, int slot,
                           hipStream_t st)
{
    // many small workgroups spread the scattered reads over more CUs
    hipLaunchKernelGGL(k_pop_blur, dim3(128), dim3(128), 0, st, s, pkt_events, step, slot);
    return hipGetLastError();
}

hipError_t launch_commit(const State& s, const StepScratch* prev, uint32_t prev_events,
                         int slot_in, int slot_out, int spatial, hipStream_t st)
{
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, st, s, prev, prev_events, slot_in,
                       slot_out, spatial);
    return hipGetLastError();
}

hipError_t launch_readout(const State& s, int spatial, const StepScratch* prev,
                          uint32_t prev_events, int slot, float* L, float* pbar, uint8_t* stale,
                          uint32_t* cnt, int64_t* last, float* log_age, uint32_t* tcnt,
                          hipStream_t st)
{
    const uint64_t npx = (uint64_t)s.W * s.H;
    uint64_t blocks = (npx + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_readout, dim3((uint32_t)blocks), dim3(256), 0, st, s, spatial, prev,
                       prev_events, slot, L, pbar, stale, cnt, last, log_age, tcnt);
    return hipGetLastError();
}

}  // namespace fibar
