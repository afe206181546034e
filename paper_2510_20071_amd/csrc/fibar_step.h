// Device functions of the in-order steps (apply a chunk, pop the window,
// blur stale pixels, commit the window scalars, read out), shared by the
// single-stream kernels and the multi-stream work-queue kernels.  Internal
// header.
#pragma once

#include "fibar_tile.h"

namespace fibar {
namespace step {
namespace {

using namespace tile;

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

// Window head before and after the pops of a step whose packet has
// `pkt_events` events, from the scalars committed after the previous step.
__device__ __forceinline__ void pop_bounds(const DevScalars& c, uint32_t pkt_events,
                                           uint64_t* h_old, uint64_t* h_new)
{
    const uint64_t k_end = (uint64_t)(c.k + (int64_t)pkt_events);
    *h_old = c.h;
    *h_new = c.h;
    if (k_end + 1 > c.Q && k_end + 1 - c.Q > c.h) *h_new = k_end + 1 - c.Q;
}

// Item i of a chunk's apply, in two parts so that a kernel can issue the
// loads that need only the chunk (segment record, event coordinates) before
// it waits for the window head: load_item, then apply_loaded, which pushes
// event i to the back of the window and applies the composed map of segment
// i (one distinct pixel) to the state, counting activations of pixels and
// tiles.  i < kChunk: a chunk slot always holds kChunk records.
struct Item {
    SegRec rec;
    uint32_t ex, ey;
};

__device__ __forceinline__ Item load_item(const ChunkDesc& cd, const SegRec* __restrict__ seg,
                                          uint32_t i, int spatial)
{
    Item it;
    it.rec = seg[i];
    it.ex = 0u;
    it.ey = 0u;
    if (spatial && i < cd.n) {
        it.ex = cd.x[i];
        it.ey = cd.y[i];
    }
    return it;
}

__device__ __forceinline__ void apply_loaded(const State& s, const Item& it, uint32_t n,
                                             uint32_t nseg, uint32_t i, uint64_t first,
                                             uint64_t h0, int spatial, uint32_t& dP, uint32_t& dT)
{
    if (spatial && i < n) s.ring[(first + i) & s.ring_mask] = it.ey * s.W + it.ex;
    if (i < nseg) {
        const SegRec& r = it.rec;
        const uint32_t pix = r.pix;
        const float pb = s.pbar[pix];
        float2 lp = s.Lp[pix];
        float l = lp.x;
        int64_t last_old = 0;
        uint32_t old = 0u;
        if (spatial) {
            last_old = s.last[pix];
            old = s.cnt[pix];
            // a stale (or never seen) pixel's current value is its blurred one
            l = last_old < (int64_t)h0 ? lp.y : lp.x;
        }
        s.pbar[pix] = fmaf(r.a, pb, r.u1);
        lp.x = fmaf(r.g, pb, fmaf(r.b, l, r.u2));
        s.Lp[pix] = lp;
        s.last[pix] = (int64_t)(first + (r.n_last & 0xffffu));
        if (spatial) {
            s.cnt[pix] = old + (r.n_last >> 16);
            if (old == 0u) {
                dP += 1u;
                if (atomicAdd(&s.tcnt[tile_of(s, pix)], 1u) == 0u) dT += 1u;
            }
        }
    }
}

// Pops j = start, start + stride, ... below h_new: pixels whose last queued
// event leaves the window go stale and get their blurred value in Lb,
// computed from the image as it was before this step's blurs.
__device__ __forceinline__ void pop_range(const State& s, uint64_t start, uint64_t h_new,
                                          uint64_t stride, uint64_t h_old, uint32_t& dP,
                                          uint32_t& dT)
{
    for (uint64_t j = start; j < h_new; j += stride) {
        const uint32_t pix = s.ring[j & s.ring_mask];
        // The neighbourhood is read before the count update returns (most
        // pops end a pixel's activity, so few of these reads are wasted):
        // the values do not depend on the update, since a pixel that goes
        // stale in this step is still read as L.
        const float b = blur_at(s, pix, (int64_t)h_old);
        if (atomicSub(&s.cnt[pix], 1u) == 1u) {
            ++dP;
            if (atomicSub(&s.tcnt[tile_of(s, pix)], 1u) == 1u) ++dT;
            s.Lp[pix].y = b;
        }
    }
}

// Add a workgroup's activation (slot 0, 1) or deactivation (slot 2, 3)
// counts to the step's scratch.
__device__ __forceinline__ void add_counts(StepScratch* step, int first_slot, uint32_t a, uint32_t b)
{
    block_sum2(a, b);
    if (threadIdx.x == 0 && (a | b)) {
        uint32_t* part = step->part[blockIdx.x % kSpread];
        atomicAdd(&part[first_slot], a);
        atomicAdd(&part[first_slot + 1], b);
    }
}

// Readout of pixel i given the newest index k and window head h.
__device__ __forceinline__ void readout_pixel(const State& s, int spatial, int64_t k, int64_t h,
                                              uint64_t i, float* L, float* pbar, uint8_t* stale,
                                              uint32_t* cnt, int64_t* last, float* log_age)
{
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

}  // namespace
}  // namespace step
}  // namespace fibar
