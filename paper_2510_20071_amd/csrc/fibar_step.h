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

// A chunk's records are sorted tile-major (2x2 tile index, then the pixel's
// position in its tile), so the records of one tile are consecutive, at most
// four.  The first record of a tile (the group head) applies all of them:
// it sees every pixel of its tile before and after, so the activations of
// pixels and of the tile follow from last-event indices (a pixel is active
// iff its newest event is inside the window, last >= h) with no atomics.
// Item i also pushes event i to the back of the window.
//
// In two parts, so that a kernel can issue the loads that need only the
// chunk (records i - 1 .. i + 3, event coordinates) before it waits for the
// window head: load_group, then apply_group.  i < kChunk, and a chunk's
// record slot is followed by at least 3 more records of memory.
struct Group {
    uint32_t prev_key;       // sort key of record i - 1, all ones for i = 0
    SegRec r[4];             // records i .. i + 3
    uint32_t ex, ey;         // event i
};

__device__ __forceinline__ Group load_group(const ChunkDesc& cd, const SegRec* __restrict__ seg,
                                           uint32_t i, int spatial)
{
    Group g;
    const uint32_t pk = seg[i > 0 ? i - 1 : 0].key;          // unconditional: no wait
    g.prev_key = i > 0 ? pk : 0xffffffffu;
#pragma unroll
    for (int q = 0; q < 4; ++q) g.r[q] = seg[i + q];
    g.ex = 0u;
    g.ey = 0u;
    if (spatial && i < cd.n) {
        g.ex = cd.x[i];
        g.ey = cd.y[i];
    }
    return g;
}

// Every load is unconditional, from a valid address (values not needed are
// masked afterwards), so that all of them are in flight together.
__device__ __forceinline__ void apply_group(const State& s, const Group& g, uint32_t n,
                                            uint32_t nseg, uint32_t i, uint64_t first,
                                            uint64_t h0, int spatial, uint32_t& dP, uint32_t& dT)
{
    if (spatial && i < n) s.ring[(first + i) & s.ring_mask] = g.ey * s.W + g.ex;
    if (i >= nseg) return;
    const uint32_t t = g.r[0].key >> 2;
    if (i > 0 && (g.prev_key >> 2) == t) return;              // not the head of its tile
    bool mem[4];
    uint32_t pix[4];
    mem[0] = true;
#pragma unroll
    for (int k = 1; k < 4; ++k) mem[k] = mem[k - 1] && i + k < nseg && (g.r[k].key >> 2) == t;
#pragma unroll
    for (int k = 0; k < 4; ++k) pix[k] = mem[k] ? g.r[k].pix : g.r[0].pix;
    // the tile's pixels: quad q at (2 tx + (q & 1), 2 ty + (q >> 1))
    const uint32_t k0 = g.r[0].key;
    const uint32_t base = pix[0] - (k0 & 1u) - ((k0 >> 1) & 1u) * s.W;
    const uint32_t ty = t / s.TW, tx = t - ty * s.TW;
    const bool has_x1 = 2 * tx + 1 < s.W, has_y1 = 2 * ty + 1 < s.H;
    int64_t lq[4];
    float pb[4];
    float2 lp[4];
    uint32_t cn[4];
    if (spatial) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool ok = (!(q & 1) || has_x1) && (!(q & 2) || has_y1);
            lq[q] = s.last[ok ? base + (q & 1) + (q >> 1) * s.W : base];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pb[k] = s.pbar[pix[k]];
        lp[k] = s.Lp[pix[k]];
        cn[k] = spatial ? s.cnt[pix[k]] : 0u;
    }
    bool tile_was_active = false;
    if (spatial) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool ok = (!(q & 1) || has_x1) && (!(q & 2) || has_y1);
            if (!ok) lq[q] = -1;
            tile_was_active |= lq[q] >= (int64_t)h0;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!mem[k]) continue;
        const SegRec& r = g.r[k];
        float l = lp[k].x;
        if (spatial) {
            const uint32_t q = r.key & 3u;
            const int64_t last_old = q == 3 ? lq[3] : q == 2 ? lq[2] : q == 1 ? lq[1] : lq[0];
            // a stale (or never seen) pixel's current value is its blurred one
            if (last_old < (int64_t)h0) {
                l = lp[k].y;
                dP += 1u;
            }
        }
        s.pbar[pix[k]] = fmaf(r.a, pb[k], r.u1);
        float2 o = lp[k];
        o.x = fmaf(r.g, pb[k], fmaf(r.b, l, r.u2));
        s.Lp[pix[k]] = o;
        s.last[pix[k]] = (int64_t)(first + (r.n_last & 0xffffu));
        if (spatial) s.cnt[pix[k]] = cn[k] + (r.n_last >> 16);
    }
    if (spatial && !tile_was_active) dT += 1u;
}

// Pops j = start, start + stride, ... below h_new.  A pixel goes stale when
// its newest event leaves the window, i.e. exactly when the popped j is its
// last index; it then gets its blurred value in Lp.y, computed from the image
// as it was before this step's blurs.  Its 2x2 tile goes inactive when no
// pixel of the tile has a newer event: the pixel with the largest last
// index of the tile (unique, and popped in this same step) counts it.  The
// whole 3x3 neighbourhood (which holds the tile) is loaded for every pop,
// before the decision; the count update needs no result.
__device__ __forceinline__ void pop_range(const State& s, uint64_t start, uint64_t h_new,
                                          uint64_t stride, uint64_t h_old, uint32_t& dP,
                                          uint32_t& dT)
{
    for (uint64_t j = start; j < h_new; j += stride) {
        const uint32_t pix = s.ring[j & s.ring_mask];
        const uint32_t y = pix / s.W, x = pix - y * s.W;
        const uint32_t xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < s.W ? x + 1 : s.W - 1};
        const uint32_t ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < s.H ? y + 1 : s.H - 1};
        int64_t lst[3][3];
        float2 lp[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const size_t q = (size_t)ys[a] * s.W + xs[b];
                lst[a][b] = s.last[q];
                lp[a][b] = s.Lp[q];
            }
        atomicSub(&s.cnt[pix], 1u);
        if (lst[1][1] != (int64_t)j) continue;
        ++dP;
        float c[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                c[a][b] = lst[a][b] < (int64_t)h_old ? lp[a][b].y : lp[a][b].x;
        // 3x3 binomial blur, clamp-to-edge, fixed summation order
        const float r0 = c[0][0] + 2.f * c[0][1] + c[0][2];
        const float r1 = c[1][0] + 2.f * c[1][1] + c[1][2];
        const float r2 = c[2][0] + 2.f * c[2][1] + c[2][2];
        s.Lp[pix].y = (r0 + 2.f * r1 + r2) * 0.0625f;
        // the tile's other pixels: column x ^ 1 and row y ^ 1, where they
        // exist (selected with fixed indices: a register array indexed at run
        // time would be moved to memory)
        const bool ox = x & 1u, oy = y & 1u;
        const bool hx = ox || x + 1 < s.W, hy = oy || y + 1 < s.H;
        const int64_t lx = ox ? lst[1][0] : lst[1][2];
        const int64_t ly = oy ? lst[0][1] : lst[2][1];
        const int64_t lxy = oy ? (ox ? lst[0][0] : lst[0][2]) : (ox ? lst[2][0] : lst[2][2]);
        const int64_t me = lst[1][1];
        const bool newest = !(hx && lx > me) && !(hy && ly > me) && !(hx && hy && lxy > me);
        if (newest) ++dT;
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

// Active pixels of tile t (their newest event is inside the window).
__device__ __forceinline__ uint32_t tile_active_pixels(const State& s, uint64_t t, int64_t h)
{
    const uint32_t ty = (uint32_t)(t / s.TW), tx = (uint32_t)(t - (uint64_t)ty * s.TW);
    uint32_t n = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t px = 2 * tx + (q & 1), py = 2 * ty + (q >> 1);
        if (px < s.W && py < s.H && s.last[(size_t)py * s.W + px] >= h) ++n;
    }
    return n;
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
        if (cnt) cnt[i] = s.cnt[i];
        if (stale) stale[i] = (li >= 0 && li < h) ? 1u : 0u;
    }
}

}  // namespace
}  // namespace step
}  // namespace fibar
