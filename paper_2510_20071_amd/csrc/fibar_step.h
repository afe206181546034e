// Device functions of the in-order steps (apply a chunk, pop the window,
// blur stale pixels, commit the window scalars, read out), shared by the
// single-stream kernels and the multi-stream work-queue kernels.  Internal
// header.
#pragma once

#include "fibar_tile.h"

// Keeps every memory access above it above it and every one below below
// (an empty statement; it neither waits for nor touches memory).
#define FIBAR_ISSUE_FENCE() asm volatile("" ::: "memory")

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
// Kernels of step b store their activation / deactivation counts into the
// step's scratch (one slot per wave).  Nobody waits for the last workgroup:
// the *next* kernel that needs the scalars after step b derives them from
// the last committed scalars plus step b's counters (every workgroup
// computes the same values), and its workgroup 0 stores them into the other
// of two slots.  So no kernel reads a slot that a kernel running at the same
// time writes.
// ---------------------------------------------------------------------------
// min(floor(num / den), cap) with num = q * fill_num * 4 * T, exact.  The
// factors q and f = fill_num * 4 * T (< 2^48) and den (< 2^48) are exact in
// double, so the double quotient is within a relative 2^-51 of the true one;
// exact 128-bit products then fix the last unit (no 128-bit division or
// conversion, which are slow here).
__device__ uint64_t target_div(uint64_t q, uint64_t fill_num, uint64_t T, uint64_t den,
                               uint64_t cap)
{
    const uint64_t f = fill_num * 4u * T;
    const double est = ((double)q * (double)f) / (double)den;
    if (est > (double)cap + 4096.0) return cap;
    const unsigned __int128 num = (unsigned __int128)q * f;
    uint64_t v = (uint64_t)est;
    while (v > 0 && (unsigned __int128)v * den > num) --v;
    while ((unsigned __int128)(v + 1) * den <= num) ++v;
    return v < cap ? v : cap;
}

// Window head and newest index after the pending step (cheap part of a
// commit: what every thread of the next kernel needs).  Selects, not
// branches, so that the status load is issued together with the scalars.
__device__ __forceinline__ void step_head(const DevScalars& c, uint32_t status, uint32_t n,
                                          int spatial, int64_t* k, uint64_t* h)
{
    const int64_t ck = c.k;
    const uint64_t ch = c.h, cQ = c.Q;
    const uint64_t k_end = (uint64_t)(ck + (int64_t)n);
    const bool move = spatial && k_end + 1 > cQ && k_end + 1 - cQ > ch;
    *k = status ? ck : (int64_t)k_end;
    *h = (status || !move) ? ch : k_end + 1 - cQ;
}

// A step's counts: activated pixels and tiles, stale pixels, deactivated
// tiles.
struct StepCounts {
    uint32_t act, tact, stale, toff;
};

// Sum of a step's count slots and overflow counters by one full wave (the
// same in every lane).  Every load is issued before any is used: a fixed
// number per lane from clamped addresses, the surplus zeroed afterwards (a
// loop would wait for each load in turn).
__device__ StepCounts gather_counts(const StepScratch* st)
{
    constexpr uint32_t kA = kApplySlots / 2, kP = kPopSlots / 2;   // slot pairs
    constexpr int kJa = (int)((kA + 63) / 64), kJp = (int)((kP + 63) / 64);
    const uint4* wa = reinterpret_cast<const uint4*>(st->wave_apply);
    const uint4* wp = reinterpret_cast<const uint4*>(st->wave_pop);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ov = lane < (uint32_t)kSpread ? lane : 0u;
    uint4 qa[kJa], qp[kJp];
#pragma unroll
    for (int j = 0; j < kJa; ++j) {
        const uint32_t i = lane + 64u * j;
        qa[j] = wa[i < kA ? i : 0u];
    }
#pragma unroll
    for (int j = 0; j < kJp; ++j) {
        const uint32_t i = lane + 64u * j;
        qp[j] = wp[i < kP ? i : 0u];
    }
    uint4 qo = *reinterpret_cast<const uint4*>(st->part[ov]);
    FIBAR_ISSUE_FENCE();
    // no sum is hoisted between the loads (it would wait for the first ones
    // before the last are issued)
#pragma unroll
    for (int j = 0; j < kJa; ++j)
        asm volatile("" : "+v"(qa[j].x), "+v"(qa[j].y), "+v"(qa[j].z), "+v"(qa[j].w));
#pragma unroll
    for (int j = 0; j < kJp; ++j)
        asm volatile("" : "+v"(qp[j].x), "+v"(qp[j].y), "+v"(qp[j].z), "+v"(qp[j].w));
    asm volatile("" : "+v"(qo.x), "+v"(qo.y), "+v"(qo.z), "+v"(qo.w));
    uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < kJa; ++j) {
        const bool ok = lane + 64u * j < kA;
        v[0] += ok ? qa[j].x + qa[j].z : 0u;
        v[1] += ok ? qa[j].y + qa[j].w : 0u;
    }
#pragma unroll
    for (int j = 0; j < kJp; ++j) {
        const bool ok = lane + 64u * j < kP;
        v[2] += ok ? qp[j].x + qp[j].z : 0u;
        v[3] += ok ? qp[j].y + qp[j].w : 0u;
    }
    const bool ook = lane < (uint32_t)kSpread;
    v[0] += ook ? qo.x : 0u;
    v[1] += ook ? qo.y : 0u;
    v[2] += ook ? qo.z : 0u;
    v[3] += ook ? qo.w : 0u;
    StepCounts r;
    r.act = wave_sum(v[0]);
    r.tact = wave_sum(v[1]);
    r.stale = wave_sum(v[2]);
    r.toff = wave_sum(v[3]);
    return r;
}

// Full commit of the pending step (validation status, counts): Eq. (20),
// statistics.
__device__ DevScalars commit_step(const DevScalars& c, uint32_t status, uint32_t n,
                                  const State& s, int spatial, const StepCounts& cn)
{
    DevScalars r = c;
    r.stepped = 0;
    if (status) {
        if (r.err == 0) r.err = (status & 1u) ? -2 : -3;   // FIBAR_E_RANGE / FIBAR_E_POLARITY
        return r;
    }
    int64_t k;
    uint64_t h_new;
    step_head(c, status, n, spatial, &k, &h_new);
    r.k = k;
    if (!spatial) return r;
    const uint32_t act = cn.act, tact = cn.tact, stale = cn.stale, toff = cn.toff;
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
    r.stepped = 1;
    r.last_stale = stale;
    r.total_stale += stale;
    return r;
}

// Commit of the pending step `prev` (n events) on top of the scalars at
// sc_in, by one full wave (the same in every lane).  The scalars and the
// status are loaded before the count slots, so that one memory round trip
// serves all of them.
__device__ DevScalars commit_by_wave(const DevScalars* sc_in, const StepScratch* prev,
                                          uint32_t n, const State& s, int spatial)
{
    const DevScalars c = *sc_in;
    const uint32_t status = prev->status;
    FIBAR_ISSUE_FENCE();
    const StepCounts cn = spatial ? gather_counts(prev) : StepCounts{0u, 0u, 0u, 0u};
    return commit_step(c, status, n, s, spatial, cn);
}

// Store a commit `r` of a step of n events (one lane): the scalars, and the
// step's record into the telemetry buffer when the commit was a regulation
// step and the buffer has room.
__device__ __forceinline__ void store_commit(const State& s, DevScalars* out, const DevScalars& r,
                                             uint32_t n)
{
    *out = r;
    if (s.tel && r.stepped && r.n_reg - 1 < s.tel_cap) {
        StepRecord t;
        t.k = r.k;
        t.h = r.h;
        t.q = (uint64_t)(r.k + 1) - r.h;
        t.Q = r.Q;
        t.P = r.P;
        t.T = r.T;
        t.stale = r.last_stale;
        t.n = n;
        s.tel[r.n_reg - 1] = t;
    }
}

// Read in place of a pending step's scratch when there is none (its value
// is not used; reading it keeps the load unconditional).
__device__ StepScratch no_pending_step;

// The scalars that (k, h) after the pending step follow from, loaded
// together (load_head), and the head computed from them (head_after).
struct HeadIn {
    int64_t k;
    uint64_t h, Q;
    uint32_t pending_status;
    bool pending;
};

__device__ __forceinline__ HeadIn load_head(const DevScalars* sc_in, const StepScratch* prev)
{
    const DevScalars& c = *sc_in;
    HeadIn r;
    r.k = c.k;
    r.h = c.h;
    r.Q = c.Q;
    r.pending_status = (prev ? prev : &no_pending_step)->status;
    r.pending = prev != nullptr;
    return r;
}

__device__ __forceinline__ void head_after(const HeadIn& c, uint32_t prev_events, int spatial,
                                           int64_t* k, uint64_t* h)
{
    const uint64_t k_end = (uint64_t)(c.k + (int64_t)prev_events);
    const bool move = spatial && k_end + 1 > c.Q && k_end + 1 - c.Q > c.h;
    const bool adv = c.pending && !c.pending_status;
    *k = adv ? (int64_t)k_end : c.k;
    *h = (adv && move) ? k_end + 1 - c.Q : c.h;
}

// (k, h) after the pending step, for every thread of a kernel.
__device__ __forceinline__ void current_head(const State& s, int slot_in, const StepScratch* prev,
                                             uint32_t prev_events, int spatial, int64_t* k,
                                             uint64_t* h)
{
    head_after(load_head(s.sc + slot_in, prev), prev_events, spatial, k, h);
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
// In parts, so that a kernel can issue the loads that need only the chunk
// (records i - 1 .. i + 3, event coordinates) and then the tile's state
// before it waits for the window head: load_group, load_tile, apply_tile.
// i < kChunk (callers clamp), and a chunk's record slot is followed by at
// least 3 more records of memory.
struct Group {
    uint32_t prev_key;       // sort key of record i - 1, all ones for i = 0
    SegRec r[4];             // records i .. i + 3
    uint32_t ex, ey;         // event i
};

__device__ __forceinline__ Group load_group(const ChunkDesc& cd, const SegRec* __restrict__ seg,
                                           uint32_t i)
{
    Group g;
    const uint32_t pk = seg[i > 0 ? i - 1 : 0].key;          // unconditional: no wait
    g.prev_key = i > 0 ? pk : 0xffffffffu;
#pragma unroll
    for (int q = 0; q < 4; ++q) g.r[q] = seg[i + q];
    // unconditional too (the chunk holds at least one event): a load under a
    // branch leaves the kernel-argument loads pending at the join, and the
    // next use of one then waits for every outstanding scalar load
    const uint32_t e = i < cd.n ? i : 0u;
    g.ex = cd.x[e];
    g.ey = cd.y[e];
    return g;
}

// The state of the tile of record i, loaded before the scalars (rejection
// status, record count, window head) are waited for: its addresses need
// only the records.  Records past the chunk's count are stale memory, so
// every address is clamped into the image and the values are masked later.
// No branch surrounds the loads (a value merged at a join is copied there,
// and the copy waits for its load); the records of a tile's other pixels
// repeat the head's addresses, which coalesce within the wavefront.
struct TileIn {
    bool head;               // first record of its tile
    bool same[4];            // records i .. i + 3 belong to the tile
    uint32_t pix[4];
    int64_t qlast[4];        // last-event index of the tile's four quads
    float L[4], Lb[4];       // the records' pixels
    int64_t last[4];
    float pbar[4];
    uint32_t cnt[4];
    uint64_t tot[4];
};

__device__ __forceinline__ TileIn load_tile(const State& s, const Group& g, uint32_t i)
{
    TileIn ti;
    const uint32_t npx = s.W * s.H;
    const uint32_t t = g.r[0].key >> 2;
    ti.head = i == 0 || (g.prev_key >> 2) != t;
    ti.same[0] = true;
#pragma unroll
    for (int k = 1; k < 4; ++k) ti.same[k] = ti.same[k - 1] && (g.r[k].key >> 2) == t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t p = ti.same[k] ? g.r[k].pix : g.r[0].pix;
        ti.pix[k] = p < npx ? p : 0u;
    }
    // the tile's pixels: quad q at (2 tx + (q & 1), 2 ty + (q >> 1))
    const uint32_t k0 = g.r[0].key;
    const uint32_t base = ti.pix[0] - (k0 & 1u) - ((k0 >> 1) & 1u) * s.W;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t p = base + (q & 1) + (q >> 1) * s.W;
        ti.qlast[q] = s.px[p < npx ? p : 0u].last;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const PixL v = s.px[ti.pix[k]];
        ti.L[k] = v.L;
        ti.Lb[k] = v.Lb;
        ti.last[k] = v.last;
        const PixP w = s.pp[ti.pix[k]];
        ti.pbar[k] = w.pbar;
        ti.cnt[k] = w.cnt;
        ti.tot[k] = w.tot;
    }
    return ti;
}

// Push event i to the window; if record i heads its tile, apply the tile's
// records and count pixel and tile activations.
__device__ __forceinline__ void apply_tile(const State& s, const Group& g, const TileIn& ti,
                                           uint32_t n, uint32_t nseg, bool rejected, uint32_t i,
                                           uint64_t first, uint64_t h0, int spatial, uint32_t& dP,
                                           uint32_t& dT)
{
    if (rejected) return;
    if (spatial && i < n) s.ring[(first + i) & s.ring_mask] = g.ey * s.W + g.ex;
    if (i >= nseg || !ti.head) return;
    const uint32_t t = g.r[0].key >> 2;
    const uint32_t ty = t / s.TW, tx = t - ty * s.TW;
    const bool has_x1 = 2 * tx + 1 < s.W, has_y1 = 2 * ty + 1 < s.H;
    bool tile_was_active = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool ok = (!(q & 1) || has_x1) && (!(q & 2) || has_y1);
        tile_was_active |= ok && ti.qlast[q] >= (int64_t)h0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!ti.same[k] || i + k >= nseg) continue;
        const SegRec& r = g.r[k];
        const uint32_t px = ti.pix[k];
        float l = ti.L[k];
        // a stale (or never seen) pixel's current value is its blurred one
        if (spatial && ti.last[k] < (int64_t)h0) {
            l = ti.Lb[k];
            dP += 1u;
        }
        const float pb = ti.pbar[k];
        PixL o;
        o.L = fmaf(r.g, pb, fmaf(r.b, l, r.u2));
        o.Lb = ti.Lb[k];
        o.last = (int64_t)(first + (r.n_last & 0xffffu));
        s.px[px] = o;
        PixP op;
        op.pbar = fmaf(r.a, pb, r.u1);
        op.cnt = spatial ? ti.cnt[k] + (r.n_last >> 16) : ti.cnt[k];
        op.tot = ti.tot[k] + (r.n_last >> 16);
        s.pp[px] = op;
    }
    if (spatial && !tile_was_active) dT += 1u;
}

// Passes scalar-loaded values through an empty statement placed after the
// state loads, so that no arithmetic on them (which waits for every
// outstanding scalar load) is scheduled before those loads are issued.
__device__ __forceinline__ void scalars_after_loads(HeadIn& h, uint32_t& status, uint32_t& nseg)
{
    asm volatile("" : "+s"(h.k), "+s"(h.h), "+s"(h.Q), "+s"(h.pending_status), "+s"(status),
                 "+s"(nseg)::"memory");
}

// Pop event j (at pixel pix).  A pixel goes stale when
// its newest event leaves the window, i.e. exactly when the popped j is its
// last index; it then gets its blurred value in Lb, computed from the image
// as it was before this step's blurs.  Its 2x2 tile goes inactive when no
// pixel of the tile has a newer event: the pixel with the largest last
// index of the tile (unique, and popped in this same step) counts it.  The
// whole 3x3 neighbourhood (which holds the tile) is loaded for every pop,
// before the decision; the count update needs no result.
// In two parts, so that a kernel can issue the neighbourhood loads before
// it waits for the window head: load_pop, then decide_pop.  The caller owns
// the neighbourhood array (a struct returned by value ended up in scratch
// memory).
__device__ __forceinline__ void load_pop(const State& s, uint32_t pix, PixL (&nb)[3][3])
{
    const uint32_t y = pix / s.W, x = pix - y * s.W;
    const uint32_t xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < s.W ? x + 1 : s.W - 1};
    const uint32_t ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < s.H ? y + 1 : s.H - 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) nb[a][b] = s.px[(size_t)ys[a] * s.W + xs[b]];
}

// Blurred value of a pixel going stale in a step whose pops start at h_old:
// 3x3 binomial, clamp-to-edge, fixed summation order, over the image before
// the step's blurs (a neighbour's current value is Lb if it was stale
// before the step, else L).  It reads nothing the step's pops write.
__device__ __forceinline__ float stale_blur(const PixL (&nb)[3][3], uint64_t h_old)
{
    float c[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            c[a][b] = nb[a][b].last < (int64_t)h_old ? nb[a][b].Lb : nb[a][b].L;
    const float r0 = c[0][0] + 2.f * c[0][1] + c[0][2];
    const float r1 = c[1][0] + 2.f * c[1][1] + c[1][2];
    const float r2 = c[2][0] + 2.f * c[2][1] + c[2][2];
    return (r0 + 2.f * r1 + r2) * 0.0625f;
}

__device__ __forceinline__ void decide_pop(const State& s, uint64_t j, uint32_t pix,
                                           const PixL (&nb)[3][3], uint64_t h_old, uint32_t& dP,
                                           uint32_t& dT)
{
    const uint32_t y = pix / s.W, x = pix - y * s.W;
    atomicSub(&s.pp[pix].cnt, 1u);
    if (nb[1][1].last != (int64_t)j) return;
    ++dP;
    s.px[pix].Lb = stale_blur(nb, h_old);
    // the tile's other pixels: column x ^ 1 and row y ^ 1, where they
    // exist (selected with fixed indices: a register array indexed at run
    // time would be moved to memory)
    const bool ox = x & 1u, oy = y & 1u;
    const bool hx = ox || x + 1 < s.W, hy = oy || y + 1 < s.H;
    const int64_t lx = ox ? nb[1][0].last : nb[1][2].last;
    const int64_t ly = oy ? nb[0][1].last : nb[2][1].last;
    const int64_t lxy = oy ? (ox ? nb[0][0].last : nb[0][2].last)
                           : (ox ? nb[2][0].last : nb[2][2].last);
    const int64_t me = nb[1][1].last;
    const bool newest = !(hx && lx > me) && !(hy && ly > me) && !(hx && hy && lxy > me);
    if (newest) ++dT;
}

__device__ __forceinline__ void pop_one(const State& s, uint64_t j, uint32_t pix, uint64_t h_old,
                                        uint32_t& dP, uint32_t& dT)
{
    PixL nb[3][3];
    load_pop(s, pix, nb);
    decide_pop(s, j, pix, nb, h_old, dP, dT);
}

// Pops j = start, start + stride, ... below h_new, pixels from the ring.
__device__ __forceinline__ void pop_range(const State& s, uint64_t start, uint64_t h_new,
                                          uint64_t stride, uint64_t h_old, uint32_t& dP,
                                          uint32_t& dT)
{
    for (uint64_t j = start; j < h_new; j += stride)
        pop_one(s, j, s.ring[j & s.ring_mask], h_old, dP, dT);
}

// Store a wave's activation (pops = false) or deactivation (pops = true)
// counts into the step's scratch.  g is the thread's index in the step's
// grid of that kind, so the wave's slot is g / 64; waves past the slots add
// to the overflow counters.  Zero counts are not stored (the scratch starts
// zeroed).
__device__ __forceinline__ void add_counts(StepScratch* step, bool pops, uint32_t g, uint32_t a,
                                           uint32_t b)
{
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63u) == 0 && (a | b)) {
        const uint32_t w = g >> 6;
        if (w < (pops ? kPopSlots : kApplySlots)) {
            (pops ? step->wave_pop : step->wave_apply)[w] = make_uint2(a, b);
        } else {
            uint32_t* part = step->part[w % kSpread] + (pops ? 2 : 0);
            atomicAdd(&part[0], a);
            atomicAdd(&part[1], b);
        }
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
        if (px < s.W && py < s.H && s.px[(size_t)py * s.W + px].last >= h) ++n;
    }
    return n;
}

// Readout of pixel i after a step whose pops move the head from h_old to
// h_new, taken while those pops run: a pixel going stale in the step
// (h_old <= last < h_new) gets the blurred value its pop writes, computed
// here from the same operands.  Every output but the window count (which
// the pops decrement) is available this way.
__device__ __forceinline__ void readout_pixel_after_pops(const State& s, int64_t k, uint64_t h_old,
                                                         uint64_t h_new, uint64_t i, const PixL& v,
                                                         float* L, float* pbar, uint8_t* stale,
                                                         int64_t* last, float* log_age,
                                                         uint64_t* tot)
{
    const int64_t li = v.last;
    float val = v.L;
    if (li < (int64_t)h_new) {
        val = v.Lb;
        if (li >= (int64_t)h_old) {
            PixL nb[3][3];
            load_pop(s, (uint32_t)i, nb);
            val = stale_blur(nb, h_old);
        }
    }
    L[i] = val;
    if (pbar) pbar[i] = s.pp[i].pbar;
    if (tot) tot[i] = s.pp[i].tot;
    if (last) last[i] = li;
    if (log_age) log_age[i] = log1pf((float)(k - li));
    if (stale) stale[i] = (li >= 0 && li < (int64_t)h_new) ? 1u : 0u;
}

// Readout of pixel i given the newest index k and window head h.
__device__ __forceinline__ void readout_pixel(const State& s, int spatial, int64_t k, int64_t h,
                                              uint64_t i, float* L, float* pbar, uint8_t* stale,
                                              uint32_t* cnt, int64_t* last, float* log_age,
                                              uint64_t* tot)
{
    const PixL v = s.px[i];
    const int64_t li = v.last;
    L[i] = (spatial && li < h) ? v.Lb : v.L;
    if (pbar) pbar[i] = s.pp[i].pbar;
    if (tot) tot[i] = s.pp[i].tot;
    if (last) last[i] = li;
    if (log_age) log_age[i] = log1pf((float)(k - li));
    if (spatial) {
        if (cnt) cnt[i] = s.pp[i].cnt;
        if (stale) stale[i] = (li >= 0 && li < h) ? 1u : 0u;
    }
}

}  // namespace
}  // namespace step
}  // namespace fibar
