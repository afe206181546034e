// Per-tile event queues (the paper's Limitations: event queues operated
// separately for each tile of the image).  The sensor is cut into tiles of
// R x R pixels (R even, <= 32, so that the 2x2 cells of Eq. (19) never
// straddle two tiles); each tile keeps its own FIFO window of its own
// events, its own active pixel and cell counts and its own target of
// Eq. (20), clamped to [min(q_min, n), n] for a tile of n pixels.  A tile
// that no longer registers events still advances: an event also leaves once
// age_max newer events have arrived anywhere on the sensor.  Regulation is
// per packet, with the blurs of a step simultaneous, as in the single-queue
// path.
//
// Per batch (bulk, like the blur-off path): k_tq_count histograms each
// chunk's events per tile, the blur-off scan and base kernels place the
// tiles' slices, and k_tq_scatter moves every event into its tile's slice
// (chunk order, then arrival order).  Per packet, two launches:
//   k_tq_step  one 1024-thread workgroup per tile, a thread per pixel: the
//              tile's events of the packet are applied in time order per
//              pixel, pushed to the tile's ring, then the tile pops (target
//              and age), finds its stale pixels (a pixel goes stale when its
//              newest event leaves), updates its counts and target, and
//              lists the stale pixels;
//   k_tq_blur  every listed pixel gets its one-time 3x3 blur into Lb, from
//              the image before the step's blurs.
// A pixel's current brightness is Lb when its newest event is older than
// its tile's window front (the global index of the tile's oldest window
// event), else L.  Fronts are kept for two consecutive steps, so that the
// blur reads every neighbour's tile front from before the step.
#include "fibar_ctx.h"
#include "fibar_internal.h"
#include "fibar_tile.h"

namespace fibar {
namespace {

using namespace tile;

constexpr uint64_t kNoPix = 0xffffffffull;

struct TQGeom {
    uint32_t W, H, R, RW, RH;
};

__device__ __forceinline__ uint32_t tq_tile_of(const TQGeom& g, uint32_t pix)
{
    const uint32_t y = pix / g.W, x = pix - y * g.W;
    return (y / g.R) * g.RW + x / g.R;
}

// Exclusive sum over the 1024-thread workgroup (block_exscan_u32) used as a
// plain sum.
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* scan1)
{
    uint32_t total;
    (void)block_exscan_u32(v, scan1, &total);
    return total;
}

__global__ __launch_bounds__(1024) void k_tq_count(const ChunkDesc* __restrict__ chunks, TQGeom g,
                                                   uint32_t n_tiles, uint32_t* __restrict__ cnt,
                                                   StepScratch* __restrict__ scratch)
{
    __shared__ uint32_t hist[kMaxRegions];
    __shared__ uint32_t bad_sh;
    const ChunkDesc cd = chunks[blockIdx.x];
    for (uint32_t r = threadIdx.x; r < n_tiles; r += blockDim.x) hist[r] = 0u;
    if (threadIdx.x == 0) bad_sh = 0u;
    __syncthreads();
    uint32_t bad = 0u;
    for (uint32_t e = threadIdx.x; e < cd.n; e += blockDim.x) {
        const uint32_t x = cd.x[e], y = cd.y[e], p = cd.p[e];
        const bool inr = x < g.W && y < g.H;
        bad |= inr ? 0u : 1u;
        bad |= p > 1u ? 2u : 0u;
        atomicAdd(&hist[inr ? (y / g.R) * g.RW + x / g.R : 0u], 1u);
    }
    if (bad) atomicOr(&bad_sh, bad);
    __syncthreads();
    if (threadIdx.x == 0 && bad_sh) atomicOr(&scratch[cd.pkt].status, bad_sh);
    uint32_t* row = cnt + (size_t)blockIdx.x * n_tiles;
    for (uint32_t r = threadIdx.x; r < n_tiles; r += blockDim.x) row[r] = hist[r];
}

// Per chunk: stable LDS sort by tile, then every event to its tile's slice.
// Payload: global pixel (or kNoPix for a rejected packet) << 32 | chunk << 15
// | arrival index << 1 | polarity.
__global__ __launch_bounds__(kSortThreads) void k_tq_scatter(
    const ChunkDesc* __restrict__ chunks, TQGeom g, int tile_bits,
    const uint32_t* __restrict__ offs, uint32_t n_tiles, const uint64_t* __restrict__ base,
    const StepScratch* __restrict__ scratch, uint64_t* __restrict__ payload)
{
    __shared__ uint32_t keypol[kChunk];
    __shared__ __align__(16) uint16_t idxA[kChunk];
    __shared__ __align__(16) uint16_t idxB[kChunk];
    __shared__ uint64_t scan4[kWaves + 1][4];
    __shared__ uint32_t scan1[kWaves + 1];
    const ChunkDesc cd = chunks[blockIdx.x];
    const uint32_t cn = cd.n;
    for (uint32_t e = threadIdx.x; e < cn; e += kSortThreads) {
        const uint32_t x = cd.x[e], y = cd.y[e], p = cd.p[e];
        const bool inr = x < g.W && y < g.H;
        const uint32_t tl = inr ? (y / g.R) * g.RW + x / g.R : 0u;
        keypol[e] = (tl << 1) | (p & 1u);
        idxA[e] = (uint16_t)e;
    }
    __syncthreads();
    const uint16_t* sorted = tile_sort(keypol, idxA, idxB, cn, tile_bits, scan4);
    const bool valid = scratch[cd.pkt].status == 0u;
    const uint32_t* off_row = offs + (size_t)blockIdx.x * n_tiles;
    // rank among the chunk's items of the same tile: position minus the
    // position of the tile's first item
    const uint32_t beg = threadIdx.x * kSortItems;
    uint32_t lmax = 0;
    uint32_t prev = (beg > 0 && beg - 1 < cn) ? keypol[sorted[beg - 1]] >> 1 : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t sidx = beg + j;
        if (sidx < cn) {
            const uint32_t tl = keypol[sorted[sidx]] >> 1;
            if (sidx == 0 || tl != prev) lmax = sidx;
            prev = tl;
        }
    }
    // exclusive max-scan of the heads (the thread's last head, or 0)
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        uint32_t inc = lmax;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc = max(inc, o);
        }
        if (lane == 63) scan1[wave] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t t = scan1[w];
                scan1[w] = run;
                run = max(run, t);
            }
        }
        __syncthreads();
        uint32_t ex = __shfl_up(inc, 1, 64);
        if (lane == 0) ex = 0;
        lmax = max(scan1[wave], ex);
    }
    uint32_t head = lmax;
    prev = (beg > 0 && beg - 1 < cn) ? keypol[sorted[beg - 1]] >> 1 : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t sidx = beg + j;
        if (sidx < cn) {
            const uint32_t oid = sorted[sidx];
            const uint32_t kp = keypol[oid];
            const uint32_t tl = kp >> 1;
            if (sidx == 0 || tl != prev) head = sidx;
            prev = tl;
            const uint64_t dest = base[tl] + off_row[tl] + (sidx - head);
            const uint64_t pixf = valid ? (uint64_t)cd.y[oid] * g.W + cd.x[oid] : kNoPix;
            payload[dest] = (pixf << 32) | ((uint64_t)blockIdx.x << 15) | ((uint64_t)oid << 1) |
                            (uint64_t)(kp & 1u);
        }
    }
}

// Initial tile state: empty windows (front 0 = the first event), targets at
// the tile's pixel count.
__global__ __launch_bounds__(256) void k_tq_init(TQTile* tiles, uint64_t* front, TQGeom g,
                                                 uint32_t n_tiles)
{
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t tx = t % g.RW, ty = t / g.RW;
    const uint32_t w = min(g.R, g.W - tx * g.R), h = min(g.R, g.H - ty * g.R);
    TQTile z;
    z.head = z.tail = 0u;
    z.Q = w * h;
    z.P = z.T = 0u;
    z.npix = w * h;
    z.pad[0] = z.pad[1] = 0u;
    tiles[t] = z;
    front[t] = 0u;
    front[n_tiles + t] = 0u;
}

struct TQStep {
    uint32_t c0, c1, n_chunks, pkt;
    int parity;
    int slot;
};

// Work grows with the tile's events and pops, not with its pixels: only the
// 2x2 cells that an event or a pop touches load and store their state.
// Events are taken in pieces of up to 1024 (time order); each owner thread
// scans a piece for its own pixel and applies those events in order.
constexpr uint32_t kPiece = 1024;

__global__ __launch_bounds__(1024) void k_tq_step(State s, TQGeom g, TQTile* __restrict__ tiles,
                                                  uint64_t* __restrict__ front,
                                                  uint2* __restrict__ ring, uint32_t ring_mask,
                                                  uint32_t* __restrict__ stale_list,
                                                  RegionBuffers rb, StepScratch* __restrict__ scratch,
                                                  TQStep st, uint64_t age_max, Coef coef)
{
    __shared__ uint32_t ent_key[kPiece];     // local pixel << 1 | polarity
    __shared__ uint32_t ent_gi[kPiece];      // global index, low 32 bits
    __shared__ uint32_t pop_cnt[1024];
    __shared__ uint8_t touched[1024];        // an event or a pop of this pixel
    __shared__ uint8_t act_b[1024], act_a[1024], act_p[1024];
    __shared__ uint32_t counts[6];           // dP, dT, old events, stale, cells gone, any work

    const uint32_t t = blockIdx.x, n_tiles = gridDim.x;
    const uint32_t tid = threadIdx.x;
    const uint64_t* front_old = front + (size_t)st.parity * n_tiles;
    uint64_t* front_new = front + (size_t)(st.parity ^ 1) * n_tiles;
    const uint64_t f_old = front_old[t];
    if (scratch[st.pkt].status != 0u) {   // a rejected packet changes nothing
        if (tid == 0) front_new[t] = f_old;
        return;
    }
    const TQTile tl = tiles[t];
    const uint32_t tx0 = (t % g.RW) * g.R, ty0 = (t / g.RW) * g.R;
    const uint32_t tw = min(g.R, g.W - tx0), th = min(g.R, g.H - ty0);
    const uint32_t lx = tid % g.R, ly = tid / g.R;
    const bool own = ly < th && lx < tw && tid < g.R * g.R;
    const uint64_t gp = own ? (uint64_t)(ty0 + ly) * g.W + tx0 + lx : 0u;
    const int64_t k_after = rb.chunk_k[st.c1] - 1;

    // the tile's events of this packet: [lo, hi) of its slice
    const uint64_t bt = rb.base[t];
    const uint64_t lo = bt + rb.cnt[(size_t)st.c0 * n_tiles + t];
    const uint64_t hi = st.c1 < st.n_chunks ? bt + rb.cnt[(size_t)st.c1 * n_tiles + t]
                                             : bt + rb.total[t];
    const uint32_t n_new = (uint32_t)(hi - lo);
    const uint32_t tail = tl.tail + n_new;
    const uint32_t q = tail - tl.head;
    const size_t rbase = (size_t)t * (ring_mask + 1);
    auto global_of = [&](uint32_t lo32) {   // a window event is < 2^32 events old
        return (uint64_t)k_after - (uint32_t)((uint32_t)k_after - lo32);
    };

    // a tile without new events, within its target and whose oldest event
    // is young enough, does nothing but move an empty window's front
    if (n_new == 0 && q <= tl.Q) {
        bool idle = true;
        if (q > 0) {
            const uint64_t e0 = global_of(ring[rbase + (tl.head & ring_mask)].x);
            idle = (uint64_t)k_after - e0 < age_max;
        }
        if (idle) {
            if (tid == 0) front_new[t] = q > 0 ? f_old : (uint64_t)k_after + 1;
            return;
        }
    }

    touched[tid] = 0u;
    pop_cnt[tid] = 0u;
    if (tid < 6) counts[tid] = 0u;
    __syncthreads();

    // events: into the ring (time order) and marked
    for (uint64_t cur = lo; cur < hi; cur += 1024) {
        const uint64_t e = cur + tid;
        if (e < hi) {
            const uint64_t pl = rb.payload[e];
            const uint32_t pix = (uint32_t)(pl >> 32);
            const uint32_t py = pix / g.W, px = pix - py * g.W;
            const uint32_t lk = (py - ty0) * g.R + (px - tx0);
            const uint32_t ch = (uint32_t)(pl >> 15) & 0xffu;
            const uint64_t ge = (uint64_t)(rb.chunk_k[ch] + (int64_t)((pl >> 1) & 0x3fffu));
            ring[rbase + ((tl.tail + (uint32_t)(e - lo)) & ring_mask)] = make_uint2((uint32_t)ge, lk);
            touched[lk] = 1u;
        }
    }
    __syncthreads();   // the pushed entries are read back below
    // pops: while the window is longer than the target, or its oldest event
    // is age_max or more events old (both hold for a prefix of the window)
    uint32_t my_old = 0u;
    if ((uint64_t)k_after + 1 > age_max) {
        const uint64_t lim = (uint64_t)k_after - age_max;   // events at or below leave
        for (uint32_t i = tid; i < q; i += 1024) {
            const uint2 en = ring[rbase + ((tl.head + i) & ring_mask)];
            my_old += global_of(en.x) <= lim ? 1u : 0u;
        }
    }
    if (my_old) atomicAdd(&counts[2], my_old);
    __syncthreads();
    const uint32_t n_len = q > tl.Q ? q - tl.Q : 0u;
    const uint32_t n_pop = counts[2] > n_len ? counts[2] : n_len;
    for (uint32_t i = tid; i < n_pop; i += 1024) {
        const uint2 en = ring[rbase + ((tl.head + i) & ring_mask)];
        atomicAdd(&pop_cnt[en.y], 1u);
        touched[en.y] = 1u;
    }
    __syncthreads();
    const uint32_t head1 = tl.head + n_pop;
    uint64_t f_new = (uint64_t)k_after + 1;
    if (n_pop < q) f_new = global_of(ring[rbase + (head1 & ring_mask)].x);

    // the pixels of touched 2x2 cells load their state
    const uint32_t cx = lx & ~1u, cy = ly & ~1u;
    const uint32_t c0 = cy * g.R + cx;
    const bool cell_touched = own && (touched[c0] | (cx + 1 < tw ? touched[c0 + 1] : 0u) |
                                      (cy + 1 < th ? touched[c0 + g.R] : 0u) |
                                      (cx + 1 < tw && cy + 1 < th ? touched[c0 + g.R + 1] : 0u));
    float pb = 0.f, l = 0.f, lb = 0.f, gain = 1.f;
    int64_t last = -1;
    uint32_t cnt = 0u;
    uint64_t tot = 0u;
    if (cell_touched) {
        const PixL v = s.px[gp];
        last = v.last;
        lb = v.Lb;
        l = v.last < (int64_t)f_old ? v.Lb : v.L;
        if (touched[tid]) {
            const PixP w = s.pp[gp];
            pb = w.pbar;
            cnt = w.cnt;
            tot = w.tot;
            if (s.gain) gain = s.gain[gp];
        }
    }
    const bool was_active = cell_touched && last >= (int64_t)f_old;

    // the owner applies its pixel's events in time order (Eq. (7), then
    // Eq. (6) and (10)), a piece of up to 1024 events at a time
    const float c = (0.5f + 0.5f * coef.beta) * gain;
    uint32_t got = 0u;
    for (uint64_t cur = lo; cur < hi; cur += kPiece) {
        const uint32_t m = (uint32_t)(hi - cur < kPiece ? hi - cur : kPiece);
        __syncthreads();
        if (tid < m) {
            const uint2 en = ring[rbase + ((tl.tail + (uint32_t)(cur - lo) + tid) & ring_mask)];
            const uint64_t pl = rb.payload[cur + tid];
            ent_key[tid] = (en.y << 1) | (uint32_t)(pl & 1u);
            ent_gi[tid] = en.x;
        }
        __syncthreads();
        if (own && touched[tid]) {
            for (uint32_t e = 0; e < m; ++e) {
                const uint32_t kp = ent_key[e];
                if ((kp >> 1) != tid) continue;
                const float p = (kp & 1u) ? 1.f : -1.f;
                pb = fmaf(coef.alpha, pb, coef.one_m_alpha * p);
                l = fmaf(coef.beta, l, c * (p - pb));
                ++got;
                last = (int64_t)global_of(ent_gi[e]);
            }
        }
    }
    tot += got;
    const bool active_a = was_active || got > 0u;
    // a pixel goes stale when its newest event leaves: its last index is
    // below the new front while it was active
    const bool stale_now = own && active_a && last < (int64_t)f_new;
    act_b[tid] = was_active ? 1u : 0u;
    act_a[tid] = active_a ? 1u : 0u;
    act_p[tid] = (active_a && !stale_now) ? 1u : 0u;
    __syncthreads();
    const bool cell_head = cell_touched && (lx & 1u) == 0u && (ly & 1u) == 0u;
    auto cell_any = [&](const uint8_t* a) {
        uint32_t v = a[tid];
        if (lx + 1 < tw) v |= a[tid + 1];
        if (ly + 1 < th) v |= a[tid + g.R];
        if (lx + 1 < tw && ly + 1 < th) v |= a[tid + g.R + 1];
        return v != 0u;
    };
    if (own && !was_active && active_a) atomicAdd(&counts[0], 1u);
    if (cell_head) {
        const bool b = cell_any(act_b), a_ = cell_any(act_a), p_ = cell_any(act_p);
        if (!b && a_) atomicAdd(&counts[1], 1u);
        if (a_ && !p_) atomicAdd(&counts[4], 1u);
    }
    if (stale_now) {
        atomicAdd(&counts[3], 1u);
        const uint32_t at = atomicAdd(&scratch[st.pkt].part[0][0], 1u);
        stale_list[at] = (uint32_t)gp;
    }
    if (own && touched[tid]) {
        cnt = cnt + got - pop_cnt[tid];
        if (got) {
            PixL v;
            v.L = l;
            v.Lb = lb;
            v.last = last;
            s.px[gp] = v;
        }
        PixP w;
        w.pbar = pb;
        w.cnt = cnt;
        w.tot = tot;
        s.pp[gp] = w;
    }
    __syncthreads();
    if (tid == 0) {
        TQTile o = tl;
        o.head = head1;
        o.tail = tail;
        o.P = tl.P + counts[0] - counts[3];
        o.T = tl.T + counts[1] - counts[4];
        const uint32_t q1 = tail - head1;
        if (o.P > 0) {
            // Eq. (20): floor(q num 4 T / (den P)) from a double quotient
            // (numerator below 2^53) fixed by one integer check
            const uint64_t num = (uint64_t)q1 * o.T * (4u * s.fill_num);
            const uint64_t dv = (uint64_t)s.fill_den * o.P;
            uint64_t v = (uint64_t)((double)num / (double)dv);
            if (v * dv > num) --v;
            else if ((v + 1) * dv <= num) ++v;
            const uint32_t lo_q = s.q_min < tl.npix ? (uint32_t)s.q_min : tl.npix;
            o.Q = v > tl.npix ? tl.npix : (v < lo_q ? lo_q : (uint32_t)v);
        }
        tiles[t] = o;
        front_new[t] = f_new;
    }
}

// The one-time blur of every pixel listed by the step (3x3 binomial,
// clamp-to-edge, fixed order), each neighbour taken as Lb when it was stale
// before the step (its newest event below its tile's old front), else L.
// One thread also stores the step's scalars: newest index, step count,
// stale pixels.
__global__ __launch_bounds__(256) void k_tq_blur(State s, TQGeom g, const uint64_t* __restrict__ front,
                                                 uint32_t n_tiles, const uint32_t* __restrict__ stale_list,
                                                 StepScratch* __restrict__ scratch,
                                                 const int64_t* __restrict__ chunk_k, TQStep st)
{
    const uint64_t* front_old = front + (size_t)st.parity * n_tiles;
    const uint32_t n = scratch[st.pkt].status ? 0u : scratch[st.pkt].part[0][0];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const uint32_t j = stale_list[i];
        const uint32_t y = j / g.W, x = j - y * g.W;
        const uint32_t xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < g.W ? x + 1 : g.W - 1};
        const uint32_t ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < g.H ? y + 1 : g.H - 1};
        float cv[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint32_t pix = ys[a] * g.W + xs[b];
                const PixL v = s.px[pix];
                const uint64_t f = front_old[(ys[a] / g.R) * g.RW + xs[b] / g.R];
                cv[a][b] = v.last < (int64_t)f ? v.Lb : v.L;
            }
        const float r0 = cv[0][0] + 2.f * cv[0][1] + cv[0][2];
        const float r1 = cv[1][0] + 2.f * cv[1][1] + cv[1][2];
        const float r2 = cv[2][0] + 2.f * cv[2][1] + cv[2][2];
        s.px[j].Lb = (r0 + 2.f * r1 + r2) * 0.0625f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && scratch[st.pkt].status == 0u) {
        DevScalars& sc = s.sc[st.slot];
        sc.k = chunk_k[st.c1] - 1;
        sc.n_reg += 1;
        sc.last_stale = n;
        sc.total_stale += n;
    }
}

__global__ __launch_bounds__(256) void k_tq_readout(State s, TQGeom g, const uint64_t* __restrict__ front,
                                                    int slot, float* L, float* pbar, uint8_t* stale,
                                                    uint32_t* cnt, int64_t* last, float* log_age,
                                                    uint32_t* tcnt, uint64_t* tot)
{
    const uint64_t npx = (uint64_t)g.W * g.H;
    const int64_t k = s.sc[slot].k;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < npx; i += stride) {
        const PixL v = s.px[i];
        const uint64_t f = front[tq_tile_of(g, (uint32_t)i)];
        const bool st = v.last < (int64_t)f;
        L[i] = st ? v.Lb : v.L;
        if (pbar) pbar[i] = s.pp[i].pbar;
        if (tot) tot[i] = s.pp[i].tot;
        if (last) last[i] = v.last;
        if (log_age) log_age[i] = log1pf((float)(k - v.last));
        if (cnt) cnt[i] = s.pp[i].cnt;
        if (stale) stale[i] = (v.last >= 0 && st) ? 1u : 0u;
    }
    if (tcnt) {
        const uint32_t TW = (g.W + 1) / 2, nt = TW * ((g.H + 1) / 2);
        for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < nt; c += stride) {
            const uint32_t cx = (uint32_t)(c % TW), cy = (uint32_t)(c / TW);
            uint32_t a = 0;
            for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t x = 2 * cx + (q & 1), y = 2 * cy + (q >> 1);
                if (x < g.W && y < g.H) {
                    const uint32_t pix = y * g.W + x;
                    a += s.px[pix].last >= (int64_t)front[tq_tile_of(g, pix)] ? 1u : 0u;
                }
            }
            tcnt[c] = a;
        }
    }
}

inline TQGeom geom_of(const fibar_ctx* c)
{
    TQGeom g;
    g.W = c->W;
    g.H = c->H;
    g.R = c->tq_R;
    g.RW = c->tq_RW;
    g.RH = c->tq_RH;
    return g;
}

}  // namespace

hipError_t tq_init(fibar_ctx* c)
{
    const uint32_t n = c->tq_RW * c->tq_RH;
    hipLaunchKernelGGL(k_tq_init, dim3((n + 255) / 256), dim3(256), 0, c->st, c->tq_tiles,
                       c->tq_front, geom_of(c), n);
    c->tq_parity = 0;
    return hipGetLastError();
}

hipError_t tq_bulk(fibar_ctx* c, uint32_t n_chunks)
{
    const uint32_t n = c->tq_RW * c->tq_RH;
    const TQGeom g = geom_of(c);
    hipLaunchKernelGGL(k_tq_count, dim3(n_chunks), dim3(1024), 0, c->st, c->d_chunks, g, n,
                       c->rb.cnt, c->scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_region_scan_bases(c->s, c->cur_slot, c->d_chunks, n_chunks, c->scratch, c->rb,
                                 false, c->st);
    if (e != hipSuccess) return e;
    int bits = 1;
    while ((1u << bits) < n) ++bits;
    hipLaunchKernelGGL(k_tq_scatter, dim3(n_chunks), dim3(kSortThreads), 0, c->st, c->d_chunks, g,
                       bits, (const uint32_t*)c->rb.cnt, n, (const uint64_t*)c->rb.base,
                       (const StepScratch*)c->scratch, c->rb.payload);
    return hipGetLastError();
}

hipError_t tq_step(fibar_ctx* c, uint32_t c0, uint32_t c1, uint32_t n_chunks, uint32_t pkt)
{
    const uint32_t n = c->tq_RW * c->tq_RH;
    const TQGeom g = geom_of(c);
    TQStep st;
    st.c0 = c0;
    st.c1 = c1;
    st.n_chunks = n_chunks;
    st.pkt = pkt;
    st.parity = c->tq_parity;
    st.slot = c->cur_slot;
    hipLaunchKernelGGL(k_tq_step, dim3(n), dim3(1024), 0, c->st, c->s, g, c->tq_tiles,
                       c->tq_front, c->tq_ring, c->tq_cap - 1, c->tq_stale, c->rb, c->scratch, st,
                       c->tq_age, c->coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tq_blur, dim3(64), dim3(256), 0, c->st, c->s, g,
                       (const uint64_t*)c->tq_front, n, (const uint32_t*)c->tq_stale, c->scratch,
                       (const int64_t*)c->rb.chunk_k, st);
    c->tq_parity ^= 1;
    return hipGetLastError();
}

hipError_t tq_readout(fibar_ctx* c, float* L, float* pbar, uint8_t* stale, uint32_t* cnt,
                      int64_t* last, float* log_age, uint32_t* tcnt, uint64_t* tot)
{
    const uint32_t n = c->tq_RW * c->tq_RH;
    const uint64_t blocks = (c->npx + 255) / 256;
    hipLaunchKernelGGL(k_tq_readout, dim3((uint32_t)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                       c->st, c->s, geom_of(c),
                       (const uint64_t*)(c->tq_front + (size_t)c->tq_parity * n), c->cur_slot, L,
                       pbar, stale, cnt, last, log_age, tcnt, tot);
    return hipGetLastError();
}

}  // namespace fibar
