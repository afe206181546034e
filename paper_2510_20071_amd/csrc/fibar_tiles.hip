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
//   k_tq_step  a workgroup per tile, a thread per 2x2 cell: the tile's
//              events of the packet are pushed to its ring, the tile pops
//              (target and age), the cells touched by an event or a pop
//              apply their pixels' events
//              in time order and find their stale pixels (a pixel goes stale
//              when its newest event leaves), and the tile updates its
//              counts and target and lists the stale pixels;
//   k_tq_blur  a workgroup per tile: every listed pixel gets its one-time
//              3x3 blur into Lb, from the image before the step's blurs.
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
    const ChunkDesc cd = global_chunk(chunks[blockIdx.x]);
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
    // the chunk's validation bits, in its own slot (the base kernel gathers
    // them per packet)
    if (threadIdx.x == 0) scratch[blockIdx.x].pad[0] = bad_sh;
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
    const ChunkDesc cd = global_chunk(chunks[blockIdx.x]);
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

// One workgroup per tile, one thread per 2x2 cell (R <= 32: at most 256
// cells), and work that grows with the tile's events and pops, not with its
// pixels: only the cells that an event or a pop touches load and store their
// state.  The dependent memory round trips are few: the tile's scalars; then
// its new events, the oldest part of its window (the likely pops, into LDS)
// and the step's chunk indices together; then the touched cells' state.
// Events are bucketed by cell in pieces of kPiece (a count per cell, a scan,
// a scatter), so a thread reads only its own cell's events and applies them
// by increasing index.
constexpr uint32_t kTqThreads = 256;
constexpr uint32_t kPiece = 512;
constexpr uint32_t kPre = 512;   // window entries prefetched into LDS
static_assert(kPre % kTqThreads == 0, "the prefetch takes kPre / kTqThreads entries per thread");
constexpr uint32_t kPer = kPiece / kTqThreads;
static_assert(kMaxBatchChunks <= kTqThreads, "a step's chunk indices are staged one per thread");

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if ((int)lane >= o) v += u;
    }
    return v;
}

// The pointers the first loads need lead the argument list (16 dwords, which
// arrive preloaded in scalar registers): the fronts before and after the
// step, the packet's scratch record, the tiles, the step's end index
// (chunk_k of its end chunk), the region bases and the count rows of the
// step's first and end chunk (the totals when the step ends the batch).
__global__ __launch_bounds__(kTqThreads, 4) void k_tq_step(
    const uint64_t* __restrict__ front_old, StepScratch* __restrict__ pkt_scratch,
    TQTile* __restrict__ tiles, const int64_t* __restrict__ k_end,
    const uint64_t* __restrict__ base, const uint32_t* __restrict__ cnt_lo,
    const uint32_t* __restrict__ cnt_hi, uint64_t* __restrict__ front_new, State s, TQGeom g,
    uint2* __restrict__ ring, uint32_t ring_mask, uint32_t* __restrict__ stale_list,
    uint32_t* __restrict__ nstale, RegionBuffers rb, TQStep st, uint64_t age_max, Coef coef)
{
    __shared__ uint32_t touched_w[256];           // a byte per pixel: event or pop
    __shared__ uint32_t popc[1024];               // pops per pixel
    __shared__ uint32_t keys[kPiece];             // bucketed events: pixel << 1 | polarity
    __shared__ uint32_t gis[kPiece];              // global index, low 32 bits
    __shared__ uint32_t ccnt[kTqThreads];         // a piece's events per cell
    __shared__ uint32_t cstart[kTqThreads];       // and where each cell's begin
    __shared__ int64_t ck[kTqThreads];            // first global index of the step's chunks
    __shared__ uint2 pre[kPre];                   // the window's oldest entries
    __shared__ uint2 newe[kPiece];                // and its entries pushed by the step
    __shared__ uint32_t wtot[kTqThreads / 64];
    __shared__ uint32_t sh_first, sh_nstale, sh_red[3];

    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t t = blockIdx.x;
    uint8_t* touched = reinterpret_cast<uint8_t*>(touched_w);
    // the tile's scalars, all loaded together: the empty asm statement takes
    // the loaded values as they are, so that all loads are issued before one
    // wait (else the loads that only the full path needs would follow the
    // status test's wait, and arithmetic on one value would wait for it alone)
    const uint64_t f_old = front_old[t];
    const uint32_t status = pkt_scratch->status;
    const TQTile tl = tiles[t];
    const int64_t k_end_v = *k_end;
    const uint64_t bt = base[t];
    const uint32_t c_lo = cnt_lo[t], c_hi = cnt_hi[t];
    asm volatile("" ::"s"(f_old), "s"(status), "s"(tl.head), "s"(tl.tail), "s"(tl.Q), "s"(tl.P),
                 "s"(tl.T), "s"(k_end_v), "s"(bt), "s"(c_lo), "s"(c_hi));
    const int64_t k_after = k_end_v - 1;
    const uint64_t lo = bt + c_lo;
    const uint64_t hi = bt + c_hi;
    if (status != 0u) {   // a rejected packet changes nothing
        if (tid == 0) {
            front_new[t] = f_old;
            nstale[t] = 0u;
        }
        return;
    }
    const uint32_t tx0 = (t % g.RW) * g.R, ty0 = (t / g.RW) * g.R;
    const uint32_t tw = min(g.R, g.W - tx0), th = min(g.R, g.H - ty0);
    // this tile's stale pixels of the step go to its own part of the list
    uint32_t* my_stale = stale_list + (size_t)t * g.R * g.R;
    const uint32_t n_new = (uint32_t)(hi - lo);
    const uint32_t q_old = tl.tail - tl.head;
    const uint32_t tail = tl.tail + n_new;
    const uint32_t q = tail - tl.head;
    const size_t rbase = (size_t)t * (ring_mask + 1);
    auto global_of = [&](uint32_t lo32) {   // a window event is < 2^32 events old
        return (uint64_t)k_after - (uint32_t)((uint32_t)k_after - lo32);
    };
    const bool can_age = (uint64_t)k_after + 1 > age_max;
    const uint64_t lim = can_age ? (uint64_t)k_after - age_max : 0u;   // at or below: leave

    // a tile without new events, within its target and whose oldest event
    // is young enough, only moves an empty window's front
    if (n_new == 0 && q <= tl.Q) {
        bool idle = true;
        if (q > 0 && can_age) idle = global_of(ring[rbase + (tl.head & ring_mask)].x) > lim;
        if (idle) {
            if (tid == 0) {
                front_new[t] = q > 0 ? f_old : (uint64_t)k_after + 1;
                nstale[t] = 0u;
            }
            return;
        }
    }

    const uint32_t n_len = q > tl.Q ? q - tl.Q : 0u;   // pops by target
    uint32_t npre = n_len + 64u;
    npre = npre < q_old ? npre : q_old;
    npre = npre < kPre ? npre : kPre;
    touched_w[tid] = 0u;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) popc[tid + kTqThreads * j] = 0u;
    // the step's chunk indices and the window's oldest entries: every load
    // issued (from clamped, valid indices) before any is stored to LDS, so
    // that they travel together (a load stored at once waits for itself)
    const bool has_ck = tid < st.c1 - st.c0;
    const int64_t ckv = rb.chunk_k[st.c0 + (has_ck ? tid : 0u)];
    uint2 prv[kPre / kTqThreads];
#pragma unroll
    for (uint32_t j = 0; j < kPre / kTqThreads; ++j) {
        const uint32_t i = tid + kTqThreads * j;
        prv[j] = ring[rbase + ((tl.head + (i < npre ? i : 0u)) & ring_mask)];
    }
    // the step's first piece of events, kept in registers for the bucketing
    // (loaded from entry 0 where a thread has none, then zeroed)
    uint64_t pl0[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t i = tid + kTqThreads * j;
        pl0[j] = rb.payload[i < n_new ? lo + i : 0u];
    }
    if (has_ck) ck[tid] = ckv;
#pragma unroll
    for (uint32_t j = 0; j < kPre / kTqThreads; ++j) {
        const uint32_t i = tid + kTqThreads * j;
        if (i < npre) pre[i] = prv[j];
    }
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) pl0[j] = tid + kTqThreads * j < n_new ? pl0[j] : 0ull;
    if (tid == 0) {
        sh_first = q;
        sh_nstale = 0u;
        sh_red[0] = sh_red[1] = sh_red[2] = 0u;
    }
    __syncthreads();

    // an event's local pixel and global index (low 32 bits) from its payload
    auto decode = [&](uint64_t pl, uint32_t& lk, uint32_t& gi) {
        const uint32_t pix = (uint32_t)(pl >> 32);
        const uint32_t py = pix / g.W, px = pix - py * g.W;
        lk = (py - ty0) * g.R + (px - tx0);
        const uint32_t ch = (uint32_t)(pl >> 15) & 0xffu;
        // a step's chunks are chunks of one batch (at most kMaxBatchChunks =
        // kTqThreads), all staged in ck
        const int64_t kc = ck[ch - st.c0];
        gi = (uint32_t)(uint64_t)(kc + (int64_t)((pl >> 1) & 0x3fffu));
    };

    // the packet's events join the back of the window
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t i = tid + kTqThreads * j;
        if (i < n_new) {
            uint32_t lk, gi;
            decode(pl0[j], lk, gi);
            ring[rbase + ((tl.tail + i) & ring_mask)] = make_uint2(gi, lk);
            newe[i] = make_uint2(gi, lk);
            touched[lk] = 1u;
        }
    }
    for (uint32_t i = tid + kPiece; i < n_new; i += kTqThreads) {
        uint32_t lk, gi;
        decode(rb.payload[lo + i], lk, gi);
        ring[rbase + ((tl.tail + i) & ring_mask)] = make_uint2(gi, lk);
        touched[lk] = 1u;
    }
    // window entry i (0 = oldest): prefetched, pushed by this step (the
    // first kPiece), else from the ring
    auto entry = [&](uint32_t i) {
        if (i < npre) return pre[i];
        if (i >= q_old && i - q_old < kPiece) return newe[i - q_old];
        return ring[rbase + ((tl.head + i) & ring_mask)];
    };
    // the ring stores above need to be visible to the workgroup only when a
    // pushed entry beyond the first kPiece may be read back
    if (n_new > kPiece) __threadfence_block();
    __syncthreads();

    // events that leave: a prefix of the window, by target and by age.  The
    // oldest entries are in LDS; the ring is read only when all of them are
    // too old (the first young entry is nearly always among the first few)
    uint32_t n_old = 0;
    if (can_age) {
        // a wave's young entries have ascending indices, so only its first
        // young lane takes the LDS minimum: one atomic per wave, not one per
        // lane (a uniform-address atomic is serialised over active lanes)
        for (uint32_t i = tid; i < npre; i += kTqThreads) {
            const bool young = global_of(pre[i].x) > lim;
            const uint64_t m = __ballot(young);
            if (young && lane == (uint32_t)__builtin_ctzll(m)) atomicMin(&sh_first, i);
        }
        __syncthreads();
        n_old = sh_first;
        if (n_old == q && npre < q) {
            __syncthreads();   // read by all before the updates below
            for (uint32_t b = npre; b < q; b += kTqThreads) {
                const uint32_t i = b + tid;
                const bool young = i < q && global_of(entry(i).x) > lim;
                const uint64_t m = __ballot(young);
                if (young && lane == (uint32_t)__builtin_ctzll(m)) atomicMin(&sh_first, i);
                __syncthreads();
                n_old = sh_first;
                __syncthreads();   // read by all before the next chunk's updates
                if (n_old < q) break;
            }
        }
    }
    const uint32_t n_pop = n_old > n_len ? n_old : n_len;
    for (uint32_t i = tid; i < n_pop; i += kTqThreads) {
        const uint32_t lk = entry(i).y;
        atomicAdd(&popc[lk], 1u);
        touched[lk] = 1u;
    }
    const uint32_t head1 = tl.head + n_pop;
    uint64_t f_new = (uint64_t)k_after + 1;
    if (n_pop < q) f_new = global_of(entry(n_pop).x);
    __syncthreads();

    // this thread's cell: pixels q = 0..3 at (cx + (q & 1), cy + (q >> 1))
    const uint32_t CR = g.R / 2;
    const uint32_t cell = tid;
    const uint32_t cx = (cell % CR) * 2, cy = (cell / CR) * 2;
    const bool inc = cell < CR * CR;
    const float cgain = 0.5f + 0.5f * coef.beta;
    // pixel q's local and global indices, recomputed where needed
    auto lk_of = [&](int qq) { return (cy + (qq >> 1)) * g.R + cx + (qq & 1); };
    auto gp_of = [&](int qq) {
        return (uint64_t)(ty0 + cy + (qq >> 1)) * g.W + tx0 + cx + (qq & 1);
    };
    bool in[4], tch[4];
    float pb[4], l[4], c[4];
    int64_t last[4];
    uint32_t cnt[4], got[4];
    uint64_t tot[4];
    bool was[4];
    bool has = false;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const uint32_t lx = cx + (qq & 1), ly = cy + (qq >> 1);
        in[qq] = inc && lx < tw && ly < th;
        tch[qq] = in[qq] && touched[lk_of(qq)];
        has |= tch[qq];
    }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        in[qq] = in[qq] && has;
        pb[qq] = l[qq] = 0.f;
        c[qq] = cgain;
        last[qq] = -1;
        cnt[qq] = got[qq] = 0u;
        tot[qq] = 0u;
    }
    // a touched cell loads all four pixels' records before it waits for any
    // (one round trip, not one per pixel: loads under per-pixel conditions
    // were each followed by their own wait), pixels outside the tile from
    // the cell's first pixel, which is inside it, and keeps what it needs
    if (has) {
        PixL v[4];
        PixP w[4];
        float gn[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const uint64_t gq = gp_of(in[qq] ? qq : 0);
            v[qq] = s.px[gq];
            w[qq] = s.pp[gq];
            gn[qq] = s.gain ? s.gain[gq] : 1.f;
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            if (in[qq]) {
                last[qq] = v[qq].last;
                l[qq] = v[qq].last < (int64_t)f_old ? v[qq].Lb : v[qq].L;
            }
            if (tch[qq]) {
                pb[qq] = w[qq].pbar;
                cnt[qq] = w[qq].cnt;
                tot[qq] = w[qq].tot;
                if (s.gain) c[qq] = cgain * gn[qq];
            }
        }
    }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) was[qq] = in[qq] && last[qq] >= (int64_t)f_old;

    // the cell's events in time order (Eq. (7), then Eq. (6) and (10))
    for (uint32_t p0 = 0; p0 < n_new; p0 += kPiece) {
        const uint32_t m = n_new - p0 < kPiece ? n_new - p0 : kPiece;
        ccnt[tid] = 0u;
        __syncthreads();
        uint32_t ek[kPer], eg[kPer], ec[kPer], es[kPer];
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            const uint32_t i = tid + kTqThreads * j;
            ec[j] = 0xffffffffu;
            if (i < m) {
                const uint64_t pl = p0 == 0 ? pl0[j] : rb.payload[lo + p0 + i];
                uint32_t k2, gi;
                decode(pl, k2, gi);
                ek[j] = (k2 << 1) | (uint32_t)(pl & 1u);
                eg[j] = gi;
                ec[j] = (k2 / g.R / 2) * CR + (k2 % g.R) / 2;
                es[j] = atomicAdd(&ccnt[ec[j]], 1u);
            }
        }
        __syncthreads();
        const uint32_t nk = ccnt[tid];
        const uint32_t incl = wave_incl_scan(nk, lane);
        if (lane == 63) wtot[wv] = incl;
        __syncthreads();
        uint32_t b0 = incl - nk;
        for (uint32_t w = 0; w < wv; ++w) b0 += wtot[w];
        cstart[tid] = b0;
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            if (ec[j] != 0xffffffffu) {
                const uint32_t pos = cstart[ec[j]] + es[j];
                keys[pos] = ek[j];
                gis[pos] = eg[j];
            }
        }
        __syncthreads();
        if (has && nk) {
            // order the bucket by index: insertion sort, close to linear as
            // the scatter leaves it nearly ordered
            for (uint32_t a = 1; a < nk; ++a) {
                const uint32_t kg = gis[b0 + a], kk = keys[b0 + a];
                const uint64_t gv = global_of(kg);
                uint32_t b = a;
                while (b > 0 && global_of(gis[b0 + b - 1]) > gv) {
                    gis[b0 + b] = gis[b0 + b - 1];
                    keys[b0 + b] = keys[b0 + b - 1];
                    --b;
                }
                gis[b0 + b] = kg;
                keys[b0 + b] = kk;
            }
            for (uint32_t e = 0; e < nk; ++e) {
                const uint32_t kp = keys[b0 + e];
                const uint32_t pk = kp >> 1;
                const int qq = (int)((pk & 1u) | (((pk / g.R) & 1u) << 1));
                const float p = (kp & 1u) ? 1.f : -1.f;
                const int64_t ge = (int64_t)global_of(gis[b0 + e]);
                // fixed register indices: a run-time index would move the
                // arrays to scratch
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    if (z != qq) continue;
                    pb[z] = fmaf(coef.alpha, pb[z], coef.one_m_alpha * p);
                    l[z] = fmaf(coef.beta, l[z], c[z] * (p - pb[z]));
                    ++got[z];
                    last[z] = ge;
                }
            }
        }
        __syncthreads();   // the next piece reuses the buckets
    }

    bool b_any = false, a_any = false, p_any = false;
    bool stale[4];
    uint32_t my_n = 0, dP = 0;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const bool act = was[qq] || got[qq] > 0u;
        // a pixel goes stale when its newest event leaves: its last index
        // is below the new front while it was active
        stale[qq] = in[qq] && act && last[qq] < (int64_t)f_new;
        b_any |= was[qq];
        a_any |= act;
        p_any |= act && !stale[qq];
        dP += (!was[qq] && act) ? 1u : 0u;
        my_n += stale[qq] ? 1u : 0u;
    }
    // places in the tile's list: a scan over the wave, one LDS atomic per wave
    const uint32_t incl = wave_incl_scan(my_n, lane);
    uint32_t wbase = 0;
    if (lane == 63 && incl) wbase = atomicAdd(&sh_nstale, incl);
    wbase = __shfl(wbase, 63, 64);
    uint32_t at = wbase + incl - my_n;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
        if (stale[qq]) my_stale[at++] = (uint32_t)gp_of(qq);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        if (tch[qq]) {
            PixL* pl = s.px + gp_of(qq);
            if (got[qq]) {   // Lb stays
                pl->L = l[qq];
                pl->last = last[qq];
            }
            PixP w;
            w.pbar = pb[qq];
            w.cnt = cnt[qq] + got[qq] - popc[lk_of(qq)];
            w.tot = tot[qq] + got[qq];
            s.pp[gp_of(qq)] = w;
        }
    }
    const uint32_t dT = wave_sum((has && !b_any && a_any) ? 1u : 0u);
    const uint32_t n_gone = wave_sum((has && a_any && !p_any) ? 1u : 0u);
    dP = wave_sum(dP);
    if (lane == 0) {
        if (dP) atomicAdd(&sh_red[0], dP);
        if (dT) atomicAdd(&sh_red[1], dT);
        if (n_gone) atomicAdd(&sh_red[2], n_gone);
    }
    __syncthreads();
    if (tid == 0) {
        const uint32_t n_stale = sh_nstale;
        TQTile o = tl;
        o.head = head1;
        o.tail = tail;
        o.P = tl.P + sh_red[0] - n_stale;
        o.T = tl.T + sh_red[1] - sh_red[2];
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
        nstale[t] = n_stale;
        if (n_stale) atomicAdd(&pkt_scratch->part[0][0], n_stale);
    }
}

// The one-time blur of every pixel listed by the step (3x3 binomial,
// clamp-to-edge, fixed order), each neighbour taken as Lb when it was stale
// before the step (its newest event below its tile's old front), else L.
// One thread also stores the step's scalars: newest index, step count,
// stale pixels.
__global__ __launch_bounds__(256) void k_tq_blur(State s, TQGeom g, const uint64_t* __restrict__ front,
                                                 uint32_t n_tiles, const uint32_t* __restrict__ stale_list,
                                                 const uint32_t* __restrict__ nstale,
                                                 StepScratch* __restrict__ scratch,
                                                 const int64_t* __restrict__ chunk_k, TQStep st)
{
    const uint64_t* front_old = front + (size_t)st.parity * n_tiles;
    const uint32_t n = scratch[st.pkt].status ? 0u : scratch[st.pkt].part[0][0];
    // a workgroup per tile, over the tile's own list
    const uint32_t t = blockIdx.x;
    const uint32_t nt = nstale[t];
    const uint32_t* list = stale_list + (size_t)t * g.R * g.R;
    for (uint32_t i = threadIdx.x; i < nt; i += 256) {
        const uint32_t j = list[i];
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
    const uint64_t* f_old = c->tq_front + (size_t)c->tq_parity * n;
    uint64_t* f_new = c->tq_front + (size_t)(c->tq_parity ^ 1) * n;
    const uint32_t* cnt_lo = c->rb.cnt + (size_t)c0 * n;
    const uint32_t* cnt_hi = c1 < n_chunks ? c->rb.cnt + (size_t)c1 * n : c->rb.total;
    hipLaunchKernelGGL(k_tq_step, dim3(n), dim3(kTqThreads), 0, c->st, f_old, c->scratch + pkt,
                       c->tq_tiles, (const int64_t*)c->rb.chunk_k + c1,
                       (const uint64_t*)c->rb.base, cnt_lo, cnt_hi, f_new, c->s, g, c->tq_ring,
                       c->tq_cap - 1, c->tq_stale, c->tq_nstale, c->rb, st, c->tq_age, c->coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tq_blur, dim3(n), dim3(256), 0, c->st, c->s, g,
                       (const uint64_t*)c->tq_front, n, (const uint32_t*)c->tq_stale,
                       (const uint32_t*)c->tq_nstale, c->scratch, (const int64_t*)c->rb.chunk_k, st);
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
