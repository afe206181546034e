// HIP kernels of libfibar for gfx950 (MI355X).
//
// Per pushed packet the work splits into a part that does not depend on the
// reconstruction state (grouping the packet's events by pixel and composing
// each pixel's temporal-filter updates) and an in-order part (applying the
// compositions to the state, moving the active-event window, detecting and
// blurring stale pixels).  The first part runs for many packets in one bulk
// launch (k_sort_compose, one 1024-thread workgroup per <=16384-event chunk);
// the second runs packet by packet (k_apply, then k_pop_blur, whose extra
// workgroups also write a readout that directly follows the packet).
//
// Blurred values of stale pixels live in a second image Lb (stored next to
// L and the last-event index, px[i] = (L, Lb, last)): a pixel's current
// brightness is Lb[i] when it is stale (its newest event has left the
// window, last[i] < h) and L[i] otherwise.  The pop kernel of a step writes
// only Lb of the pixels that go stale in that step and reads neighbours with
// the window head h of the previous step, so every blur of the step sees the
// pre-blur image (the blurs of one step are simultaneous) without a separate
// write pass.
//
// Paper references: temporal filter Eq. (6), (7), (10); active event queue
// and its regulation Eq. (19), (20) (Method, "Spatial filtering"); one-time
// 3x3 Gaussian blur of stale pixels (same section).
#include "fibar_step.h"

namespace fibar {
namespace {

using namespace tile;
using namespace step;


// ---------------------------------------------------------------------------
// Bulk kernel: validate, stable LDS radix sort by pixel, segmented scan of
// the per-event affine maps.  One workgroup per chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_sort_compose(
    const ChunkDesc* __restrict__ chunks, SegRec* __restrict__ seg, uint32_t* __restrict__ seg_count,
    StepScratch* __restrict__ scratch, uint32_t W, uint32_t H, int key_bits, Coef coef,
    const float* __restrict__ gain)
{
    __shared__ uint32_t keypol[kChunk];                 // (tile-major key << 1) | polarity
    __shared__ __align__(16) uint16_t idxA[kChunk];     // permutation ping
    __shared__ __align__(16) uint16_t idxB[kChunk];     // permutation pong
    __shared__ uint64_t scan4[kWaves + 1][4];
    __shared__ SegPair scanp[kWaves];
    __shared__ uint32_t scan1[kWaves + 1];
    __shared__ uint32_t bad_sh;

    const ChunkDesc cd = global_chunk(chunks[blockIdx.x]);
    const uint32_t cn = cd.n;
    const int tid = threadIdx.x;
    if (tid == 0) bad_sh = 0u;
    __syncthreads();

    // key: 2x2 tile index, then the pixel's position in its tile, so that a
    // tile's pixels are consecutive after the sort
    const uint32_t TW = (W + 1) >> 1;
    uint32_t bad = 0u;
    for (uint32_t e = tid; e < cn; e += kSortThreads) {
        const uint32_t x = cd.x[e], y = cd.y[e], p = cd.p[e];
        const bool inr = x < W && y < H;
        bad |= inr ? 0u : 1u;
        bad |= p > 1u ? 2u : 0u;
        const uint32_t key = inr ? ((((y >> 1) * TW + (x >> 1)) << 2) | ((y & 1u) << 1) | (x & 1u))
                                 : 0u;
        keypol[e] = (key << 1) | (p & 1u);
        idxA[e] = (uint16_t)e;
    }
    if (bad) atomicOr(&bad_sh, bad);
    __syncthreads();
    if (tid == 0 && bad_sh) atomicOr(&scratch[cd.pkt].status, bad_sh);

    const uint16_t* sorted = tile_sort(keypol, idxA, idxB, cn, key_bits, scan4);
    SegRec* out = seg + (size_t)blockIdx.x * kChunk;
    const uint32_t total = tile_compose(keypol, sorted, cn, coef, scanp, scan1,
        [&](uint32_t key, const Aff& acc, uint32_t oid, uint32_t rank) {
            const uint32_t t = key >> 2, ty = t / TW, tx = t - ty * TW;
            SegRec r;
            r.pix = (2 * ty + ((key >> 1) & 1u)) * W + 2 * tx + (key & 1u);
            r.n_last = (acc.n << 16) | oid;
            r.a = acc.a;
            r.g = acc.g;
            r.b = acc.b;
            r.u1 = acc.u1;
            r.u2 = acc.u2;
            r.key = key;
            if (gain) {
                // every event map of the pixel has its increment scaled by
                // the same C'_i, and so has their composition: the pbar
                // column of the L row and the L offset
                const float c = gain[r.pix];
                r.g *= c;
                r.u2 *= c;
            }
            out[rank] = r;
        });
    if (tid == 0) seg_count[blockIdx.x] = total;
}

// ---------------------------------------------------------------------------
// In-order kernels (one stream)
// ---------------------------------------------------------------------------

// Apply one chunk's compositions to the state; push the chunk's events to
// the back of the window (spatial filter); count activations.  Workgroup 0
// only commits the previous step's scalars (sc_in -> sc_out).
//
// The values the first loads need lead the argument list, so that they
// arrive in preloaded scalar registers; nothing before the record loads
// waits for another argument (the workgroup size is a constant and the
// commit workgroup is found without the grid size).  n_prev holds the
// chunk's event count and, in bit 31, whether a step is pending; a pending
// step's scratch is the one before this step's.
constexpr uint32_t kPendingBit = 1u << 31;

__global__ __launch_bounds__(kApplyBlock) void k_apply(
    const SegRec* __restrict__ seg, const uint32_t* __restrict__ seg_count, StepScratch* step,
    const DevScalars* sc_in, const uint16_t* ex, const uint16_t* ey, uint32_t n_prev, State s,
    uint32_t chunk_offset, uint32_t prev_events, DevScalars* sc_out, int spatial)
{
    const StepScratch* prev = (n_prev & kPendingBit) ? step - 1 : nullptr;
    const uint32_t n = n_prev & ~kPendingBit;
    if (blockIdx.x == 0) {
        if (prev && sc_out && threadIdx.x < 64) {
            const DevScalars r = commit_by_wave(sc_in, prev, prev_events, s, spatial);
            if (threadIdx.x == 0) store_commit(s, sc_out, r, prev_events);
        }
        return;
    }
    // every load that needs only the arguments is issued before any is used
    const uint32_t i = (blockIdx.x - 1) * kApplyBlock + threadIdx.x;
    ChunkDesc cd;
    cd.x = ex;
    cd.y = ey;
    cd.n = n;
    const Group g = load_group(cd, seg, i);
    uint32_t status = step->status;
    uint32_t nseg = *seg_count;
    HeadIn hin = load_head(sc_in, prev);
    FIBAR_ISSUE_FENCE();
    const TileIn ti = load_tile(s, g, i);
    scalars_after_loads(hin, status, nseg);
    int64_t k0;
    uint64_t h0;
    head_after(hin, prev_events, spatial, &k0, &h0);
    const uint64_t first = (uint64_t)(k0 + 1) + chunk_offset;
    uint32_t dP = 0u, dT = 0u;
    apply_tile(s, g, ti, cd.n, nseg, status != 0, i, first, h0, spatial, dP, dT);
    if (spatial) add_counts(step, false, chunk_offset + i, dP, dT);
}

// Move the window head by the target of the previous step (Eq. (20)),
// detect pixels whose last queued event leaves the window, and write their
// blurred values to Lb.  `sc` holds the scalars after the previous step.
// Leading arguments as in k_apply.  The pops take pop_threads(pkt_events)
// threads, the first workgroups; workgroups past them write the readout
// that directly follows the step, if there is one (`ro`), kRoPix pixels per
// thread.
constexpr int kRoPix = 1;   // 2 and 4 (fewer workgroups) were slower

__global__ __launch_bounds__(kPopBlock) void k_pop_blur(const DevScalars* sc, StepScratch* step,
                                                        const uint32_t* ring, uint64_t ring_mask,
                                                        PixL* px, uint32_t W, uint32_t H,
                                                        uint32_t pkt_events, State s, PopReadout ro)
{
    s.ring = const_cast<uint32_t*>(ring);
    s.ring_mask = ring_mask;
    s.px = px;
    s.W = W;
    s.H = H;
    // from preloaded arguments only: a readout workgroup knows it is one
    // without waiting for any load
    const uint32_t threads = pop_threads(pkt_events);
    const uint32_t pop_blocks = threads / kPopBlock;
    if (blockIdx.x >= pop_blocks) {
        // the readout of the state after the step; what it reads is not
        // written by the pops (see readout_pixel_after_pops).  The first
        // pass's pixels are loaded before the window scalars.
        const uint64_t npx = (uint64_t)W * H;
        const uint32_t rb = blockIdx.x - pop_blocks, nrb = gridDim.x - pop_blocks;
        const uint64_t span = (uint64_t)nrb * kPopBlock * kRoPix;
        const uint64_t first = (uint64_t)rb * kPopBlock * kRoPix + threadIdx.x;
        PixL v[kRoPix];
#pragma unroll
        for (int q = 0; q < kRoPix; ++q) {
            const uint64_t i = first + (uint64_t)q * kPopBlock;
            v[q] = px[i < npx ? i : 0];
        }
        FIBAR_ISSUE_FENCE();
        const uint32_t status = step->status;
        const DevScalars c = *sc;
        uint64_t h_old, h_new;
        pop_bounds(c, pkt_events, &h_old, &h_new);
        if (status) h_new = h_old;   // a rejected packet pops nothing
        const int64_t k = status ? c.k : c.k + (int64_t)pkt_events;
        for (uint64_t base = first; base < npx; base += span) {
            if (base != first) {
#pragma unroll
                for (int q = 0; q < kRoPix; ++q) {
                    const uint64_t i = base + (uint64_t)q * kPopBlock;
                    v[q] = px[i < npx ? i : 0];
                }
            }
#pragma unroll
            for (int q = 0; q < kRoPix; ++q) {
                const uint64_t i = base + (uint64_t)q * kPopBlock;
                if (i < npx)
                    readout_pixel_after_pops(s, k, h_old, h_new, i, v[q], ro.L, ro.pbar,
                                             ro.stale, ro.last, ro.log_age, ro.tot);
            }
        }
        if (ro.tcnt) {
            const uint64_t nt = (uint64_t)s.TW * ((H + 1) / 2);
            const uint64_t tstride = (uint64_t)nrb * kPopBlock;
            for (uint64_t t = (uint64_t)rb * kPopBlock + threadIdx.x; t < nt; t += tstride)
                ro.tcnt[t] = tile_active_pixels(s, t, h_new);
        }
        return;
    }
    // the status and the scalars are loaded together (a select, not a branch)
    const uint32_t status = step->status;
    const DevScalars c = *sc;
    uint64_t h_old, h_new;
    pop_bounds(c, pkt_events, &h_old, &h_new);
    if (status) h_new = h_old;   // a rejected packet pops nothing
    uint32_t dP = 0u, dT = 0u;
    pop_range(s, h_old + blockIdx.x * kPopBlock + threadIdx.x, h_new, threads, h_old, dP, dT);
    add_counts(step, true, blockIdx.x * kPopBlock + threadIdx.x, dP, dT);
}

// Initial per-pixel state.
__global__ __launch_bounds__(256) void k_init_state(State s)
{
    const uint64_t npx = (uint64_t)s.W * s.H;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += stride) {
        PixL v;
        v.L = 0.f;
        v.Lb = 0.f;
        v.last = -1;
        s.px[i] = v;
        PixP p;
        p.pbar = 0.f;
        p.cnt = 0u;
        p.tot = 0u;
        s.pp[i] = p;
    }
}

// Commit a pending step into the other slot (one wave).
__global__ __launch_bounds__(64) void k_commit(State s, const StepScratch* prev,
                                                uint32_t prev_events, int slot_in, int slot_out,
                                                int spatial)
{
    const DevScalars r = commit_by_wave(s.sc + slot_in, prev, prev_events, s, spatial);
    if (threadIdx.x == 0) store_commit(s, s.sc + slot_out, r, prev_events);
}

__global__ __launch_bounds__(256) void k_readout(State s, int spatial, const StepScratch* prev,
                                                 uint32_t prev_events, int slot, float* L,
                                                 float* pbar, uint8_t* stale, uint32_t* cnt,
                                                 int64_t* last, float* log_age, uint32_t* tcnt,
                                                 uint64_t* tot)
{
    int64_t k;
    uint64_t hu;
    current_head(s, slot, prev, prev_events, spatial, &k, &hu);
    const uint64_t npx = (uint64_t)s.W * s.H;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += stride)
        readout_pixel(s, spatial, k, (int64_t)hu, i, L, pbar, stale, cnt, last, log_age, tot);
    if (spatial && tcnt) {
        const uint64_t nt = (uint64_t)s.TW * ((s.H + 1) / 2);
        for (uint64_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride)
            tcnt[t] = tile_active_pixels(s, t, (int64_t)hu);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sort_compose(const ChunkDesc* d_chunks, uint32_t n_chunks, SegRec* seg,
                               uint32_t* seg_count, StepScratch* scratch, uint32_t W,
                               uint32_t H, int key_bits, Coef coef, const float* gain,
                               hipStream_t st, const LaunchTiming& tm)
{
    if (n_chunks == 0) return hipSuccess;
    return launch_timed(k_sort_compose, dim3(n_chunks), dim3(kSortThreads), st, tm.start, tm.stop,
                        d_chunks, seg, seg_count, scratch, W, H, key_bits, coef, gain);
}

hipError_t launch_apply(const State& s, const ChunkDesc* d_chunk, const SegRec* seg,
                        const uint32_t* seg_count, uint32_t chunk_events, uint32_t chunk_offset,
                        StepScratch* step, const StepScratch* prev, uint32_t prev_events,
                        int slot_in, int slot_out, int spatial, hipStream_t st,
                        const LaunchTiming& tm)
{
    // one extra workgroup (the first) commits the previous step's scalars
    if (prev && prev != step - 1) return hipErrorInvalidValue;   // scratch layout
    if (chunk_events == 0 || chunk_events > (uint32_t)kChunk) return hipErrorInvalidValue;
    const uint32_t blocks = (chunk_events + kApplyBlock - 1) / kApplyBlock + 1;
    DevScalars* sc_out = slot_out >= 0 ? s.sc + slot_out : nullptr;
    return launch_timed(k_apply, dim3(blocks), dim3(kApplyBlock), st, tm.start, tm.stop, seg,
                        seg_count, step, (const DevScalars*)(s.sc + slot_in), d_chunk->x,
                        d_chunk->y, chunk_events | (prev ? kPendingBit : 0u), s, chunk_offset,
                        prev_events, sc_out, spatial);
}

hipError_t launch_pop_blur(const State& s, uint32_t pkt_events, StepScratch* step, int slot,
                           const PopReadout* ro, hipStream_t st, const LaunchTiming& tm)
{
    const uint32_t threads = pop_threads(pkt_events);
    if (threads == 0 || (ro && !ro->L)) return hipErrorInvalidValue;
    const uint32_t pop_blocks = threads / kPopBlock;   // the kernel derives the same
    uint32_t ro_blocks = 0;
    PopReadout r{};
    if (ro) {
        // kRoPix pixels per thread; the pop workgroups come first
        const uint64_t per = (uint64_t)kPopBlock * kRoPix;
        const uint64_t b = ((uint64_t)s.W * s.H + per - 1) / per;
        ro_blocks = (uint32_t)(b < kReadoutMaxBlocks ? (b > 0 ? b : 1) : kReadoutMaxBlocks);
        r = *ro;
    }
    return launch_timed(k_pop_blur, dim3(pop_blocks + ro_blocks), dim3(kPopBlock), st, tm.start,
                        tm.stop, (const DevScalars*)(s.sc + slot), step, (const uint32_t*)s.ring,
                        s.ring_mask, s.px, s.W, s.H, pkt_events, s, r);
}

hipError_t launch_init_state(const State& s, hipStream_t st)
{
    const uint64_t npx = (uint64_t)s.W * s.H;
    uint64_t blocks = (npx + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_state, dim3((uint32_t)blocks), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_commit(const State& s, const StepScratch* prev, uint32_t prev_events,
                         int slot_in, int slot_out, int spatial, hipStream_t st)
{
    return launch_timed(k_commit, dim3(1), dim3(64), st, nullptr, nullptr, s, prev, prev_events,
                        slot_in, slot_out, spatial);
}

hipError_t launch_readout(const State& s, int spatial, const StepScratch* prev,
                          uint32_t prev_events, int slot, float* L, float* pbar, uint8_t* stale,
                          uint32_t* cnt, int64_t* last, float* log_age, uint32_t* tcnt,
                          uint64_t* tot, hipStream_t st, const LaunchTiming& tm)
{
    const uint64_t npx = (uint64_t)s.W * s.H;
    uint64_t blocks = (npx + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    return launch_timed(k_readout, dim3((uint32_t)blocks), dim3(256), st, tm.start, tm.stop, s,
                        spatial, prev, prev_events, slot, L, pbar, stale, cnt, last, log_age,
                        tcnt, tot);
}

}  // namespace fibar
