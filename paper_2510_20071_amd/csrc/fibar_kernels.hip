// HIP kernels of libfibar for gfx950 (MI355X).
//
// Per pushed packet the work splits into a part that does not depend on the
// reconstruction state (grouping the packet's events by pixel and composing
// each pixel's temporal-filter updates) and an in-order part (applying the
// compositions to the state, moving the active-event window, detecting and
// blurring stale pixels).  The first part runs for many packets in one bulk
// launch (k_sort_compose, one 1024-thread workgroup per <=16384-event chunk);
// the second runs packet by packet (k_step: the pops of one packet together
// with the pushes of the next, and a readout between them if there is one).
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
    StepScratch* __restrict__ scratch, uint32_t W, uint32_t H, int key_bits, Coef coef)
{
    __shared__ uint32_t keypol[kChunk];                 // (tile-major key << 1) | polarity
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
            out[rank] = r;
        });
    if (tid == 0) seg_count[blockIdx.x] = total;
}

// ---------------------------------------------------------------------------
// In-order kernel (one stream): one launch per packet.
//
// A launch may commit the scalars of a step, pop the window of the step
// after it, and apply one chunk of the packet after that, all at once: the
// pops of step b and the pushes of packet b + 1 need the same committed
// scalars, and neither reads a value the other writes, except through two
// hand-offs.  (1) The tiles of packet b + 1 (tagged with its sequence number
// by the launch before) are left by the pops to the packet's apply, which
// sees their records before rewriting them.  (2) A record rewritten by the
// apply keeps, in Lb, the value the blurs of step b read (preblur_value).
// The pops read their pixels from a staging list that the launch before
// wrote at a fixed place, so that their neighbourhoods load in the second
// memory round trip.  Workgroups: pops, then apply, then readout.
// ---------------------------------------------------------------------------
constexpr uint32_t kPendingBit = 1u << 31;   // n_pop: a step is committed here
constexpr uint32_t kHeadBit = 1u << 30;      // n_pop: the head step is given
constexpr uint32_t kPopsBit = 1u << 29;      // n_pop: the head step is popped here
constexpr uint32_t kCountMask = kPopsBit - 1u;
constexpr uint32_t kFusedFlag = 1u;
constexpr uint32_t kReadoutFlag = 2u;
constexpr uint32_t kSpatialFlag = 4u;

__device__ StepScratch no_step;              // read in place of an absent step

__global__ __launch_bounds__(kPopBlock) void k_step(const SegRec* __restrict__ seg,
                                                    const uint32_t* __restrict__ stage_in,
                                                    const DevScalars* sc_in, StepScratch* sp_head,
                                                    const uint64_t* __restrict__ ttag_in,
                                                    const uint16_t* ex, const uint16_t* ey,
                                                    uint32_t n_pop, uint32_t n_app, State s,
                                                    StepAux a)
{
    const uint32_t n_head = n_pop & kCountMask;
    const bool pending = (n_pop & kPendingBit) != 0u, has_head = (n_pop & kHeadBit) != 0u;
    const bool pops = (n_pop & kPopsBit) != 0u;
    const bool fused = (a.flags & kFusedFlag) != 0u;
    const int spatial = (a.flags & kSpatialFlag) != 0u ? 1 : 0;
    // workgroup roles, from preloaded arguments only
    const uint32_t pop_blocks = pops ? pop_threads(n_head) / kPopBlock : 0u;
    const uint32_t app_blocks = (n_app + kPopBlock - 1) / kPopBlock;
    const uint32_t blk = blockIdx.x, tid = threadIdx.x;
    const int role = blk < pop_blocks ? 0 : blk < pop_blocks + app_blocks ? 1 : 2;
    const StepScratch* hd = has_head ? sp_head : &no_step;
    const StepScratch* cm = pending ? a.sp_commit : &no_step;

    // first round trip: the role's own loads, then the scalars and the
    // commit's counts
    uint32_t sp_pix = 0u;
    Group g;
    uint32_t nseg = 0u, st_app = 0u, next_key = 0u, next_n = 0u, st_next = 1u;
    PixL rv;
    uint64_t rtag = 0u;
    const uint32_t gi = (role == 0 ? blk : role == 1 ? blk - pop_blocks
                                                     : blk - pop_blocks - app_blocks) *
                            kPopBlock + tid;
    const uint64_t npx = (uint64_t)s.W * s.H;
    if (role == 0) {
        if (stage_in) sp_pix = stage_in[gi < kStage ? gi : 0u];
    } else if (role == 1) {
        ChunkDesc cd;
        cd.x = ex;
        cd.y = ey;
        cd.n = n_app;
        g = load_group(cd, seg, gi);
        nseg = *a.seg_count;
        st_app = a.sp_app->status;
        if (a.next_seg) {
            next_key = a.next_seg[gi < kChunk ? gi : 0u].key;
            next_n = *a.next_count;
            st_next = a.sp_next->status;
        }
    } else {
        const uint64_t i = gi < npx ? gi : 0u;
        rv = load_rec(&s.px[i]);
        if (fused) {
            const uint32_t y = (uint32_t)(i / s.W), x = (uint32_t)(i - (uint64_t)y * s.W);
            rtag = ttag_in[(y >> 1) * s.TW + (x >> 1)];
        }
    }
    const DevScalars cin = *sc_in;
    const uint32_t st_head = hd->status, st_commit = cm->status;
    FIBAR_ISSUE_FENCE();
    const StepCounts cn = pending && spatial ? gather_counts(cm) : StepCounts{0u, 0u, 0u, 0u};
    const DevScalars c = pending ? commit_step(cin, st_commit, a.n_commit, s, spatial, cn) : cin;
    if (blk == 0 && tid == 0 && pending) store_commit(s, a.sc_out, c, a.n_commit);
    // the window around the head step
    StepWin w;
    w.h_old = c.h;
    int64_t k_end = c.k;
    uint64_t h_new = c.h;
    if (has_head) step_head(c, st_head, n_head, spatial, &k_end, &h_new);
    w.h_new = h_new;
    w.k_prev = k_end;
    w.fused = fused;
    w.spatial = spatial != 0;
    w.kpost = fused ? k_end + 1 : kNoPost;
    w.first = (uint64_t)(k_end + 1) + a.chunk_offset;
    const uint64_t seq = fused ? a.seq : ~0ull;

    if (role == 0) {
        // pop j = h_old + gi (and, past the first pass, every pop_threads-th
        // after it, with pixels from the ring)
        const uint32_t G = pop_blocks * kPopBlock;
        const uint64_t j = w.h_old + gi;
        // without a staging list (the first pops of a batch) the pixel comes
        // from the window ring
        if (!stage_in) sp_pix = s.ring[j & s.ring_mask];
        const uint32_t pix = sp_pix < npx ? sp_pix : 0u;
        PixL nb[3][3];
        load_pop(s, pix, nb);
        uint64_t tag = 0u;
        if (fused) tag = ttag_in[tile_of(s, pix)];
        // the next pop step's staging list: window events that are pushed
        // already (the apply below stages the packet it pushes)
        for (uint32_t k = gi; k < a.copy_count; k += G) {
            const uint64_t jj = h_new + k;
            if ((int64_t)jj <= k_end) a.stage_out[k] = s.ring[jj & s.ring_mask];
        }
        uint32_t dP = 0u, dT = 0u;
        if (j < h_new) {
            if (gi < kStage || !stage_in) {
                step_pop(s, j, pix, nb, tag, seq, w.h_old, w.kpost, dP, dT);
            } else {
                const uint32_t p2 = s.ring[j & s.ring_mask];
                PixL nb2[3][3];
                load_pop(s, p2, nb2);
                const uint64_t tag2 = fused ? ttag_in[tile_of(s, p2)] : 0u;
                step_pop(s, j, p2, nb2, tag2, seq, w.h_old, w.kpost, dP, dT);
            }
        }
        add_counts(sp_head, kCountPop, gi, dP, dT);
        // pops past the first pass; their counts are summed over the whole
        // wave afterwards (a wave sum needs every lane)
        uint32_t eP = 0u, eT = 0u;
        for (uint64_t jj = j + G; jj < h_new; jj += G) {
            const uint32_t p2 = s.ring[jj & s.ring_mask];
            PixL nb2[3][3];
            load_pop(s, p2, nb2);
            const uint64_t tag2 = fused ? ttag_in[tile_of(s, p2)] : 0u;
            step_pop(s, jj, p2, nb2, tag2, seq, w.h_old, w.kpost, eP, eT);
        }
        add_overflow_counts(sp_head, kCountPop, gi, eP, eT);
        return;
    }
    if (role == 1) {
        const TileIn ti = load_tile(s, g, gi);
        const bool rejected = st_app != 0u;
        uint32_t act = 0u, tact = 0u, hst = 0u, hoff = 0u;
        const PopReadout ro = a.ro;
        const bool want_ro = (a.flags & kReadoutFlag) && fused;
        apply_tile_step(s, g, ti, n_app, nseg, rejected, gi, w, act, tact, hst, hoff, ro,
                        want_ro);
        // stage the pushed event for the next pop step, tag the next packet's
        // tiles for the launch that pops this one
        if (!rejected && gi < n_app) {
            const uint64_t rel = w.first + gi - h_new;
            if (rel < a.copy_count) a.stage_out[rel] = g.ey * s.W + g.ex;
        }
        if (a.next_seg && st_next == 0u) {
            const uint32_t G = app_blocks * kPopBlock;
            for (uint32_t k = gi; k < next_n; k += G) {
                const uint32_t key = k == gi ? next_key : a.next_seg[k].key;
                a.ttag_out[key >> 2] = a.seq + 1u;
            }
        }
        add_counts(a.sp_app, kCountApply, a.chunk_offset + gi, act, tact);
        if (fused) add_counts(sp_head, kCountHead, gi, hst, hoff);
        return;
    }
    // readout of the state after the head step's pops (workgroups past the
    // pops and the apply, one pixel per thread)
    const PopReadout ro = a.ro;
    const uint32_t nrb = gridDim.x - pop_blocks - app_blocks;
    const uint64_t span = (uint64_t)nrb * kPopBlock;
    for (uint64_t i = gi; i < npx; i += span) {
        if (i != gi) {
            rv = load_rec(&s.px[i]);
            if (fused) {
                const uint32_t y = (uint32_t)(i / s.W), x = (uint32_t)(i - (uint64_t)y * s.W);
                rtag = ttag_in[(y >> 1) * s.TW + (x >> 1)];
            }
        }
        if (fused && rtag == seq) continue;   // written by the tile's head
        readout_pixel_after_pops(s, k_end, w.h_old, h_new, i, rv, ro.L, ro.pbar, ro.stale,
                                 ro.last, ro.log_age, ro.tot, w.kpost);
    }
    if (ro.tcnt) {
        const uint64_t nt = (uint64_t)s.TW * ((s.H + 1) / 2);
        for (uint64_t t = gi; t < nt; t += span)
            if (!fused || ttag_in[t] != seq) ro.tcnt[t] = tile_active_pixels(s, t, h_new);
    }
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
        p.pad = 0u;
        p.tot = 0u;
        s.pp[i] = p;
        s.cnt[i] = 0u;
    }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
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
                               uint32_t H, int key_bits, Coef coef, hipStream_t st,
                               const LaunchTiming& tm)
{
    if (n_chunks == 0) return hipSuccess;
    return launch_timed(k_sort_compose, dim3(n_chunks), dim3(kSortThreads), st, tm.start, tm.stop,
                        d_chunks, seg, seg_count, scratch, W, H, key_bits, coef);
}

hipError_t launch_step(const State& s, const StepLaunch& L, hipStream_t st,
                       const LaunchTiming& tm)
{
    const bool pops = L.pops && L.head && L.spatial;
    if (L.n_app > (uint32_t)kChunk || (L.n_app && (!L.app || !L.seg || !L.seg_count))) return hipErrorInvalidValue;
    if (L.fused && !(pops && L.n_app && L.ttag_in)) return hipErrorInvalidValue;
    if (L.commit && (L.slot_out < 0 || L.slot_out > 1)) return hipErrorInvalidValue;
    if (L.n_head > kCountMask || L.n_commit > kCountMask) return hipErrorInvalidValue;
    if (L.ro && (!L.ro->L || !pops)) return hipErrorInvalidValue;
    if (L.copy_count > kStage || (L.copy_count && !L.stage_out)) return hipErrorInvalidValue;
    if (L.next_seg && !(L.next_count && L.next && L.ttag_out)) return hipErrorInvalidValue;
    const uint32_t pop_blocks = pops ? pop_threads(L.n_head) / kPopBlock : 0u;
    const uint32_t app_blocks = (L.n_app + kPopBlock - 1) / kPopBlock;
    uint32_t ro_blocks = 0;
    StepAux a{};
    if (L.ro) {
        const uint64_t b = ((uint64_t)s.W * s.H + kPopBlock - 1) / kPopBlock;
        ro_blocks = (uint32_t)(b < kReadoutMaxBlocks ? (b > 0 ? b : 1) : kReadoutMaxBlocks);
        a.ro = *L.ro;
        a.flags |= kReadoutFlag;
    }
    const uint32_t blocks = pop_blocks + app_blocks + ro_blocks;
    if (blocks == 0) return hipSuccess;
    uint32_t n_pop = L.n_head;
    if (L.commit) n_pop |= kPendingBit;
    if (L.head) n_pop |= kHeadBit;
    if (pops) n_pop |= kPopsBit;
    if (L.fused) a.flags |= kFusedFlag;
    if (L.spatial) a.flags |= kSpatialFlag;
    a.sp_commit = L.commit;
    a.sp_app = L.app;
    a.n_commit = L.n_commit;
    a.chunk_offset = L.chunk_offset;
    a.copy_count = L.copy_count;
    a.seg_count = L.seg_count;
    a.sc_out = L.commit ? s.sc + L.slot_out : nullptr;
    a.stage_out = L.stage_out;
    a.ttag_out = L.ttag_out;
    a.next_seg = L.next_seg;
    a.next_count = L.next_count;
    a.sp_next = L.next;
    a.seq = L.seq;
    return launch_timed(k_step, dim3(blocks), dim3(kPopBlock), st, tm.start, tm.stop, L.seg,
                        L.stage_in, (const DevScalars*)(s.sc + L.slot_in), L.head,
                        L.ttag_in, L.ex, L.ey, n_pop, L.n_app, s, a);
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

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, st, p, (uint64_t)n, v);
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
