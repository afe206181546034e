// Host runtime and C ABI of libfibar (see include/fibar.h).
//
// Every public call is turned into a list of operations (pushes and
// readouts) executed in batches:
//   1. one bulk launch groups and composes the events of every packet of the
//      batch (state independent, all packets in parallel);
//   2. the packets are then applied in order: compositions -> state, window
//      pops / stale detection / blur values, blur write; readouts run at
//      their place in the sequence.
// All work is ordered on the context's stream.
#include "fibar.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "fibar_ctx.h"

using namespace fibar;

namespace {

constexpr uint32_t kMaxPacket = 1u << 20;
constexpr uint64_t kMaxKeySpan = 1ull << 31;

// Eq. (17) and Eq. (18), evaluated in double precision.
void filter_coefficients(double t_cut, double* alpha, double* beta)
{
    const double w = 2.0 * M_PI / t_cut;
    *alpha = (1.0 - sin(w)) / cos(w);
    const double a = 2.0 - cos(w);
    *beta = a - sqrt(a * a - 1.0);
}

}  // namespace

namespace {


hipEvent_t pooled_event(fibar_ctx* c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t ev = c->event_pool.back();
        c->event_pool.pop_back();
        return ev;
    }
    // timing only: without the system-scope fence that an event's
    // completion otherwise carries (a write-back of the L2 at the end of
    // the timed kernel, which made it ~1.8 us slower); the times are read
    // after a stream synchronisation
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return ev;
}

// Launch through `fn`; every time_every-th launch of a timed kernel kind
// carries start/stop events on its dispatch.  Launches count under `kind`
// and their times are kept under `store` (a pop launch that also writes a
// readout counts as a pop and is kept apart).  A recorded batch counts from
// its own start, so that batches of the same shape time the same launches
// (and replay the same graph).
template <class F>
hipError_t timed_launch(fibar_ctx* c, int kind, int store, F&& fn)
{
    uint64_t& seq = c->recording ? c->batch_seq[kind] : c->time_seq[kind];
    if (!(c->time_mask & (1u << kind)) || (seq++ % c->time_every) != 0)
        return fn(LaunchTiming());
    LaunchTiming tm;
    tm.start = pooled_event(c);
    tm.stop = pooled_event(c);
    if (!tm.start || !tm.stop) return hipErrorOutOfMemory;
    const hipError_t e = fn(tm);
    c->timed[store].emplace_back(tm.start, tm.stop);
    return e;
}
template <class F>
hipError_t timed_launch(fibar_ctx* c, int kind, F&& fn)
{
    return timed_launch(c, kind, kind, fn);
}

// ---- batch graphs ------------------------------------------------------------

#define HIP_CHECK_RET(expr)                   \
    do {                                      \
        const hipError_t e_ = (expr);         \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

void destroy_graph(BatchGraph* g)
{
    for (int e = 0; e < 2; ++e) {
        if (g->done[e]) {
            (void)hipEventSynchronize(g->done[e]);
            (void)hipEventDestroy(g->done[e]);
        }
        if (g->exec[e]) (void)hipGraphExecDestroy(g->exec[e]);
    }
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

hipKernelNodeParams node_params(RecordedLaunch& L)
{
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(L.func);
    kp.gridDim = L.grid;
    kp.blockDim = L.block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = L.params.data();
    kp.extra = nullptr;
    return kp;
}

// A chain of the recorded launches, instantiated twice.
hipError_t build_graph(std::vector<RecordedLaunch>& ls, BatchGraph* g)
{
    const size_t n = ls.size();
    g->funcs.resize(n);
    g->timed.resize(n);
    g->knode.assign(n, nullptr);
    g->ev_start.assign(n, nullptr);
    g->ev_stop.assign(n, nullptr);
    hipError_t e = hipGraphCreate(&g->graph, 0);
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        RecordedLaunch& L = ls[i];
        g->funcs[i] = L.func;
        g->timed[i] = L.start ? 1 : 0;
        if (L.start) {
            e = hipGraphAddEventRecordNode(&g->ev_start[i], g->graph, prev ? &prev : nullptr,
                                           prev ? 1 : 0, L.start);
            prev = g->ev_start[i];
        }
        const hipKernelNodeParams kp = node_params(L);
        if (e == hipSuccess)
            e = hipGraphAddKernelNode(&g->knode[i], g->graph, prev ? &prev : nullptr,
                                      prev ? 1 : 0, &kp);
        prev = g->knode[i];
        if (e == hipSuccess && L.stop) {
            e = hipGraphAddEventRecordNode(&g->ev_stop[i], g->graph, &prev, 1, L.stop);
            prev = g->ev_stop[i];
        }
    }
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipGraphInstantiate(&g->exec[k], g->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done[k], hipEventDisableTiming);
    }
    g->fresh[0] = true;   // copy 0 runs this batch as instantiated; copy 1 is updated first
    return e;
}

bool same_sequence(const BatchGraph* g, const std::vector<RecordedLaunch>& ls)
{
    if (g->funcs.size() != ls.size()) return false;
    for (size_t i = 0; i < ls.size(); ++i)
        if (g->funcs[i] != ls[i].func || g->timed[i] != (ls[i].start ? 1 : 0)) return false;
    return true;
}

constexpr size_t kMaxGraphs = 8;

// Run the recorded batch: the cached graph of the same kernel sequence with
// this batch's parameters, or a new one.
hipError_t replay_batch(fibar_ctx* c)
{
    std::vector<RecordedLaunch>& ls = c->rec.launches;
    if (ls.empty()) return hipSuccess;
    BatchGraph* g = nullptr;
    for (BatchGraph* b : c->graphs)
        if (same_sequence(b, ls)) {
            g = b;
            break;
        }
    if (!g) {
        if (c->graphs.size() >= kMaxGraphs) {
            size_t lru = 0;
            for (size_t i = 1; i < c->graphs.size(); ++i)
                if (c->graphs[i]->last_use < c->graphs[lru]->last_use) lru = i;
            destroy_graph(c->graphs[lru]);
            c->graphs.erase(c->graphs.begin() + (long)lru);
        }
        g = new BatchGraph();
        const hipError_t e = build_graph(ls, g);
        if (e != hipSuccess) {
            destroy_graph(g);
            return e;
        }
        c->graphs.push_back(g);
    }
    g->last_use = ++c->graph_clock;
    const int k = g->next;
    g->next ^= 1;
    // the copy's previous launch must be over before its parameters change
    if (g->launched[k]) HIP_CHECK_RET(hipEventSynchronize(g->done[k]));
    if (!g->fresh[k]) {
        for (size_t i = 0; i < ls.size(); ++i) {
            const hipKernelNodeParams kp = node_params(ls[i]);
            HIP_CHECK_RET(hipGraphExecKernelNodeSetParams(g->exec[k], g->knode[i], &kp));
            if (ls[i].start) {
                HIP_CHECK_RET(hipGraphExecEventRecordNodeSetEvent(g->exec[k], g->ev_start[i],
                                                                  ls[i].start));
                HIP_CHECK_RET(hipGraphExecEventRecordNodeSetEvent(g->exec[k], g->ev_stop[i],
                                                                  ls[i].stop));
            }
        }
    }
    g->fresh[k] = false;
    HIP_CHECK_RET(hipGraphLaunch(g->exec[k], c->st));
    HIP_CHECK_RET(hipEventRecord(g->done[k], c->st));
    g->launched[k] = true;
    return hipSuccess;
}

// Records the launches of its scope (graph mode) and replays them at finish().
struct BatchRecording {
    fibar_ctx* c;
    bool on;
    BatchRecording(fibar_ctx* ctx, bool enable) : c(ctx), on(enable)
    {
        if (!on) return;
        c->rec.launches.clear();
        for (auto& q : c->batch_seq) q = 0;
        c->recording = true;
        tl_recorder = &c->rec;
    }
    void stop()
    {
        if (!on) return;
        tl_recorder = nullptr;
        c->recording = false;
    }
    hipError_t finish()
    {
        if (!on) return hipSuccess;
        stop();
        const hipError_t e = replay_batch(c);
        c->rec.launches.clear();
        on = false;
        return e;
    }
    ~BatchRecording()
    {
        stop();
        if (c) c->rec.launches.clear();
    }
};

void free_ctx(fibar_ctx* c)
{
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    else (void)hipDeviceSynchronize();
    (void)hipFree(c->s.px);
    (void)hipFree(c->s.pp);
    (void)hipFree(c->s.ring);
    (void)hipFree(c->gain);
    (void)hipFree(c->tq_tiles);
    (void)hipFree(c->tq_front);
    (void)hipFree(c->tq_ring);
    (void)hipFree(c->tq_stale);
    (void)hipFree(c->tq_nstale);
    (void)hipFree(c->s.sc);
    (void)hipFree(c->d_chunks);
    (void)hipFree(c->seg);
    (void)hipFree(c->seg_count);
    (void)hipFree(c->scratch);
    (void)hipFree(c->stg_x);
    (void)hipFree(c->stg_y);
    (void)hipFree(c->stg_p);
    if (c->hs_x) (void)hipHostFree(c->hs_x);
    if (c->hs_y) (void)hipHostFree(c->hs_y);
    if (c->hs_p) (void)hipHostFree(c->hs_p);
    if (c->hs_done) (void)hipEventDestroy(c->hs_done);
    (void)hipFree(c->rb.cnt);
    (void)hipFree(c->rb.base);
    (void)hipFree(c->rb.total);
    (void)hipFree(c->rb.chunk_k);
    (void)hipFree(c->rb.payload);
    // rb.ro and h_ro (blur off) are parts of d_chunks and h_chunks
    if (c->ro_free) (void)hipEventDestroy(c->ro_free);
    if (c->h_chunks) (void)hipHostFree(c->h_chunks);
    if (c->h_sc) (void)hipHostFree(c->h_sc);
    if (c->chunks_free) (void)hipEventDestroy(c->chunks_free);
    for (auto& v : c->timed)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t ev : c->event_pool) (void)hipEventDestroy(ev);
    for (BatchGraph* g : c->graphs) destroy_graph(g);
    delete c;
}

// One operation of an execution list.
struct Op {
    int kind;  // 0 push, 1 readout
    const uint16_t* x;
    const uint16_t* y;
    const uint8_t* p;
    uint32_t n;
    fibar_readout_buf ro;
};

int host_validate(const fibar_ctx* c, const fibar_packet* pk)
{
    for (size_t e = 0; e < pk->n; ++e)
        if (pk->x[e] >= c->W || pk->y[e] >= c->H) return FIBAR_E_RANGE;
    for (size_t e = 0; e < pk->n; ++e)
        if (pk->p[e] > 1) return FIBAR_E_POLARITY;
    return FIBAR_OK;
}

int do_readout_kernel(fibar_ctx* c, const fibar_readout_buf& ro, const StepScratch* pend,
                      uint32_t pend_n)
{
    const int sp = (int)c->prm.spatial_filter;
    const int slot = c->cur_slot;
    if (ro.on_device) {
        if (c->tq)
            return map_err(tq_readout(c, ro.brightness, ro.pbar, ro.stale_mask, ro.active_count,
                                      ro.last_index, ro.log_age, ro.tile_count, ro.total_count));
        HIP_TRY(timed_launch(c, 4, [&](const LaunchTiming& tm) {
            return launch_readout(c->s, sp, pend, pend_n, slot, ro.brightness, ro.pbar,
                                  ro.stale_mask, ro.active_count, ro.last_index, ro.log_age,
                                  ro.tile_count, ro.total_count, c->st, tm);
        }));
        return FIBAR_OK;
    }
    // host outputs: stage on the device, copy back, synchronise
    const size_t npx = c->npx;
    size_t bytes = npx * 4;                       // brightness
    if (ro.pbar) bytes += npx * 4;
    if (ro.stale_mask) bytes += (npx + 255) & ~size_t(255);
    if (ro.active_count) bytes += npx * 4;
    if (ro.last_index) bytes += npx * 8;
    if (ro.log_age) bytes += npx * 4;
    if (ro.tile_count) bytes += c->ntiles * 4;
    if (ro.total_count) bytes += npx * 8;
    bytes += 8 * 256;
    uint8_t* stage = nullptr;
    HIP_TRY(hipMallocAsync((void**)&stage, bytes, c->st));
    uint8_t* cur = stage;
    auto take = [&](size_t n) { uint8_t* r = cur; cur += (n + 255) & ~size_t(255); return r; };
    float* dL = (float*)take(npx * 4);
    float* dP = ro.pbar ? (float*)take(npx * 4) : nullptr;
    uint8_t* dS = ro.stale_mask ? take(npx) : nullptr;
    uint32_t* dC = ro.active_count ? (uint32_t*)take(npx * 4) : nullptr;
    int64_t* dLi = ro.last_index ? (int64_t*)take(npx * 8) : nullptr;
    float* dA = ro.log_age ? (float*)take(npx * 4) : nullptr;
    uint32_t* dT = ro.tile_count ? (uint32_t*)take(c->ntiles * 4) : nullptr;
    uint64_t* dN = ro.total_count ? (uint64_t*)take(npx * 8) : nullptr;
    hipError_t e = c->tq ? tq_readout(c, dL, dP, dS, dC, dLi, dA, dT, dN)
                         : launch_readout(c->s, sp, pend, pend_n, slot, dL, dP, dS, dC, dLi, dA,
                                          dT, dN, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(ro.brightness, dL, npx * 4, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dP) e = hipMemcpyAsync(ro.pbar, dP, npx * 4, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dS) e = hipMemcpyAsync(ro.stale_mask, dS, npx, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dC) e = hipMemcpyAsync(ro.active_count, dC, npx * 4, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dLi) e = hipMemcpyAsync(ro.last_index, dLi, npx * 8, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dA) e = hipMemcpyAsync(ro.log_age, dA, npx * 4, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dT) e = hipMemcpyAsync(ro.tile_count, dT, c->ntiles * 4, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && dN) e = hipMemcpyAsync(ro.total_count, dN, npx * 8, hipMemcpyDeviceToHost, c->st);
    hipError_t e2 = hipFreeAsync(stage, c->st);
    hipError_t e3 = hipStreamSynchronize(c->st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = e3;
    return map_err(e);
}

// Wait until the latest blur-off batch that read its descriptors in place
// has read them (its base launch stored its number).  The stream is queried
// only after a millisecond of waiting (a query can put a marker into the
// stream, which costs as much as an event); if it has gone idle without the
// number, the launch did not run.
hipError_t wait_descriptors_read(fibar_ctx* c)
{
    if (!c->h_done) return hipSuccess;
    auto next_query = std::chrono::steady_clock::now() + std::chrono::milliseconds(1);
    while (*c->h_done < c->done_seq) {
        if (std::chrono::steady_clock::now() < next_query) continue;
        const hipError_t q = hipStreamQuery(c->st);
        if (q == hipSuccess && *c->h_done < c->done_seq) return hipErrorLaunchFailure;
        if (q != hipSuccess && q != hipErrorNotReady) return q;
        next_query = std::chrono::steady_clock::now() + std::chrono::milliseconds(1);
    }
    return hipSuccess;
}

// Blur-off batch: pushes and device readouts in one region-path pass.
int run_region_batch(fibar_ctx* c, const Op* ops, size_t n, uint32_t n_chunks, uint32_t n_steps)
{
    HIP_TRY(wait_descriptors_read(c));
    HIP_TRY(hipEventSynchronize(c->chunks_free));
    HIP_TRY(hipEventSynchronize(c->ro_free));
    uint32_t ci = 0, step = 0, nr = 0;
    bool any_opt = false;   // a readout asks for more than the brightness
    for (size_t i = 0; i < n; ++i) {
        if (ops[i].kind == 1) {
            RegionReadout& d = c->h_ro[nr++];
            d.chunk_end = ci;
            d.pad = 0;
            d.L = ops[i].ro.brightness;
            d.pbar = ops[i].ro.pbar;
            d.last = ops[i].ro.last_index;
            d.log_age = ops[i].ro.log_age;
            d.tot = ops[i].ro.total_count;
            any_opt = any_opt || d.pbar || d.last || d.log_age || d.tot;
            continue;
        }
        for (uint32_t off = 0; off < ops[i].n; off += kChunk) {
            ChunkDesc& d = c->h_chunks[ci++];
            const uint32_t m = ops[i].n - off < (uint32_t)kChunk ? ops[i].n - off : (uint32_t)kChunk;
            d.x = ops[i].x + off;
            d.y = ops[i].y + off;
            d.p = ops[i].p + off;
            d.n = m;
            d.pkt = step;
        }
        ++step;
    }
    // the first kernel reads the descriptors from host memory and keeps the
    // device copy (no copy in the stream), and a later one then stores the
    // batch's number into h_done; a batch of readouts only has no such kernel
    // and takes one copy: the chunk descriptors, and the readout descriptors
    // after all kMaxBatchChunks slots
    const bool direct = n_chunks > 0 && c->h_chunks_dev;
    if (!direct) {
        const size_t bytes = nr ? kMaxBatchChunks * sizeof(ChunkDesc) + (size_t)nr * sizeof(RegionReadout)
                                : (size_t)n_chunks * sizeof(ChunkDesc);
        if (bytes) HIP_TRY(hipMemcpyAsync(c->d_chunks, c->h_chunks, bytes, hipMemcpyHostToDevice, c->st));
        HIP_TRY(hipEventRecord(c->chunks_free, c->st));
        HIP_TRY(hipEventRecord(c->ro_free, c->st));
    }
    // no clearing of the step scratch: the kernels write each chunk's and
    // each packet's validation bits whole
    (void)n_steps;
    const uint64_t seq = direct ? c->done_seq + 1 : 0;
    HIP_TRY(timed_launch(c, 0, [&](const LaunchTiming& tm) {
        return launch_region_batch(c->s, c->cur_slot, c->d_chunks, n_chunks, c->scratch, c->rb, nr,
                                   any_opt, c->key_bits, c->coef, c->st, tm,
                                   direct ? c->h_chunks_dev : nullptr, c->d_done, seq);
    }));
    if (direct) c->done_seq = seq;
    return FIBAR_OK;
}

// Per-event regulation: one launch per packet, readouts between them.
int run_event_batch(fibar_ctx* c, const Op* ops, size_t n)
{
    for (size_t i = 0; i < n; ++i) {
        if (ops[i].kind == 1) {
            int rc = do_readout_kernel(c, ops[i].ro, nullptr, 0);
            if (rc) return rc;
            continue;
        }
        HIP_TRY(launch_event_packet(c->s, c->cur_slot, ops[i].x, ops[i].y, ops[i].p, ops[i].n,
                                    c->coef, c->ev_cap, c->ev_lds, c->st));
    }
    return FIBAR_OK;
}

// Per-tile queues: the batch's events bucketed by tile, then per packet
// the tiles' steps and the blur; readouts between them.
int run_tq_batch(fibar_ctx* c, const Op* ops, size_t n, uint32_t n_chunks, uint32_t n_steps)
{
    if (n_chunks > 0) {
        HIP_TRY(hipEventSynchronize(c->chunks_free));
        uint32_t ci = 0, step = 0;
        for (size_t i = 0; i < n; ++i) {
            if (ops[i].kind != 0) continue;
            for (uint32_t off = 0; off < ops[i].n; off += kChunk) {
                ChunkDesc& d = c->h_chunks[ci++];
                const uint32_t m = ops[i].n - off < (uint32_t)kChunk ? ops[i].n - off : (uint32_t)kChunk;
                d.x = ops[i].x + off;
                d.y = ops[i].y + off;
                d.p = ops[i].p + off;
                d.n = m;
                d.pkt = step;
            }
            ++step;
        }
        HIP_TRY(hipMemcpyAsync(c->d_chunks, c->h_chunks, (size_t)n_chunks * sizeof(ChunkDesc),
                               hipMemcpyHostToDevice, c->st));
        HIP_TRY(hipEventRecord(c->chunks_free, c->st));
        HIP_TRY(hipMemsetAsync(c->scratch, 0, (size_t)n_steps * sizeof(StepScratch), c->st));
        HIP_TRY(tq_bulk(c, n_chunks));
    }
    uint32_t ci = 0, step = 0;
    for (size_t i = 0; i < n; ++i) {
        if (ops[i].kind == 1) {
            int rc = do_readout_kernel(c, ops[i].ro, nullptr, 0);
            if (rc) return rc;
            continue;
        }
        const uint32_t nc = (ops[i].n + kChunk - 1) / kChunk;
        HIP_TRY(tq_step(c, ci, ci + nc, n_chunks, step));
        ci += nc;
        ++step;
    }
    return FIBAR_OK;
}

// Execute ops[0..n): bulk sort for all pushes, then the in-order steps.
int run_batch(fibar_ctx* c, const Op* ops, size_t n, uint32_t n_chunks, uint32_t n_steps)
{
    if (n == 0) return FIBAR_OK;
    if (c->region_path) return run_region_batch(c, ops, n, n_chunks, n_steps);
    if (c->event_mode) return run_event_batch(c, ops, n);
    if (c->tq) return run_tq_batch(c, ops, n, n_chunks, n_steps);
    // graph mode replays the batch's kernels as one graph; a readout into
    // host memory (copies and a wait between the kernels) keeps the batch on
    // direct launches
    bool graph = c->graph_mode;
    for (size_t i = 0; graph && i < n; ++i)
        if (ops[i].kind == 1 && !ops[i].ro.on_device) graph = false;
    if (n_chunks > 0) {
        // the pinned descriptor buffer may still feed a previous copy
        HIP_TRY(hipEventSynchronize(c->chunks_free));
        uint32_t ci = 0, step = 0;
        for (size_t i = 0; i < n; ++i) {
            if (ops[i].kind != 0) continue;
            for (uint32_t off = 0; off < ops[i].n; off += kChunk) {
                ChunkDesc& d = c->h_chunks[ci++];
                const uint32_t m = ops[i].n - off < (uint32_t)kChunk ? ops[i].n - off : (uint32_t)kChunk;
                d.x = ops[i].x + off;
                d.y = ops[i].y + off;
                d.p = ops[i].p + off;
                d.n = m;
                d.pkt = step;
            }
            ++step;
        }
        HIP_TRY(hipMemcpyAsync(c->d_chunks, c->h_chunks, (size_t)n_chunks * sizeof(ChunkDesc),
                               hipMemcpyHostToDevice, c->st));
        HIP_TRY(hipEventRecord(c->chunks_free, c->st));
        HIP_TRY(hipMemsetAsync(c->scratch, 0, (size_t)n_steps * sizeof(StepScratch), c->st));
    }
    BatchRecording recording(c, graph);   // the kernels from here on
    if (n_chunks > 0) {
        HIP_TRY(timed_launch(c, 0, [&](const LaunchTiming& tm) {
            return launch_sort_compose(c->d_chunks, n_chunks, c->seg, c->seg_count, c->scratch,
                                       c->W, c->H, c->key_bits, c->coef, c->s.gain, c->st, tm);
        }));
    }
    uint32_t ci = 0, step = 0;
    const int sp = (int)c->prm.spatial_filter;
    const StepScratch* pend = nullptr;   // step applied but not yet committed
    uint32_t pend_n = 0;
    for (size_t i = 0; i < n; ++i) {
        if (ops[i].kind == 1) {
            int rc = do_readout_kernel(c, ops[i].ro, pend, pend_n);
            if (rc) return rc;
            continue;
        }
        StepScratch* stp = c->scratch + step;
        const uint32_t nev = ops[i].n;
        const int slot_in = c->cur_slot;
        const int slot_out = pend ? (slot_in ^ 1) : -1;
        for (uint32_t off = 0; off < nev; off += kChunk) {
            const uint32_t m = nev - off < (uint32_t)kChunk ? nev - off : (uint32_t)kChunk;
            HIP_TRY(timed_launch(c, 1, [&](const LaunchTiming& tm) {
                return launch_apply(c->s, &c->h_chunks[ci], c->seg + (size_t)ci * kChunk,
                                    c->seg_count + ci, m, off, stp, pend, pend_n, slot_in,
                                    slot_out, sp, c->st, tm);
            }));
            ++ci;
        }
        if (pend) c->cur_slot ^= 1;
        if (sp) {
            const int slot = c->cur_slot;
            // a device readout right after the step (without the window
            // count, which the pops change) is taken by the pop launch
            const bool fuse = i + 1 < n && ops[i + 1].kind == 1 && ops[i + 1].ro.on_device &&
                              !ops[i + 1].ro.active_count;
            if (fuse) {
                const fibar_readout_buf& rb = ops[i + 1].ro;
                PopReadout pr{rb.brightness, rb.pbar,     rb.stale_mask,
                              rb.last_index, rb.log_age, rb.tile_count,
                              rb.total_count};
                if (graph) {
                    // counted as a pop, so that the timed launches of a
                    // batch do not depend on where its readouts fall
                    HIP_TRY(timed_launch(c, 2, 3, [&](const LaunchTiming& tm) {
                        return launch_pop_blur(c->s, nev, stp, slot, &pr, c->st, tm);
                    }));
                } else {
                    HIP_TRY(launch_pop_blur(c->s, nev, stp, slot, &pr, c->st));
                }
                ++i;   // the readout op is done
            } else {
                HIP_TRY(timed_launch(c, 2, [&](const LaunchTiming& tm) {
                    return launch_pop_blur(c->s, nev, stp, slot, nullptr, c->st, tm);
                }));
            }
        }
        pend = stp;
        pend_n = nev;
        ++step;
    }
    if (pend) {
        HIP_TRY(launch_commit(c->s, pend, pend_n, c->cur_slot, c->cur_slot ^ 1, sp, c->st));
        c->cur_slot ^= 1;
    }
    HIP_TRY(recording.finish());
    return FIBAR_OK;
}

// Check, stage and execute a list of public ops.
int execute(fibar_ctx* c, const fibar_op* ops, size_t n_ops)
{
    std::vector<Op> batch;
    batch.reserve(n_ops < 4096 ? n_ops : 4096);
    uint32_t n_chunks = 0, n_steps = 0, n_readouts = 0;
    for (size_t i = 0; i < n_ops; ++i) {
        const fibar_op& op = ops[i];
        if (op.kind == FIBAR_OP_PUSH) {
            const fibar_packet& pk = op.packet;
            if (pk.n == 0) continue;
            if (pk.n > c->prm.max_packet || !pk.x || !pk.y || !pk.p) {
                int rc = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                return rc ? rc : FIBAR_E_INVALID_ARG;
            }
            const uint32_t need = (uint32_t)((pk.n + kChunk - 1) / kChunk);
            const bool host = !pk.on_device;
            const bool wrap = host && c->hs_pos + pk.n > c->stg_cap;
            if (n_chunks + need > kMaxBatchChunks || wrap) {
                int rc = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                if (rc) return rc;
                batch.clear();
                n_chunks = n_steps = 0;
                n_readouts = 0;
            }
            if (wrap) {
                // the pinned ring starts over once every copy from it has run
                HIP_TRY(hipEventSynchronize(c->hs_done));
                c->hs_pos = 0;
            }
            Op o{};
            o.kind = 0;
            o.n = (uint32_t)pk.n;
            if (host) {
                int rc = host_validate(c, &pk);
                if (rc) {
                    int rc2 = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                    return rc2 ? rc2 : rc;
                }
                // the caller's arrays are free when the call returns: copy
                // them into the pinned ring, then to the device in stream
                // order (the device staging is reused in stream order too)
                const size_t at = c->hs_pos;
                memcpy(c->hs_x + at, pk.x, pk.n * 2);
                memcpy(c->hs_y + at, pk.y, pk.n * 2);
                memcpy(c->hs_p + at, pk.p, pk.n);
                HIP_TRY(hipMemcpyAsync(c->stg_x + at, c->hs_x + at, pk.n * 2, hipMemcpyHostToDevice,
                                       c->st));
                HIP_TRY(hipMemcpyAsync(c->stg_y + at, c->hs_y + at, pk.n * 2, hipMemcpyHostToDevice,
                                       c->st));
                HIP_TRY(hipMemcpyAsync(c->stg_p + at, c->hs_p + at, pk.n, hipMemcpyHostToDevice,
                                       c->st));
                HIP_TRY(hipEventRecord(c->hs_done, c->st));
                o.x = c->stg_x + at;
                o.y = c->stg_y + at;
                o.p = c->stg_p + at;
                c->hs_pos = at + pk.n;
                if (pk.t && pk.t[pk.n - 1] > c->t_hi) c->t_hi = pk.t[pk.n - 1];
            } else {
                o.x = pk.x;
                o.y = pk.y;
                o.p = pk.p;
            }
            batch.push_back(o);
            n_chunks += need;
            n_steps += 1;
        } else if (op.kind == FIBAR_OP_READOUT) {
            const fibar_readout_buf& ro = op.readout;
            int rc = FIBAR_OK;
            if (!ro.brightness) rc = FIBAR_E_INVALID_ARG;
            else if (!c->prm.spatial_filter &&
                     (ro.stale_mask || ro.active_count || ro.tile_count)) rc = FIBAR_E_UNSUPPORTED;
            else if (op.t < c->t_hi) rc = FIBAR_E_TIME;
            if (rc) {
                int rc2 = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                return rc2 ? rc2 : rc;
            }
            c->t_hi = op.t;
            Op o{};
            o.kind = 1;
            o.ro = ro;
            if (c->region_path) {
                if (!ro.on_device) {
                    // host outputs: finish the batch, then read the state
                    int rc2 = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                    if (rc2) return rc2;
                    batch.clear();
                    n_chunks = n_steps = 0;
                    rc2 = do_readout_kernel(c, ro, nullptr, 0);
                    if (rc2) return rc2;
                    continue;
                }
                if (n_readouts == kMaxBatchReadouts) {
                    int rc2 = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
                    if (rc2) return rc2;
                    batch.clear();
                    n_chunks = n_steps = 0;
                    n_readouts = 0;
                }
                ++n_readouts;
            }
            batch.push_back(o);
        } else {
            int rc2 = run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
            return rc2 ? rc2 : FIBAR_E_INVALID_ARG;
        }
    }
    return run_batch(c, batch.data(), batch.size(), n_chunks, n_steps);
}

// Initial state: zero images, no events seen, target length q_max.
hipError_t init_state(fibar_ctx* c)
{
    c->h_sc->k = -1;
    c->h_sc->h = 0;
    c->h_sc->Q = c->prm.q_max;
    c->h_sc->P = c->h_sc->T = 0;
    c->h_sc->n_reg = c->h_sc->last_stale = c->h_sc->total_stale = 0;
    c->h_sc->err = 0;
    c->h_sc->stepped = 0;
    c->cur_slot = 0;
    hipError_t e = launch_init_state(c->s, c->st);
    if (e == hipSuccess && c->tq) e = tq_init(c);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->s.sc + c->cur_slot, c->h_sc, sizeof(DevScalars), hipMemcpyHostToDevice,
                           c->st);
    // the pinned source must not change before the copy has run
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    c->t_hi = 0;
    return e;
}

int fetch_scalars(fibar_ctx* c)
{
    HIP_TRY(hipMemcpyAsync(c->h_sc, c->s.sc + c->cur_slot, sizeof(DevScalars),
                           hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return FIBAR_OK;
}

// Report and clear a device-side packet error.
int take_device_error(fibar_ctx* c)
{
    const int err = c->h_sc->err;
    if (err) {
        const int32_t zero = 0;
        HIP_TRY(hipMemcpyAsync(&c->s.sc[c->cur_slot].err, &zero, sizeof(zero),
                               hipMemcpyHostToDevice, c->st));
        HIP_TRY(hipStreamSynchronize(c->st));
    }
    return err;
}

}  // namespace

extern "C" {

void fibar_default_params(fibar_params* p)
{
    if (!p) return;
    p->t_cut = 40.0;
    p->fill_num = 1;
    p->fill_den = 2;
    p->q_min = 64;
    p->q_max = 0;
    p->spatial_filter = 1;
    p->regulation = FIBAR_REG_PACKET;
    p->max_packet = 65536;
    p->stream = nullptr;
    p->region = 0;
    p->age_max = 0;
}

int fibar_create(uint32_t width, uint32_t height, const fibar_params* prm, fibar_ctx** out)
{
    if (!out) return FIBAR_E_INVALID_ARG;
    *out = nullptr;
    fibar_params p;
    if (prm) p = *prm;
    else fibar_default_params(&p);
    if (width == 0 || height == 0 || width > 65535 || height > 65535) return FIBAR_E_INVALID_ARG;
    if (!(p.t_cut > 4.0) || !isfinite(p.t_cut)) return FIBAR_E_INVALID_ARG;
    if (p.fill_num == 0 || p.fill_den == 0 || p.fill_num > p.fill_den || p.fill_den > 65535)
        return FIBAR_E_INVALID_ARG;
    if (p.spatial_filter > 1 || p.regulation > FIBAR_REG_EVENT) return FIBAR_E_INVALID_ARG;
    if (p.max_packet == 0 || p.max_packet > kMaxPacket) return FIBAR_E_INVALID_ARG;
    const uint64_t npx = (uint64_t)width * height;
    // the sort key of an event is (tile-major pixel key << 1) | polarity in
    // 32 bits, with 4 keys per 2x2 tile
    const uint64_t key_span = 4ull * ((width + 1) / 2) * ((height + 1) / 2);
    if (key_span > kMaxKeySpan) return FIBAR_E_INVALID_ARG;
    if (p.q_max == 0) p.q_max = (uint32_t)npx;
    if (p.q_min == 0 || p.q_min > p.q_max) return FIBAR_E_INVALID_ARG;
    // per-event regulation with the spatial filter on keeps a packet's state
    // in one workgroup's LDS (without the filter there is nothing to regulate)
    const bool event_mode = p.regulation == FIBAR_REG_EVENT && p.spatial_filter;
    // per-tile queues: tiles of whole 2x2 cells that fit one 1024-thread
    // workgroup, packet regulation
    const bool tq = p.region != 0;
    uint32_t tq_RW = 0, tq_RH = 0, tq_cap = 1;
    if (tq) {
        if ((p.region & 1u) || p.region > 32 || !p.spatial_filter ||
            p.regulation != FIBAR_REG_PACKET)
            return FIBAR_E_INVALID_ARG;
        tq_RW = (width + p.region - 1) / p.region;
        tq_RH = (height + p.region - 1) / p.region;
        if ((uint64_t)tq_RW * tq_RH > kMaxRegions) return FIBAR_E_INVALID_ARG;
        while (tq_cap < p.region * p.region + p.max_packet) tq_cap <<= 1;
    }
    uint32_t ev_cap = 1;
    if (event_mode) {
        if (npx > kEventMaxPixels || p.q_max > kEventMaxRing - 2) return FIBAR_E_INVALID_ARG;
        while (ev_cap < p.q_max + 2) ev_cap <<= 1;
    }

    fibar_ctx* c = new (std::nothrow) fibar_ctx();
    if (!c) return FIBAR_E_NOMEM;
    c->W = width;
    c->H = height;
    c->TW = (width + 1) / 2;
    c->TH = (height + 1) / 2;
    c->npx = npx;
    c->ntiles = (uint64_t)c->TW * c->TH;
    c->prm = p;
    c->st = (hipStream_t)p.stream;
    double a, b;
    filter_coefficients(p.t_cut, &a, &b);
    c->coef.alpha = (float)a;
    c->coef.one_m_alpha = (float)(1.0 - a);
    c->coef.beta = (float)b;
    c->coef.c_alpha = (float)(0.5 * (1.0 + b) * a);
    // sort keys are tile-major: 4 per 2x2 tile
    int kb = 1;
    while (kb < 32 && (1ull << kb) < 4 * c->ntiles) ++kb;
    c->key_bits = kb;

    uint64_t ring = 1;
    while (ring < (uint64_t)p.q_max + p.max_packet) ring <<= 1;
    const uint64_t stg = (uint64_t)kMaxBatchChunks * kChunk;

    const uint64_t n_regions = (npx + kRegion - 1) / kRegion;
    c->region_path = !p.spatial_filter && n_regions <= kMaxRegions;
    c->event_mode = event_mode;
    c->tq = tq;
    if (tq) {
        c->tq_R = p.region;
        c->tq_RW = tq_RW;
        c->tq_RH = tq_RH;
        c->tq_cap = tq_cap;
        c->tq_age = p.age_max ? p.age_max : npx;
    }
    if (event_mode) {
        c->ev_cap = ev_cap;
        c->ev_lds = event_lds_bytes(width, height, c->TW, ev_cap);
    }

    hipError_t e = hipSuccess;
    auto alloc = [&](void** ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, bytes);
    };
    alloc((void**)&c->s.px, npx * sizeof(PixL));
    alloc((void**)&c->s.pp, npx * sizeof(PixP));
    alloc((void**)&c->s.ring, ring * 4);
    alloc((void**)&c->s.sc, 2 * sizeof(DevScalars));
    // blur off: the readout descriptors of a batch follow its chunk
    // descriptors in the same buffers, so that one copy carries both
    const size_t desc_bytes = kMaxBatchChunks * sizeof(ChunkDesc) +
                              (c->region_path ? kMaxBatchReadouts * sizeof(RegionReadout) : 0);
    alloc((void**)&c->d_chunks, desc_bytes);
    // 4 spare records: an item reads records up to i + 3 of its chunk
    alloc((void**)&c->seg, ((size_t)kMaxBatchChunks * kChunk + 4) * sizeof(SegRec));
    alloc((void**)&c->seg_count, kMaxBatchChunks * 4);
    alloc((void**)&c->scratch, kMaxBatchChunks * sizeof(StepScratch));
    alloc((void**)&c->stg_x, stg * 2);
    alloc((void**)&c->stg_y, stg * 2);
    alloc((void**)&c->stg_p, stg);
    if (tq) {
        const uint64_t nt = (uint64_t)tq_RW * tq_RH;
        c->rb.n_regions = (uint32_t)nt;
        alloc((void**)&c->rb.cnt, (size_t)kMaxBatchChunks * nt * 4);
        alloc((void**)&c->rb.base, (nt + 1) * 8);
        alloc((void**)&c->rb.total, nt * 4);
        alloc((void**)&c->rb.chunk_k, (kMaxBatchChunks + 1) * 8);
        alloc((void**)&c->rb.payload, (size_t)kMaxBatchChunks * kChunk * 8);
        alloc((void**)&c->tq_tiles, nt * sizeof(TQTile));
        alloc((void**)&c->tq_front, 2 * nt * 8);
        alloc((void**)&c->tq_ring, nt * tq_cap * sizeof(uint2));
        alloc((void**)&c->tq_stale, nt * p.region * p.region * 4);
        alloc((void**)&c->tq_nstale, nt * 4);
    }
    if (c->region_path) {
        c->rb.n_regions = (uint32_t)n_regions;
        alloc((void**)&c->rb.cnt, (size_t)kMaxBatchChunks * n_regions * 4);
        alloc((void**)&c->rb.base, (n_regions + 1) * 8);
        alloc((void**)&c->rb.total, n_regions * 4);
        alloc((void**)&c->rb.chunk_k, (kMaxBatchChunks + 1) * 8);
        alloc((void**)&c->rb.payload, (size_t)kMaxBatchChunks * kChunk * 8);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ro_free, hipEventDisableTiming);
    }
    // blur off: the descriptors are read by a kernel where the host wrote
    // them (mapped and coherent, so a kernel sees the host's latest writes)
    // (and the word after them that says a batch's descriptors were read)
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->h_chunks, desc_bytes + (c->region_path ? 64 : 0),
                          c->region_path ? hipHostMallocMapped | hipHostMallocCoherent : 0u);
    if (e == hipSuccess && c->region_path) {
        c->rb.ro = reinterpret_cast<RegionReadout*>(c->d_chunks + kMaxBatchChunks);
        c->h_ro = reinterpret_cast<RegionReadout*>(c->h_chunks + kMaxBatchChunks);
        void* dev = nullptr;
        if (hipHostGetDevicePointer(&dev, c->h_chunks, 0) == hipSuccess && dev) {
            c->h_chunks_dev = static_cast<const ChunkDesc*>(dev);
            c->h_done = reinterpret_cast<volatile uint64_t*>(
                reinterpret_cast<char*>(c->h_chunks) + desc_bytes);
            *c->h_done = 0;
            c->d_done = reinterpret_cast<uint64_t*>(static_cast<char*>(dev) + desc_bytes);
        } else {
            (void)hipGetLastError();   // no device view: each batch copies its descriptors
        }
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->hs_x, stg * 2, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->hs_y, stg * 2, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->hs_p, stg, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->hs_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_sc, sizeof(DevScalars), 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->chunks_free, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = map_err(e);
        free_ctx(c);
        return rc;
    }
    c->stg_cap = stg;
    c->s.ring_mask = ring - 1;
    c->s.W = width;
    c->s.H = height;
    c->s.TW = c->TW;
    c->s.fill_num = p.fill_num;
    c->s.fill_den = p.fill_den;
    c->s.q_min = p.q_min;
    c->s.q_max = p.q_max;

    if (event_mode) e = prepare_event_kernel(c->ev_lds);
    if (e == hipSuccess) e = init_state(c);
    if (e == hipSuccess) e = hipEventRecord(c->chunks_free, c->st);
    if (e == hipSuccess) e = hipEventRecord(c->hs_done, c->st);
    if (e == hipSuccess && c->ro_free) e = hipEventRecord(c->ro_free, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        int rc = map_err(e);
        free_ctx(c);
        return rc;
    }
    *out = c;
    return FIBAR_OK;
}

int fibar_push_events(fibar_ctx* c, const fibar_packet* pkt)
{
    if (!c || !pkt) return FIBAR_E_INVALID_ARG;
    fibar_op op{};
    op.kind = FIBAR_OP_PUSH;
    op.packet = *pkt;
    return execute(c, &op, 1);
}

int fibar_readout(fibar_ctx* c, uint64_t t, const fibar_readout_buf* out)
{
    if (!c || !out) return FIBAR_E_INVALID_ARG;
    fibar_op op{};
    op.kind = FIBAR_OP_READOUT;
    op.t = t;
    op.readout = *out;
    int rc = execute(c, &op, 1);
    if (rc) return rc;
    if (!out->on_device) {
        rc = fetch_scalars(c);
        if (rc) return rc;
        return take_device_error(c);
    }
    return FIBAR_OK;
}

int fibar_submit(fibar_ctx* c, const fibar_op* ops, size_t n_ops)
{
    if (!c || (!ops && n_ops)) return FIBAR_E_INVALID_ARG;
    return execute(c, ops, n_ops);
}

void fibar_destroy(fibar_ctx* c) { free_ctx(c); }

int fibar_get_stats(fibar_ctx* c, fibar_stats* s)
{
    if (!c || !s) return FIBAR_E_INVALID_ARG;
    int rc = fetch_scalars(c);
    if (rc) return rc;
    const DevScalars& d = *c->h_sc;
    s->k = d.k;
    s->h = d.h;
    s->q = (uint64_t)(d.k + 1) - d.h;
    s->Q = d.Q;
    s->P = d.P;
    s->T = d.T;
    if (c->tq) {
        // sums over the tiles
        const size_t nt = (size_t)c->tq_RW * c->tq_RH;
        std::vector<TQTile> t(nt);
        HIP_TRY(hipMemcpy(t.data(), c->tq_tiles, nt * sizeof(TQTile), hipMemcpyDeviceToHost));
        uint64_t q = 0, Q = 0, P = 0, T = 0;
        for (const TQTile& x : t) {
            q += x.tail - x.head;
            Q += x.Q;
            P += x.P;
            T += x.T;
        }
        s->q = q;
        s->h = (uint64_t)(d.k + 1) - q;
        s->Q = Q;
        s->P = P;
        s->T = T;
    }
    s->n_regulations = d.n_reg;
    s->last_stale = d.last_stale;
    s->total_stale = d.total_stale;
    return take_device_error(c);
}

int fibar_synchronize(fibar_ctx* c)
{
    if (!c) return FIBAR_E_INVALID_ARG;
    int rc = fetch_scalars(c);
    if (rc) return rc;
    return take_device_error(c);
}

int fibar_reset(fibar_ctx* c)
{
    if (!c) return FIBAR_E_INVALID_ARG;
    return map_err(init_state(c));
}

int fibar_set_kernel_timing(fibar_ctx* c, uint32_t kernel_mask, uint32_t every)
{
    if (!c || kernel_mask >= (1u << 5) || every == 0) return FIBAR_E_INVALID_ARG;
    c->time_mask = kernel_mask;
    c->time_every = every;
    for (auto& q : c->time_seq) q = 0;
    return FIBAR_OK;
}

int fibar_tile_stats(fibar_ctx* c, uint64_t* q, uint64_t* Q, uint64_t* P, uint64_t* T,
                     uint64_t* front)
{
    if (!c) return FIBAR_E_INVALID_ARG;
    if (!c->tq) return FIBAR_E_UNSUPPORTED;
    int rc = fetch_scalars(c);
    if (rc) return rc;
    const size_t nt = (size_t)c->tq_RW * c->tq_RH;
    std::vector<TQTile> t(nt);
    std::vector<uint64_t> f(nt);
    HIP_TRY(hipMemcpy(t.data(), c->tq_tiles, nt * sizeof(TQTile), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(f.data(), c->tq_front + (size_t)c->tq_parity * nt, nt * 8,
                      hipMemcpyDeviceToHost));
    for (size_t i = 0; i < nt; ++i) {
        if (q) q[i] = t[i].tail - t[i].head;
        if (Q) Q[i] = t[i].Q;
        if (P) P[i] = t[i].P;
        if (T) T[i] = t[i].T;
        if (front) front[i] = f[i];
    }
    return take_device_error(c);
}

int fibar_set_telemetry(fibar_ctx* c, fibar_step_record* records, uint64_t capacity)
{
    if (!c || (!records && capacity)) return FIBAR_E_INVALID_ARG;
    if ((!c->prm.spatial_filter || c->event_mode || c->tq) && records) return FIBAR_E_UNSUPPORTED;
    // launches already queued keep the buffer they were given
    c->s.tel = capacity ? reinterpret_cast<StepRecord*>(records) : nullptr;
    c->s.tel_cap = capacity;
    return FIBAR_OK;
}

int fibar_set_launch_mode(fibar_ctx* c, int mode)
{
    if (!c || (mode != FIBAR_LAUNCH_DIRECT && mode != FIBAR_LAUNCH_GRAPH)) return FIBAR_E_INVALID_ARG;
    c->graph_mode = mode == FIBAR_LAUNCH_GRAPH;
    return FIBAR_OK;
}

int fibar_kernel_time(fibar_ctx* c, int kernel, double* total_ms, uint64_t* launches)
{
    if (!c || kernel < 0 || kernel >= 5 || !total_ms || !launches) return FIBAR_E_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize(c->st));
    double sum = 0.0;
    for (auto& pr : c->timed[kernel]) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        sum += ms;
        c->event_pool.push_back(pr.first);
        c->event_pool.push_back(pr.second);
    }
    *launches = c->timed[kernel].size();
    *total_ms = sum;
    c->timed[kernel].clear();
    return FIBAR_OK;
}

const char* fibar_status_string(int status)
{
    switch (status) {
    case FIBAR_OK: return "ok";
    case FIBAR_E_INVALID_ARG: return "invalid argument";
    case FIBAR_E_RANGE: return "event coordinate out of range";
    case FIBAR_E_POLARITY: return "polarity byte not 0 or 1";
    case FIBAR_E_TIME: return "readout time earlier than a previous time";
    case FIBAR_E_NOMEM: return "out of memory";
    case FIBAR_E_DEVICE: return "device error";
    case FIBAR_E_UNSUPPORTED: return "output not maintained in this mode";
    default: return "unknown status";
    }
}

}  // extern "C"
