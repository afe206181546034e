// Multi-stream executor of libfibar: many independent event streams (each a
// fibar_ctx with its own resolution, packet sizes and state) advance
// together, one packet per stream per round.
//
// A round is a fixed sequence of launches shared by every stream:
//   k_multi_apply (sub-round 0, and sub-round 1 when some packet has a second
//   chunk), k_multi_pop, and k_multi_readout when some stream reads out.
// The host plans every round of a batch up front: one self-contained record
// per stream holds everything its step needs (the stream's state pointers,
// chunk descriptors, scratch, scalar slots) and, per kind of launch, the
// cumulative count of workgroup tasks up to that stream.  A workgroup finds
// the stream owning task t with one ballot over those counts (one stream
// per lane).  Each launch has a fixed number of resident workgroups,
// workgroup w taking tasks w, w + grid, ...
//
// Up to kUnroll consecutive rounds form one HIP graph (readouts only in its
// last round, so the launch sequence is fixed).  Its first node copies the
// records of its rounds from the batch table (at the index of the graph's
// first round, kept on the device and advanced by the graph's last node)
// into a fixed ring; the round kernels read ring slot j, an address fixed at
// capture.  So reaching the per-pixel work takes one dependent load, the
// stream record -- dependent misses, not bandwidth, bound the small rounds.
// Within a stream the order of steps is the single-stream order (apply,
// pop/blur, lagged commit), so results are identical to running each stream
// alone.
//
// The launch shape (workgroup size, number of resident workgroups) does not
// change any result: only integer atomics are reordered and every float is
// computed from the same operands.  The autotuner times the candidate shapes
// on interleaved groups of rounds of a submission and keeps the fastest.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fibar_ctx.h"
#include "fibar_step.h"

namespace fibar {
namespace {

using namespace tile;
using namespace step;

constexpr uint32_t kMultiMaxStreams = 64;       // one wave's lanes
constexpr uint32_t kMultiChunks = 1024;         // chunks grouped per multi batch
constexpr uint32_t kMultiMaxRounds = 1024;
constexpr uint32_t kMultiMaxReadouts = 1024;
constexpr uint32_t kMultiMaxRoTasks = 1u << 20;
constexpr uint32_t kReadoutBlock = 1024;        // pixels per readout task
constexpr uint32_t kUnroll = 64;                // rounds per graph replay
constexpr uint32_t kTuneLen = 4;                // rounds per timed group while tuning
constexpr uint32_t kTuneGroups = 3;             // timed groups per candidate shape
constexpr uint32_t kNone = 0xffffffffu;
constexpr uint32_t kMaxDirectGrid = 1u << 16;   // workgroups of a direct launch

// Task kinds of a round: apply sub-round 0 (a stream with a pending step
// gets one extra task, its first, that commits it), apply sub-round 1, pops.
constexpr int kKinds = 3;

// One stream's step in one round; read by every workgroup working on it.
// Records of streams without a step in the round have end[] = the round's
// totals and own no task.
struct alignas(16) StreamStep {
    uint32_t end[kKinds];            // cumulative tasks of records 0..this one
    uint32_t ro_off, ro_cnt;         // the round's readout tasks (record 0)
    State s;
    ChunkDesc chunk[2];
    const SegRec* seg[2];            // the chunks' composed records
    const uint32_t* nseg[2];         // and their counts
    StepScratch* step;               // this step's counters and status
    const StepScratch* prev;         // the pending (uncommitted) step, or null
    uint32_t events, prev_events;
    int32_t slot_in;                 // committed scalars before this round
    int32_t slot_out;                // where the pending step is committed
    int32_t pop_slot;                // committed scalars the pops start from
    uint32_t pop_blocks;             // workgroup tasks sharing the pops
};

struct RoTask {
    uint32_t rec;                    // stream record in the round
    uint32_t ro;                     // readout slot in the batch
    uint32_t blk;                    // pixel block
    uint32_t pad;
};

struct MultiReadout {
    float* L;
    float* pbar;
    uint8_t* stale;
    uint32_t* cnt;
    int64_t* last;
    float* log_age;
    uint64_t* tot;
};

struct CommitDesc {
    State s;
    const StepScratch* prev;
    uint32_t prev_events;
    int32_t slot_in, slot_out;
};

struct MultiArgs {
    const RoTask* rot;
    const MultiReadout* ros;
    uint32_t S;
};

// Each lane of a wave holds one record's cumulative task count of a kind
// (lanes >= S: no record); the last record's is the round's total.
__device__ __forceinline__ uint32_t lane_end(const StreamStep* rec, uint32_t S, int kind,
                                             uint32_t* total)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t e = lane < S ? rec[lane].end[kind] : 0xffffffffu;
    *total = (uint32_t)__builtin_amdgcn_readlane((int)e, (int)S - 1);   // S is uniform
    return e;
}

// Record owning task t: the number of records whose range ends at or before
// t (wave-uniform).  *start gets the record's first task.
__device__ __forceinline__ uint32_t owner(uint32_t e, uint32_t t, uint32_t* start)
{
    const uint32_t k = (uint32_t)__popcll(__ballot(e <= t));
    const uint32_t prev_end = (uint32_t)__builtin_amdgcn_readlane((int)e, (int)(k > 0 ? k - 1 : 0));
    *start = k > 0 ? prev_end : 0u;
    return k;
}

// The owner's record fields come from the lane that holds them: every lane
// loads its own record's fields together with its task count, so finding
// the owner costs no second dependent load.  k is wave-uniform.
__device__ __forceinline__ uint32_t bcast32(uint32_t v, uint32_t k)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)k);
}
template <typename P>
__device__ __forceinline__ P* bcast_ptr(P* p, uint32_t k)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint64_t r = (uint64_t)bcast32((uint32_t)v, k) | ((uint64_t)bcast32((uint32_t)(v >> 32), k) << 32);
    return as_global(reinterpret_cast<P*>(r));   // every record pointer is device memory
}
__device__ __forceinline__ uint64_t bcast64(uint64_t v, uint32_t k)
{
    return (uint64_t)bcast32((uint32_t)v, k) | ((uint64_t)bcast32((uint32_t)(v >> 32), k) << 32);
}

// A stream's State as held per lane (the fields the round kernels use).
struct LaneState {
    PixL* px;
    PixP* pp;
    uint32_t* ring;
    uint64_t ring_mask;
    DevScalars* sc;
    uint32_t W, H, TW, fill_num, fill_den;
    uint64_t q_min, q_max;
    StepRecord* tel;
    uint64_t tel_cap;
};

__device__ __forceinline__ LaneState lane_state(const StreamStep* rr, uint32_t S)
{
    const uint32_t lane = threadIdx.x & 63u;
    const StreamStep* e = rr + (lane < S ? lane : 0u);
    LaneState l;
    l.px = e->s.px;
    l.pp = e->s.pp;
    l.ring = e->s.ring;
    l.ring_mask = e->s.ring_mask;
    l.sc = e->s.sc;
    l.W = e->s.W;
    l.H = e->s.H;
    l.TW = e->s.TW;
    l.fill_num = e->s.fill_num;
    l.fill_den = e->s.fill_den;
    l.q_min = e->s.q_min;
    l.q_max = e->s.q_max;
    l.tel = e->s.tel;
    l.tel_cap = e->s.tel_cap;
    return l;
}

__device__ __forceinline__ State owner_state(const LaneState& l, uint32_t k)
{
    State s;
    s.px = bcast_ptr(l.px, k);
    s.pp = bcast_ptr(l.pp, k);
    s.ring = bcast_ptr(l.ring, k);
    s.ring_mask = bcast64(l.ring_mask, k);
    s.sc = bcast_ptr(l.sc, k);
    s.W = bcast32(l.W, k);
    s.H = bcast32(l.H, k);
    s.TW = bcast32(l.TW, k);
    s.fill_num = bcast32(l.fill_num, k);
    s.fill_den = bcast32(l.fill_den, k);
    s.q_min = bcast64(l.q_min, k);
    s.q_max = bcast64(l.q_max, k);
    s.tel = bcast_ptr(l.tel, k);
    s.tel_cap = bcast64(l.tel_cap, k);
    return s;
}

// Every round kernel gets `rr`, the round's S records, as its leading
// arguments: plain ones, so that they arrive preloaded in scalar registers
// (a leading struct argument stops the preloading, and every kernel then
// began with a round trip for its arguments).
__global__ __launch_bounds__(256) void k_multi_apply(const StreamStep* rr, uint32_t S, int sub)
{
    // this lane's record: the fields an apply task needs, loaded together with
    // the task counts (the fence keeps them from sinking behind the lookup)
    const uint32_t lane = threadIdx.x & 63u;
    const StreamStep* mine = rr + (lane < S ? lane : 0u);
    const LaneState ls = lane_state(rr, S);
    const StepScratch* l_prev = mine->prev;
    StepScratch* l_step = mine->step;
    const uint16_t* l_x = mine->chunk[sub].x;
    const uint16_t* l_y = mine->chunk[sub].y;
    const uint32_t l_n = mine->chunk[sub].n;
    const SegRec* l_seg = mine->seg[sub];
    const uint32_t* l_nseg = mine->nseg[sub];
    const uint32_t l_prev_events = mine->prev_events;
    const int32_t l_slot_in = mine->slot_in, l_slot_out = mine->slot_out;
    uint32_t total;
    const uint32_t le = lane_end(rr, S, sub, &total);
    FIBAR_ISSUE_FENCE();
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        uint32_t start;
        const uint32_t k = owner(le, t, &start);
        const State s = owner_state(ls, k);
        const StepScratch* prev = bcast_ptr(l_prev, k);
        const uint32_t prev_events = bcast32(l_prev_events, k);
        const int32_t slot_in = (int32_t)bcast32((uint32_t)l_slot_in, k);
        uint32_t b = t - start;
        if (sub == 0 && prev) {
            if (b == 0) {
                if (threadIdx.x < 64) {
                    const DevScalars r = commit_by_wave(s.sc + slot_in, prev, prev_events, s, 1);
                    const int32_t slot_out = (int32_t)bcast32((uint32_t)l_slot_out, k);
                    if (threadIdx.x == 0) store_commit(s, s.sc + slot_out, r, prev_events);
                }
                continue;
            }
            --b;
        }
        StepScratch* stp = bcast_ptr(l_step, k);
        ChunkDesc cd;
        cd.x = bcast_ptr(l_x, k);
        cd.y = bcast_ptr(l_y, k);
        cd.n = bcast32(l_n, k);
        // i < kChunk: task counts are ceil(n / block) and every block size
        // divides kChunk; a chunk slot holds kChunk records and 3 more follow
        const uint32_t i = b * blockDim.x + threadIdx.x;
        // every load that only needs the record is issued before any is used
        const Group g = load_group(cd, bcast_ptr(l_seg, k), i);
        const uint32_t status = stp->status;
        const uint32_t nseg = *bcast_ptr(l_nseg, k);
        const HeadIn hin = load_head(s.sc + slot_in, prev);
        FIBAR_ISSUE_FENCE();
        const TileIn ti = load_tile(s, g, i);
        FIBAR_ISSUE_FENCE();
        int64_t k0;
        uint64_t h0;
        head_after(hin, prev_events, 1, &k0, &h0);
        const uint64_t first = (uint64_t)(k0 + 1) + (uint64_t)sub * kChunk;
        uint32_t dP = 0u, dT = 0u;
        apply_tile(s, g, ti, cd.n, nseg, status != 0, i, first, h0, 1, dP, dT);
        add_counts(stp, false, (uint32_t)sub * kChunk + i, dP, dT);
    }
}

__global__ __launch_bounds__(256) void k_multi_pop(const StreamStep* rr, uint32_t S)
{
    const uint32_t lane = threadIdx.x & 63u;
    const StreamStep* mine = rr + (lane < S ? lane : 0u);
    const LaneState ls = lane_state(rr, S);
    StepScratch* l_step = mine->step;
    const uint32_t l_events = mine->events, l_pop_blocks = mine->pop_blocks;
    const int32_t l_pop_slot = mine->pop_slot;
    uint32_t total;
    const uint32_t le = lane_end(rr, S, 2, &total);
    FIBAR_ISSUE_FENCE();
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        uint32_t start;
        const uint32_t k = owner(le, t, &start);
        const State s = owner_state(ls, k);
        StepScratch* stp = bcast_ptr(l_step, k);
        const uint32_t events = bcast32(l_events, k), pop_blocks = bcast32(l_pop_blocks, k);
        const int32_t pop_slot = (int32_t)bcast32((uint32_t)l_pop_slot, k);
        const uint32_t status = stp->status;
        uint64_t h_old, h_new;
        pop_bounds(s.sc[pop_slot], events, &h_old, &h_new);
        if (status) h_new = h_old;   // a rejected packet pops nothing
        uint32_t dP = 0u, dT = 0u;
        pop_range(s, h_old + (uint64_t)(t - start) * blockDim.x + threadIdx.x, h_new,
                  (uint64_t)pop_blocks * blockDim.x, h_old, dP, dT);
        add_counts(stp, true, (t - start) * blockDim.x + threadIdx.x, dP, dT);
    }
}

__global__ __launch_bounds__(256) void k_multi_readout(const StreamStep* rr, MultiArgs a)
{
    const uint32_t off = rr->ro_off, cnt = rr->ro_cnt;
    for (uint32_t t = blockIdx.x; t < cnt; t += gridDim.x) {
        const RoTask task = a.rot[off + t];
        const MultiReadout ro = a.ros[task.ro];
        const StreamStep* e = rr + task.rec;
        const State s = global_state(e->s);
        int64_t k;
        uint64_t h;
        current_head(s, e->pop_slot, e->step, e->events, 1, &k, &h);
        const uint64_t npx = (uint64_t)s.W * s.H;
        const uint64_t p0 = (uint64_t)task.blk * kReadoutBlock;
        for (uint64_t i = p0 + threadIdx.x; i < npx && i < p0 + kReadoutBlock; i += blockDim.x)
            readout_pixel(s, 1, k, (int64_t)h, i, as_global(ro.L), as_global(ro.pbar),
                          as_global(ro.stale), as_global(ro.cnt), as_global(ro.last),
                          as_global(ro.log_age), as_global(ro.tot));
    }
}

// Copy the records of the graph's rounds (n16 16-byte words from round
// *base of the batch table) into the ring.
__global__ __launch_bounds__(256) void k_multi_stage(const StreamStep* __restrict__ rec,
                                                     StreamStep* __restrict__ ring,
                                                     const uint32_t* __restrict__ base,
                                                     uint32_t S, uint32_t n16)
{
    const uint4* src = reinterpret_cast<const uint4*>(rec + (size_t)*base * S);
    uint4* dst = reinterpret_cast<uint4*>(ring);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_multi_advance(uint32_t* base, uint32_t rounds)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += rounds;
}

// One wave per commit.
__global__ __launch_bounds__(64) void k_multi_commit(const CommitDesc* __restrict__ cd, uint32_t n)
{
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        CommitDesc c = cd[i];
        c.s = global_state(c.s);
        c.prev = as_global(c.prev);
        const DevScalars r = commit_by_wave(c.s.sc + c.slot_in, c.prev, c.prev_events, c.s, 1);
        if (threadIdx.x == 0) store_commit(c.s, c.s.sc + c.slot_out, r, c.prev_events);
    }
}

// Launch configurations the autotuner chooses from: workgroup size,
// workgroups, and whether groups of rounds are replayed as HIP graphs or the
// round kernels are launched one by one.
struct Shape {
    uint32_t block, grid;
    int graph;
};
constexpr Shape kShapes[] = {{128, 512, 1}, {64, 1024, 1}, {128, 1024, 1}, {256, 256, 1},
                             {256, 512, 1}, {128, 512, 0}, {64, 1024, 0}, {128, 1024, 0},
                             {256, 256, 0}, {256, 512, 0}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Launch sequence of a group of rounds: bit 0 = second apply sub-round,
// bit 1 = readouts after the last round.
constexpr int kVariants = 4;

}  // namespace
}  // namespace fibar

using namespace fibar;

struct fibar_multi {
    std::vector<fibar_ctx*> ctx;
    hipStream_t st = nullptr;        // internal stream (graphs are captured on it)
    hipStream_t user = nullptr;      // the caller's stream
    uint32_t n = 0;
    // device tables
    StreamStep* d_rec = nullptr;     // the batch's records, round by round
    StreamStep* d_ring = nullptr;    // the current graph's records
    RoTask* d_rot = nullptr;
    MultiReadout* d_ros = nullptr;
    CommitDesc* d_commits = nullptr;
    ChunkDesc* d_chunks = nullptr;
    SegRec* seg = nullptr;
    uint32_t* seg_count = nullptr;
    StepScratch* scratch = nullptr;
    uint32_t* base = nullptr;
    // host staging (pinned)
    StreamStep* h_rec = nullptr;
    RoTask* h_rot = nullptr;
    MultiReadout* h_ros = nullptr;
    CommitDesc* h_commits = nullptr;
    ChunkDesc* h_chunks = nullptr;
    hipEvent_t staging_free = nullptr;
    hipEvent_t commits_free = nullptr;
    // graphs: [shape][rounds - 1][launch sequence]
    hipGraphExec_t graph[kNumShapes][kUnroll][kVariants] = {};
    // autotuning
    int shape = 0;                 // chosen shape
    int tune = 0;                  // 1: time the candidates on the next submissions
    uint32_t tune_next = 0;        // shape of the next timed group
    double tune_ms[kNumShapes] = {};
    double tune_events[kNumShapes] = {};
    uint32_t tune_groups[kNumShapes] = {};
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
};

namespace {

void multi_free(fibar_multi* m)
{
    if (!m) return;
    if (m->st) (void)hipStreamSynchronize(m->st);
    for (auto& a : m->graph)
        for (auto& b : a)
            for (auto& g : b)
                if (g) (void)hipGraphExecDestroy(g);
    void* dev[] = {m->d_rec, m->d_ring, m->d_rot, m->d_ros, m->d_commits, m->d_chunks,
                   m->seg, m->seg_count, m->scratch, m->base};
    for (void* p : dev) (void)hipFree(p);
    void* host[] = {m->h_rec, m->h_rot, m->h_ros, m->h_commits, m->h_chunks};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (m->staging_free) (void)hipEventDestroy(m->staging_free);
    if (m->commits_free) (void)hipEventDestroy(m->commits_free);
    if (m->ev_a) (void)hipEventDestroy(m->ev_a);
    if (m->ev_b) (void)hipEventDestroy(m->ev_b);
    if (m->st) (void)hipStreamDestroy(m->st);
    delete m;
}

MultiArgs multi_args(const fibar_multi* m)
{
    return MultiArgs{m->d_rot, m->d_ros, m->n};
}

// Queue the kernels of `rounds` rounds with launch sequence `var` whose
// records start at `rec` (stride S).
// With the host copy of the records (direct launches), every launch gets one
// workgroup per task of its round, so no workgroup takes a second task (a
// second dependent chain); a graph's launches keep the shape's fixed grid.
void launch_round_kernels(fibar_multi* m, const Shape& sh, const StreamStep* rec,
                          const StreamStep* host_rec, uint32_t rounds, int var)
{
    const MultiArgs a = multi_args(m);
    auto grid = [&](uint32_t j, int kind) -> uint32_t {
        if (!host_rec) return sh.grid;
        const StreamStep& last = host_rec[(size_t)j * m->n + (m->n - 1)];
        const uint32_t tasks = kind < kKinds ? last.end[kind] : host_rec[(size_t)j * m->n].ro_cnt;
        return std::min<uint32_t>(std::max<uint32_t>(tasks, 1u), kMaxDirectGrid);
    };
    for (uint32_t j = 0; j < rounds; ++j) {
        const StreamStep* rr = rec + (size_t)j * m->n;
        hipLaunchKernelGGL(k_multi_apply, dim3(grid(j, 0)), dim3(sh.block), 0, m->st, rr, a.S, 0);
        if (var & 1)
            hipLaunchKernelGGL(k_multi_apply, dim3(grid(j, 1)), dim3(sh.block), 0, m->st, rr, a.S, 1);
        hipLaunchKernelGGL(k_multi_pop, dim3(grid(j, 2)), dim3(sh.block), 0, m->st, rr, a.S);
    }
    if (var & 2)
        hipLaunchKernelGGL(k_multi_readout, dim3(grid(rounds - 1, kKinds)), dim3(sh.block), 0,
                           m->st, rec + (size_t)(rounds - 1) * m->n, a);
}

// The launches of a graph: stage the records, the rounds on the ring, advance.
hipError_t launch_rounds(fibar_multi* m, const Shape& sh, uint32_t rounds, int var)
{
    const uint32_t n16 = (uint32_t)(rounds * m->n * sizeof(StreamStep) / 16);
    hipLaunchKernelGGL(k_multi_stage, dim3(std::min<uint32_t>(64, (n16 + 255) / 256)), dim3(256), 0,
                       m->st, m->d_rec, m->d_ring, m->base, m->n, n16);
    launch_round_kernels(m, sh, m->d_ring, nullptr, rounds, var);
    hipLaunchKernelGGL(k_multi_advance, dim3(1), dim3(64), 0, m->st, m->base, rounds);
    return hipGetLastError();
}

hipError_t rounds_graph(fibar_multi* m, int shape, uint32_t rounds, int var, hipGraphExec_t* out)
{
    hipGraphExec_t& g = m->graph[shape][rounds - 1][var];
    if (!g) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(m->st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = launch_rounds(m, kShapes[shape], rounds, var);
        e = hipStreamEndCapture(m->st, &graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
    }
    *out = g;
    return hipSuccess;
}

// Per-stream execution state while a submission is planned.
struct StreamPlan {
    const fibar_op* ops = nullptr;
    size_t n_ops = 0, next = 0;      // next op to plan
    int cur_slot = 0;
    uint32_t pend_idx = kNone;       // scratch slot of the pending step
    uint32_t pend_events = 0;
};

// Pending steps at the end of a batch are committed in one launch.
int commit_pending(fibar_multi* m, std::vector<StreamPlan>& plans)
{
    // the staged descriptors of the previous batch's commits must have been
    // copied before they are overwritten
    HIP_TRY(hipEventSynchronize(m->commits_free));
    uint32_t nc = 0;
    for (uint32_t i = 0; i < m->n; ++i) {
        StreamPlan& p = plans[i];
        if (p.pend_idx == kNone) continue;
        CommitDesc& c = m->h_commits[nc++];
        c.s = m->ctx[i]->s;
        c.prev = m->scratch + p.pend_idx;
        c.prev_events = p.pend_events;
        c.slot_in = p.cur_slot;
        c.slot_out = p.cur_slot ^ 1;
        p.cur_slot ^= 1;
        p.pend_idx = kNone;
    }
    if (nc) {
        HIP_TRY(hipMemcpyAsync(m->d_commits, m->h_commits, nc * sizeof(CommitDesc),
                               hipMemcpyHostToDevice, m->st));
        HIP_TRY(hipEventRecord(m->commits_free, m->st));
        hipLaunchKernelGGL(k_multi_commit, dim3(nc), dim3(64), 0, m->st, m->d_commits, nc);
        HIP_TRY(hipGetLastError());
    }
    return FIBAR_OK;
}

// Plan and run one batch: as many rounds as fit the batch buffers.
// *done is set when every stream's ops are consumed.
int run_multi_batch(fibar_multi* m, std::vector<StreamPlan>& plans, bool* done)
{
    HIP_TRY(hipEventSynchronize(m->staging_free));
    const uint32_t S = m->n;
    uint32_t n_chunks = 0, n_steps = 0, n_rounds = 0, n_ro = 0, n_rot = 0;
    struct PendingChunk {
        uint32_t round, rec, sub;
        ChunkDesc d;
    };
    std::vector<std::vector<PendingChunk>> chunks_of(S);
    std::vector<int> round_var;
    std::vector<uint64_t> round_events;
    *done = true;
    for (;;) {
        bool more = false;
        uint32_t need_chunks = 0, need_ro = 0, need_rot = 0;
        for (uint32_t i = 0; i < S; ++i) {
            const StreamPlan& p = plans[i];
            if (p.next >= p.n_ops) continue;
            more = true;
            need_chunks += (uint32_t)((p.ops[p.next].packet.n + kChunk - 1) / kChunk);
            for (size_t q = p.next + 1; q < p.n_ops && p.ops[q].kind == FIBAR_OP_READOUT; ++q) {
                ++need_ro;
                need_rot += (uint32_t)((m->ctx[i]->npx + kReadoutBlock - 1) / kReadoutBlock);
            }
        }
        if (!more) break;
        if (n_rounds == kMultiMaxRounds || n_chunks + need_chunks > kMultiChunks ||
            n_ro + need_ro > kMultiMaxReadouts || n_rot + need_rot > kMultiMaxRoTasks) {
            *done = false;
            break;
        }
        const uint32_t ro_off = n_rot;
        uint64_t ev = 0;
        int var = 0;
        uint32_t nrec = 0;
        for (uint32_t i = 0; i < S; ++i) {
            StreamPlan& p = plans[i];
            if (p.next >= p.n_ops) continue;         // this stream is done
            const fibar_packet& pk = p.ops[p.next].packet;
            ++p.next;
            const uint32_t k = nrec++;
            StreamStep& e = m->h_rec[(size_t)n_rounds * S + k];
            memset(&e, 0, sizeof(e));
            e.s = m->ctx[i]->s;
            const uint32_t nev = (uint32_t)pk.n;
            ev += nev;
            e.events = nev;
            const uint32_t step_idx = n_steps++;
            e.step = m->scratch + step_idx;
            const uint32_t nch = (nev + kChunk - 1) / kChunk;
            for (uint32_t c = 0; c < nch; ++c) {
                PendingChunk pc;
                const uint32_t off = c * kChunk;
                pc.round = n_rounds;
                pc.rec = k;
                pc.sub = c;
                pc.d.x = pk.x + off;
                pc.d.y = pk.y + off;
                pc.d.p = pk.p + off;
                pc.d.n = nev - off < (uint32_t)kChunk ? nev - off : (uint32_t)kChunk;
                pc.d.pkt = step_idx;
                e.chunk[c] = pc.d;
                chunks_of[i].push_back(pc);
                ++n_chunks;
            }
            e.prev = p.pend_idx == kNone ? nullptr : m->scratch + p.pend_idx;
            e.prev_events = p.pend_events;
            e.slot_in = p.cur_slot;
            e.slot_out = -1;
            if (p.pend_idx != kNone) {
                e.slot_out = p.cur_slot ^ 1;
                p.cur_slot ^= 1;
            }
            e.pop_slot = p.cur_slot;
            if (nch == 2) var |= 1;
            p.pend_idx = step_idx;
            p.pend_events = nev;
            while (p.next < p.n_ops && p.ops[p.next].kind == FIBAR_OP_READOUT) {
                const fibar_readout_buf& rb = p.ops[p.next].readout;
                MultiReadout& ro = m->h_ros[n_ro];
                ro.L = rb.brightness;
                ro.pbar = rb.pbar;
                ro.stale = rb.stale_mask;
                ro.cnt = rb.active_count;
                ro.last = rb.last_index;
                ro.log_age = rb.log_age;
                ro.tot = rb.total_count;
                for (uint64_t blk = 0; blk * kReadoutBlock < m->ctx[i]->npx; ++blk)
                    m->h_rot[n_rot++] = RoTask{k, n_ro, (uint32_t)blk, 0u};
                ++n_ro;
                ++p.next;
                var |= 2;
            }
        }
        for (uint32_t k = nrec; k < S; ++k)
            memset(&m->h_rec[(size_t)n_rounds * S + k], 0, sizeof(StreamStep));
        m->h_rec[(size_t)n_rounds * S].ro_off = ro_off;
        m->h_rec[(size_t)n_rounds * S].ro_cnt = n_rot - ro_off;
        round_var.push_back(var);
        round_events.push_back(ev);
        ++n_rounds;
    }
    if (n_rounds == 0) return FIBAR_OK;

    // Groups of rounds replayed as one graph: at most kUnroll rounds
    // (kTuneLen while tuning, each group with the next candidate shape) of
    // the same second-sub-round flag, ending at the first round with
    // readouts.
    struct Group {
        uint32_t r0, len;
        int shape, var;
        uint64_t events;
    };
    std::vector<Group> groups;
    for (uint32_t r = 0; r < n_rounds;) {
        const int two = round_var[r] & 1;
        const int shape = m->tune ? (int)(m->tune_next++ % kNumShapes) : m->shape;
        const uint32_t cap = m->tune ? kTuneLen : kUnroll;
        Group g{r, 0, shape, two, 0};
        while (r < n_rounds && (round_var[r] & 1) == two && g.len < cap) {
            g.events += round_events[r];
            ++g.len;
            const bool ro = round_var[r] & 2;
            ++r;
            if (ro) {
                g.var |= 2;
                break;
            }
        }
        groups.push_back(g);
    }

    // task counts of each round for the workgroup size of its group
    for (const Group& g : groups) {
        const uint32_t B = kShapes[g.shape].block;
        for (uint32_t r = g.r0; r < g.r0 + g.len; ++r) {
            uint32_t acc[kKinds] = {0, 0, 0};
            for (uint32_t k = 0; k < S; ++k) {
                StreamStep& e = m->h_rec[(size_t)r * S + k];
                if (e.events) {
                    // 1/8 headroom for a shrinking target length
                    e.pop_blocks = (e.events + e.events / 8 + B - 1) / B;
                    acc[0] += (e.chunk[0].n + B - 1) / B + (e.prev ? 1u : 0u);
                    acc[1] += (e.chunk[1].n + B - 1) / B;
                    acc[2] += e.pop_blocks;
                }
                // records without a step come last and get the totals
                for (int q = 0; q < kKinds; ++q) e.end[q] = acc[q];
            }
        }
    }

    // chunk records laid out stream by stream, so that one group+compose
    // launch per stream (its own size and filter constants) covers them
    std::vector<uint32_t> first(S + 1, 0);
    uint32_t slot = 0;
    for (uint32_t i = 0; i < S; ++i) {
        first[i] = slot;
        for (const PendingChunk& pc : chunks_of[i]) {
            m->h_chunks[slot] = pc.d;
            StreamStep& e = m->h_rec[(size_t)pc.round * S + pc.rec];
            e.seg[pc.sub] = m->seg + (size_t)slot * kChunk;
            e.nseg[pc.sub] = m->seg_count + slot;
            ++slot;
        }
    }
    first[S] = slot;

    HIP_TRY(hipMemcpyAsync(m->d_chunks, m->h_chunks, n_chunks * sizeof(ChunkDesc),
                           hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipMemcpyAsync(m->d_rec, m->h_rec, (size_t)n_rounds * S * sizeof(StreamStep),
                           hipMemcpyHostToDevice, m->st));
    if (n_rot)
        HIP_TRY(hipMemcpyAsync(m->d_rot, m->h_rot, n_rot * sizeof(RoTask), hipMemcpyHostToDevice,
                               m->st));
    if (n_ro)
        HIP_TRY(hipMemcpyAsync(m->d_ros, m->h_ros, n_ro * sizeof(MultiReadout),
                               hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipEventRecord(m->staging_free, m->st));
    HIP_TRY(hipMemsetAsync(m->scratch, 0, n_steps * sizeof(StepScratch), m->st));
    HIP_TRY(hipMemsetAsync(m->base, 0, sizeof(uint32_t), m->st));

    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t cnt = first[i + 1] - first[i];
        if (!cnt) continue;
        const fibar_ctx* c = m->ctx[i];
        HIP_TRY(launch_sort_compose(m->d_chunks + first[i], cnt, m->seg + (size_t)first[i] * kChunk,
                                    m->seg_count + first[i], m->scratch, c->W, c->H, c->key_bits,
                                    c->coef, c->s.gain, m->st));
    }

    // index of the last group replayed as a graph (the device round index is
    // only read by graphs)
    int last_graph = -1;
    for (size_t q = 0; q < groups.size(); ++q)
        if (kShapes[groups[q].shape].graph) last_graph = (int)q;
    for (size_t q = 0; q < groups.size(); ++q) {
        const Group& g = groups[q];
        hipGraphExec_t ge = nullptr;
        if (kShapes[g.shape].graph) HIP_TRY(rounds_graph(m, g.shape, g.len, g.var, &ge));
        if (m->tune) HIP_TRY(hipEventRecord(m->ev_a, m->st));
        if (ge) {
            HIP_TRY(hipGraphLaunch(ge, m->st));
        } else {
            // direct launches; a later graph's first round index moves past
            // these rounds too
            launch_round_kernels(m, kShapes[g.shape], m->d_rec + (size_t)g.r0 * S,
                                 m->h_rec + (size_t)g.r0 * S, g.len, g.var);
            if ((int)q < last_graph)
                hipLaunchKernelGGL(k_multi_advance, dim3(1), dim3(64), 0, m->st, m->base, g.len);
            HIP_TRY(hipGetLastError());
        }
        if (m->tune) {
            HIP_TRY(hipEventRecord(m->ev_b, m->st));
            HIP_TRY(hipEventSynchronize(m->ev_b));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, m->ev_a, m->ev_b));
            m->tune_ms[g.shape] += ms;
            m->tune_events[g.shape] += (double)g.events;
            ++m->tune_groups[g.shape];
        }
    }
    if (m->tune) {
        // once every shape has run its groups: the fastest time per event
        bool enough = true;
        for (int k = 0; k < kNumShapes; ++k) enough = enough && m->tune_groups[k] >= kTuneGroups;
        if (enough) {
            int best = 0;
            for (int k = 1; k < kNumShapes; ++k)
                if (m->tune_ms[k] / m->tune_events[k] < m->tune_ms[best] / m->tune_events[best])
                    best = k;
            m->shape = best;
            m->tune = 0;
        }
    }
    return commit_pending(m, plans);
}

}  // namespace

extern "C" {

int fibar_multi_create(fibar_ctx* const* ctxs, uint32_t n, void* stream, fibar_multi** out)
{
    if (!out) return FIBAR_E_INVALID_ARG;
    *out = nullptr;
    if (!ctxs || n == 0 || n > kMultiMaxStreams) return FIBAR_E_INVALID_ARG;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return FIBAR_E_INVALID_ARG;
        if (!ctxs[i]->prm.spatial_filter || ctxs[i]->event_mode || ctxs[i]->tq)
            return FIBAR_E_UNSUPPORTED;
        for (uint32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return FIBAR_E_INVALID_ARG;
    }
    fibar_multi* m = new (std::nothrow) fibar_multi();
    if (!m) return FIBAR_E_NOMEM;
    m->ctx.assign(ctxs, ctxs + n);
    m->n = n;
    m->user = (hipStream_t)stream;
    hipError_t e = hipStreamCreate(&m->st);
    auto dalloc = [&](void** p, size_t b) {
        if (e == hipSuccess) e = hipMalloc(p, b);
    };
    auto halloc = [&](void** p, size_t b) {
        if (e == hipSuccess) e = hipHostMalloc(p, b, 0);
    };
    const size_t recs = (size_t)kMultiMaxRounds * n;
    dalloc((void**)&m->d_rec, recs * sizeof(StreamStep));
    dalloc((void**)&m->d_ring, (size_t)kUnroll * n * sizeof(StreamStep));
    dalloc((void**)&m->d_rot, kMultiMaxRoTasks * sizeof(RoTask));
    dalloc((void**)&m->d_ros, kMultiMaxReadouts * sizeof(MultiReadout));
    dalloc((void**)&m->d_commits, kMultiMaxStreams * sizeof(CommitDesc));
    dalloc((void**)&m->d_chunks, kMultiChunks * sizeof(ChunkDesc));
    // 4 spare records: an item reads records up to i + 3 of its chunk
    dalloc((void**)&m->seg, ((size_t)kMultiChunks * kChunk + 4) * sizeof(SegRec));
    dalloc((void**)&m->seg_count, kMultiChunks * sizeof(uint32_t));
    // every step has at least one chunk (empty packets are rejected)
    dalloc((void**)&m->scratch, kMultiChunks * sizeof(StepScratch));
    dalloc((void**)&m->base, sizeof(uint32_t));
    halloc((void**)&m->h_rec, recs * sizeof(StreamStep));
    halloc((void**)&m->h_rot, kMultiMaxRoTasks * sizeof(RoTask));
    halloc((void**)&m->h_ros, kMultiMaxReadouts * sizeof(MultiReadout));
    halloc((void**)&m->h_commits, kMultiMaxStreams * sizeof(CommitDesc));
    halloc((void**)&m->h_chunks, kMultiChunks * sizeof(ChunkDesc));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staging_free, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->commits_free, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&m->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&m->ev_b);
    if (e == hipSuccess) e = hipEventRecord(m->staging_free, m->st);
    if (e == hipSuccess) e = hipEventRecord(m->commits_free, m->st);
    if (e == hipSuccess) e = hipStreamSynchronize(m->st);
    if (e != hipSuccess) {
        multi_free(m);
        return map_err(e);
    }
    *out = m;
    return FIBAR_OK;
}

int fibar_multi_submit(fibar_multi* m, const fibar_op* const* ops, const size_t* n_ops)
{
    if (!m || !ops || !n_ops) return FIBAR_E_INVALID_ARG;
    std::vector<StreamPlan> plans(m->n);
    // check everything before any work is queued
    for (uint32_t i = 0; i < m->n; ++i) {
        fibar_ctx* c = m->ctx[i];
        if (n_ops[i] && !ops[i]) return FIBAR_E_INVALID_ARG;
        uint64_t t_hi = c->t_hi;
        for (size_t j = 0; j < n_ops[i]; ++j) {
            const fibar_op& op = ops[i][j];
            if (op.kind == FIBAR_OP_PUSH) {
                const fibar_packet& pk = op.packet;
                if (pk.n == 0 || pk.n > c->prm.max_packet || pk.n > 2u * kChunk || !pk.on_device ||
                    !pk.x || !pk.y || !pk.p)
                    return FIBAR_E_INVALID_ARG;
            } else if (op.kind == FIBAR_OP_READOUT) {
                const fibar_readout_buf& rb = op.readout;
                if (j == 0 || !rb.brightness || !rb.on_device) return FIBAR_E_INVALID_ARG;
                if (rb.tile_count) return FIBAR_E_UNSUPPORTED;
                if (op.t < t_hi) return FIBAR_E_TIME;
                t_hi = op.t;
            } else {
                return FIBAR_E_INVALID_ARG;
            }
        }
        plans[i].ops = ops[i];
        plans[i].n_ops = n_ops[i];
        plans[i].cur_slot = c->cur_slot;
    }
    // work already queued on the caller's and the contexts' streams first
    HIP_TRY(hipEventRecord(m->ev_a, m->user));
    HIP_TRY(hipStreamWaitEvent(m->st, m->ev_a, 0));
    for (uint32_t i = 0; i < m->n; ++i) HIP_TRY(hipStreamSynchronize(m->ctx[i]->st));
    bool done = false;
    while (!done) {
        int rc = run_multi_batch(m, plans, &done);
        if (rc) return rc;
    }
    for (uint32_t i = 0; i < m->n; ++i) {
        fibar_ctx* c = m->ctx[i];
        c->cur_slot = plans[i].cur_slot;
        for (size_t j = 0; j < n_ops[i]; ++j)
            if (ops[i][j].kind == FIBAR_OP_READOUT) c->t_hi = ops[i][j].t;
    }
    // later work on the caller's stream and the contexts' streams runs after
    HIP_TRY(hipEventRecord(m->ev_b, m->st));
    HIP_TRY(hipStreamWaitEvent(m->user, m->ev_b, 0));
    for (uint32_t i = 0; i < m->n; ++i) HIP_TRY(hipStreamWaitEvent(m->ctx[i]->st, m->ev_b, 0));
    return FIBAR_OK;
}

int fibar_multi_autotune(fibar_multi* m)
{
    if (!m) return FIBAR_E_INVALID_ARG;
    m->tune = 1;
    m->tune_next = 0;
    for (int k = 0; k < kNumShapes; ++k) {
        m->tune_ms[k] = m->tune_events[k] = 0.0;
        m->tune_groups[k] = 0;
    }
    return FIBAR_OK;
}

int fibar_multi_get_shape(fibar_multi* m, uint32_t* block, uint32_t* grid)
{
    if (!m || !block || !grid) return FIBAR_E_INVALID_ARG;
    *block = kShapes[m->shape].block;
    *grid = kShapes[m->shape].grid;
    return FIBAR_OK;
}

int fibar_multi_get_config(fibar_multi* m, uint32_t* index)
{
    if (!m || !index) return FIBAR_E_INVALID_ARG;
    *index = (uint32_t)m->shape;
    return FIBAR_OK;
}

int fibar_multi_set_shape(fibar_multi* m, uint32_t index)
{
    if (!m || index >= (uint32_t)kNumShapes) return FIBAR_E_INVALID_ARG;
    m->shape = (int)index;
    m->tune = 0;
    return FIBAR_OK;
}

void fibar_multi_destroy(fibar_multi* m) { multi_free(m); }

}  // extern "C"
