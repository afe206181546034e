// Multi-stream executor of libfibar: many independent event streams (each a
// fibar_ctx with its own resolution, packet sizes and state) advance
// together, one packet per stream per round.
//
// A round is a fixed sequence of launches shared by every stream:
//   k_multi_apply (sub-round 0, and sub-round 1 when a packet has a second
//   chunk), k_multi_pop, k_multi_readout, k_multi_advance.
// Each of them consumes the round's device task list -- (stream, slice)
// tasks of equal size, planned on the host -- with a fixed number of resident
// workgroups, workgroup w taking tasks w, w + grid, w + 2 grid, ...  (a
// shared dequeue counter would serialise: same-address atomics cost ~10 ns
// each), so streams of different sizes share the GPU without a launch per
// stream.  Every launch reads the round index from device memory; the round
// is captured once as a HIP graph and replayed for every round.  Within a
// stream the order of steps is the single-stream order (apply, pop/blur,
// lagged commit), so results are identical to running each stream alone.
//
// The launch shape (workgroup size, number of resident workgroups) does not
// change any result: only integer atomics are reordered and every float is
// computed from the same operands.  The autotuner times the candidate shapes
// on the first rounds of a submission and keeps the fastest.
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

constexpr uint32_t kMultiMaxStreams = 64;
constexpr uint32_t kMultiChunks = 1024;        // chunks grouped per multi batch
constexpr uint32_t kMultiMaxRounds = 1024;
constexpr uint32_t kMultiMaxReadouts = 1024;
constexpr uint32_t kMultiMaxTasks = 1u << 20;  // per task kind per batch
constexpr uint32_t kReadoutBlock = 4096;       // pixels per readout task
constexpr uint32_t kNone = 0xffffffffu;

// One stream's step in one round.
struct MultiStep {
    ChunkDesc chunk[2];
    uint32_t seg_chunk[2];   // chunk slot in the batch's record buffer
    uint32_t n_chunks;       // 0: the stream has no step in this round
    uint32_t events;
    uint32_t step_idx;       // scratch slot of this step
    uint32_t prev_idx;       // scratch slot of the pending step, or kNone
    uint32_t prev_events;
    uint32_t pop_blocks;     // virtual workgroups sharing this step's pops
    int32_t slot_in, slot_out, pop_slot;
    uint32_t pad;
};

struct RoundDesc {
    uint32_t apply_off[2], apply_cnt[2];
    uint32_t pop_off, pop_cnt;
    uint32_t ro_off, ro_cnt;
    uint32_t step_off;       // MultiStep of stream 0 in this round
    uint32_t pad;
};

struct Task {
    uint32_t stream;
    uint32_t idx;            // apply: item block (kNone = commit); pop: virtual block;
                             // readout: readout slot in the high bits, pixel block low
};

struct MultiReadout {
    uint32_t stream;
    uint32_t pad;
    float* L;
    float* pbar;
    uint8_t* stale;
    uint32_t* cnt;
    int64_t* last;
    float* log_age;
};

struct CommitDesc {
    uint32_t stream;
    uint32_t prev_idx;
    uint32_t prev_events;
    int32_t slot_in, slot_out;
};

struct MultiCtl {
    const State* states;
    const MultiStep* steps;
    const RoundDesc* rounds;
    const Task* apply_tasks;
    const Task* pop_tasks;
    const Task* ro_tasks;
    const MultiReadout* ros;
    const SegRec* seg;
    const uint32_t* seg_count;
    StepScratch* scratch;
    uint32_t* round;
};

__global__ __launch_bounds__(256) void k_multi_apply(const MultiCtl* __restrict__ ctl, int sub)
{
    const uint32_t r = *ctl->round;
    const RoundDesc rd = ctl->rounds[r];
    for (uint32_t t = blockIdx.x; t < rd.apply_cnt[sub]; t += gridDim.x) {
        const Task task = ctl->apply_tasks[rd.apply_off[sub] + t];
        const MultiStep& st = ctl->steps[rd.step_off + task.stream];
        const State s = ctl->states[task.stream];
        const StepScratch* prev = st.prev_idx == kNone ? nullptr : ctl->scratch + st.prev_idx;
        if (task.idx == kNone) {
            if (threadIdx.x == 0 && prev && st.slot_out >= 0)
                s.sc[st.slot_out] = commit_step(s.sc[st.slot_in], prev, st.prev_events, s, 1);
            continue;
        }
        StepScratch* stp = ctl->scratch + st.step_idx;
        if (stp->status) continue;
        int64_t k0;
        uint64_t h0;
        current_head(s, st.slot_in, prev, st.prev_events, 1, &k0, &h0);
        const uint64_t first = (uint64_t)(k0 + 1) + (uint64_t)sub * kChunk;
        const uint32_t i = task.idx * blockDim.x + threadIdx.x;
        const uint32_t sc = st.seg_chunk[sub];
        uint32_t dP = 0u, dT = 0u;
        apply_item(s, st.chunk[sub], ctl->seg + (size_t)sc * kChunk, ctl->seg_count[sc], i, first,
                   h0, 1, dP, dT);
        add_counts(stp, 0, dP, dT);
    }
}

__global__ __launch_bounds__(256) void k_multi_pop(const MultiCtl* __restrict__ ctl)
{
    const uint32_t r = *ctl->round;
    const RoundDesc rd = ctl->rounds[r];
    for (uint32_t t = blockIdx.x; t < rd.pop_cnt; t += gridDim.x) {
        const Task task = ctl->pop_tasks[rd.pop_off + t];
        const MultiStep& st = ctl->steps[rd.step_off + task.stream];
        StepScratch* stp = ctl->scratch + st.step_idx;
        if (stp->status) continue;
        const State s = ctl->states[task.stream];
        uint64_t h_old, h_new;
        pop_bounds(s.sc[st.pop_slot], st.events, &h_old, &h_new);
        uint32_t dP = 0u, dT = 0u;
        pop_range(s, h_old + (uint64_t)task.idx * blockDim.x + threadIdx.x, h_new,
                  (uint64_t)st.pop_blocks * blockDim.x, h_old, dP, dT);
        add_counts(stp, 2, dP, dT);
    }
}

__global__ __launch_bounds__(256) void k_multi_readout(const MultiCtl* __restrict__ ctl)
{
    const uint32_t r = *ctl->round;
    const RoundDesc rd = ctl->rounds[r];
    for (uint32_t t = blockIdx.x; t < rd.ro_cnt; t += gridDim.x) {
        const Task task = ctl->ro_tasks[rd.ro_off + t];
        const MultiReadout ro = ctl->ros[task.idx >> 12];
        const MultiStep& st = ctl->steps[rd.step_off + ro.stream];
        const State s = ctl->states[ro.stream];
        int64_t k;
        uint64_t h;
        current_head(s, st.pop_slot, ctl->scratch + st.step_idx, st.events, 1, &k, &h);
        const uint64_t npx = (uint64_t)s.W * s.H;
        const uint64_t p0 = (uint64_t)(task.idx & 0xfffu) * kReadoutBlock;
        for (uint64_t i = p0 + threadIdx.x; i < npx && i < p0 + kReadoutBlock; i += blockDim.x)
            readout_pixel(s, 1, k, (int64_t)h, i, ro.L, ro.pbar, ro.stale, ro.cnt, ro.last,
                          ro.log_age);
    }
}

__global__ void k_multi_advance(const MultiCtl* __restrict__ ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctl->round += 1u;
}

__global__ void k_multi_commit(const MultiCtl* __restrict__ ctl, const CommitDesc* __restrict__ cd,
                               uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CommitDesc c = cd[i];
    const State s = ctl->states[c.stream];
    s.sc[c.slot_out] = commit_step(s.sc[c.slot_in], ctl->scratch + c.prev_idx, c.prev_events, s, 1);
}

// Launch shapes the autotuner chooses from: (workgroup size, workgroups).
struct Shape {
    uint32_t block, grid;
};
constexpr Shape kShapes[] = {{128, 512}, {64, 1024}, {128, 1024}, {256, 256}, {256, 512}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

}  // namespace
}  // namespace fibar

using namespace fibar;

struct fibar_multi {
    std::vector<fibar_ctx*> ctx;
    hipStream_t st = nullptr;        // internal stream (graphs are captured on it)
    hipStream_t user = nullptr;      // the caller's stream
    uint32_t n = 0;
    // device tables
    State* d_states = nullptr;
    MultiStep* d_steps = nullptr;
    RoundDesc* d_rounds = nullptr;
    Task* d_apply = nullptr;
    Task* d_pop = nullptr;
    Task* d_rot = nullptr;
    MultiReadout* d_ros = nullptr;
    CommitDesc* d_commits = nullptr;
    ChunkDesc* d_chunks = nullptr;
    SegRec* seg = nullptr;
    uint32_t* seg_count = nullptr;
    StepScratch* scratch = nullptr;
    uint32_t* round = nullptr;
    MultiCtl* d_ctl = nullptr;
    // host staging (pinned)
    MultiStep* h_steps = nullptr;
    RoundDesc* h_rounds = nullptr;
    Task* h_apply = nullptr;
    Task* h_pop = nullptr;
    Task* h_rot = nullptr;
    MultiReadout* h_ros = nullptr;
    CommitDesc* h_commits = nullptr;
    ChunkDesc* h_chunks = nullptr;
    hipEvent_t staging_free = nullptr;
    // graphs: [shape][with second apply sub-round]
    hipGraphExec_t graph[kNumShapes][2] = {};
    // autotuning
    int shape = 0;                 // chosen shape
    int tune = 0;                  // 1: time the candidates on the next submission
    double tune_ms[kNumShapes] = {};
    double tune_events[kNumShapes] = {};
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
};

namespace {

void multi_free(fibar_multi* m)
{
    if (!m) return;
    if (m->st) (void)hipStreamSynchronize(m->st);
    for (auto& g : m->graph)
        for (auto& e : g)
            if (e) (void)hipGraphExecDestroy(e);
    void* dev[] = {m->d_states, m->d_steps, m->d_rounds, m->d_apply, m->d_pop, m->d_rot,
                   m->d_ros, m->d_commits, m->d_chunks, m->seg, m->seg_count, m->scratch,
                   m->round, m->d_ctl};
    for (void* p : dev) (void)hipFree(p);
    void* host[] = {m->h_steps, m->h_rounds, m->h_apply, m->h_pop, m->h_rot, m->h_ros,
                    m->h_commits, m->h_chunks};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (m->staging_free) (void)hipEventDestroy(m->staging_free);
    if (m->ev_a) (void)hipEventDestroy(m->ev_a);
    if (m->ev_b) (void)hipEventDestroy(m->ev_b);
    if (m->st) (void)hipStreamDestroy(m->st);
    delete m;
}

// Launch one round (not captured) with a given shape.
hipError_t launch_round(fibar_multi* m, const Shape& sh, bool two)
{
    hipLaunchKernelGGL(k_multi_apply, dim3(sh.grid), dim3(sh.block), 0, m->st, m->d_ctl, 0);
    if (two) hipLaunchKernelGGL(k_multi_apply, dim3(sh.grid), dim3(sh.block), 0, m->st, m->d_ctl, 1);
    hipLaunchKernelGGL(k_multi_pop, dim3(sh.grid), dim3(sh.block), 0, m->st, m->d_ctl);
    hipLaunchKernelGGL(k_multi_readout, dim3(sh.grid), dim3(sh.block), 0, m->st, m->d_ctl);
    hipLaunchKernelGGL(k_multi_advance, dim3(1), dim3(64), 0, m->st, m->d_ctl);
    return hipGetLastError();
}

hipError_t round_graph(fibar_multi* m, int shape, bool two, hipGraphExec_t* out)
{
    hipGraphExec_t& g = m->graph[shape][two ? 1 : 0];
    if (!g) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(m->st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = launch_round(m, kShapes[shape], two);
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
    uint32_t nc = 0;
    for (uint32_t i = 0; i < m->n; ++i) {
        StreamPlan& p = plans[i];
        if (p.pend_idx == kNone) continue;
        CommitDesc& c = m->h_commits[nc++];
        c.stream = i;
        c.prev_idx = p.pend_idx;
        c.prev_events = p.pend_events;
        c.slot_in = p.cur_slot;
        c.slot_out = p.cur_slot ^ 1;
        p.cur_slot ^= 1;
        p.pend_idx = kNone;
    }
    if (nc) {
        HIP_TRY(hipMemcpyAsync(m->d_commits, m->h_commits, nc * sizeof(CommitDesc),
                               hipMemcpyHostToDevice, m->st));
        hipLaunchKernelGGL(k_multi_commit, dim3((nc + 63) / 64), dim3(64), 0, m->st, m->d_ctl,
                           m->d_commits, nc);
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
    uint32_t n_chunks = 0, n_steps = 0, n_rounds = 0, n_ro = 0;
    uint32_t n_apply = 0, n_pop = 0, n_rot = 0;
    uint64_t events_in_group[kNumShapes] = {};
    bool any_two = false;
    struct PendingChunk {
        uint32_t round, sub;
        ChunkDesc d;
    };
    std::vector<std::vector<PendingChunk>> chunks_of(S);
    std::vector<int> round_shape;
    std::vector<uint64_t> round_events;
    const uint32_t tune_group = 4;   // rounds per candidate shape while tuning
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
            n_ro + need_ro > kMultiMaxReadouts || n_apply + need_chunks * kChunk + S > kMultiMaxTasks ||
            n_pop + need_chunks * kChunk + S > kMultiMaxTasks || n_rot + need_rot > kMultiMaxTasks) {
            *done = false;
            break;
        }
        const int shape = m->tune ? (int)((n_rounds / tune_group) % kNumShapes) : m->shape;
        const uint32_t B = kShapes[shape].block;
        RoundDesc& rd = m->h_rounds[n_rounds];
        memset(&rd, 0, sizeof(rd));
        rd.step_off = n_rounds * S;
        rd.apply_off[0] = n_apply;
        rd.pop_off = n_pop;
        rd.ro_off = n_rot;
        uint64_t ev = 0;
        std::vector<Task> second;
        for (uint32_t i = 0; i < S; ++i) {
            StreamPlan& p = plans[i];
            MultiStep& st = m->h_steps[n_rounds * S + i];
            memset(&st, 0, sizeof(st));
            st.prev_idx = kNone;
            st.slot_out = -1;
            if (p.next >= p.n_ops) continue;         // this stream is done
            const fibar_packet& pk = p.ops[p.next].packet;
            ++p.next;
            const uint32_t nev = (uint32_t)pk.n;
            ev += nev;
            st.events = nev;
            st.n_chunks = (nev + kChunk - 1) / kChunk;
            st.step_idx = n_steps++;
            for (uint32_t c = 0; c < st.n_chunks; ++c) {
                PendingChunk pc;
                const uint32_t off = c * kChunk;
                pc.round = n_rounds;
                pc.sub = c;
                pc.d.x = pk.x + off;
                pc.d.y = pk.y + off;
                pc.d.p = pk.p + off;
                pc.d.n = nev - off < (uint32_t)kChunk ? nev - off : (uint32_t)kChunk;
                pc.d.pkt = st.step_idx;
                st.chunk[c] = pc.d;
                chunks_of[i].push_back(pc);
                ++n_chunks;
            }
            st.prev_idx = p.pend_idx;
            st.prev_events = p.pend_events;
            st.slot_in = p.cur_slot;
            if (p.pend_idx != kNone) {
                st.slot_out = p.cur_slot ^ 1;
                m->h_apply[n_apply++] = Task{i, kNone};   // commit of the previous step
                ++rd.apply_cnt[0];
                p.cur_slot ^= 1;
            }
            st.pop_slot = p.cur_slot;
            for (uint32_t b = 0; b * B < st.chunk[0].n; ++b) {
                m->h_apply[n_apply++] = Task{i, b};
                ++rd.apply_cnt[0];
            }
            if (st.n_chunks == 2) {
                any_two = true;
                for (uint32_t b = 0; b * B < st.chunk[1].n; ++b) second.push_back(Task{i, b});
            }
            st.pop_blocks = std::max<uint32_t>(1, (nev + B - 1) / B);
            for (uint32_t v = 0; v < st.pop_blocks; ++v) {
                m->h_pop[n_pop++] = Task{i, v};
                ++rd.pop_cnt;
            }
            p.pend_idx = st.step_idx;
            p.pend_events = nev;
            while (p.next < p.n_ops && p.ops[p.next].kind == FIBAR_OP_READOUT) {
                const fibar_readout_buf& rb = p.ops[p.next].readout;
                MultiReadout& ro = m->h_ros[n_ro];
                ro.stream = i;
                ro.pad = 0;
                ro.L = rb.brightness;
                ro.pbar = rb.pbar;
                ro.stale = rb.stale_mask;
                ro.cnt = rb.active_count;
                ro.last = rb.last_index;
                ro.log_age = rb.log_age;
                for (uint64_t blk = 0; blk * kReadoutBlock < m->ctx[i]->npx; ++blk) {
                    m->h_rot[n_rot++] = Task{i, (n_ro << 12) | (uint32_t)blk};
                    ++rd.ro_cnt;
                }
                ++n_ro;
                ++p.next;
            }
        }
        rd.apply_off[1] = n_apply;
        for (const Task& t : second) m->h_apply[n_apply++] = t;
        rd.apply_cnt[1] = (uint32_t)second.size();
        round_shape.push_back(shape);
        round_events.push_back(ev);
        ++n_rounds;
    }
    if (n_rounds == 0) return FIBAR_OK;

    // chunk records laid out stream by stream, so that one group+compose
    // launch per stream (its own size and filter constants) covers them
    std::vector<uint32_t> first(S + 1, 0);
    uint32_t slot = 0;
    for (uint32_t i = 0; i < S; ++i) {
        first[i] = slot;
        for (const PendingChunk& pc : chunks_of[i]) {
            m->h_chunks[slot] = pc.d;
            m->h_steps[pc.round * S + i].seg_chunk[pc.sub] = slot;
            ++slot;
        }
    }
    first[S] = slot;

    HIP_TRY(hipMemcpyAsync(m->d_chunks, m->h_chunks, n_chunks * sizeof(ChunkDesc),
                           hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipMemcpyAsync(m->d_steps, m->h_steps, (size_t)n_rounds * S * sizeof(MultiStep),
                           hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipMemcpyAsync(m->d_rounds, m->h_rounds, n_rounds * sizeof(RoundDesc),
                           hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipMemcpyAsync(m->d_apply, m->h_apply, n_apply * sizeof(Task), hipMemcpyHostToDevice,
                           m->st));
    HIP_TRY(hipMemcpyAsync(m->d_pop, m->h_pop, n_pop * sizeof(Task), hipMemcpyHostToDevice, m->st));
    if (n_rot)
        HIP_TRY(hipMemcpyAsync(m->d_rot, m->h_rot, n_rot * sizeof(Task), hipMemcpyHostToDevice, m->st));
    if (n_ro)
        HIP_TRY(hipMemcpyAsync(m->d_ros, m->h_ros, n_ro * sizeof(MultiReadout),
                               hipMemcpyHostToDevice, m->st));
    HIP_TRY(hipEventRecord(m->staging_free, m->st));
    HIP_TRY(hipMemsetAsync(m->scratch, 0, n_steps * sizeof(StepScratch), m->st));
    HIP_TRY(hipMemsetAsync(m->round, 0, sizeof(uint32_t), m->st));

    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t cnt = first[i + 1] - first[i];
        if (!cnt) continue;
        const fibar_ctx* c = m->ctx[i];
        HIP_TRY(launch_sort_compose(m->d_chunks + first[i], cnt, m->seg + (size_t)first[i] * kChunk,
                                    m->seg_count + first[i], m->scratch, c->W, c->H, c->key_bits,
                                    c->coef, m->st));
    }

    // the rounds: one graph replay each
    for (uint32_t r = 0; r < n_rounds;) {
        const int shape = round_shape[r];
        uint32_t r1 = r;
        uint64_t ev = 0;
        while (r1 < n_rounds && round_shape[r1] == shape) ev += round_events[r1++];
        hipGraphExec_t g = nullptr;
        HIP_TRY(round_graph(m, shape, any_two, &g));
        if (m->tune) HIP_TRY(hipEventRecord(m->ev_a, m->st));
        for (uint32_t q = r; q < r1; ++q) HIP_TRY(hipGraphLaunch(g, m->st));
        if (m->tune) {
            HIP_TRY(hipEventRecord(m->ev_b, m->st));
            HIP_TRY(hipEventSynchronize(m->ev_b));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, m->ev_a, m->ev_b));
            m->tune_ms[shape] += ms;
            m->tune_events[shape] += (double)ev;
            events_in_group[shape] += ev;
        }
        r = r1;
    }
    if (m->tune) {
        // fastest time per event over the rounds each shape ran
        int best = -1;
        double best_rate = 0.0;
        for (int k = 0; k < kNumShapes; ++k) {
            if (!events_in_group[k]) continue;
            const double rate = m->tune_ms[k] / m->tune_events[k];
            if (best < 0 || rate < best_rate) {
                best = k;
                best_rate = rate;
            }
        }
        if (best >= 0) {
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
        if (!ctxs[i]->prm.spatial_filter) return FIBAR_E_UNSUPPORTED;
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
    const size_t steps = (size_t)kMultiMaxRounds * n;
    dalloc((void**)&m->d_states, n * sizeof(State));
    dalloc((void**)&m->d_steps, steps * sizeof(MultiStep));
    dalloc((void**)&m->d_rounds, kMultiMaxRounds * sizeof(RoundDesc));
    dalloc((void**)&m->d_apply, kMultiMaxTasks * sizeof(Task));
    dalloc((void**)&m->d_pop, kMultiMaxTasks * sizeof(Task));
    dalloc((void**)&m->d_rot, kMultiMaxTasks * sizeof(Task));
    dalloc((void**)&m->d_ros, kMultiMaxReadouts * sizeof(MultiReadout));
    dalloc((void**)&m->d_commits, kMultiMaxStreams * sizeof(CommitDesc));
    dalloc((void**)&m->d_chunks, kMultiChunks * sizeof(ChunkDesc));
    dalloc((void**)&m->seg, (size_t)kMultiChunks * kChunk * sizeof(SegRec));
    dalloc((void**)&m->seg_count, kMultiChunks * sizeof(uint32_t));
    dalloc((void**)&m->scratch, steps * sizeof(StepScratch));
    dalloc((void**)&m->round, sizeof(uint32_t));
    dalloc((void**)&m->d_ctl, sizeof(MultiCtl));
    halloc((void**)&m->h_steps, steps * sizeof(MultiStep));
    halloc((void**)&m->h_rounds, kMultiMaxRounds * sizeof(RoundDesc));
    halloc((void**)&m->h_apply, kMultiMaxTasks * sizeof(Task));
    halloc((void**)&m->h_pop, kMultiMaxTasks * sizeof(Task));
    halloc((void**)&m->h_rot, kMultiMaxTasks * sizeof(Task));
    halloc((void**)&m->h_ros, kMultiMaxReadouts * sizeof(MultiReadout));
    halloc((void**)&m->h_commits, kMultiMaxStreams * sizeof(CommitDesc));
    halloc((void**)&m->h_chunks, kMultiChunks * sizeof(ChunkDesc));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staging_free, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&m->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&m->ev_b);
    if (e != hipSuccess) {
        multi_free(m);
        return map_err(e);
    }
    std::vector<State> states(n);
    for (uint32_t i = 0; i < n; ++i) states[i] = ctxs[i]->s;
    MultiCtl ctl{m->d_states, m->d_steps, m->d_rounds, m->d_apply, m->d_pop, m->d_rot, m->d_ros,
                 m->seg, m->seg_count, m->scratch, m->round};
    e = hipMemcpyAsync(m->d_states, states.data(), n * sizeof(State), hipMemcpyHostToDevice, m->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, m->st);
    if (e == hipSuccess) e = hipEventRecord(m->staging_free, m->st);
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
    for (int k = 0; k < kNumShapes; ++k) m->tune_ms[k] = m->tune_events[k] = 0.0;
    return FIBAR_OK;
}

int fibar_multi_get_shape(fibar_multi* m, uint32_t* block, uint32_t* grid)
{
    if (!m || !block || !grid) return FIBAR_E_INVALID_ARG;
    *block = kShapes[m->shape].block;
    *grid = kShapes[m->shape].grid;
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
