// Internal declarations shared by the host runtime and the kernels of
// libfibar.  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <tuple>
#include <utility>
#include <vector>

namespace fibar {

// One LDS sort tile: 1024 threads x 16 events.  A packet larger than this is
// cut into consecutive chunks that are applied in order.
constexpr int kSortThreads = 1024;
constexpr int kSortItems = 16;
constexpr int kChunk = kSortThreads * kSortItems;

// Chunks grouped and composed per bulk launch (one batch).
constexpr uint32_t kMaxBatchChunks = 256;

// Filter constants, derived on the host in double precision and rounded once.
//   one event of polarity p maps the state s = (pbar, L) to
//   [[alpha, 0], [-c*alpha, beta]] s + [(1-alpha) p, c*alpha p],
//   c = (1 + beta) / 2  -- Eq. (7), then Eq. (6) and Eq. (10) substituted.
struct Coef {
    float alpha;
    float one_m_alpha;
    float beta;
    float c_alpha;
};

// The composition of all events of one pixel inside one chunk:
//   s -> [[a, 0], [g, b]] s + [u1, u2]
// n_last packs the event count (high 16 bits) and the chunk-local index of
// the pixel's newest event (low 16 bits); key is the pixel's sort key (2x2
// tile index << 2 | position in the tile).
struct alignas(32) SegRec {
    uint32_t pix;
    uint32_t n_last;
    float a, g, b, u1, u2;
    uint32_t key;
};

// Per-chunk work item of the bulk sort kernel.
struct ChunkDesc {
    const uint16_t* x;
    const uint16_t* y;
    const uint8_t* p;
    uint32_t n;        // events in this chunk (<= kChunk)
    uint32_t pkt;      // packet slot in the current batch
};

// A pointer that a kernel loads from memory (a descriptor, a record) is a
// generic pointer to the compiler, and its accesses become flat
// instructions, which also count as LDS accesses: every later LDS wait then
// waits for them as well.  Passed through an integer into the global address
// space, the compiler emits global instructions (all such pointers here are
// device or pinned host allocations).
template <class T>
__device__ __forceinline__ T* as_global(T* p)
{
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ __forceinline__ ChunkDesc global_chunk(ChunkDesc cd)
{
    cd.x = as_global(cd.x);
    cd.y = as_global(cd.y);
    cd.p = as_global(cd.p);
    return cd;
}

// Window scalars of one context after a regulation step (device resident).
struct DevScalars {
    int64_t k;             // index of the newest applied event (-1: none)
    uint64_t h;            // index of the oldest event in the window
    uint64_t Q;            // target window length
    uint64_t P;            // active pixels
    uint64_t T;            // active 2x2 tiles
    uint64_t n_reg;        // regulation steps so far
    uint64_t last_stale;   // pixels blurred in the last step
    uint64_t total_stale;  // pixels blurred so far
    int32_t err;           // first device-side packet error (0: none)
    int32_t stepped;       // 1: the commit that wrote these was a regulation step
};

// Per-packet scratch of one batch (zeroed at the start of the batch).
// Every 64-thread wave of a step's kernels stores its (activation or
// deactivation) counts into a slot of its own, numbered by the wave's first
// thread in the step's grid of that kind: plain stores, no atomics, which
// had cost a few tenths of a microsecond at the end of every launch.  Waves
// past the slots (packets above one chunk) add to the overflow counters,
// spread over kSpread cache lines.  A commit sums slots and overflow.
constexpr int kSpread = 8;
constexpr int kLineWords = 32;       // 128-byte cache line
constexpr uint32_t kApplySlots = kChunk / 64;              // one chunk's apply waves
constexpr uint32_t kPopSlots = (kChunk + kChunk / 8) / 64 + 32;   // its pops' waves
struct alignas(128) StepScratch {
    uint32_t status;                 // validation bits: 1 = range, 2 = polarity
    uint32_t pad[kLineWords - 1];
    uint32_t part[kSpread][kLineWords];   // overflow, [0..3]: activated pixels,
                                          // activated tiles, stale pixels,
                                          // deactivated tiles
    uint2 wave_apply[kApplySlots];        // (activated pixels, activated tiles)
    uint2 wave_pop[kPopSlots];            // (stale pixels, deactivated tiles)
};
static_assert(kApplySlots % 2 == 0 && kPopSlots % 2 == 0, "slots are read in pairs");

// Per-pixel state, in two arrays of structures so that what one kernel
// needs of a pixel comes in one load: the window kernels read brightness and
// last-event index together (the 3x3 blur reads both for every neighbour),
// and only the filter update reads pbar, the queued-event count and the
// event total.
struct alignas(16) PixL {
    float L;        // brightness of active / never-seen pixels
    float Lb;       // brightness of stale pixels (their one-time blur)
    int64_t last;   // index of the newest event (-1: none)
};
struct alignas(16) PixP {
    float pbar;     // low-passed polarity
    uint32_t cnt;   // events of the pixel in the window
    uint64_t tot;   // events of the pixel so far
};

// Window scalars after one regulation step, as recorded for the caller's
// telemetry buffer (the layout of fibar_step_record in fibar.h).
struct StepRecord {
    int64_t k;
    uint64_t h, q, Q, P, T, stale, n;
};

// Device pointers of one context's state.
struct State {
    PixL* px;
    PixP* pp;
    uint32_t* ring;
    uint64_t ring_mask;
    DevScalars* sc;   // two slots; see the commit scheme in fibar_kernels.hip
    uint32_t W, H, TW;
    uint32_t fill_num, fill_den;
    uint64_t q_min, q_max;
    StepRecord* tel;   // per-step telemetry (null: none), tel_cap records
    uint64_t tel_cap;
    const float* gain; // per-pixel multiplier of Eq. (6)'s increment (null: none)
};

// A State loaded from memory (a record), with its pointers global (as_global).
__device__ __forceinline__ State global_state(State s)
{
    s.px = as_global(s.px);
    s.pp = as_global(s.pp);
    s.ring = as_global(s.ring);
    s.sc = as_global(s.sc);
    s.tel = as_global(s.tel);
    s.gain = as_global(s.gain);
    return s;
}

// Optional HIP events attached to a launch's dispatch (hipExtLaunchKernel):
// the runtime stamps them with the dispatch's own start and end, as a
// profiler does.  For a launcher that queues several kernels, `start` goes on
// the first and `stop` on the last.  Null events: an ordinary launch.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Launch recording: while a recorder is set on the calling thread,
// launch_timed appends the launch (kernel, shape, a copy of its parameters
// converted to the kernel's parameter types, timing events) instead of
// issuing it.  The host then replays a batch's launches as one HIP graph.
struct RecordedLaunch {
    const void* func = nullptr;
    dim3 grid, block;
    std::shared_ptr<void> args;      // the parameters (a std::tuple)
    std::vector<void*> params;       // pointers to each of them
    hipEvent_t start = nullptr, stop = nullptr;
};
struct LaunchRecorder {
    std::vector<RecordedLaunch> launches;
};
inline thread_local LaunchRecorder* tl_recorder = nullptr;

// A batch's recorded launches as an instantiated HIP graph: a chain of kernel
// nodes, with event-record nodes around the timed ones.  Two executable
// copies are used in turn, so that one is updated while the other may still
// run; `done` marks the end of each copy's last launch.
struct BatchGraph {
    std::vector<const void*> funcs;          // the kernels, in order
    std::vector<uint8_t> timed;              // 1: launch carries events
    hipGraph_t graph = nullptr;
    std::vector<hipGraphNode_t> knode, ev_start, ev_stop;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool launched[2] = {false, false};
    bool fresh[2] = {false, false};          // holds exactly the recorded parameters
    int next = 0;
    uint64_t last_use = 0;
};

template <typename T, size_t... I>
inline std::vector<void*> tuple_ptrs(T& t, std::index_sequence<I...>)
{
    return {static_cast<void*>(&std::get<I>(t))...};
}

template <typename... P, typename... A>
inline hipError_t launch_timed(void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t st,
                               hipEvent_t start, hipEvent_t stop, A... args)
{
    if (LaunchRecorder* r = tl_recorder) {
        auto t = std::make_shared<std::tuple<std::decay_t<P>...>>(
            static_cast<std::decay_t<P>>(args)...);
        RecordedLaunch L;
        L.func = reinterpret_cast<const void*>(kernel);
        L.grid = grid;
        L.block = block;
        L.params = tuple_ptrs(*t, std::index_sequence_for<P...>{});
        L.args = std::move(t);
        L.start = start;
        L.stop = stop;
        r->launches.push_back(std::move(L));
        return hipSuccess;
    }
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, start, stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    return hipGetLastError();
}

// ---- blur-off batch path (fibar_region.hip) --------------------------------
// Pixels are split into regions of kRegion consecutive pixels; a batch's
// events are bucketed by region (stable), and one workgroup per region
// applies them in time order with the region's state held in LDS.
constexpr uint32_t kRegion = 1024;
constexpr uint32_t kMaxRegions = 16384;
constexpr uint32_t kMaxBatchReadouts = 256;
// Events of a region's slice that the blur-off apply kernel orders at a time.
constexpr uint32_t kApplyTile = 8192;

// A readout placed inside a blur-off batch: it sees the events of chunks
// [0, chunk_end).
struct RegionReadout {
    uint32_t chunk_end;
    uint32_t pad;
    float* L;
    float* pbar;
    int64_t* last;
    float* log_age;
    uint64_t* tot;
};

struct RegionBuffers {
    uint32_t* cnt;        // [chunks][regions]: counts, then offsets within region
    uint64_t* base;       // [regions + 1]: first slot of each region
    uint32_t* total;      // [regions]
    int64_t* chunk_k;     // [chunks + 1]: global index of each chunk's first event
    uint64_t* payload;    // bucketed events
    RegionReadout* ro;    // [kMaxBatchReadouts]
    uint32_t n_regions;
};

// Scan of the per-(chunk, region) counts and the region bases / chunk
// indices of a batch (the first two stages of launch_region_batch); with
// set_k the newest event index of the batch is stored in the scalars.
hipError_t launch_region_scan_bases(const State& s, int slot, const ChunkDesc* d_chunks,
                                    uint32_t n_chunks, StepScratch* scratch,
                                    const RegionBuffers& rb, bool set_k, hipStream_t st);

// Per-tile event queues (fibar_tiles.hip): one tile's window and counts.
struct TQTile {
    uint32_t head, tail;   // ring positions of the window [head, tail)
    uint32_t Q, P, T;      // target, active pixels, active 2x2 cells
    uint32_t npix;         // pixels of the tile
    uint32_t pad[2];
};

// any_opt: some readout of the batch asks for more than the brightness.
// src (may be null): the batch's descriptors in mapped, coherent host memory,
// laid out as in d_chunks (chunk descriptors, readout descriptors after
// kMaxBatchChunks slots); the first launch reads them there and keeps the
// device copy that the later launches read, and a later launch stores src_seq
// into src_done (host memory, as the device sees it) once that launch has
// ended, so that the host rewrites src only after it ran.  Null src: the
// descriptors are in d_chunks already.
hipError_t launch_region_batch(const State& s, int slot, const ChunkDesc* d_chunks,
                               uint32_t n_chunks, StepScratch* scratch, const RegionBuffers& rb,
                               uint32_t n_readouts, bool any_opt, int key_bits, Coef coef,
                               hipStream_t st, const LaunchTiming& tm = LaunchTiming(),
                               const ChunkDesc* src = nullptr, uint64_t* src_done = nullptr,
                               uint64_t src_seq = 0);

// ---- in-order path (fibar_kernels.hip) -----------------------------------
// Workgroup sizes of the in-order kernels (on the 1280x720 stream with
// 16384-event packets, 64- and 256-thread workgroups were both slower).
constexpr uint32_t kApplyBlock = 128;
constexpr uint32_t kPopBlock = 128;
// Workgroups of a pop launch's readout, one pixel per thread (1, 2, 4 and 8
// pixels per thread were tried: 1 was fastest on the 1280x720 stream), at
// most this many (more pixels loop).
constexpr uint32_t kReadoutMaxBlocks = 16384;

// Threads of a step's pop launch: one pop each.  A step pops its packet's
// events plus the amount the target length shrank by, so the grid has 1/8
// headroom (a thread that had to take a second pop would double the
// kernel's latency).
inline __host__ __device__ uint32_t pop_threads(uint32_t pkt_events)
{
    return (pkt_events + pkt_events / 8 + kPopBlock - 1) / kPopBlock * kPopBlock;
}


// ---- launchers (fibar_kernels.hip) ---------------------------------------
// `gain` (null: none) scales each pixel's composed increment (the relative
// threshold C'_i multiplying Eq. (6)).
hipError_t launch_sort_compose(const ChunkDesc* d_chunks, uint32_t n_chunks, SegRec* seg,
                               uint32_t* seg_count, StepScratch* scratch, uint32_t W,
                               uint32_t H, int key_bits, Coef coef, const float* gain,
                               hipStream_t st, const LaunchTiming& tm = LaunchTiming());

// In-order launches.  `slot_in` holds the last committed scalars; when
// `prev` is not null the step it describes (with `prev_events` events) is
// committed on top of them, and the result is written to `slot_out`.
hipError_t launch_apply(const State& s, const ChunkDesc* d_chunk, const SegRec* seg,
                        const uint32_t* seg_count, uint32_t chunk_events,
                        uint32_t chunk_offset, StepScratch* step, const StepScratch* prev,
                        uint32_t prev_events, int slot_in, int slot_out, int spatial,
                        hipStream_t st, const LaunchTiming& tm = LaunchTiming());

// Outputs of a readout taken in the pop launch of the step before it (any
// may be null but L; no window count: the pops change it).
struct PopReadout {
    float* L;
    float* pbar;
    uint8_t* stale;
    int64_t* last;
    float* log_age;
    uint32_t* tcnt;
    uint64_t* tot;
};

// With `ro` the launch also writes the readout of the state after the step.
hipError_t launch_pop_blur(const State& s, uint32_t pkt_events, StepScratch* step, int slot,
                           const PopReadout* ro, hipStream_t st,
                           const LaunchTiming& tm = LaunchTiming());

// Initial per-pixel state: zero brightness and polarity, no events.
hipError_t launch_init_state(const State& s, hipStream_t st);

hipError_t launch_commit(const State& s, const StepScratch* prev, uint32_t prev_events,
                         int slot_in, int slot_out, int spatial, hipStream_t st);

hipError_t launch_readout(const State& s, int spatial, const StepScratch* prev,
                          uint32_t prev_events, int slot, float* L, float* pbar,
                          uint8_t* stale, uint32_t* cnt, int64_t* last, float* log_age,
                          uint32_t* tcnt, uint64_t* tot, hipStream_t st,
                          const LaunchTiming& tm = LaunchTiming());

// Per-event regulation (fibar_event.hip): one packet in one workgroup with
// the state in LDS.  Limits of a context regulated per event: at most
// kEventMaxPixels pixels, and windows of at most kEventMaxRing - 2 events
// (the LDS ring of pixel ids has kEventMaxRing entries at most).
constexpr uint32_t kEventMaxPixels = 8192;
constexpr uint32_t kEventMaxRing = 16384;
size_t event_lds_bytes(uint32_t W, uint32_t H, uint32_t TW, uint32_t cap);
hipError_t prepare_event_kernel(size_t lds_bytes);
hipError_t launch_event_packet(const State& s, int slot, const uint16_t* x, const uint16_t* y,
                               const uint8_t* p, uint32_t n, const Coef& coef, uint32_t cap,
                               size_t lds_bytes, hipStream_t st);

}  // namespace fibar
