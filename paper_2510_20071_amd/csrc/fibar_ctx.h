// Host-side context of libfibar, shared by the C-ABI implementation and the
// multi-stream executor.  Internal header.
#pragma once

#include <utility>
#include <vector>

#include "fibar.h"
#include "fibar_internal.h"

struct fibar_ctx {
    uint32_t W = 0, H = 0, TW = 0, TH = 0;
    uint64_t npx = 0, ntiles = 0;
    fibar_params prm{};
    fibar::Coef coef{};
    int key_bits = 4;
    hipStream_t st = nullptr;
    fibar::State s{};
    // batch resources
    fibar::ChunkDesc* d_chunks = nullptr;
    fibar::ChunkDesc* h_chunks = nullptr;      // pinned
    const fibar::ChunkDesc* h_chunks_dev = nullptr;   // blur off: h_chunks as kernels see it
    // blur off: the word after the descriptors in h_chunks, where a launch of
    // the batch that read them in place stores its number once they are read
    volatile uint64_t* h_done = nullptr;
    uint64_t* d_done = nullptr;          // the same word as kernels see it
    uint64_t done_seq = 0;               // number of the latest such batch
    hipEvent_t chunks_free = nullptr;   // h_chunks may be rewritten once this fired
    fibar::SegRec* seg = nullptr;
    uint32_t* seg_count = nullptr;
    fibar::StepScratch* scratch = nullptr;
    uint16_t* stg_x = nullptr;          // device staging for host packets
    uint16_t* stg_y = nullptr;
    uint8_t* stg_p = nullptr;
    size_t stg_cap = 0;
    // host packets go through a pinned ring of the same size: copied there on
    // the host, then to the device staging with asynchronous copies; the
    // cursor runs across calls, and only a wrap waits for the copies so far
    uint16_t* hs_x = nullptr;
    uint16_t* hs_y = nullptr;
    uint8_t* hs_p = nullptr;
    size_t hs_pos = 0;
    hipEvent_t hs_done = nullptr;       // after the latest host-packet copy
    fibar::DevScalars* h_sc = nullptr;         // pinned copy for stats
    int cur_slot = 0;                   // scalar slot holding the committed state
    uint64_t t_hi = 0;
    // blur-off batch path
    bool region_path = false;
    // per-event regulation: packets run in one LDS-resident workgroup
    bool event_mode = false;
    float* gain = nullptr;              // relative thresholds, once set
    // per-tile event queues (region > 0): tiles of tq_R x tq_R pixels
    bool tq = false;
    uint32_t tq_R = 0, tq_RW = 0, tq_RH = 0;
    uint32_t tq_cap = 0;                // ring entries per tile (a power of two)
    uint64_t tq_age = 0;                // events older than this leave
    fibar::TQTile* tq_tiles = nullptr;
    uint64_t* tq_front = nullptr;       // [2][tiles]: oldest window event, two steps
    uint2* tq_ring = nullptr;           // [tiles][tq_cap]: (global index low 32 bits, local pixel)
    uint32_t* tq_stale = nullptr;       // [tiles][region^2]: pixels going stale in the step
    uint32_t* tq_nstale = nullptr;      // [tiles]: how many
    int tq_parity = 0;                  // which front row is current
    uint32_t ev_cap = 0;                // LDS ring entries (a power of two)
    size_t ev_lds = 0;                  // dynamic LDS bytes of the event kernel
    fibar::RegionBuffers rb{};
    fibar::RegionReadout* h_ro = nullptr;      // pinned
    hipEvent_t ro_free = nullptr;
    // optional per-kernel timing: every time_every-th launch of a selected
    // kind carries a pair of events
    uint32_t time_mask = 0, time_every = 1;
    uint64_t time_seq[5] = {};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[5];
    std::vector<hipEvent_t> event_pool;
    // graph launches (blur on): a batch's kernels are recorded and replayed
    // as one HIP graph; graphs are cached by their sequence of kernels
    bool graph_mode = false;
    bool recording = false;             // the current batch is being recorded
    uint64_t batch_seq[5] = {};         // timing counters of the recorded batch
    fibar::LaunchRecorder rec;
    std::vector<fibar::BatchGraph*> graphs;
    uint64_t graph_clock = 0;
};


namespace fibar {

// Per-tile event queues (fibar_tiles.hip).
hipError_t tq_init(fibar_ctx* c);
hipError_t tq_bulk(fibar_ctx* c, uint32_t n_chunks);
hipError_t tq_step(fibar_ctx* c, uint32_t c0, uint32_t c1, uint32_t n_chunks, uint32_t pkt);
hipError_t tq_readout(fibar_ctx* c, float* L, float* pbar, uint8_t* stale, uint32_t* cnt,
                      int64_t* last, float* log_age, uint32_t* tcnt, uint64_t* tot);

inline int map_err(hipError_t e)
{
    if (e == hipSuccess) return FIBAR_OK;
    if (e == hipErrorOutOfMemory) return FIBAR_E_NOMEM;
    return FIBAR_E_DEVICE;
}

}  // namespace fibar

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return ::fibar::map_err(e_); \
    } while (0)
