// Blur-off (FIBAR-NSF) batch path of libfibar for gfx950.
//
// Without the spatial filter every event only updates its own pixel
// (temporal filter, Eq. (6), (7), (10)), so packet boundaries do not matter
// and a whole batch of packets -- with the readouts placed between them --
// can be processed at once:
//
//   k_region_count   per chunk: validate (the chunk's bits to its own
//                    scratch slot), histogram of events per region; it
//                    reads the batch's chunk and readout descriptors where
//                    the host wrote them (mapped host memory) and keeps the
//                    device copy the later launches read
//   k_region_scan    per region: offsets of each chunk's events in the
//                    region's slice (exclusive scan over chunks)
//   k_region_bases   one workgroup: each packet's status from its chunks'
//                    bits, region slice bases, first global event index of
//                    every chunk (rejected packets do not count), new
//                    newest-event index
//   k_region_scatter per chunk: stable counting sort by region (up to
//                    kRegion regions, else a stable LDS radix sort), then
//                    every event goes to its region's slice (chunk order,
//                    then arrival order)
//   k_region_apply   per region, one thread per pixel holding that pixel's
//                    pbar, L and last index in registers; the slice is
//                    consumed in tiles of kApplyTile events (stable counting
//                    sort by pixel), each owner applies its pixel's events in
//                    time order and writes the pixel into every readout of
//                    the batch as it passes the readout's position.
//
// HBM traffic per event: the packet (5 B) is read twice, an 8-byte bucket
// entry is written and read once; the state is read and written once per
// batch per region, and each readout writes 4 B per pixel.
#include "fibar_tile.h"

namespace fibar {
namespace {

using namespace tile;

constexpr uint64_t kSentinelPix = 0xffffffffull;

// A readout of a blur-off batch as k_region_apply keeps it in LDS: its
// position in the region's slice, its chunk end (bit 31: outputs beyond the
// brightness), and the brightness output.
typedef __attribute__((address_space(1))) float GlobalF32;

struct RoLds {
    uint32_t pos;
    uint32_t ce;
    float* L;
};

// Exclusive max-scan of u32 over a 1024-thread workgroup.
__device__ uint32_t block_exscan_max(uint32_t x, uint32_t* lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc = max(inc, o);
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = lds[w];
            lds[w] = run;
            run = max(run, t);
        }
    }
    __syncthreads();
    uint32_t ex = __shfl_up(inc, 1, 64);
    if (lane == 0) ex = 0;
    const uint32_t res = max(lds[wave], ex);
    __syncthreads();
    return res;
}

// Exclusive sum over a 256-thread workgroup; *total = sum of all.
__device__ uint32_t block256_exscan(uint32_t x, uint32_t* lds, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
        const uint32_t t = lds[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    *total = all;
    __syncthreads();
    return before + inc - x;
}

// Atomic add to a 16-bit LDS counter (the aligned 32-bit word that holds it;
// counters never exceed 16384, so no carry crosses into the neighbour);
// returns the counter's old value.
__device__ __forceinline__ uint32_t lds_add_u16(uint16_t* base, uint32_t i, uint32_t v)
{
    uint32_t* w = reinterpret_cast<uint32_t*>(base) + (i >> 1);
    const uint32_t sh = (i & 1u) * 16u;
    return (atomicAdd(w, v << sh) >> sh) & 0xffffu;
}

// Puts a bucket of event indices [at, at + n) in increasing order.  The
// counting sorts below leave a bucket as a run of step groups: the events of
// one key in one 64-event step of a wave (indices step * 64 + 0..63) take
// consecutive slots in whatever order one LDS atomic returned them, and the
// groups follow one another by step.  A check with independent loads comes
// first; a bucket out of order has each group rewritten from a 64-bit mask of
// its indices, which is linear in the bucket's size.
__device__ __forceinline__ void order_bucket(uint16_t* idx, uint32_t at, uint32_t n)
{
    bool ordered = true;
    for (uint32_t a = at + 1; a < at + n; ++a) ordered &= idx[a - 1] < idx[a];
    if (ordered) return;
    const uint32_t end = at + n;
    uint32_t a = at;
    while (a < end) {
        const uint32_t g0 = a;
        const uint32_t step = idx[a] >> 6;
        uint64_t mask = 0;
        for (; a < end; ++a) {
            const uint32_t v = idx[a];
            if ((v >> 6) != step) break;
            mask |= 1ull << (v & 63u);
        }
        for (uint32_t p = g0; mask; ++p) {
            idx[p] = (uint16_t)(step * 64u + (uint32_t)__builtin_ctzll(mask));
            mask &= mask - 1ull;
        }
    }
}

// f(e, key, pol) for every event of the chunk, e = threadIdx.x + k * 1024;
// the coordinates of eight events are loaded before any is used, so that
// a thread has eight loads in flight rather than one.
template <class F>
__device__ __forceinline__ void for_chunk_events(const ChunkDesc& cd, uint32_t W, uint32_t H,
                                                 uint32_t* bad, F&& f)
{
    constexpr uint32_t kU = 8;
    for (uint32_t e0 = threadIdx.x; e0 < cd.n; e0 += kU * kSortThreads) {
        uint32_t x[kU], y[kU], p[kU];
#pragma unroll
        for (uint32_t j = 0; j < kU; ++j) {
            const uint32_t e = e0 + j * kSortThreads;
            x[j] = e < cd.n ? cd.x[e] : 0u;
            y[j] = e < cd.n ? cd.y[e] : 0u;
            p[j] = e < cd.n ? cd.p[e] : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kU; ++j) {
            const uint32_t e = e0 + j * kSortThreads;
            if (e < cd.n) {
                const bool inr = x[j] < W && y[j] < H;
                *bad |= inr ? 0u : 1u;
                *bad |= p[j] > 1u ? 2u : 0u;
                f(e, inr ? y[j] * W + x[j] : 0u, p[j] & 1u);
            }
        }
    }
}

// Exclusive scan of u32 over a 1024-thread workgroup (as block_exscan_u32)
// for k_region_apply, whose tile loop calls it once per tile: the lane index
// passes through an empty asm statement at each call and the wave index is
// scalar, so that the shuffle and LDS addresses are made at the call rather
// than hoisted out of the loop into registers (at 64 VGPRs they spilled).
__device__ __forceinline__ uint32_t block_exscan_u32_at_call(uint32_t x, uint32_t* lds,
                                                              uint32_t* total)
{
    uint32_t lane = threadIdx.x & 63u;
    asm volatile("" : "+v"(lane));
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t inc = x;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t src = lane >= off ? lane - off : lane;
        const uint32_t o = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)inc);
        if (lane >= off) inc += o;
    }
    if (lane == 63u) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = lds[w];
            lds[w] = run;
            run += v;
        }
        lds[kWaves] = run;
    }
    __syncthreads();
    const uint32_t res = lds[wave] + inc - x;
    *total = lds[kWaves];
    __syncthreads();
    return res;
}

// What the first loads and the descriptor copy need leads the argument list
// (the leading arguments arrive preloaded in scalar registers; a loaded one
// would wait together with the descriptor's load from host memory).
__global__ __launch_bounds__(1024) void k_region_count(
    const ChunkDesc* __restrict__ chunks, ChunkDesc* __restrict__ chunks_out,
    const RegionReadout* __restrict__ ro_in, RegionReadout* __restrict__ ro_out,
    uint32_t n_chunks, uint32_t n_readouts, uint32_t W, uint32_t H, uint32_t n_regions,
    uint32_t* __restrict__ cnt, StepScratch* __restrict__ scratch)
{
    __shared__ uint32_t hist[kMaxRegions];
    __shared__ uint32_t bad_sh;
    const ChunkDesc raw = chunks[blockIdx.x];
    const ChunkDesc cd = global_chunk(raw);
    // descriptors read from host memory: the device copy for the batch's
    // later launches (workgroup b takes chunk b and readouts b, b + n_chunks,
    // ...; the readouts' loads first, so that they travel with the chunk's)
    if (chunks_out) {
        const uint32_t r = blockIdx.x + n_chunks * threadIdx.x;
        if (r < n_readouts) ro_out[r] = ro_in[r];
        if (threadIdx.x == 0) chunks_out[blockIdx.x] = raw;
    }
    for (uint32_t r = threadIdx.x; r < n_regions; r += 1024u) hist[r] = 0u;
    if (threadIdx.x == 0) bad_sh = 0u;
    __syncthreads();
    uint32_t bad = 0u;
    for_chunk_events(cd, W, H, &bad, [&](uint32_t, uint32_t key, uint32_t) {
        atomicAdd(&hist[key / kRegion], 1u);
    });
    if (bad) atomicOr(&bad_sh, bad);
    __syncthreads();
    // the chunk's validation bits, in its own slot (k_region_bases gathers
    // them per packet, so no slot needs clearing first)
    if (threadIdx.x == 0) scratch[blockIdx.x].pad[0] = bad_sh;
    uint32_t* row = cnt + (size_t)blockIdx.x * n_regions;
    for (uint32_t r = threadIdx.x; r < n_regions; r += 1024u) row[r] = hist[r];
}

__global__ __launch_bounds__(256) void k_region_scan(uint32_t* __restrict__ cnt, uint32_t n_chunks,
                                                     uint32_t n_regions,
                                                     uint32_t* __restrict__ total)
{
    __shared__ uint32_t lds[4];
    const uint32_t r = blockIdx.x, c = threadIdx.x;
    const uint32_t v = c < n_chunks ? cnt[(size_t)c * n_regions + r] : 0u;
    uint32_t tot;
    const uint32_t ex = block256_exscan(v, lds, &tot);
    if (c < n_chunks) cnt[(size_t)c * n_regions + r] = ex;
    if (c == 0) total[r] = tot;
}

// done (may be null): a word of host memory that gets done_seq, telling the
// host that the launch before this one (k_region_count, which reads the
// batch's descriptors in host memory) has ended.
__global__ __launch_bounds__(1024) void k_region_bases(State s, int slot,
                                                       const ChunkDesc* __restrict__ chunks,
                                                       uint32_t n_chunks,
                                                       StepScratch* __restrict__ scratch,
                                                       RegionBuffers rb, int set_k,
                                                       uint64_t* done, uint64_t done_seq)
{
    __shared__ uint32_t scan1[kWaves + 1];
    __shared__ uint32_t pst[kMaxBatchChunks];   // validation bits per packet
    if (done && threadIdx.x == 0)
        __hip_atomic_store(done, done_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    // a packet's status: the validation bits of its chunks, written for every
    // packet of the batch (the per-chunk bits are in each chunk's own slot)
    for (uint32_t i = threadIdx.x; i < kMaxBatchChunks; i += blockDim.x) pst[i] = 0u;
    __syncthreads();
    if (threadIdx.x < n_chunks) {
        const uint32_t b = scratch[threadIdx.x].pad[0];
        if (b) atomicOr(&pst[chunks[threadIdx.x].pkt], b);
    }
    __syncthreads();
    if (threadIdx.x < n_chunks) {
        const uint32_t pk = chunks[threadIdx.x].pkt;
        scratch[pk].status = pst[pk];
    }
    const uint32_t per = (rb.n_regions + blockDim.x - 1) / blockDim.x;
    const uint32_t r0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (r0 + i < rb.n_regions) local += rb.total[r0 + i];
    uint32_t all;
    uint32_t run = block_exscan_u32(local, scan1, &all);
    for (uint32_t i = 0; i < per; ++i) {
        if (r0 + i < rb.n_regions) {
            rb.base[r0 + i] = run;
            run += rb.total[r0 + i];
        }
    }
    // first global event index of every chunk: prefix over chunks of the
    // sizes of chunks whose packet passed validation (<= 256 chunks)
    const uint32_t ci = threadIdx.x;
    uint32_t st = 0u, sz = 0u;
    if (ci < n_chunks) {
        st = pst[chunks[ci].pkt];
        sz = st == 0u ? chunks[ci].n : 0u;
    }
    uint32_t nvalid;
    const uint32_t before = block_exscan_u32(sz, scan1, &nvalid);
    const int64_t k0 = s.sc[slot].k;
    if (ci < n_chunks) rb.chunk_k[ci] = k0 + 1 + before;
    // first rejected chunk decides the reported error
    const uint32_t bad_ci = block_exscan_max(st ? (kMaxBatchChunks - ci) : 0u, scan1);
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {
        uint32_t first_bad = max(bad_ci, (ci < n_chunks && st) ? kMaxBatchChunks - ci : 0u);
        rb.base[rb.n_regions] = all;
        rb.chunk_k[n_chunks] = k0 + 1 + nvalid;
        DevScalars& c = s.sc[slot];
        if (set_k) c.k = k0 + nvalid;
        if (first_bad && c.err == 0) {
            const uint32_t st0 = pst[chunks[kMaxBatchChunks - first_bad].pkt];
            c.err = (st0 & 1u) ? -2 : -3;   // FIBAR_E_RANGE / FIBAR_E_POLARITY
        }
    }
}

__global__ __launch_bounds__(kSortThreads) void k_region_scatter(
    const ChunkDesc* __restrict__ chunks, uint32_t W, uint32_t H, int region_bits,
    const uint32_t* __restrict__ offs, uint32_t n_regions, const uint64_t* __restrict__ base,
    const StepScratch* __restrict__ scratch, uint64_t* __restrict__ payload)
{
    __shared__ uint32_t keypol[kChunk];
    __shared__ __align__(16) uint16_t idxA[kChunk];
    __shared__ __align__(16) uint16_t idxB[kChunk];
    __shared__ uint64_t scan4[kWaves + 1][4];
    __shared__ uint32_t scan1[kWaves + 1];
    __shared__ uint32_t rcnt[kRegion];   // per region: bucket start
    const ChunkDesc cd = global_chunk(chunks[blockIdx.x]);
    const uint32_t cn = cd.n;
    const uint32_t t = threadIdx.x;
    // up to kRegion regions: a counting sort (per-wave counters in idxB)
    const bool fast = n_regions <= kRegion;
    if (fast) {
        uint16_t* wrow = idxB + (size_t)(t >> 6) * kRegion;
#pragma unroll
        for (uint32_t j = 0; j < kRegion / 64; ++j) wrow[(t & 63) + 64 * j] = 0u;
    }
    uint32_t bad = 0u;
    for_chunk_events(cd, W, H, &bad, [&](uint32_t e, uint32_t key, uint32_t pol) {
        keypol[e] = (key << 1) | pol;
        idxA[e] = (uint16_t)e;
    });
    __syncthreads();
    const bool valid = scratch[cd.pkt].status == 0u;
    const uint32_t* off_row = offs + (size_t)blockIdx.x * n_regions;
    if (fast) {
        // counting sort by region: wave w takes a contiguous part of the
        // chunk in order, 64 events at a time, and row w of idxB counts, then
        // places, the wave's events of each region (LDS atomics); a
        // region's bucket is then in arrival order except where one step of
        // a wave had several of its events, which the region's owner puts
        // right by insertion sort
        const uint32_t wave = t >> 6, lane = t & 63;
        uint16_t* wrow = idxB + (size_t)wave * kRegion;
        const uint32_t seg = ((cn + kWaves - 1) / kWaves + 63u) & ~63u;
        const uint32_t w0 = wave * seg, w1 = min(w0 + seg, cn);
        for (uint32_t s0e = w0 + lane; s0e < w1; s0e += 64)
            lds_add_u16(wrow, (keypol[s0e] >> 1) / kRegion, 1u);
        __syncthreads();
        // region t's owner: its count, the bucket start, each wave's place
        uint32_t cr = 0;
        if (t < n_regions) {
#pragma unroll
            for (uint32_t w = 0; w < (uint32_t)kWaves; ++w) cr += idxB[w * kRegion + t];
        }
        uint32_t all;
        const uint32_t s0 = block_exscan_u32(cr, scan1, &all);   // ends with a barrier
        if (t < n_regions) {
            rcnt[t] = s0;
            uint32_t at = s0;
#pragma unroll
            for (uint32_t w = 0; w < (uint32_t)kWaves; ++w) {
                const uint32_t cw = idxB[w * kRegion + t];
                idxB[w * kRegion + t] = (uint16_t)at;
                at += cw;
            }
        }
        __syncthreads();
        for (uint32_t s0e = w0 + lane; s0e < w1; s0e += 64)
            idxA[lds_add_u16(wrow, (keypol[s0e] >> 1) / kRegion, 1u)] = (uint16_t)s0e;
        __syncthreads();
        if (t < n_regions) order_bucket(idxA, rcnt[t], cr);
        __syncthreads();
        for (uint32_t sidx = t; sidx < cn; sidx += kSortThreads) {
            const uint32_t oid = idxA[sidx];
            const uint32_t kp = keypol[oid];
            const uint32_t pix = kp >> 1;
            const uint32_t reg = pix / kRegion;
            const uint64_t dest = base[reg] + off_row[reg] + (sidx - rcnt[reg]);
            const uint64_t pixf = valid ? (uint64_t)pix : kSentinelPix;
            payload[dest] = (pixf << 32) | ((uint64_t)blockIdx.x << 15) |
                            ((uint64_t)oid << 1) | (uint64_t)(kp & 1u);
        }
        return;
    }
    // group by region only (stable, so arrival order is kept inside a region)
    const uint16_t* sorted = tile_sort(keypol, idxA, idxB, cn, region_bits, scan4, 10);

    // rank of each item among the chunk's items of its region: position
    // minus the position of the region's first item (last head at or before)
    const uint32_t beg = threadIdx.x * kSortItems;
    uint32_t lmax = 0;
    uint32_t prev_reg = (beg > 0 && beg - 1 < cn) ? (keypol[sorted[beg - 1]] >> 1) / kRegion
                                                  : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t sidx = beg + j;
        if (sidx < cn) {
            const uint32_t reg = (keypol[sorted[sidx]] >> 1) / kRegion;
            if (sidx == 0 || reg != prev_reg) lmax = sidx;
            prev_reg = reg;
        }
    }
    uint32_t head = block_exscan_max(lmax, scan1);
    prev_reg = (beg > 0 && beg - 1 < cn) ? (keypol[sorted[beg - 1]] >> 1) / kRegion : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint32_t sidx = beg + j;
        if (sidx < cn) {
            const uint32_t oid = sorted[sidx];
            const uint32_t kp = keypol[oid];
            const uint32_t pix = kp >> 1;
            const uint32_t reg = pix / kRegion;
            if (sidx == 0 || reg != prev_reg) head = sidx;
            prev_reg = reg;
            const uint64_t dest = base[reg] + off_row[reg] + (sidx - head);
            const uint64_t pixf = valid ? (uint64_t)pix : kSentinelPix;
            payload[dest] = (pixf << 32) | ((uint64_t)blockIdx.x << 15) | ((uint64_t)oid << 1) |
                            (uint64_t)(kp & 1u);
        }
    }
}

// One workgroup per region, thread t owns pixel p0 + t.  The region's slice
// (chunk order, then arrival order) is consumed in tiles of up to kApplyTile
// events: a stable counting sort by local pixel puts each pixel's events of
// the tile together, in time order, and the owner thread applies them one by
// one (Eq. (7), then Eq. (6) and (10)).  The readouts of the batch are
// visited in order by the whole workgroup: every owner first applies its
// events that precede the readout (those at lower slice positions), then all
// write the readout together (coalesced).  70 KB of LDS and at most 64 VGPRs
// keep two workgroups on a CU.
// kOpt: the batch has readouts with outputs beyond the brightness; without,
// the kernel has no code path that loads while readouts are written (such a
// path makes the compiler wait for every store in flight at each readout).
// kTile: events ordered at a time.  kApplyTile (8192) with at most 64 VGPRs
// fits two workgroups on a CU; sensors of few regions, whose workgroups run
// in one round anyway, take twice that (fewer rounds of the tile loop).
template <bool kOpt, uint32_t kTile>
__global__ __launch_bounds__(kSortThreads, kTile == kApplyTile ? 8 : 4) void k_region_apply(
    State s, RegionBuffers rb,
                                                               uint32_t n_chunks,
                                                               uint32_t n_readouts, Coef coef)
{
    // keypol: local pixel, kRegion for rejected packets (bits 1..11) |
    // polarity (bit 0)
    __shared__ uint16_t keypol[kTile];
    __shared__ __align__(16) uint16_t idxA[kTile];
    __shared__ __align__(16) uint16_t wcnt[kWaves * kRegion];   // per wave and pixel
    __shared__ uint32_t scan1[kWaves + 1];
    __shared__ RoLds ro_s[kMaxBatchReadouts];

    const uint32_t r = blockIdx.x;
    const uint32_t t = threadIdx.x;
    const uint64_t npx = (uint64_t)s.W * s.H;
    const uint64_t p0 = (uint64_t)r * kRegion;
    const bool own = p0 + t < npx;
    const uint32_t gp = (uint32_t)(p0 + t);   // W x H < 2^31
    // the increment's factor, times the pixel's relative threshold if any
    float c = 0.5f + 0.5f * coef.beta;
    float pb = 0.f, l = 0.f;
    // with readouts of the brightness only, the last index does not stay in
    // registers (no spill at 64 VGPRs: a kernel with scratch memory waits
    // ~5 us longer to start): it is stored when it is resolved
    int64_t last = -1;
    uint64_t tot = 0u;
    if (own) {
        const PixL v = s.px[gp];
        const PixP w = s.pp[gp];
        pb = w.pbar;
        tot = w.tot;
        l = v.L;
        if constexpr (kOpt) last = v.last;
        if (s.gain) c *= s.gain[gp];
    }
    // slice offsets of a batch stay below kMaxBatchChunks x kChunk (2^22)
    const uint32_t lo = (uint32_t)rb.base[r], hi = (uint32_t)rb.base[r + 1];
    // the batch's readout descriptors, loaded once by all threads together
    // (a descriptor load per readout inside the uniform loop below would be
    // a dependent round trip each)
    for (uint32_t i = t; i < n_readouts; i += kSortThreads) {
        const RegionReadout d = rb.ro[i];
        const uint32_t ce = d.chunk_end;
        const bool opt = d.pbar || d.tot || d.last || d.log_age;
        RoLds q;
        q.pos = ce < n_chunks ? rb.cnt[(size_t)ce * rb.n_regions + r] : (uint32_t)(hi - lo);
        q.ce = ce | (opt ? 0x80000000u : 0u);
        q.L = d.L;
        ro_s[i] = q;
    }
    __syncthreads();
    // the pixel's state is in registers from here on: a first use inside the
    // loops below would wait there for every memory access in flight, and
    // stores (the readouts) count among them
    if constexpr (kOpt) asm volatile("" ::"v"(pb), "v"(l), "v"(c), "v"(last), "v"(tot));
    else asm volatile("" ::"v"(pb), "v"(l), "v"(c), "v"(tot));
    uint32_t next_ro = 0;   // first readout not written yet (uniform)

    // own events of the current tile: sorted positions [run_at, run_end)
    uint32_t run_at = 0, run_end = 0;
    uint32_t last_pos = 0xffffffffu;   // sorted position of the newest applied event
    const uint16_t* sorted = idxA;
    uint32_t tile0 = lo;

    auto resolve_last = [&]() {
        if (last_pos != 0xffffffffu) {
            const uint32_t oid = sorted[last_pos];
            const uint64_t pl = rb.payload[tile0 + oid];
            const int64_t lv =
                rb.chunk_k[(uint32_t)(pl >> 15) & 0x1ffffu] + (int64_t)((pl >> 1) & 0x3fffu);
            if constexpr (kOpt) {
                last = lv;
            } else {   // an owner's (events were applied); the address made here
                uint32_t g = gp;
                asm volatile("" : "+v"(g));
                *as_global(&s.px[g].last) = lv;
            }
            last_pos = 0xffffffffu;
        }
    };
    // the owner's next event of the tile: its position in the region's
    // slice << 1 | polarity, loaded one event ahead (trel: the tile's first
    // position).  The slice is in chunk order, so the events before a
    // readout are those at positions below the readout's.
    uint32_t nkp = 0u, trel = 0u;
    auto key_at = [&](uint32_t a) {
        const uint32_t e = sorted[a];
        return ((trel + e) << 1) | (uint32_t)(keypol[e] & 1u);
    };
    // apply own events of the tile at slice positions below `pos_limit`
    auto advance = [&](uint32_t pos_limit) {
        while (run_at < run_end) {
            const uint32_t kp = nkp;
            if ((kp >> 1) >= pos_limit) break;
            if (run_at + 1 < run_end) nkp = key_at(run_at + 1);
            const float p = (kp & 1u) ? 1.f : -1.f;
            pb = fmaf(coef.alpha, pb, coef.one_m_alpha * p);    // Eq. (7)
            l = fmaf(coef.beta, l, c * (p - pb));                 // Eq. (6), (10)
            ++tot;
            last_pos = run_at;
            ++run_at;
        }
    };
    auto write_readout = [&](uint32_t i, const RoLds& q) {
        if (!kOpt || !(q.ce >> 31)) {   // brightness only
            // a global (not flat) store: a flat store would also count as an
            // LDS access and make every later LDS read wait for it
            if (own) ((GlobalF32*)q.L)[gp] = l;
            return;
        }
        const RegionReadout d = rb.ro[i];
        if (d.last || d.log_age) resolve_last();
        if (own) {
            d.L[gp] = l;
            if (d.pbar) d.pbar[gp] = pb;
            if (d.tot) d.tot[gp] = tot;
            if (d.last) d.last[gp] = last;
            if (d.log_age) d.log_age[gp] = log1pf((float)(rb.chunk_k[d.chunk_end] - 1 - last));
        }
    };

    for (uint32_t cursor = lo; cursor < hi;) {
        const uint32_t cn = (uint32_t)(hi - cursor < kTile ? hi - cursor : kTile);
        const uint32_t rel1 = (uint32_t)(cursor - lo) + cn;
        // counting sort by pixel: wave w takes a contiguous part of the tile
        // in order, 64 events at a time, and wcnt[w][pixel] counts, then
        // places, the wave's events of each pixel (LDS atomics); a pixel's
        // bucket is then in slice (= time) order except where one step of a
        // wave had several of its events, which the owner puts right
        // (order_bucket)
        const uint32_t wave = t >> 6, lane = t & 63;
        uint16_t* wrow = wcnt + (size_t)wave * kRegion;
#pragma unroll
        for (uint32_t j = 0; j < kRegion / 64; ++j) wrow[lane + 64 * j] = 0u;
        for (uint32_t e0 = 0; e0 < cn; e0 += 2 * kSortThreads) {
            uint64_t pl[2];
#pragma unroll
            for (uint32_t j = 0; j < 2; ++j) {
                const uint32_t e = e0 + t + j * kSortThreads;
                pl[j] = e < cn ? rb.payload[cursor + e] : 0ull;
            }
#pragma unroll
            for (uint32_t j = 0; j < 2; ++j) {
                const uint32_t e = e0 + t + j * kSortThreads;
                if (e < cn) {
                    const uint64_t pix = pl[j] >> 32;
                    const uint32_t lk = pix == kSentinelPix ? kRegion : (uint32_t)(pix - p0);
                    keypol[e] = (uint16_t)((lk << 1) | (uint32_t)(pl[j] & 1u));
                }
            }
        }
        __syncthreads();
        const uint32_t seg = ((cn + kWaves - 1) / kWaves + 63u) & ~63u;
        const uint32_t w0 = wave * seg, w1 = min(w0 + seg, cn);
        // rejected packets' events (pixel kRegion) take part in none
        for (uint32_t e = w0 + lane; e < w1; e += 64) {
            const uint32_t lk = (keypol[e] >> 1) & 0x7ffu;
            if (lk < kRegion) lds_add_u16(wrow, lk, 1u);
        }
        __syncthreads();
        // the owner: its pixel's count, the bucket start, and each wave's
        // place in the bucket
        uint32_t my_cnt = 0;
#pragma unroll
        for (uint32_t w = 0; w < (uint32_t)kWaves; ++w) my_cnt += wcnt[w * kRegion + t];
        uint32_t total;
        run_at = block_exscan_u32_at_call(my_cnt, scan1, &total);   // ends with a barrier
        run_end = run_at + my_cnt;
        {
            uint32_t at = run_at;
#pragma unroll
            for (uint32_t w = 0; w < (uint32_t)kWaves; ++w) {
                const uint32_t cw = wcnt[w * kRegion + t];
                wcnt[w * kRegion + t] = (uint16_t)at;
                at += cw;
            }
        }
        __syncthreads();
        for (uint32_t e = w0 + lane; e < w1; e += 64) {
            const uint32_t lk = (keypol[e] >> 1) & 0x7ffu;
            if (lk < kRegion) idxA[lds_add_u16(wrow, lk, 1u)] = (uint16_t)e;
        }
        __syncthreads();
        order_bucket(idxA, run_at, my_cnt);
        sorted = idxA;   // an owner reads only its own bucket from here on
        tile0 = cursor;
        if (!own) run_end = run_at;
        trel = (uint32_t)(cursor - lo);
        if (run_at < run_end) nkp = key_at(run_at);
        // readouts that fall inside this tile (the next descriptor is loaded
        // while the current one is written)
        if (next_ro < n_readouts) {
            RoLds q = ro_s[next_ro];
            while (q.pos < rel1) {
                const RoLds qn = ro_s[next_ro + 1 < n_readouts ? next_ro + 1 : next_ro];
                advance(q.pos);
                write_readout(next_ro, q);
                ++next_ro;
                if (next_ro >= n_readouts) break;
                q = qn;
            }
        }
        advance(0xffffffffu);
        resolve_last();
        __syncthreads();
        cursor += cn;
    }
    for (; next_ro < n_readouts; ++next_ro) write_readout(next_ro, ro_s[next_ro]);
    if (own) {
        // the records' addresses from here, not kept from the loads above
        uint32_t g = gp;
        asm volatile("" : "+v"(g));
        s.pp[g].pbar = pb;
        s.pp[g].tot = tot;
        s.px[g].L = l;
        if constexpr (kOpt) s.px[g].last = last;
    }
}

}  // namespace

hipError_t launch_region_scan_bases(const State& s, int slot, const ChunkDesc* d_chunks,
                                    uint32_t n_chunks, StepScratch* scratch,
                                    const RegionBuffers& rb, bool set_k, hipStream_t st)
{
    hipLaunchKernelGGL(k_region_scan, dim3(rb.n_regions), dim3(256), 0, st, rb.cnt, n_chunks,
                       rb.n_regions, rb.total);
    hipLaunchKernelGGL(k_region_bases, dim3(1), dim3(1024), 0, st, s, slot, d_chunks, n_chunks,
                       scratch, rb, set_k ? 1 : 0, (uint64_t*)nullptr, (uint64_t)0);
    return hipGetLastError();
}

hipError_t launch_region_batch(const State& s, int slot, const ChunkDesc* d_chunks,
                               uint32_t n_chunks, StepScratch* scratch, const RegionBuffers& rb,
                               uint32_t n_readouts, bool any_opt, int key_bits, Coef coef,
                               hipStream_t st, const LaunchTiming& tm, const ChunkDesc* src,
                               uint64_t* src_done, uint64_t src_seq)
{
    if (n_chunks > 0) {
        const RegionReadout* ro_src =
            src ? reinterpret_cast<const RegionReadout*>(src + kMaxBatchChunks) : nullptr;
        const hipError_t e = launch_timed(
            k_region_count, dim3(n_chunks), dim3(1024), st, tm.start, nullptr,
            src ? src : d_chunks, src ? const_cast<ChunkDesc*>(d_chunks) : nullptr, ro_src,
            src ? rb.ro : nullptr, n_chunks, src ? n_readouts : 0u, s.W, s.H, rb.n_regions, rb.cnt,
            scratch);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_region_scan, dim3(rb.n_regions), dim3(256), 0, st, rb.cnt, n_chunks,
                           rb.n_regions, rb.total);
        // src is free once the count launch has ended: the base launch says
        // so in host memory (an event fired by a launch's end put ~5 us into
        // the stream, one recorded apart from it ~10 us)
        hipLaunchKernelGGL(k_region_bases, dim3(1), dim3(1024), 0, st, s, slot, d_chunks, n_chunks,
                           scratch, rb, 1, src ? src_done : (uint64_t*)nullptr, src_seq);
        int region_bits = 1;
        while ((1u << region_bits) < rb.n_regions) ++region_bits;
        hipLaunchKernelGGL(k_region_scatter, dim3(n_chunks), dim3(kSortThreads), 0, st, d_chunks,
                           s.W, s.H, region_bits, rb.cnt, rb.n_regions, rb.base, scratch,
                           rb.payload);
    } else {
        // readouts only: empty slices
        const hipError_t e = launch_timed(k_region_scan, dim3(rb.n_regions), dim3(256), st,
                                          tm.start, nullptr, rb.cnt, 0u, rb.n_regions, rb.total);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_region_bases, dim3(1), dim3(1024), 0, st, s, slot, d_chunks, 0u,
                           scratch, rb, 1, (uint64_t*)nullptr, (uint64_t)0);
    }
    // up to 256 regions: one round of workgroups in any case, the larger tile
    const bool big = rb.n_regions <= 256;
    if (any_opt && big)
        return launch_timed(k_region_apply<true, 2 * kApplyTile>, dim3(rb.n_regions),
                            dim3(kSortThreads), st, nullptr, tm.stop, s, rb, n_chunks, n_readouts,
                            coef);
    if (any_opt)
        return launch_timed(k_region_apply<true, kApplyTile>, dim3(rb.n_regions),
                            dim3(kSortThreads), st, nullptr, tm.stop, s, rb, n_chunks, n_readouts,
                            coef);
    if (big)
        return launch_timed(k_region_apply<false, 2 * kApplyTile>, dim3(rb.n_regions),
                            dim3(kSortThreads), st, nullptr, tm.stop, s, rb, n_chunks, n_readouts,
                            coef);
    return launch_timed(k_region_apply<false, kApplyTile>, dim3(rb.n_regions), dim3(kSortThreads),
                        st, nullptr, tm.stop, s, rb, n_chunks, n_readouts, coef);
}

}  // namespace fibar
