// Device helpers shared by the kernels of libfibar: affine maps of the
// temporal filter, workgroup scans, and the LDS tile sort + segmented
// composition used for grouping events by pixel.  Internal header.
#pragma once

#include "fibar_internal.h"

namespace fibar {
namespace tile {
namespace {

constexpr int kWaves = kSortThreads / 64;

// ---------------------------------------------------------------------------
// Affine maps of the 2-vector state s = (pbar, L):  s -> [[a,0],[g,b]] s + u
// ---------------------------------------------------------------------------
struct Aff {
    float a, g, b, u1, u2;
    uint32_t n;
};

__device__ __forceinline__ Aff aff_identity()
{
    Aff r;
    r.a = 1.f; r.g = 0.f; r.b = 1.f; r.u1 = 0.f; r.u2 = 0.f; r.n = 0u;
    return r;
}

// One event of polarity byte `pol` (1 -> +1, 0 -> -1):
//   pbar' = alpha pbar + (1 - alpha) p                       Eq. (7)
//   L'    = beta L + c (p - pbar') = beta L - c alpha pbar + c alpha p
//                                                           Eq. (6), (10)
__device__ __forceinline__ Aff aff_event(const Coef& c, uint32_t pol)
{
    const float p = pol ? 1.f : -1.f;
    Aff r;
    r.a = c.alpha;
    r.g = -c.c_alpha;
    r.b = c.beta;
    r.u1 = c.one_m_alpha * p;
    r.u2 = c.c_alpha * p;
    r.n = 1u;
    return r;
}

// Apply `f` first, then `s`.
__device__ __forceinline__ Aff aff_then(const Aff& f, const Aff& s)
{
    Aff r;
    r.a = s.a * f.a;
    r.g = fmaf(s.g, f.a, s.b * f.g);
    r.b = s.b * f.b;
    r.u1 = fmaf(s.a, f.u1, s.u1);
    r.u2 = fmaf(s.g, f.u1, fmaf(s.b, f.u2, s.u2));
    r.n = f.n + s.n;
    return r;
}

// Segmented-scan element: `flag` = a segment starts inside this span.
struct SegPair {
    uint32_t flag;
    Aff v;
};

// x precedes y.
__device__ __forceinline__ SegPair seg_combine(const SegPair& x, const SegPair& y)
{
    SegPair r;
    r.flag = x.flag | y.flag;
    r.v = y.flag ? y.v : aff_then(x.v, y.v);
    return r;
}

__device__ __forceinline__ SegPair shfl_up_pair(const SegPair& v, int off)
{
    SegPair r;
    r.flag = __shfl_up(v.flag, off, 64);
    r.v.a = __shfl_up(v.v.a, off, 64);
    r.v.g = __shfl_up(v.v.g, off, 64);
    r.v.b = __shfl_up(v.v.b, off, 64);
    r.v.u1 = __shfl_up(v.v.u1, off, 64);
    r.v.u2 = __shfl_up(v.v.u2, off, 64);
    r.v.n = __shfl_up(v.v.n, off, 64);
    return r;
}

// Exclusive segmented scan over the workgroup (thread order).
__device__ SegPair block_exscan_pair(const SegPair& x, SegPair* lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    SegPair inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        SegPair o = shfl_up_pair(inc, off);
        if (lane >= off) inc = seg_combine(o, inc);
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        SegPair run;
        run.flag = 0u;
        run.v = aff_identity();
        for (int w = 0; w < kWaves; ++w) {
            SegPair t = lds[w];
            lds[w] = run;
            run = seg_combine(run, t);
        }
    }
    __syncthreads();
    SegPair ex = shfl_up_pair(inc, 1);
    if (lane == 0) {
        ex.flag = 0u;
        ex.v = aff_identity();
    }
    SegPair res = seg_combine(lds[wave], ex);
    __syncthreads();
    return res;
}

// Exclusive sum over the workgroup; *total receives the sum of all threads.
__device__ uint32_t block_exscan_u32(uint32_t x, uint32_t* lds, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            uint32_t t = lds[w];
            lds[w] = run;
            run += t;
        }
        lds[kWaves] = run;
    }
    __syncthreads();
    uint32_t res = lds[wave] + inc - x;
    *total = lds[kWaves];
    __syncthreads();
    return res;
}

// ---------------------------------------------------------------------------
// Radix digit counters: 16 bins of 16 bits packed into four 64-bit words.
// A bin never exceeds 16384 (the chunk size), so fields never overflow and
// packed vectors can be added and scanned as plain integers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t dig_field(const uint64_t v[4], uint32_t d)
{
    const uint32_t q = d >> 2;
    const uint64_t w = q == 0 ? v[0] : q == 1 ? v[1] : q == 2 ? v[2] : v[3];
    return (uint32_t)(w >> ((d & 3u) * 16u)) & 0xffffu;
}

__device__ __forceinline__ void dig_add(uint64_t v[4], uint32_t d)
{
    const uint64_t inc = 1ull << ((d & 3u) * 16u);
    const uint32_t q = d >> 2;
    v[0] += q == 0 ? inc : 0ull;
    v[1] += q == 1 ? inc : 0ull;
    v[2] += q == 2 ? inc : 0ull;
    v[3] += q == 3 ? inc : 0ull;
}

__device__ void block_exscan4(const uint64_t x[4], uint64_t ex[4], uint64_t tot[4],
                              uint64_t (*lds)[4])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc[4] = {x[0], x[1], x[2], x[3]};
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint64_t o = __shfl_up(inc[q], off, 64);
            if (lane >= off) inc[q] += o;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < 4; ++q) lds[wave][q] = inc[q];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        uint64_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            uint64_t t = lds[w][q];
            lds[w][q] = run;
            run += t;
        }
        lds[kWaves][q] = run;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ex[q] = lds[wave][q] + inc[q] - x[q];
        tot[q] = lds[kWaves][q];
    }
    __syncthreads();
}

// Sum over a full wave (all 64 lanes active), in every lane: DPP adds make
// each 16-lane row's sum (quads, half rows, rows), then the four rows' sums
// are read out to scalars.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    constexpr int kQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
    constexpr int kQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
    constexpr int kRowHalfMirror = 0x141;
    constexpr int kRowMirror = 0x140;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap2, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowHalfMirror, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowMirror, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of a tile's index permutation (1024 threads x 16
// items, blocked: thread t owns sorted positions [16t, 16t + 16)).  The key
// of item e is bits [1 + key_lo, 1 + key_lo + key_bits) of keypol[e] (bit 0
// is the polarity; bits outside the key may carry other data).  4 bits per pass; every pass is stable, so items with equal
// keys keep their original (arrival) order.  Returns the buffer holding the
// sorted permutation (idxA or idxB).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t* tile_sort(const uint32_t* keypol, uint16_t* idxA, uint16_t* idxB,
                               uint32_t cn, int key_bits, uint64_t (*scan4)[4], int key_lo = 0)
{
    uint16_t* src = idxA;
    uint16_t* dst = idxB;
    const uint32_t beg = (uint32_t)threadIdx.x * kSortItems;
    for (int shift = 0; shift < key_bits; shift += 4) {
        uint16_t id[kSortItems];
        uint32_t dg[kSortItems];
        {
            const uint4 v0 = *reinterpret_cast<const uint4*>(src + beg);
            const uint4 v1 = *reinterpret_cast<const uint4*>(src + beg + 8);
            const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                id[2 * j] = (uint16_t)(w[j] & 0xffffu);
                id[2 * j + 1] = (uint16_t)(w[j] >> 16);
            }
        }
        uint64_t c[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            dg[j] = 0u;
            if (beg + j < cn) {
                dg[j] = (keypol[id[j]] >> (1 + key_lo + shift)) & 15u;
                dig_add(c, dg[j]);
            }
        }
        uint64_t ex[4], tot[4];
        block_exscan4(c, ex, tot, scan4);
        // exclusive prefix over bins, packed the same way (<= 16384 fits)
        uint64_t sum[4] = {ex[0], ex[1], ex[2], ex[3]};
        {
            uint32_t acc = 0u;
#pragma unroll
            for (int d = 0; d < 16; ++d) {
                sum[d >> 2] += (uint64_t)acc << ((d & 3) * 16);
                acc += dig_field(tot, (uint32_t)d);
            }
        }
        uint64_t run[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (beg + j < cn) {
                const uint32_t pos = dig_field(sum, dg[j]) + dig_field(run, dg[j]);
                dst[pos] = id[j];
                dig_add(run, dg[j]);
            }
        }
        __syncthreads();
        uint16_t* t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// ---------------------------------------------------------------------------
// Segmented composition over a sorted tile: for every run of equal keys
// (one pixel), the composition of its events' affine maps in arrival order.
// emit(key, acc, oid, rank) is called once per run, by the thread that owns
// the run's last item: acc is the composed map (acc.n = events in the run),
// oid the arrival index of the run's newest event, rank the run's index in
// key order.  Returns the number of runs.
// ---------------------------------------------------------------------------
template <class Emit>
__device__ uint32_t tile_compose(const uint32_t* keypol, const uint16_t* sorted, uint32_t cn,
                                 const Coef& coef, SegPair* scanp, uint32_t* scan1, Emit&& emit)
{
    const uint32_t beg = (uint32_t)threadIdx.x * kSortItems;
    uint32_t key[kSortItems], pol[kSortItems], oid[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        key[j] = 0xffffffffu;
        pol[j] = 0u;
        oid[j] = 0u;
        if (beg + j < cn) {
            oid[j] = sorted[beg + j];
            const uint32_t kp = keypol[oid[j]];
            key[j] = kp >> 1;
            pol[j] = kp & 1u;
        }
    }
    const uint32_t prevkey = (beg > 0 && beg - 1 < cn) ? (keypol[sorted[beg - 1]] >> 1) : 0xffffffffu;
    const uint32_t nextkey = (beg + kSortItems < cn) ? (keypol[sorted[beg + kSortItems]] >> 1)
                                                     : 0xffffffffu;
    SegPair agg;
    agg.flag = 0u;
    agg.v = aff_identity();
    uint32_t ntail = 0u;
    uint32_t headm = 0u, tailm = 0u;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (beg + j < cn) {
            const uint32_t pk = j == 0 ? prevkey : key[j - 1];
            const bool head = (beg + j == 0) || key[j] != pk;
            const uint32_t nk = j == kSortItems - 1 ? nextkey : key[j + 1];
            const bool tail = (beg + j == cn - 1) || key[j] != nk;
            headm |= head ? (1u << j) : 0u;
            tailm |= tail ? (1u << j) : 0u;
            const Aff e = aff_event(coef, pol[j]);
            if (head) {
                agg.flag = 1u;
                agg.v = e;
            } else {
                agg.v = aff_then(agg.v, e);
            }
            ntail += tail ? 1u : 0u;
        }
    }
    const SegPair carry = block_exscan_pair(agg, scanp);
    uint32_t total;
    uint32_t rank = block_exscan_u32(ntail, scan1, &total);
    Aff acc = carry.v;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (beg + j < cn) {
            const Aff e = aff_event(coef, pol[j]);
            acc = (headm >> j) & 1u ? e : aff_then(acc, e);
            if ((tailm >> j) & 1u) emit(key[j], acc, oid[j], rank++);
        }
    }
    return total;
}

}  // namespace
}  // namespace tile
}  // namespace fibar
