// Per-event regulation (the paper's literal procedure; Method, "Spatial
// filtering", steps 1-3, with the target of Eq. (20) updated after every
// event): for every event in order, the temporal filter of its pixel
// (Eq. (6), (7), (10)), its entry at the back of the window, then old events
// leave from the front while the window is longer than the target; a pixel
// whose last window event leaves goes stale and is blurred at once (3x3
// binomial, clamp-to-edge) from the current image, so a later blur of the
// same step sees an earlier one; then the target is recomputed from the
// active pixel and tile counts.
//
// The chain of one event depends on the one before it (window head, target,
// counts, and the image through the blur), so a packet runs in one
// workgroup with the whole state in LDS: brightness, polarity average,
// per-pixel window counts, per-tile active counts, the window's pixel ids,
// and the pixels' relative thresholds (1 without them).  One wave walks the events; the others only help load and store the
// state around it.  Sensors up to kEventMaxPixels pixels, windows up to
// kEventMaxRing - 2 events.
#include "fibar_internal.h"
#include "fibar_step.h"

namespace fibar {
namespace {

constexpr int kEvBlock = 256;

struct EvLayout {
    uint32_t npx, ntiles, cap;
    size_t off_pb, off_gn, off_ring, off_cnt, off_tcnt, bytes;
};

__host__ __device__ inline size_t ev_align(size_t v) { return (v + 15) & ~size_t(15); }

__host__ __device__ inline EvLayout ev_layout(uint32_t W, uint32_t H, uint32_t TW, uint32_t cap)
{
    EvLayout l;
    l.npx = W * H;
    l.ntiles = TW * ((H + 1) / 2);
    l.cap = cap;
    l.off_pb = ev_align((size_t)l.npx * 4);
    l.off_gn = l.off_pb + ev_align((size_t)l.npx * 4);
    l.off_ring = l.off_gn + ev_align((size_t)l.npx * 4);
    l.off_cnt = l.off_ring + ev_align((size_t)cap * 2);
    l.off_tcnt = l.off_cnt + ev_align((size_t)l.npx * 2);
    l.bytes = l.off_tcnt + ev_align(l.ntiles);
    return l;
}

// Row of pixel j (j < 2^16, so the float quotient is off by at most one).
__device__ __forceinline__ uint32_t ev_row(uint32_t j, uint32_t W, float inv_w)
{
    uint32_t y = (uint32_t)((float)j * inv_w);
    if (y * W > j) --y;
    else if ((y + 1) * W <= j) ++y;
    return y;
}

__global__ __launch_bounds__(kEvBlock) void k_event_packet(State s, int slot,
                                                           const uint16_t* __restrict__ ex,
                                                           const uint16_t* __restrict__ ey,
                                                           const uint8_t* __restrict__ ep,
                                                           uint32_t n, Coef coef, uint32_t cap,
                                                           float inv_w)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t bad;
    __shared__ uint64_t fin_h;
    __shared__ int64_t fin_k;
    const EvLayout lay = ev_layout(s.W, s.H, s.TW, cap);
    float* L = reinterpret_cast<float*>(lds);
    float* pb = reinterpret_cast<float*>(lds + lay.off_pb);
    float* gn = reinterpret_cast<float*>(lds + lay.off_gn);   // relative thresholds
    uint16_t* ring = reinterpret_cast<uint16_t*>(lds + lay.off_ring);
    uint16_t* cnt = reinterpret_cast<uint16_t*>(lds + lay.off_cnt);
    uint8_t* tcnt = lds + lay.off_tcnt;
    const uint32_t tid = threadIdx.x;
    const uint32_t W = s.W, H = s.H, TW = s.TW;
    const uint32_t cmask = cap - 1;

    // all-or-nothing validation: range errors take precedence
    if (tid == 0) bad = 0;
    __syncthreads();
    uint32_t my = 0;
    for (uint32_t e = tid; e < n; e += kEvBlock) {
        if (ex[e] >= W || ey[e] >= H) my |= 1u;
        if (ep[e] > 1) my |= 2u;
    }
    if (my) atomicOr(&bad, my);
    __syncthreads();
    if (bad) {
        if (tid == 0 && s.sc[slot].err == 0) s.sc[slot].err = (bad & 1u) ? -2 : -3;
        return;
    }

    // the state into LDS: a pixel's current brightness is Lb when stale
    const DevScalars c0 = s.sc[slot];
    for (uint32_t i = tid; i < lay.npx; i += kEvBlock) {
        const PixL v = s.px[i];
        L[i] = v.last < (int64_t)c0.h ? v.Lb : v.L;
        const PixP w = s.pp[i];
        pb[i] = w.pbar;
        cnt[i] = (uint16_t)w.cnt;
        gn[i] = s.gain ? s.gain[i] : 1.f;
    }
    for (uint64_t e = c0.h + tid; (int64_t)e <= c0.k; e += kEvBlock)
        ring[e & cmask] = (uint16_t)s.ring[e & s.ring_mask];
    __syncthreads();
    for (uint32_t t = tid; t < lay.ntiles; t += kEvBlock) {
        const uint32_t tx = t % TW, ty = t / TW;
        uint32_t a = 0;
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t x = 2 * tx + (q & 1), y = 2 * ty + (q >> 1);
            if (x < W && y < H && cnt[y * W + x] != 0) ++a;
        }
        tcnt[t] = (uint8_t)a;
    }
    __syncthreads();

    if (tid < 64) {
        // wave 0 loads the events, 64 per block with the next block in
        // flight; lane 0 alone walks them (one lane issues every LDS access
        // of the walk).  Inside a packet the window head, the newest index,
        // the counts and the target fit 32 bits: indices are taken relative
        // to the head the packet starts from.
        const uint32_t lane = tid;
        const uint64_t base = c0.h;
        const uint32_t bm = (uint32_t)(base & cmask);
        uint32_t hl = 0;                                     // head - base
        uint32_t kq = (uint32_t)((uint64_t)(c0.k + 1) - base);   // newest + 1 - base
        uint32_t Q = (uint32_t)c0.Q, P = (uint32_t)c0.P, T = (uint32_t)c0.T;
        uint32_t st = 0, total = 0;
        const uint32_t num4 = 4u * s.fill_num, den = s.fill_den;
        const uint32_t q_min = (uint32_t)s.q_min, q_max = (uint32_t)s.q_max;
        const float g = 0.5f * (1.0f + coef.beta);
        auto load_block = [&](uint32_t b, uint32_t& xy, uint32_t& pol) {
            const uint32_t e = b * 64 + lane;
            const uint32_t ec = e < n ? e : n - 1;
            xy = (uint32_t)ex[ec] | ((uint32_t)ey[ec] << 16);
            pol = ep[ec];
        };
        uint32_t cur_xy, cur_p;
        load_block(0, cur_xy, cur_p);
        const uint32_t nblocks = (n + 63) / 64;
        for (uint32_t b = 0; b < nblocks; ++b) {
            uint32_t nxt_xy = 0, nxt_p = 0;
            if (b + 1 < nblocks) load_block(b + 1, nxt_xy, nxt_p);
            const uint32_t m = n - b * 64 < 64 ? n - b * 64 : 64;
            for (uint32_t e = 0; lane == 0 && e < m; ++e) {
                const uint32_t xy = __builtin_amdgcn_readlane(cur_xy, e);
                const uint32_t pol = __builtin_amdgcn_readlane(cur_p, e);
                const uint32_t x = xy & 0xffffu, y = xy >> 16;
                const uint32_t i = y * W + x, t = (y >> 1) * TW + (x >> 1);
                // step 1: the temporal filter (Eq. (7), then (6) and (10))
                const float pk = pol ? 1.f : -1.f;
                const float pbi = pb[i], Li = L[i], gi = gn[i];
                const uint32_t ci = cnt[i], tci = tcnt[t];
                const float pbn = fmaf(coef.alpha, pbi, coef.one_m_alpha * pk);
                pb[i] = pbn;
                L[i] = fmaf(coef.beta, Li, (g * gi) * (pk - pbn));
                s.px[i].last = c0.k + 1 + (int64_t)(b * 64 + e);
                atomicAdd(reinterpret_cast<unsigned long long*>(&s.pp[i].tot), 1ull);
                // step 2: the event enters the window
                if (ci == 0) {
                    ++P;
                    if (tci == 0) ++T;
                    tcnt[t] = (uint8_t)(tci + 1);
                }
                cnt[i] = (uint16_t)(ci + 1);
                ring[(bm + kq) & cmask] = (uint16_t)i;
                ++kq;
                // step 3: old events leave; a pixel without window events
                // goes stale and is blurred from the current image
                st = 0;
                while (kq - hl > Q) {
                    const uint32_t j = ring[(bm + hl) & cmask];
                    ++hl;
                    const uint32_t yj = ev_row(j, W, inv_w), xj = j - yj * W;
                    const uint32_t xs[3] = {xj > 0 ? xj - 1 : 0, xj, xj + 1 < W ? xj + 1 : W - 1};
                    const uint32_t ys[3] = {yj > 0 ? yj - 1 : 0, yj, yj + 1 < H ? yj + 1 : H - 1};
                    const uint32_t tj = (yj >> 1) * TW + (xj >> 1);
                    const uint32_t cj = cnt[j], tcj = tcnt[tj];
                    float nb[3][3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int bb = 0; bb < 3; ++bb) nb[a][bb] = L[ys[a] * W + xs[bb]];
                    cnt[j] = (uint16_t)(cj - 1);
                    if (cj == 1) {
                        --P;
                        tcnt[tj] = (uint8_t)(tcj - 1);
                        if (tcj == 1) --T;
                        const float r0 = nb[0][0] + 2.f * nb[0][1] + nb[0][2];
                        const float r1 = nb[1][0] + 2.f * nb[1][1] + nb[1][2];
                        const float r2 = nb[2][0] + 2.f * nb[2][1] + nb[2][2];
                        L[j] = (r0 + 2.f * r1 + r2) * 0.0625f;
                        ++st;
                    }
                }
                // the target of Eq. (20) from the integer counts:
                // floor(q num 4 T / (den P)); the numerator is below 2^53 and
                // the divisor below 2^32, so the double quotient is within
                // one unit and one integer check fixes it
                if (P > 0) {
                    const uint64_t num = (uint64_t)(kq - hl) * T * num4;
                    const uint64_t dv = (uint64_t)den * P;
                    uint64_t v = (uint64_t)((double)num / (double)dv);
                    if (v * dv > num) --v;
                    else if ((v + 1) * dv <= num) ++v;
                    Q = v > q_max ? q_max : (v < q_min ? q_min : (uint32_t)v);
                }
                total += st;
            }
            cur_xy = nxt_xy;
            cur_p = nxt_p;
        }
        if (lane == 0) {
            DevScalars r = c0;
            r.k = c0.k + (int64_t)n;
            r.h = base + hl;
            r.Q = Q;
            r.P = P;
            r.T = T;
            r.n_reg = c0.n_reg + n;
            r.last_stale = st;
            r.total_stale = c0.total_stale + total;
            r.stepped = 1;
            s.sc[slot] = r;
            fin_h = r.h;
            fin_k = r.k;
        }
    }
    __syncthreads();

    // back to device memory: brightness (as both L and Lb: the readouts
    // pick Lb for stale pixels), polarity average and window count, and the
    // pixel ids of this packet's events still in the window
    for (uint32_t i = tid; i < lay.npx; i += kEvBlock) {
        const float v = L[i];
        *reinterpret_cast<float2*>(&s.px[i]) = make_float2(v, v);
        *reinterpret_cast<uint2*>(&s.pp[i]) = make_uint2(__float_as_uint(pb[i]), cnt[i]);
    }
    const uint64_t lo = (uint64_t)(c0.k + 1) > fin_h ? (uint64_t)(c0.k + 1) : fin_h;
    for (uint64_t e = lo + tid; (int64_t)e <= fin_k; e += kEvBlock)
        s.ring[e & s.ring_mask] = ring[e & cmask];
}

}  // namespace

size_t event_lds_bytes(uint32_t W, uint32_t H, uint32_t TW, uint32_t cap)
{
    return ev_layout(W, H, TW, cap).bytes;
}

hipError_t prepare_event_kernel(size_t lds_bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_event_packet),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_event_packet(const State& s, int slot, const uint16_t* x, const uint16_t* y,
                               const uint8_t* p, uint32_t n, const Coef& coef, uint32_t cap,
                               size_t lds_bytes, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const float inv_w = 1.0f / (float)s.W;
    hipLaunchKernelGGL(k_event_packet, dim3(1), dim3(kEvBlock), lds_bytes, st, s, slot, x, y, p, n,
                       coef, cap, inv_w);
    return hipGetLastError();
}

}  // namespace fibar
