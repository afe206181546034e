/*
 * fibar_oracle.c -- plain, slow FP64 CPU reference of FIBAR.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * It processes events strictly one at a time, in the order the paper gives:
 *
 *   Temporal filter (Method, "Temporal digital filtering"):
 *     Eq. (7)   pbar_k = alpha * pbar_{k-1} + (1 - alpha) * p_k
 *     Eq. (6)   dLdet_k = p_k - pbar_k            (uses the updated pbar_k)
 *     Eq. (10)  L_k = beta * L_{k-1} + (1 + beta)/2 * dLdet_k
 *   with alpha and beta set from the cutoff period T_cut by Eq. (17) and
 *   Eq. (18), omega_cut = 2 pi / T_cut.  The update order (pbar, then the
 *   detrended increment, then L) is the one the paper recommends over the
 *   single recursion Eq. (15), because the spatial filter changes L only.
 *
 *   Spatial filter (Method, "Spatial filtering"), per event:
 *     1. temporal update of the event's pixel;
 *     2. append the event to the back of the active event queue and
 *        increment that pixel's active-event counter;
 *     3. remove events from the front until the queue length is at most the
 *        target q_targ; a pixel whose counter reaches zero becomes inactive
 *        ("stale") and gets a one-time 3x3 Gaussian blur of its L.
 *   The target is regulated after the removals by Eq. (20) with the fill
 *   ratio of Eq. (19) over 2x2 tiles (A = 4), evaluated with integer counts
 *   n_pix (active pixels) and n_tiles (active tiles):
 *     q_targ <- floor(q * r_fill / r_fill_k)
 *            =  floor(q * num * A * n_tiles / (den * n_pix)),  r_fill = num/den
 *   clamped to [q_min, q_max].
 *
 * Readings where the paper is silent or ambiguous (each stated in the
 * design notes as well):
 *   - initial pbar = L = 0;
 *   - the queue is first-in first-out (events enter at the back and leave
 *     from the front), so the window is always the newest events [h, k];
 *   - pops continue while q > q_targ; q_targ starts at q_max; the update is
 *     skipped while n_pix = 0;
 *   - blur weights are the binomial [1 2 1]^T [1 2 1] / 16 with
 *     clamp-to-edge borders, reading the current L of all nine pixels and
 *     writing only the centre; pbar is never blurred;
 *   - regulation granularity: EVENT mode regulates after every event and
 *     blurs each newly stale pixel immediately, in pop order (the paper's
 *     literal procedure).  PACKET mode applies all events of a pushed packet,
 *     then regulates once: pops, then blurs every pixel that went stale in
 *     that step from the same pre-blur snapshot (simultaneous update), then
 *     updates q_targ.  For one-event packets without multi-stale pop bursts
 *     the two coincide.
 *   - polarity byte 1 -> +1 (ON), 0 -> -1 (OFF); anything else is rejected.
 *   - time stamps are never used, except that a readout time may not be
 *     earlier than a previous readout or the newest pushed time stamp.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    REF_OK = 0, REF_E_INVALID_ARG = -1, REF_E_RANGE = -2, REF_E_POLARITY = -3,
    REF_E_TIME = -4, REF_E_NOMEM = -5
};
enum { REF_REG_PACKET = 0, REF_REG_EVENT = 1 };

typedef struct {
    double   t_cut;
    uint32_t fill_num, fill_den;
    uint32_t q_min, q_max;
    uint32_t spatial_filter;
    uint32_t regulation;
    uint32_t region;     /* per-tile queues: tile side in pixels (even), 0 = one queue */
    uint64_t age_max;    /* per-tile queues: events older than this leave (0 = W*H) */
} fibar_ref_params;

typedef struct {
    int64_t  k;          /* global index of the newest event, -1 before any */
    uint64_t h;          /* global index of the oldest queued event          */
    uint64_t q;          /* current queue length k - h + 1                   */
    uint64_t Q;          /* target queue length                              */
    uint64_t P;          /* active pixels                                    */
    uint64_t T;          /* active 2x2 tiles                                 */
    uint64_t n_regulations;
    uint64_t last_stale; /* pixels that went stale in the last regulation    */
    uint64_t total_stale;
} fibar_ref_stats;

typedef struct fibar_ref {
    uint32_t W, H, TW;
    fibar_ref_params prm;
    double alpha, beta, half_1pb;
    double *pbar, *L;
    uint64_t* tot;
    int64_t* last;
    uint32_t* cnt;
    uint32_t* tcnt;
    uint32_t* ring;      /* FIFO: event with global index e sits at ring[e % cap] */
    uint64_t ring_cap;
    int64_t k;
    uint64_t h, Q, P, T;
    uint64_t n_reg, last_stale, total_stale;
    uint64_t t_hi;       /* newest time stamp seen (pushes and readouts) */
    uint32_t* S;         /* stale list of one regulation step (PACKET mode) */
    double* Sval;
    size_t S_cap;
    double* gain;        /* per-pixel multiplier of Eq. (6), NULL: none */
    /* per-tile queues (region > 0): one FIFO of (global index, pixel) per tile */
    uint32_t RW, RH;     /* tiles across and down */
    struct ref_region* reg;
} fibar_ref;

typedef struct ref_region {
    uint64_t* ev;        /* global indices of the tile's window events, [head, tail) */
    uint32_t* pix;
    size_t head, tail, cap;
    uint64_t Q, P, T;
    uint64_t npix;       /* pixels of the tile (edge tiles are cut by the image) */
} ref_region;

/* Eq. (17): alpha_cut = (1 - sin w) / cos w. */
static double coef_alpha(double w) { return (1.0 - sin(w)) / cos(w); }
/* Eq. (18): beta_cut = (2 - cos w) - sqrt((2 - cos w)^2 - 1). */
static double coef_beta(double w)
{
    double a = 2.0 - cos(w);
    return a - sqrt(a * a - 1.0);
}

void fibar_ref_default_params(fibar_ref_params* p)
{
    p->t_cut = 40.0;      /* the paper's chosen cutoff period */
    p->fill_num = 1;      /* r_fill = 1/2, the paper's chosen fill ratio */
    p->fill_den = 2;
    p->q_min = 64;
    p->q_max = 0;         /* 0 -> number of pixels */
    p->spatial_filter = 1;
    p->regulation = REF_REG_PACKET;
    p->region = 0;
    p->age_max = 0;
}

void fibar_ref_coefficients(double t_cut, double* alpha, double* beta)
{
    double w = 2.0 * M_PI / t_cut;
    *alpha = coef_alpha(w);
    *beta = coef_beta(w);
}

void fibar_ref_destroy(fibar_ref* c)
{
    if (!c) return;
    free(c->pbar); free(c->L); free(c->tot); free(c->last); free(c->cnt);
    free(c->tcnt); free(c->ring); free(c->S); free(c->Sval); free(c->gain);
    if (c->reg) {
        for (uint64_t r = 0; r < (uint64_t)c->RW * c->RH; ++r) {
            free(c->reg[r].ev);
            free(c->reg[r].pix);
        }
        free(c->reg);
    }
    free(c);
}

int fibar_ref_create(uint32_t W, uint32_t H, const fibar_ref_params* prm, fibar_ref** out)
{
    if (!out) return REF_E_INVALID_ARG;
    *out = NULL;
    fibar_ref_params p;
    if (prm) p = *prm; else fibar_ref_default_params(&p);
    if (W == 0 || H == 0 || W > 65535 || H > 65535) return REF_E_INVALID_ARG;
    if (!(p.t_cut > 4.0) || !isfinite(p.t_cut)) return REF_E_INVALID_ARG;
    if (p.fill_num == 0 || p.fill_den == 0 || p.fill_num > p.fill_den ||
        p.fill_den > 65535) return REF_E_INVALID_ARG;
    if (p.regulation > 1 || p.spatial_filter > 1) return REF_E_INVALID_ARG;
    uint64_t npx = (uint64_t)W * H;
    if (p.q_max == 0) p.q_max = (uint32_t)(npx > 0xffffffffu ? 0xffffffffu : npx);
    if (p.q_min == 0 || p.q_min > p.q_max) return REF_E_INVALID_ARG;
    /* per-tile queues: even tile sides (whole 2x2 fill-ratio cells), packet
     * regulation with the spatial filter */
    if (p.region && ((p.region & 1u) || p.regulation != REF_REG_PACKET || !p.spatial_filter))
        return REF_E_INVALID_ARG;
    if (p.age_max == 0) p.age_max = npx;

    fibar_ref* c = (fibar_ref*)calloc(1, sizeof(fibar_ref));
    if (!c) return REF_E_NOMEM;
    c->W = W; c->H = H; c->TW = (W + 1) / 2;
    c->prm = p;
    fibar_ref_coefficients(p.t_cut, &c->alpha, &c->beta);
    c->half_1pb = 0.5 * (1.0 + c->beta);
    uint64_t ntiles = (uint64_t)c->TW * ((H + 1) / 2);
    c->pbar = (double*)calloc(npx, sizeof(double));
    c->L = (double*)calloc(npx, sizeof(double));
    c->tot = (uint64_t*)calloc(npx, sizeof(uint64_t));
    c->last = (int64_t*)malloc(npx * sizeof(int64_t));
    c->cnt = (uint32_t*)calloc(npx, sizeof(uint32_t));
    c->tcnt = (uint32_t*)calloc(ntiles, sizeof(uint32_t));
    c->ring_cap = 1024;
    c->ring = (uint32_t*)malloc(c->ring_cap * sizeof(uint32_t));
    if (!c->pbar || !c->L || !c->tot || !c->last || !c->cnt || !c->tcnt || !c->ring) {
        fibar_ref_destroy(c);
        return REF_E_NOMEM;
    }
    for (uint64_t i = 0; i < npx; ++i) c->last[i] = -1;
    c->k = -1;
    c->h = 0;
    c->Q = p.q_max;
    if (p.region) {
        c->RW = (W + p.region - 1) / p.region;
        c->RH = (H + p.region - 1) / p.region;
        c->reg = (ref_region*)calloc((size_t)c->RW * c->RH, sizeof(ref_region));
        if (!c->reg) {
            fibar_ref_destroy(c);
            return REF_E_NOMEM;
        }
        for (uint32_t ry = 0; ry < c->RH; ++ry)
            for (uint32_t rx = 0; rx < c->RW; ++rx) {
                ref_region* g = &c->reg[(size_t)ry * c->RW + rx];
                uint32_t w = W - rx * p.region < p.region ? W - rx * p.region : p.region;
                uint32_t h = H - ry * p.region < p.region ? H - ry * p.region : p.region;
                g->npix = (uint64_t)w * h;
                g->Q = g->npix;
            }
    }
    *out = c;
    return REF_OK;
}

static uint32_t tile_of(const fibar_ref* c, uint32_t i)
{
    uint32_t x = i % c->W, y = i / c->W;
    return (y >> 1) * c->TW + (x >> 1);
}

/* 3x3 binomial blur of L at pixel i, clamp-to-edge, reading current L. */
static double blur_at(const fibar_ref* c, uint32_t i)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int x = (int)(i % c->W), y = (int)(i / c->W);
    double acc = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        int yy = y + dy;
        if (yy < 0) yy = 0;
        if (yy >= (int)c->H) yy = (int)c->H - 1;
        for (int dx = -1; dx <= 1; ++dx) {
            int xx = x + dx;
            if (xx < 0) xx = 0;
            if (xx >= (int)c->W) xx = (int)c->W - 1;
            acc += w[dy + 1] * w[dx + 1] * c->L[(size_t)yy * c->W + xx];
        }
    }
    return acc;
}

static int ring_push(fibar_ref* c, uint32_t pix)
{
    uint64_t q = (uint64_t)(c->k + 1) - c->h; /* length before this push (k already advanced) */
    if (q >= c->ring_cap) {
        uint64_t nc = c->ring_cap * 2;
        uint32_t* nr = (uint32_t*)malloc(nc * sizeof(uint32_t));
        if (!nr) return REF_E_NOMEM;
        for (uint64_t e = c->h; e < (uint64_t)c->k; ++e) nr[e % nc] = c->ring[e % c->ring_cap];
        free(c->ring);
        c->ring = nr;
        c->ring_cap = nc;
    }
    c->ring[(uint64_t)c->k % c->ring_cap] = pix;
    return REF_OK;
}

static int stale_append(fibar_ref* c, uint32_t pix)
{
    if (c->last_stale == c->S_cap) {
        size_t nc = c->S_cap ? 2 * c->S_cap : 1024;
        uint32_t* ns = (uint32_t*)realloc(c->S, nc * sizeof(uint32_t));
        if (!ns) return REF_E_NOMEM;
        c->S = ns;
        double* nv = (double*)realloc(c->Sval, nc * sizeof(double));
        if (!nv) return REF_E_NOMEM;
        c->Sval = nv;
        c->S_cap = nc;
    }
    c->S[c->last_stale] = pix;
    return REF_OK;
}

/* Pops, stale handling and the Eq. (20) update; one regulation step. */
static int regulate(fibar_ref* c)
{
    const int event_mode = c->prm.regulation == REF_REG_EVENT;
    c->last_stale = 0;
    while ((uint64_t)(c->k + 1) - c->h > c->Q) {
        uint32_t j = c->ring[c->h % c->ring_cap];
        c->h++;
        c->cnt[j]--;
        if (c->cnt[j] == 0) {
            c->P--;
            uint32_t t = tile_of(c, j);
            c->tcnt[t]--;
            if (c->tcnt[t] == 0) c->T--;
            if (event_mode) {
                c->L[j] = blur_at(c, j);
            } else {
                int rc = stale_append(c, j);
                if (rc) return rc;
            }
            c->last_stale++;
        }
    }
    if (!event_mode) {
        for (uint64_t s = 0; s < c->last_stale; ++s) c->Sval[s] = blur_at(c, c->S[s]);
        for (uint64_t s = 0; s < c->last_stale; ++s) c->L[c->S[s]] = c->Sval[s];
    }
    c->total_stale += c->last_stale;
    uint64_t q = (uint64_t)(c->k + 1) - c->h;
    if (c->P > 0) {
        unsigned __int128 num = (unsigned __int128)q * c->prm.fill_num * 4u * c->T;
        unsigned __int128 den = (unsigned __int128)c->prm.fill_den * c->P;
        unsigned __int128 v = num / den;
        uint64_t Q = v > c->prm.q_max ? c->prm.q_max : (uint64_t)v;
        if (Q < c->prm.q_min) Q = c->prm.q_min;
        c->Q = Q;
    }
    c->n_reg++;
    return REF_OK;
}

/*
 * Per-tile queues (Limitations: event queues operated separately for each
 * tile of the image).  Readings, the paper leaving them open: tiles are
 * region x region pixels (even, so the 2x2 cells of Eq. (19) never straddle
 * two tiles; edge tiles are cut by the image); each tile keeps its own FIFO
 * window of its own events, its own active pixel and 2x2 cell counts, and its
 * own target of Eq. (20) from them, clamped to [min(q_min, n), n] with n the
 * tile's pixels and starting at n; a tile that no longer registers events
 * still advances, because an event also leaves once age_max newer events
 * have arrived anywhere on the sensor (0 = W*H, the single queue's bound).
 * Regulation is per pushed packet: after the packet's events, every tile
 * pops, all pixels gone stale are blurred from the same pre-blur image, and
 * every tile with an active pixel updates its target.
 */
static uint32_t region_of(const fibar_ref* c, uint32_t i)
{
    uint32_t x = i % c->W, y = i / c->W;
    return (y / c->prm.region) * c->RW + x / c->prm.region;
}

static int region_push(ref_region* g, uint64_t e, uint32_t pix)
{
    if (g->tail == g->cap) {
        size_t live = g->tail - g->head;
        if (g->head > 0 && live < g->cap / 2) {
            memmove(g->ev, g->ev + g->head, live * sizeof(uint64_t));
            memmove(g->pix, g->pix + g->head, live * sizeof(uint32_t));
        } else {
            size_t nc = g->cap ? 2 * g->cap : 64;
            uint64_t* ne = (uint64_t*)malloc(nc * sizeof(uint64_t));
            uint32_t* np = (uint32_t*)malloc(nc * sizeof(uint32_t));
            if (!ne || !np) { free(ne); free(np); return REF_E_NOMEM; }
            if (live) {
                memcpy(ne, g->ev + g->head, live * sizeof(uint64_t));
                memcpy(np, g->pix + g->head, live * sizeof(uint32_t));
            }
            free(g->ev); free(g->pix);
            g->ev = ne; g->pix = np; g->cap = nc;
        }
        g->head = 0;
        g->tail = live;
    }
    g->ev[g->tail] = e;
    g->pix[g->tail] = pix;
    g->tail++;
    return REF_OK;
}

static int regulate_regions(fibar_ref* c)
{
    c->last_stale = 0;
    const uint64_t nreg = (uint64_t)c->RW * c->RH;
    for (uint64_t r = 0; r < nreg; ++r) {
        ref_region* g = &c->reg[r];
        while (g->tail > g->head &&
               (g->tail - g->head > g->Q || (uint64_t)c->k - g->ev[g->head] >= c->prm.age_max)) {
            uint32_t j = g->pix[g->head];
            g->head++;
            c->cnt[j]--;
            if (c->cnt[j] == 0) {
                g->P--;
                uint32_t t = tile_of(c, j);
                c->tcnt[t]--;
                if (c->tcnt[t] == 0) g->T--;
                int rc = stale_append(c, j);
                if (rc) return rc;
                c->last_stale++;
            }
        }
    }
    for (uint64_t s = 0; s < c->last_stale; ++s) c->Sval[s] = blur_at(c, c->S[s]);
    for (uint64_t s = 0; s < c->last_stale; ++s) c->L[c->S[s]] = c->Sval[s];
    c->total_stale += c->last_stale;
    uint64_t q_all = 0, P_all = 0, T_all = 0, Q_all = 0;
    for (uint64_t r = 0; r < nreg; ++r) {
        ref_region* g = &c->reg[r];
        uint64_t q = g->tail - g->head;
        if (g->P > 0) {
            unsigned __int128 num = (unsigned __int128)q * c->prm.fill_num * 4u * g->T;
            unsigned __int128 den = (unsigned __int128)c->prm.fill_den * g->P;
            unsigned __int128 v = num / den;
            uint64_t lo = c->prm.q_min < g->npix ? c->prm.q_min : g->npix;
            uint64_t Q = v > g->npix ? g->npix : (uint64_t)v;
            if (Q < lo) Q = lo;
            g->Q = Q;
        }
        q_all += q;
        P_all += g->P;
        T_all += g->T;
        Q_all += g->Q;
    }
    /* whole-sensor figures: q, Q, P and T summed over tiles, h = k + 1 - q */
    c->h = (uint64_t)(c->k + 1) - q_all;
    c->Q = Q_all;
    c->P = P_all;
    c->T = T_all;
    c->n_reg++;
    return REF_OK;
}

/* Per-tile scalars after the last step (per-tile queues only): window
 * length, target, active pixels and cells, and the global index of the
 * oldest window event (k + 1 when the window is empty).  Arrays of
 * tiles_x * tiles_y entries, row-major; any pointer may be NULL. */
int fibar_ref_region_stats(const fibar_ref* c, uint64_t* q, uint64_t* Q, uint64_t* P, uint64_t* T,
                           uint64_t* front)
{
    if (!c || !c->reg) return REF_E_INVALID_ARG;
    const uint64_t nreg = (uint64_t)c->RW * c->RH;
    for (uint64_t r = 0; r < nreg; ++r) {
        const ref_region* g = &c->reg[r];
        if (q) q[r] = g->tail - g->head;
        if (Q) Q[r] = g->Q;
        if (P) P[r] = g->P;
        if (T) T[r] = g->T;
        if (front) front[r] = g->tail > g->head ? g->ev[g->head] : (uint64_t)(c->k + 1);
    }
    return REF_OK;
}

int fibar_ref_push_events(fibar_ref* c, const uint16_t* x, const uint16_t* y, const uint8_t* p,
                          const uint64_t* t, size_t n)
{
    if (!c) return REF_E_INVALID_ARG;
    if (n == 0) return REF_OK;
    if (!x || !y || !p) return REF_E_INVALID_ARG;
    /* validate the whole packet first: a rejected packet changes nothing */
    for (size_t e = 0; e < n; ++e)
        if (x[e] >= c->W || y[e] >= c->H) return REF_E_RANGE;
    for (size_t e = 0; e < n; ++e)
        if (p[e] > 1) return REF_E_POLARITY;

    const double a = c->alpha, b = c->beta, g = c->half_1pb;
    for (size_t e = 0; e < n; ++e) {
        uint32_t i = (uint32_t)y[e] * c->W + x[e];
        double pk = p[e] ? 1.0 : -1.0;
        c->k++;
        c->pbar[i] = a * c->pbar[i] + (1.0 - a) * pk;    /* Eq. (7)  */
        double d = pk - c->pbar[i];                      /* Eq. (6)  */
        if (c->gain) d *= c->gain[i];                    /* relative threshold C'_i */
        c->L[i] = b * c->L[i] + g * d;                   /* Eq. (10) */
        c->tot[i]++;
        c->last[i] = c->k;
        if (c->prm.spatial_filter && c->reg) {
            ref_region* g = &c->reg[region_of(c, i)];
            if (c->cnt[i] == 0) {
                g->P++;
                uint32_t tl = tile_of(c, i);
                if (c->tcnt[tl] == 0) g->T++;
                c->tcnt[tl]++;
            }
            c->cnt[i]++;
            int rc = region_push(g, (uint64_t)c->k, i);
            if (rc) return rc;
        } else if (c->prm.spatial_filter) {
            if (c->cnt[i] == 0) {
                c->P++;
                uint32_t tl = tile_of(c, i);
                if (c->tcnt[tl] == 0) c->T++;
                c->tcnt[tl]++;
            }
            c->cnt[i]++;
            int rc = ring_push(c, i);
            if (rc) return rc;
            if (c->prm.regulation == REF_REG_EVENT) {
                rc = regulate(c);
                if (rc) return rc;
            }
        }
    }
    if (c->prm.spatial_filter && c->prm.regulation == REF_REG_PACKET) {
        int rc = c->reg ? regulate_regions(c) : regulate(c);
        if (rc) return rc;
    }
    if (t && t[n - 1] > c->t_hi) c->t_hi = t[n - 1];
    return REF_OK;
}

/*
 * Copy the state out.  Any output pointer may be NULL.  stale[i] is 1 for a
 * pixel that has had events but has none left in the queue.
 */
int fibar_ref_readout(fibar_ref* c, uint64_t t, double* L, double* pbar, uint32_t* cnt,
                      uint64_t* tot, int64_t* last, uint32_t* tcnt, uint8_t* stale)
{
    if (!c) return REF_E_INVALID_ARG;
    if (t < c->t_hi) return REF_E_TIME;
    c->t_hi = t;
    uint64_t npx = (uint64_t)c->W * c->H;
    if (L) memcpy(L, c->L, npx * sizeof(double));
    if (pbar) memcpy(pbar, c->pbar, npx * sizeof(double));
    if (cnt) memcpy(cnt, c->cnt, npx * sizeof(uint32_t));
    if (tot) memcpy(tot, c->tot, npx * sizeof(uint64_t));
    if (last) memcpy(last, c->last, npx * sizeof(int64_t));
    if (tcnt) memcpy(tcnt, c->tcnt, (uint64_t)c->TW * ((c->H + 1) / 2) * sizeof(uint32_t));
    if (stale)
        for (uint64_t i = 0; i < npx; ++i)
            stale[i] = (uint8_t)(c->prm.spatial_filter && c->tot[i] > 0 && c->cnt[i] == 0);
    return REF_OK;
}

int fibar_ref_get_stats(const fibar_ref* c, fibar_ref_stats* s)
{
    if (!c || !s) return REF_E_INVALID_ARG;
    s->k = c->k;
    s->h = c->h;
    s->q = (uint64_t)(c->k + 1) - c->h;
    s->Q = c->Q;
    s->P = c->P;
    s->T = c->T;
    s->n_regulations = c->n_reg;
    s->last_stale = c->last_stale;
    s->total_stale = c->total_stale;
    return REF_OK;
}

/*
 * Relative-threshold variant (Experiments, "Inter-pixel threshold
 * variation"): the detrended increment of Eq. (6) at pixel i is multiplied
 * by gain[i] (the relative threshold C'_i of the threshold appendix).
 * gain == NULL removes the multipliers.  The values are copied.
 */
int fibar_ref_set_gain(fibar_ref* c, const double* gain)
{
    if (!c) return REF_E_INVALID_ARG;
    if (!gain) {
        free(c->gain);
        c->gain = NULL;
        return REF_OK;
    }
    uint64_t npx = (uint64_t)c->W * c->H;
    if (!c->gain) {
        c->gain = (double*)malloc(npx * sizeof(double));
        if (!c->gain) return REF_E_NOMEM;
    }
    memcpy(c->gain, gain, npx * sizeof(double));
    return REF_OK;
}

/* The coefficients in use, for tests. */
int fibar_ref_get_coefficients(const fibar_ref* c, double* alpha, double* beta)
{
    if (!c) return REF_E_INVALID_ARG;
    *alpha = c->alpha;
    *beta = c->beta;
    return REF_OK;
}
