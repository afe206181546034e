/*
 * eventsim.c -- seeded synthetic event-camera simulator with ground truth.
 *
 * Input generator shared by the tests and the benchmark.  It contains none of
 * the reconstruction method's arithmetic: it only produces events and the
 * ground-truth log-intensity frames they come from.
 *
 * Event model (paper, Notation section, Eq. (1)-(3)): brightness is the log of
 * the photocurrent; a pixel emits an ON (OFF) event each time its brightness
 * has risen (fallen) by its contrast threshold C_ON (C_OFF) since the last
 * event, so each event carries a brightness change of C_p * p.
 *
 * Scene: a static log-intensity texture on a periodic canvas of 2W x 2H
 * texels (a sum of Gaussian blobs, optionally plus a random checkerboard),
 * seen through a sensor that translates and rotates over it.  The texture is
 * rendered once and sampled bilinearly; each time step moves every pixel by at
 * most `step_px` texels.  Crossing times are interpolated linearly inside a
 * step.  Noise events are uniform over pixels, polarity and time within a
 * step.  Events of one step are ordered by (time, pixel index).
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
 * from its published definition; every draw is addressed by a counter
 * (purpose, index, sub-index), so the output depends only on the seed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ----------------------------------------------------------------------- */
/* Philox4x32-10                                                             */
/* ----------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void sim_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct { uint32_t key[2]; } rng_t;

/* Four uniforms in [0,1) for counter (purpose, a, b). */
static void rng_u4(const rng_t* r, uint32_t purpose, uint32_t a, uint32_t b, double u[4])
{
    uint32_t ctr[4] = {purpose, a, b, 0x5eedu};
    uint32_t o[4];
    sim_philox4x32_10(ctr, r->key, o);
    for (int i = 0; i < 4; ++i) u[i] = (o[i] + 0.5) * (1.0 / 4294967296.0);
}

enum { P_BLOB = 1, P_CHECK = 2, P_THR = 3, P_MOTION = 4, P_NOISE = 5 };

/* ----------------------------------------------------------------------- */
/* Parameters                                                                */
/* ----------------------------------------------------------------------- */
typedef struct {
    int32_t  width, height;
    uint64_t n_events;        /* events to produce                        */
    uint64_t seed;
    int32_t  n_blobs;
    double   amp_lo, amp_hi;  /* blob amplitude ~ U(amp_lo, amp_hi)        */
    double   sig_lo, sig_hi;  /* blob sigma (texels) ~ U(sig_lo, sig_hi)   */
    double   checker_cell;    /* checkerboard cell size in texels, 0 = off */
    double   checker_contrast;/* each cell is +-contrast/2                 */
    double   speed_px_s;      /* translation speed (texels / s)            */
    double   rot_rad_s;       /* rotation rate about the sensor centre     */
    double   thr_on, thr_off; /* mean contrast thresholds                  */
    double   thr_jitter;      /* per-pixel threshold ~ U(C - j, C + j)     */
    double   noise_frac;      /* fraction of all events that are noise     */
    double   step_px;         /* max motion of any pixel per step          */
} sim_params;

typedef struct {
    sim_params p;
    rng_t rng;
    int cw, ch;               /* canvas size */
    float* tex;               /* cw*ch texture */
    double vx, vy;            /* translation velocity */
    double dt;                /* step duration, s */
} scene_t;

static double wrap(double v, double m)
{
    double r = v - floor(v / m) * m;
    return r >= m ? r - m : r;
}

static int scene_init(scene_t* s, const sim_params* p)
{
    memset(s, 0, sizeof(*s));
    s->p = *p;
    s->rng.key[0] = (uint32_t)p->seed;
    s->rng.key[1] = (uint32_t)(p->seed >> 32) ^ 0x243F6A88u;
    s->cw = 2 * p->width;
    s->ch = 2 * p->height;
    s->tex = (float*)calloc((size_t)s->cw * s->ch, sizeof(float));
    if (!s->tex) return -1;
    double* acc = (double*)calloc((size_t)s->cw * s->ch, sizeof(double));
    if (!acc) { free(s->tex); return -1; }

    for (int b = 0; b < p->n_blobs; ++b) {
        double u[4];
        rng_u4(&s->rng, P_BLOB, (uint32_t)b, 0, u);
        double cx = u[0] * s->cw, cy = u[1] * s->ch;
        double a = p->amp_lo + (p->amp_hi - p->amp_lo) * u[2];
        double sg = p->sig_lo + (p->sig_hi - p->sig_lo) * u[3];
        int rad = (int)ceil(4.0 * sg);
        double inv2s2 = 1.0 / (2.0 * sg * sg);
        int x0 = (int)floor(cx), y0 = (int)floor(cy);
        for (int dy = -rad; dy <= rad + 1; ++dy) {
            int ty = y0 + dy;
            double ddy = ty - cy;
            int wy = ((ty % s->ch) + s->ch) % s->ch;
            for (int dx = -rad; dx <= rad + 1; ++dx) {
                int tx = x0 + dx;
                double ddx = tx - cx;
                int wx = ((tx % s->cw) + s->cw) % s->cw;
                acc[(size_t)wy * s->cw + wx] += a * exp(-(ddx * ddx + ddy * ddy) * inv2s2);
            }
        }
    }
    if (p->checker_cell > 0 && p->checker_contrast != 0) {
        int ncx = (int)ceil(s->cw / p->checker_cell);
        for (int ty = 0; ty < s->ch; ++ty) {
            int cy = (int)(ty / p->checker_cell);
            for (int tx = 0; tx < s->cw; ++tx) {
                int cx = (int)(tx / p->checker_cell);
                double u[4];
                rng_u4(&s->rng, P_CHECK, (uint32_t)(cy * ncx + cx), 0, u);
                acc[(size_t)ty * s->cw + tx] += (u[0] < 0.5 ? -0.5 : 0.5) * p->checker_contrast;
            }
        }
    }
    for (size_t i = 0; i < (size_t)s->cw * s->ch; ++i) s->tex[i] = (float)acc[i];
    free(acc);

    double u[4];
    rng_u4(&s->rng, P_MOTION, 0, 0, u);
    double phi = 2.0 * M_PI * u[0];
    s->vx = p->speed_px_s * cos(phi);
    s->vy = p->speed_px_s * sin(phi);
    double rmax = 0.5 * sqrt((double)p->width * p->width + (double)p->height * p->height);
    double vmax = p->speed_px_s + fabs(p->rot_rad_s) * rmax;
    s->dt = vmax > 0 ? p->step_px / vmax : 1e-3;
    return 0;
}

static void scene_free(scene_t* s) { free(s->tex); s->tex = NULL; }

/* Bilinear sample of the periodic texture at canvas coordinate (u, v). */
static double tex_sample(const scene_t* s, double u, double v)
{
    u = wrap(u, s->cw);
    v = wrap(v, s->ch);
    int x0 = (int)u, y0 = (int)v;
    double fx = u - x0, fy = v - y0;
    int x1 = x0 + 1 == s->cw ? 0 : x0 + 1;
    int y1 = y0 + 1 == s->ch ? 0 : y0 + 1;
    const float* r0 = s->tex + (size_t)y0 * s->cw;
    const float* r1 = s->tex + (size_t)y1 * s->cw;
    double a = r0[x0] + fx * (r0[x1] - r0[x0]);
    double b = r1[x0] + fx * (r1[x1] - r1[x0]);
    return a + fy * (b - a);
}

/* Bilinear sample at a coordinate already inside [0,cw) x [0,ch). */
static inline double tex_sample_wrapped(const scene_t* s, double u, double v)
{
    int x0 = (int)u, y0 = (int)v;
    if (x0 >= s->cw) x0 = s->cw - 1;
    if (y0 >= s->ch) y0 = s->ch - 1;
    double fx = u - x0, fy = v - y0;
    int x1 = x0 + 1 == s->cw ? 0 : x0 + 1;
    int y1 = y0 + 1 == s->ch ? 0 : y0 + 1;
    const float* r0 = s->tex + (size_t)y0 * s->cw;
    const float* r1 = s->tex + (size_t)y1 * s->cw;
    double a = r0[x0] + fx * (r0[x1] - r0[x0]);
    double b = r1[x0] + fx * (r1[x1] - r1[x0]);
    return a + fy * (b - a);
}

/* Ground-truth log intensity of every sensor pixel at time t (seconds). */
static void scene_render(const scene_t* s, double t, double* out)
{
    const int W = s->p.width, H = s->p.height;
    double th = s->p.rot_rad_s * t;
    double c = cos(th), sn = sin(th);
    double ox = 0.5 * (W - 1), oy = 0.5 * (H - 1);
    double tx = ox + 0.5 * W + s->vx * t, ty = oy + 0.5 * H + s->vy * t;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        double ry = y - oy;
        for (int x = 0; x < W; ++x) {
            double rx = x - ox;
            double u = c * rx - sn * ry + tx;
            double v = sn * rx + c * ry + ty;
            out[(size_t)y * W + x] = tex_sample(s, u, v);
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Event generation                                                          */
/* ----------------------------------------------------------------------- */
typedef struct { uint64_t t; uint32_t pix; uint8_t pol; } ev_t;

static int ev_cmp(const void* a, const void* b)
{
    const ev_t* x = (const ev_t*)a;
    const ev_t* y = (const ev_t*)b;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    if (x->pix != y->pix) return x->pix < y->pix ? -1 : 1;
    return (int)x->pol - (int)y->pol;
}

/* Growable per-thread event buffer. */
typedef struct { ev_t* v; size_t n, cap; int oom; } evbuf_t;

static void evbuf_push(evbuf_t* b, uint64_t t, uint32_t pix, uint8_t pol)
{
    if (b->n == b->cap) {
        size_t nc = b->cap ? 2 * b->cap : 4096;
        ev_t* nv = (ev_t*)realloc(b->v, nc * sizeof(ev_t));
        if (!nv) { b->oom = 1; return; }
        b->v = nv; b->cap = nc;
    }
    b->v[b->n].t = t; b->v[b->n].pix = pix; b->v[b->n].pol = pol;
    ++b->n;
}

/*
 * Produce exactly p->n_events events (fewer only if `max_steps` is hit).
 * Returns the number produced, or -1 on allocation failure.  `steps_out`
 * (optional) receives the number of time steps simulated.  Rows are
 * simulated in parallel; the result does not depend on the thread count
 * because every step's events are put in (time, pixel, polarity) order.
 */
int64_t sim_generate(const sim_params* p, uint16_t* xs, uint16_t* ys, uint8_t* ps,
                     uint64_t* ts, uint64_t max_steps, uint64_t* steps_out)
{
    if (p->width <= 0 || p->height <= 0 || p->width > 65535 || p->height > 65535) return -1;
    scene_t s;
    if (scene_init(&s, p) != 0) return -1;
    const int W = p->width, H = p->height;
    const size_t npx = (size_t)W * H;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double* cur = (double*)malloc(npx * sizeof(double));
    double* ref = (double*)malloc(npx * sizeof(double));
    double* con = (double*)malloc(npx * sizeof(double));
    double* coff = (double*)malloc(npx * sizeof(double));
    evbuf_t* tb = (evbuf_t*)calloc((size_t)nthr, sizeof(evbuf_t));
    evbuf_t all = {0};
    int64_t ret = -1;
    if (!cur || !ref || !con || !coff || !tb) goto done;
    for (size_t i = 0; i < npx; ++i) {
        double u[4];
        rng_u4(&s.rng, P_THR, (uint32_t)i, 0, u);
        con[i] = p->thr_on + p->thr_jitter * (2.0 * u[0] - 1.0);
        coff[i] = p->thr_off + p->thr_jitter * (2.0 * u[1] - 1.0);
    }
    scene_render(&s, 0.0, cur);
    memcpy(ref, cur, npx * sizeof(double));

    const double dt = s.dt;
    const double f = p->noise_frac;
    const double ox = 0.5 * (W - 1), oy = 0.5 * (H - 1);
    uint64_t produced = 0, step = 0;
    while (produced < p->n_events && step < max_steps) {
        const double t0 = step * dt, t1 = (step + 1) * dt;
        const double th = p->rot_rad_s * t1;
        const double c = cos(th), sn = sin(th);
        const double tx = ox + 0.5 * W + s.vx * t1, ty = oy + 0.5 * H + s.vy * t1;
        for (int k = 0; k < nthr; ++k) tb[k].n = 0;
        #pragma omp parallel for schedule(static)
        for (int y = 0; y < H; ++y) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            evbuf_t* b = &tb[tid];
            const double ry = y - oy;
            /* texture coordinate moves by (c, sn) per pixel along a row */
            double u = wrap(c * (0 - ox) - sn * ry + tx, s.cw);
            double v = wrap(sn * (0 - ox) + c * ry + ty, s.ch);
            for (int x = 0; x < W; ++x, u += c, v += sn) {
                if (u >= s.cw) u -= s.cw; else if (u < 0) u += s.cw;
                if (v >= s.ch) v -= s.ch; else if (v < 0) v += s.ch;
                const size_t i = (size_t)y * W + x;
                const double bv = tex_sample_wrapped(&s, u, v);
                const double a = cur[i];
                const double d = bv - a;
                for (;;) {
                    int pol;
                    if (bv - ref[i] >= con[i]) { ref[i] += con[i]; pol = 1; }
                    else if (ref[i] - bv >= coff[i]) { ref[i] -= coff[i]; pol = 0; }
                    else break;
                    double fr = d != 0.0 ? (ref[i] - a) / d : 0.5;
                    if (fr < 0) fr = 0; else if (fr > 1) fr = 1;
                    evbuf_push(b, (uint64_t)llround((t0 + fr * dt) * 1e9), (uint32_t)i, (uint8_t)pol);
                }
                cur[i] = bv;
            }
        }
        all.n = 0;
        for (int k = 0; k < nthr; ++k) {
            if (tb[k].oom) goto done;
            for (size_t j = 0; j < tb[k].n; ++j)
                evbuf_push(&all, tb[k].v[j].t, tb[k].v[j].pix, tb[k].v[j].pol);
        }
        /* noise: expected n_sig * f / (1 - f) events, stochastic rounding */
        if (f > 0 && f < 1.0) {
            double u[4];
            rng_u4(&s.rng, P_NOISE, (uint32_t)step, 0xffffffffu, u);
            size_t nn = (size_t)floor(all.n * f / (1.0 - f) + u[0]);
            for (size_t j = 0; j < nn; ++j) {
                rng_u4(&s.rng, P_NOISE, (uint32_t)step, (uint32_t)j, u);
                size_t pix = (size_t)(u[0] * npx);
                if (pix >= npx) pix = npx - 1;
                evbuf_push(&all, (uint64_t)llround((t0 + u[2] * dt) * 1e9), (uint32_t)pix,
                           (uint8_t)(u[1] < 0.5));
            }
        }
        if (all.oom) goto done;
        if (all.n > 1) qsort(all.v, all.n, sizeof(ev_t), ev_cmp);   /* a step may emit nothing */
        for (size_t j = 0; j < all.n && produced < p->n_events; ++j, ++produced) {
            xs[produced] = (uint16_t)(all.v[j].pix % (uint32_t)W);
            ys[produced] = (uint16_t)(all.v[j].pix / (uint32_t)W);
            ps[produced] = all.v[j].pol;
            if (ts) ts[produced] = all.v[j].t;
        }
        ++step;
    }
    if (steps_out) *steps_out = step;
    ret = (int64_t)produced;
done:
    if (tb) for (int k = 0; k < nthr; ++k) free(tb[k].v);
    free(tb); free(all.v);
    free(cur); free(ref); free(con); free(coff);
    scene_free(&s);
    return ret;
}

/* Ground-truth log intensity (W*H, row-major) at each of `n` times (ns). */
int sim_render_frames(const sim_params* p, const uint64_t* t_ns, size_t n, float* out)
{
    scene_t s;
    if (scene_init(&s, p) != 0) return -1;
    const size_t npx = (size_t)p->width * p->height;
    double* fr = (double*)malloc(npx * sizeof(double));
    if (!fr) { scene_free(&s); return -1; }
    for (size_t k = 0; k < n; ++k) {
        scene_render(&s, t_ns[k] * 1e-9, fr);
        for (size_t i = 0; i < npx; ++i) out[k * npx + i] = (float)fr[i];
    }
    free(fr);
    scene_free(&s);
    return 0;
}

/* Step duration (s) the scene uses, for callers that want rates. */
double sim_step_seconds(const sim_params* p)
{
    scene_t s;
    if (scene_init(&s, p) != 0) return -1.0;
    double dt = s.dt;
    scene_free(&s);
    return dt;
}
