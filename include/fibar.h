/*
 * fibar.h -- C ABI of libfibar, an MI355X (gfx950) implementation of the
 * FIBAR event-camera image reconstruction hot path (Pfrommer, "Filter-Based
 * Reconstruction of Images from Events", arXiv 2510.20071).
 *
 * The paper's problem statement (Introduction): events arrive
 * asynchronously, grouped into packets by the transport; every event updates
 * the brightness image at its own pixel; the image can be read out at any
 * time with no final processing.  The library keeps the whole reconstruction
 * state in device memory and runs every step in its own HIP kernels:
 *
 *   - temporal filter per event (Method, Eq. (6), (7), (10); coefficients
 *     from the cutoff period by Eq. (17), (18));
 *   - active-event window and 2x2 active-tile bookkeeping with the queue
 *     target regulated by Eq. (19), (20) (Method, "Spatial filtering");
 *   - one-time 3x3 Gaussian blur of pixels that go stale.
 *
 * Regulation granularity: by default the library regulates once per pushed
 * packet (all events of the packet are applied, then old events leave the
 * window, every pixel that went stale in that step is blurred from the same
 * pre-blur image, then the target length is updated).  A packet of one event
 * is the paper's per-event step.  FIBAR_REG_EVENT runs the paper's
 * procedure literally (Method, "Spatial filtering", steps 1-3; Eq. (20)
 * after every event): each event is applied, enters the window, old events
 * leave while the window is longer than the target, each pixel going stale
 * is blurred at once from the current image (so later blurs of the same
 * event see earlier ones), and the target is updated; results then do not
 * depend on how events are grouped into packets.
 *
 * Threading: a context is not thread-safe; calls on one context must be
 * serialised by the caller.  All device work of a context is ordered on the
 * stream given at creation.
 */
#ifndef FIBAR_H
#define FIBAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fibar_ctx fibar_ctx;  /* opaque; owns all device state */

typedef enum {
    FIBAR_OK = 0,
    FIBAR_E_INVALID_ARG = -1,   /* NULL pointer, bad size or parameter        */
    FIBAR_E_RANGE = -2,         /* an event has x >= width or y >= height     */
    FIBAR_E_POLARITY = -3,      /* a polarity byte is neither 0 nor 1         */
    FIBAR_E_TIME = -4,          /* readout time earlier than a previous one   */
    FIBAR_E_NOMEM = -5,         /* device or host allocation failed           */
    FIBAR_E_DEVICE = -6,        /* a HIP call failed                          */
    FIBAR_E_UNSUPPORTED = -7    /* output not maintained in this mode         */
} fibar_status;

typedef enum {
    FIBAR_REG_PACKET = 0,       /* regulate once per pushed packet            */
    FIBAR_REG_EVENT = 1         /* regulate after every event (see below)     */
} fibar_regulation;

/*
 * Parameters.  fibar_default_params() fills the paper's settings.
 *   t_cut          cutoff period in events, > 4 (Eq. (16)-(18); the paper
 *                  uses 40).  alpha and beta are derived on the host in
 *                  double precision and rounded once to float.
 *   fill_num/den   target fill ratio r_fill = num/den of Eq. (19), with
 *                  0 < num <= den <= 65535 (the paper uses 1/2).
 *   q_min, q_max   clamp of the target queue length; q_min >= 1 (the paper
 *                  only asks for a lower bound; default 64); q_max = 0 means
 *                  width*height (the paper's queue limit).
 *   spatial_filter 1 = FIBAR (stale detection + blur), 0 = FIBAR-NSF
 *                  (temporal filter only).
 *   regulation     FIBAR_REG_PACKET or FIBAR_REG_EVENT.  Per-event
 *                  regulation (with spatial_filter = 1) keeps a packet's whole
 *                  state in one workgroup's local memory: sensors of at most
 *                  8192 pixels and q_max <= 16382 (FIBAR_E_INVALID_ARG
 *                  otherwise); step telemetry and batched groups
 *                  (fibar_multi_create) are not available for such contexts
 *                  (FIBAR_E_UNSUPPORTED).  With spatial_filter = 0 nothing
 *                  is regulated and both settings are the same.
 *   max_packet     largest packet accepted by fibar_push_events (events),
 *                  1 .. 1048576; sizes device buffers.  Default 65536.
 *   stream         hipStream_t all work is ordered on; NULL = the null stream.
 *   region         per-tile event queues (Limitations: event queues operated
 *                  separately for each tile of the image): 0 (the default)
 *                  keeps the paper's single queue; an even value 2 .. 32
 *                  gives every tile of region x region pixels (edge tiles cut
 *                  by the image) its own window, active pixel and 2x2-cell
 *                  counts and target of Eq. (20), clamped to
 *                  [min(q_min, n), n] for a tile of n pixels (q_max does not
 *                  apply).  Needs spatial_filter = 1, FIBAR_REG_PACKET and at
 *                  most 16384 tiles; device memory grows by 8 bytes x tiles x
 *                  the power of two >= region^2 + max_packet (each tile's
 *                  window ring).  Telemetry and groups are not available for
 *                  such contexts (FIBAR_E_UNSUPPORTED).
 *   age_max        with per-tile queues, an event also leaves its tile's
 *                  window once age_max newer events have arrived anywhere on
 *                  the sensor, so that tiles without new events still advance
 *                  (the paper leaves this open); 0 = width*height.
 */
typedef struct {
    double   t_cut;
    uint32_t fill_num, fill_den;
    uint32_t q_min;
    uint32_t q_max;
    uint32_t spatial_filter;
    uint32_t regulation;
    uint32_t max_packet;
    void*    stream;
    uint32_t region;
    uint64_t age_max;
} fibar_params;

void fibar_default_params(fibar_params* p);

/*
 * Create a context for a width x height sensor (1..65535 each, and at most
 * 2^29 two-by-two tiles, i.e. ((width+1)/2)*((height+1)/2) <= 536870912:
 * an event's sort key holds its tile-major pixel key and polarity in 32
 * bits; larger sensors return FIBAR_E_INVALID_ARG).  Allocates all device
 * state (zero brightness, no events seen).  On success *out receives the
 * context; on failure *out is NULL and the status says why
 * (FIBAR_E_INVALID_ARG for bad sizes or parameters, FIBAR_E_NOMEM if device
 * memory is short, FIBAR_E_DEVICE for other HIP errors).
 */
int fibar_create(uint32_t width, uint32_t height, const fibar_params* p, fibar_ctx** out);

/*
 * One packet of n events, in arrival (time) order, as structure-of-arrays:
 *   x[n], y[n]  pixel coordinates (uint16),
 *   p[n]        polarity byte: 1 = ON (+1), 0 = OFF (-1),
 *   t[n]        time stamps (uint64); may be NULL.  The method never uses
 *               them (paper, Introduction and Method: each pixel runs on
 *               event time); for host packets t[n-1] is remembered for the
 *               readout-order check.
 *   on_device   0: the arrays are host memory, read before the call returns.
 *               1: the arrays are device memory, read in stream order; the
 *               caller keeps them alive until the stream has passed this
 *               call.
 */
typedef struct {
    const uint16_t* x;
    const uint16_t* y;
    const uint8_t*  p;
    const uint64_t* t;
    size_t          n;
    int             on_device;
} fibar_packet;

/*
 * Apply a packet: every event updates its pixel (temporal filter), enters
 * the active-event window, and then the window is regulated once (spatial
 * filter on).  n == 0 is a no-op.  n > max_packet -> FIBAR_E_INVALID_ARG.
 *
 * Validation is all-or-nothing: a packet with any event out of range
 * (FIBAR_E_RANGE, checked first) or any polarity byte other than 0/1
 * (FIBAR_E_POLARITY) changes no state.  Host packets are checked before
 * the call returns.  Device packets are checked on the device; a rejected
 * device packet is skipped by every kernel and its status is reported by
 * the next fibar_synchronize / fibar_get_stats / host readout (then
 * cleared).
 */
int fibar_push_events(fibar_ctx* c, const fibar_packet* pkt);

/*
 * Output buffers of a readout, width*height elements each, row-major
 * (index y*width + x).  Any pointer but `brightness` may be NULL.
 *   brightness    L, the reconstructed brightness (float).
 *   pbar          the per-pixel polarity average of Eq. (7) (float).
 *   stale_mask    1 where the pixel has had events but none is left in the
 *                 window, else 0.                        [spatial filter]
 *   active_count  events of that pixel inside the window. [spatial filter]
 *   last_index    global index (0-based) of the pixel's newest event, -1 if
 *                 none.
 *   log_age       log(1 + k - last_index), k = index of the newest event
 *                 overall (float); never-seen pixels use last_index = -1.
 *   tile_count    active pixels per 2x2 tile, ((width+1)/2)*((height+1)/2)
 *                 elements, tile (tx, ty) at ty*((width+1)/2)+tx.
 *                                                          [spatial filter]
 *   total_count   events of that pixel since creation or reset (uint64).
 *   on_device     0: host memory (the call synchronises the stream);
 *                 1: device memory, written in stream order.
 * Outputs marked [spatial filter] return FIBAR_E_UNSUPPORTED when the
 * context was created with spatial_filter = 0 and the pointer is non-NULL.
 */
typedef struct {
    float*    brightness;
    float*    pbar;
    uint8_t*  stale_mask;
    uint32_t* active_count;
    int64_t*  last_index;
    float*    log_age;
    uint32_t* tile_count;
    uint64_t* total_count;
    int       on_device;
} fibar_readout_buf;

/*
 * Read the state after all pushed events (paper, Introduction: no final
 * processing is needed at read-out).  t is the readout time; it is not used
 * by the method, but it may not be earlier than a previous readout time or
 * the newest host-packet time stamp (FIBAR_E_TIME otherwise).
 */
int fibar_readout(fibar_ctx* c, uint64_t t, const fibar_readout_buf* out);

/*
 * A list of operations executed in order, with the same results as calling
 * fibar_push_events / fibar_readout one by one.  Executing them together lets
 * the library group and compose the events of many packets in one parallel
 * pass before applying them in order, and lets a device readout that directly
 * follows a push (and asks for no window counts) be written by that push's
 * last launch, with identical results.  Host readouts inside a list do not
 * report pending device-side packet errors (the next fibar_synchronize does).
 * Execution stops at the first error the host detects, which is returned;
 * the operations before it have been carried out.
 */
typedef enum { FIBAR_OP_PUSH = 0, FIBAR_OP_READOUT = 1 } fibar_op_kind;

typedef struct {
    int               kind;     /* fibar_op_kind                   */
    fibar_packet      packet;   /* FIBAR_OP_PUSH                   */
    uint64_t          t;        /* FIBAR_OP_READOUT: readout time  */
    fibar_readout_buf readout;  /* FIBAR_OP_READOUT: outputs       */
} fibar_op;

int fibar_submit(fibar_ctx* c, const fibar_op* ops, size_t n_ops);

/* Free all resources.  NULL-safe.  Waits for the context's stream. */
void fibar_destroy(fibar_ctx* c);

/*
 * Window statistics after the last regulation step (synchronises):
 *   k  index of the newest event (-1 before any), h index of the oldest
 *   event in the window, q = k - h + 1, Q the target length, P active
 *   pixels, T active tiles, n_regulations steps so far, last_stale pixels
 *   blurred in the last step, total_stale blurred so far.
 */
typedef struct {
    int64_t  k;
    uint64_t h, q, Q, P, T;
    uint64_t n_regulations, last_stale, total_stale;
} fibar_stats;

int fibar_get_stats(fibar_ctx* c, fibar_stats* s);

/*
 * Return the context to its initial state (no events seen, zero images,
 * target length q_max), keeping its allocations.  Stream ordered.
 */
int fibar_reset(fibar_ctx* c);

/*
 * Optional per-kernel timing.  Launches of the kernels selected by
 * `kernel_mask` (bit i = kernel i below; 0 turns timing off) are counted per
 * kernel, and launch 0, every, 2 every, ... carries a pair of HIP events on
 * its dispatch (hipExtLaunchKernel), which the runtime stamps with the
 * dispatch's start and end.  Sampling (every > 1) keeps the event handling
 * off most launches, so a timed run keeps the pace of an untimed one.
 * fibar_kernel_time() synchronises the context's stream, returns the summed
 * duration (ms) and the count of the launches of kernel `kernel` timed since
 * the last call, and clears them.  Kernels: 0 group+compose (bulk; the whole
 * blur-off batch in that mode), 1 apply, 2 window pop + stale blur values
 * (launches that also write a readout are not timed with direct launches),
 * 3 pop launches that also write a readout (graph launches only), 4 readout
 * (the separate readout kernel).  With graph launches (below) the count
 * restarts with every batch, pop launches count whether or not they also
 * write a readout, and a timed launch's events are recorded by graph nodes
 * just before and after its kernel.
 */
int fibar_set_kernel_timing(fibar_ctx* c, uint32_t kernel_mask, uint32_t every);
int fibar_kernel_time(fibar_ctx* c, int kernel, double* total_ms, uint64_t* launches);

/*
 * Per-step telemetry (spatial filter on): every regulation step of the
 * context (one per pushed packet that was not rejected; Method, "Spatial
 * filtering", Eq. (19), (20)) writes one record of the window scalars after
 * that step into a caller-owned device buffer of `capacity` records, at the
 * index of the step (0-based, counting from creation or reset; steps past
 * the capacity are not recorded).  The record's fields:
 *   k      index of the newest event after the step,
 *   h      index of the oldest event left in the window,
 *   q      window length k - h + 1,
 *   Q      target length for the next step (Eq. (20)),
 *   P, T   active pixels and active 2x2 tiles after the step,
 *   stale  pixels that went stale (and were blurred) in the step,
 *   n      events of the step's packet.
 * The buffer is written in stream order by the step's device work; the
 * caller keeps it alive while that work runs and reads it after a
 * synchronising call.  NULL with capacity 0 turns recording off.  Returns
 * FIBAR_E_INVALID_ARG for NULL with a nonzero capacity and
 * FIBAR_E_UNSUPPORTED for a context without the spatial filter.
 */
typedef struct {
    int64_t  k;
    uint64_t h, q, Q, P, T, stale, n;
} fibar_step_record;

int fibar_set_telemetry(fibar_ctx* c, fibar_step_record* records, uint64_t capacity);

/*
 * How the in-order kernels of a batch are issued (spatial filter on).
 * FIBAR_LAUNCH_DIRECT (the default): one HIP launch per kernel.
 * FIBAR_LAUNCH_GRAPH: the batch's launches are recorded and replayed as one
 * HIP graph; batches with the same sequence of kernels (the usual case:
 * batches of the same packet count) reuse an instantiated graph whose node
 * parameters are updated, which costs the host much less per kernel than a
 * launch.  A batch holding a readout into host memory runs on direct
 * launches.  Results are identical in both modes.  Returns
 * FIBAR_E_INVALID_ARG for another mode.
 */
#define FIBAR_LAUNCH_DIRECT 0
#define FIBAR_LAUNCH_GRAPH 1
int fibar_set_launch_mode(fibar_ctx* c, int mode);

/*
 * Relative contrast thresholds (Experiments, "Inter-pixel threshold
 * variation"; the threshold appendix, Eq. (21)-(30)).  The temporal filter
 * already balances a pixel's ON against its OFF threshold; this variant also
 * corrects for thresholds that differ between pixels, by multiplying the
 * right-hand side of Eq. (6) at pixel i by its relative threshold C'_i (the
 * paper found no material gain in its application).
 *
 * fibar_count_polarities adds the ON and OFF events of one packet of a
 * calibration recording (device arrays x, y, p of n events, as in
 * fibar_packet) to per-pixel counters n_on and n_off (device, width*height
 * uint32 each, row-major, initialised by the caller; counts wrap at 2^32).
 * The packet is checked first and counted only if every event is in range
 * (FIBAR_E_RANGE) with a polarity byte of 0 or 1 (FIBAR_E_POLARITY), so a
 * rejected packet adds nothing.  It synchronises `stream` (hipStream_t, NULL
 * = the null stream) for that check.
 *
 * fibar_relative_thresholds forms, with N the mean of n_on + n_off over all
 * width*height pixels, C'_i = N / (n_on_i + n_off_i) (Eq. (30)) into c_rel,
 * and, when the pointers are not NULL, C'_on_i = N / (2 n_on_i) and
 * C'_off_i = N / (2 n_off_i) (device float arrays, width*height each).  A
 * pixel without events of the kind a ratio divides by gets 1.  Computed in
 * double precision and rounded once; queued on `stream` without waiting.
 *
 * fibar_set_pixel_gain makes every later push of the context multiply the
 * increment of Eq. (6) at each pixel by gain[i] (device, width*height
 * floats, copied in stream order into the context, so the caller may reuse
 * the buffer once the stream has passed the call; the values are used as
 * given, e.g. c_rel above).  NULL removes the multipliers.  Every path
 * applies them: both regulation modes, blur on and off, and groups.
 */
int fibar_count_polarities(const uint16_t* x, const uint16_t* y, const uint8_t* p, size_t n,
                           uint32_t width, uint32_t height, uint32_t* n_on, uint32_t* n_off,
                           void* stream);
int fibar_relative_thresholds(const uint32_t* n_on, const uint32_t* n_off, uint32_t width,
                              uint32_t height, float* c_rel, float* c_on_rel, float* c_off_rel,
                              void* stream);
int fibar_set_pixel_gain(fibar_ctx* c, const float* gain);

/*
 * Per-tile queues: each tile's scalars after the last regulation step, into
 * host arrays of tiles_x * tiles_y entries (row-major; tiles_x =
 * ceil(width / region), tiles_y = ceil(height / region)); any pointer may be
 * NULL.  q: window length, Q: target, P: active pixels, T: active 2x2 cells,
 * front: global index of the tile's oldest window event (k + 1 when the
 * window is empty).  Synchronises the stream.  FIBAR_E_UNSUPPORTED for a
 * context with one queue.  fibar_get_stats reports q, Q, P and T summed over
 * the tiles and h = k + 1 - q for such contexts.
 */
int fibar_tile_stats(fibar_ctx* c, uint64_t* q, uint64_t* Q, uint64_t* P, uint64_t* T,
                     uint64_t* front);

/*
 * Several independent streams advanced together.  A group holds 1..64
 * contexts (spatial filter on; the blur-off path already batches well on its
 * own); fibar_multi_submit takes one op list per context and gives the same
 * results as fibar_submit on each context separately.  Execution goes in
 * rounds -- the next packet of every stream -- and every launch of a round
 * serves all streams: its workgroups split the round's (stream, slice)
 * tasks.  Consecutive rounds are either replayed as one HIP graph or
 * launched kernel by kernel, whichever the launch configuration says.
 * Restrictions: device packets of at most 32768 events, device readouts
 * without tile counts, and each op list starts with a push.  Contexts stay
 * owned by the caller and must outlive the group; they may be used alone
 * between submissions.  The group runs on a stream of its own: a submission
 * starts after the work already queued on `stream` (hipStream_t, NULL = the
 * null stream) and on the contexts' streams, and work queued on them after
 * the call returns waits for it.
 */
typedef struct fibar_multi fibar_multi;

int fibar_multi_create(fibar_ctx* const* ctxs, uint32_t n, void* stream, fibar_multi** out);
int fibar_multi_submit(fibar_multi* m, const fibar_op* const* ops, const size_t* n_ops);

/*
 * Launch configuration of the round kernels: workgroup size x resident
 * workgroups, and HIP-graph replay or direct launches.  Candidates 0..9:
 * index % 5 picks the shape (128x512, 64x1024, 128x1024, 256x256, 256x512),
 * index / 5 the mode (0 graphs, 1 direct).  It never changes results.
 * fibar_multi_autotune() makes the next submissions time the candidates on
 * interleaved groups of rounds and keep the fastest; fibar_multi_get_shape()
 * reports the shape in use and fibar_multi_get_config() its index;
 * fibar_multi_set_shape() picks a candidate directly.
 */
int fibar_multi_autotune(fibar_multi* m);
int fibar_multi_get_shape(fibar_multi* m, uint32_t* block, uint32_t* grid);
int fibar_multi_get_config(fibar_multi* m, uint32_t* index);
int fibar_multi_set_shape(fibar_multi* m, uint32_t index);
void fibar_multi_destroy(fibar_multi* m);

/* Wait for all queued work; returns a pending device-side packet error. */
int fibar_synchronize(fibar_ctx* c);

/* Short English description of a status code (static string). */
const char* fibar_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* FIBAR_H */
