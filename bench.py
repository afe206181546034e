#!/usr/bin/env python3
"""Throughput of the FIBAR hot path on one MI355X.

Workload (hd720): a 1280x720 sensor, 100 M events from the seeded simulator
(2048 blobs, rotation 0.5 rad/s + translation 300 px/s, threshold 0.15, 2 %
noise), pushed in 16384-event packets, with readouts of the brightness image
at ~1000 random event indices (mean spacing 100 000; a readout inside a
packet splits it).  Events are resident in device memory before timing.

One step = the whole stream from a freshly reset context: every packet
pushed (temporal filter, window bookkeeping, stale blur) and every readout
written to its own device buffer, submitted through the C ABI.  The JSON
line reports Mev/s with the spatial filter on (FIBAR) and, as extra fields,
with it off (FIBAR-NSF).

Extra legs:
* the FP64 CPU oracle on one pinned host CPU over the same stream, blur on
  and off (cpu_baseline), and the GPU's final state against the oracle's;
* the 64x48 (200 000 events) and 640x480 (20 M events) configurations, blur
  on and off, each with its oracle timing and final-state parity;
* 16 independent streams of uneven resolution and rate advanced together,
  with the oracle on min(16, CPUs) pinned threads;
* the learned stale fill: trained on 200 sequences, its per-tile fallback
  threshold chosen on training frames, scored on 20 held-out sequences
  against the Gaussian fill and a per-tile ground-truth upper bound, and the
  hd720 stream reconstructed with the fill on every readout.
Every roofline figure uses the algorithmic bytes below and 8 TB/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic bytes per unit of work, at the state widths of the method
# (FP32 brightness and polarity average, 8-byte last-event index, u16 window
# count, u8 tile count; the widths the measurement section of the design
# notes states), per kernel:
#   group      : per event: x, y, p read (5 B).  The composed-map records the
#                sort writes are overhead, not algorithmic.
#   apply      : per distinct (pixel, packet): pbar, L read + write (16 B),
#                last write (8 B), window count read + write (4 B); per
#                event: ring write (4 B); per activated tile (one per stale
#                pixel in steady state): tile count read + write (2 B).
#   pop_blur   : per popped event: ring read (4 B) + window count read +
#                write (4 B); per stale pixel: 9 brightness reads (36 B),
#                the blurred value written (4 B), tile count read + write
#                (2 B).
# End to end (whole stream, readouts included), per event, with u distinct
# pixels per event and packet, s stale pixels per event, R events per readout:
#   blur off: 5 + 16/u + 8 W H / R
#   blur on : 17 + 28/u + 44 s + 8 W H / R
KERNELS = ("group_compose", "apply", "pop_blur", "pop_blur_readout", "readout")
LAUNCH_MODES = {"direct": 0, "graph": 1}
KERNEL_SOURCES = ("paper_2510_20071_amd/csrc/fibar_kernels.hip",
                  "paper_2510_20071_amd/csrc/fibar_step.h",
                  "paper_2510_20071_amd/csrc/fibar_tile.h",
                  "paper_2510_20071_amd/csrc/fibar_internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_hd720.md" % kernel)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_info():
    """The host the CPU baselines ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


class pinned:
    """Pin the calling thread to one CPU (the `i`-th it may use) while inside."""

    def __init__(self, i=0):
        cpus = sorted(os.sched_getaffinity(0))
        self.cpu = cpus[i % len(cpus)]

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {self.cpu})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)
        return False


def bytes_per_event(u, s, W, H, R, spatial):
    """Algorithmic HBM bytes per event of the whole path (readouts included)."""
    ro = 8.0 * W * H / R if R else 0.0
    if spatial:
        return 17.0 + 28.0 / u + 44.0 * s + ro
    return 5.0 + 16.0 / u + ro


def time_oracle(oracle, W, H, ev, sched, spatial=True, regulation="packet", limit=None,
                cpu=0):
    """Wall-clock of the FP64 oracle's pushes and readouts over `sched` (the
    events up to `limit`), on one pinned CPU.  Returns (seconds, events,
    oracle); the caller closes the oracle."""
    m = len(ev) if limit is None else min(limit, len(ev))
    orc = oracle.Oracle(W, H, spatial_filter=spatial, regulation=regulation)
    lo = oracle._load()
    Lbuf = np.empty(W * H, np.float64)
    sub = [it for it in sched if (it[0] == "push" and it[2] <= m) or
           (it[0] == "read" and it[1] <= m)]
    with pinned(cpu):
        t0 = time.perf_counter()
        for it in sub:
            if it[0] == "push":
                a, b = it[1], it[2]
                rc = lo.fibar_ref_push_events(orc._h, ev.x[a:b].ctypes.data,
                                              ev.y[a:b].ctypes.data, ev.p[a:b].ctypes.data,
                                              None, b - a)
                assert rc == 0, rc
            else:
                lo.fibar_ref_readout(orc._h, int(ev.t[it[1] - 1]), Lbuf.ctypes.data, None, None,
                                     None, None, None, None)
        secs = time.perf_counter() - t0
    return secs, m, orc


def final_parity(g, r, spatial):
    """Final GPU state against the oracle's: integers bit for bit, brightness
    as the largest relative error (floor 1)."""
    keys = ("cnt", "last", "stale", "tcnt", "tot") if spatial else ("last", "tot")
    ints = all(np.array_equal(g[k].astype(np.int64), r[k].astype(np.int64)) for k in keys)
    d = np.abs(g["L"].astype(np.float64) - r["L"])
    return {"integer_state_bit_exact": bool(ints),
            "max_rel_err_L": float((d / np.maximum(np.abs(r["L"]), 1.0)).max())}


def run_config(args, torch, dev, fb, eventsim, name):
    """A smaller configuration (64x48 sensor or the 640x480 one): GPU Mev/s
    with the spatial filter on and off, the oracle on one pinned CPU in both
    modes (and, on the 64x48 sensor, with per-event regulation), and the
    final state of each GPU run against the oracle's."""
    import oracle
    wl = eventsim.preset(name)
    W, H = wl.scene.width, wl.scene.height
    t0 = time.time()
    ev = eventsim.generate(wl.scene)
    n = len(ev)
    sched = eventsim.schedule(n, wl.packet, wl.readouts)
    n_push = sum(1 for it in sched if it[0] == "push")
    n_read = sum(1 for it in sched if it[0] == "read")
    log("%s: %d events generated in %.1f s" % (name, n, time.time() - t0))
    gx = torch.from_numpy(ev.x.view(np.int16)).to(dev)
    gy = torch.from_numpy(ev.y.view(np.int16)).to(dev)
    gp = torch.from_numpy(ev.p).to(dev)
    frames = torch.empty((max(n_read, 1), W * H), dtype=torch.float32, device=dev)
    ops = []
    r = 0
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            ops.append(fb.readout_op(int(ev.t[it[1] - 1]), frames[r]))
            r += 1
    stream = torch.cuda.current_stream(dev).cuda_stream
    res = {"workload": "%s: %dx%d sensor, %d events, %d-event packets, %d readouts"
                       % (name, W, H, n, wl.packet, n_read),
           "events": n, "packets": n_push}
    R = n / max(n_read, 1)
    u = distinct_per_packet(ev.x, ev.y, W, wl.packet)
    for spatial in (True, False):
        ctx = fb.Context(W, H, spatial_filter=spatial, stream=stream)
        for _ in range(args.warmup):
            assert ctx.reset() == 0 and ctx.submit(ops) == 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            assert ctx.reset() == 0 and ctx.submit(ops) == 0
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        assert ctx.synchronize() == 0
        st = ctx.stats() if spatial else None
        g = ctx.readout_host(int(ev.t[-1]))
        ctx.close()
        secs, m, orc = time_oracle(oracle, W, H, ev, sched, spatial)
        ref = orc.readout(int(ev.t[-1]))
        par = final_parity(g, ref, spatial)
        if spatial:
            par["window_scalars_equal"] = all(st[f] == orc.stats()[f]
                                              for f in ("k", "h", "Q", "P", "T"))
        orc.close()
        key = "blur_on" if spatial else "blur_off"
        mev = n / el / 1e6
        s_ev = st["total_stale"] / n if spatial else 0.0
        B = bytes_per_event(u, s_ev, W, H, R, spatial)
        res[key] = {"mev_s": round(mev, 3), "ms_per_step": round(1e3 * el, 3),
                    "bytes_per_event": round(B, 2),
                    "frac_end_to_end": round(B * mev * 1e6 / 8e12, 6),
                    "oracle_mev_s": round(m / secs / 1e6, 3), "parity": par}
        log("%s %s: %.1f Mev/s (oracle %.2f Mev/s), parity %s"
            % (name, key, mev, m / secs / 1e6, par))
    res["distinct_pixels_per_event"] = round(u, 4)
    res["event_vs_packet"] = event_vs_packet(oracle, eventsim, wl, ev, sched)
    log("%s per-event against per-packet regulation (oracle): %s" % (name, res["event_vs_packet"]))
    if name == "vga":
        res["relative_thresholds"] = thresholds_leg(args, torch, dev, fb, eventsim, oracle, W, H,
                                                    ev, sched, ops, stream, n)
    if name == "sensor64x48":
        # per-event regulation (the paper's literal procedure), GPU and oracle
        ctx = fb.Context(W, H, stream=stream, regulation="event")
        for _ in range(args.warmup):
            assert ctx.reset() == 0 and ctx.submit(ops) == 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            assert ctx.reset() == 0 and ctx.submit(ops) == 0
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        assert ctx.synchronize() == 0
        st = ctx.stats()
        g = ctx.readout_host(int(ev.t[-1]))
        ctx.close()
        secs, m, orc = time_oracle(oracle, W, H, ev, sched, True, regulation="event")
        par = final_parity(g, orc.readout(int(ev.t[-1])), True)
        par["window_scalars_equal"] = all(st[f] == orc.stats()[f]
                                          for f in ("k", "h", "Q", "P", "T", "n_regulations"))
        orc.close()
        res["event_regulation"] = {"mev_s": round(n / el / 1e6, 3),
                                   "ms_per_step": round(1e3 * el, 3),
                                   "oracle_mev_s": round(m / secs / 1e6, 3), "parity": par}
        log("%s per-event regulation: %.1f Mev/s (oracle %.2f Mev/s), parity %s"
            % (name, n / el / 1e6, m / secs / 1e6, par))
    return res


def event_vs_packet(oracle, eventsim, wl, ev, sched):
    """How far per-packet regulation (the GPU contract) is from the paper's
    per-event regulation, both from the FP64 oracle at every readout: the
    Jaccard index of the two stale sets, and each mode's PSNR against the
    simulator's ground truth (its log intensity mapped affinely onto the
    brightness over the active pixels, the whole frame scored)."""
    W, H = wl.scene.width, wl.scene.height
    reads = [it[1] for it in sched if it[0] == "read"]
    gt = eventsim.render_frames(wl.scene, [int(ev.t[k - 1]) for k in reads])
    orcs = {m: oracle.Oracle(W, H, regulation=m) for m in ("packet", "event")}
    jac, psnr = [], {m: [] for m in orcs}
    i = 0
    for it in sched:
        if it[0] == "push":
            a, b = it[1], it[2]
            for o in orcs.values():
                assert o.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
            continue
        r = {m: o.readout(0) for m, o in orcs.items()}
        se, sp = r["event"]["stale"] != 0, r["packet"]["stale"] != 0
        union = int(np.count_nonzero(se | sp))
        jac.append(int(np.count_nonzero(se & sp)) / union if union else 1.0)
        for m in orcs:
            L = r[m]["L"].reshape(H, W)
            target = eventsim.fill_target(gt[i], L, (r[m]["cnt"] > 0).reshape(H, W))
            psnr[m].append(eventsim.fill_psnr(L, target, np.ones((H, W), bool)))
        i += 1
    for o in orcs.values():
        o.close()
    return {"readouts": len(jac), "stale_jaccard_mean": round(float(np.mean(jac)), 4),
            "stale_jaccard_min": round(float(np.min(jac)), 4),
            "psnr_db_packet": round(float(np.mean(psnr["packet"])), 3),
            "psnr_db_event": round(float(np.mean(psnr["event"])), 3)}


def tiles_leg(args, torch, dev, fb, W, H, ev, sched, ops, n_ops, stream, n):
    """The hd720 stream with per-tile event queues (tiles of --tile pixels,
    age limit W x H events): GPU Mev/s, and the final state and every tile's
    window against the oracle's per-tile queues."""
    import oracle
    R = args.tile
    lib = fb.load()
    ctx = fb.Context(W, H, stream=stream, region=R)
    steps = max(1, min(args.steps, 5))
    for _ in range(max(1, min(args.warmup, 2))):
        assert ctx.reset() == 0 and lib.fibar_submit(ctx.handle, ops, n_ops) == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        assert ctx.reset() == 0 and lib.fibar_submit(ctx.handle, ops, n_ops) == 0
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    assert ctx.synchronize() == 0
    st = ctx.stats()
    g = ctx.readout_host(int(ev.t[-1]))
    gt = ctx.tile_stats()
    ctx.close()
    res = {"tile": R, "tiles": int(gt["q"].shape[0]), "age_max": W * H,
           "mev_s": round(n / el / 1e6, 2), "ms_per_step": round(1e3 * el, 3), "steps": steps}
    if not args.no_cpu_baseline:
        orc = oracle.Oracle(W, H, region=R)
        t0 = time.perf_counter()
        for it in sched:
            if it[0] == "push":
                assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
        res["oracle_mev_s"] = round(n / (time.perf_counter() - t0) / 1e6, 3)
        par = final_parity(g, orc.readout(int(ev.t[-1])), True)
        ot = orc.region_stats()
        par["tile_windows_equal"] = all(np.array_equal(gt[k], ot[k]) for k in gt)
        par["scalars_equal"] = all(st[f] == orc.stats()[f] for f in ("k", "q", "Q", "P", "T"))
        orc.close()
        res["parity"] = par
        res["total_stale"] = st["total_stale"]
    log("hd720 per-tile queues (tiles of %d): %.1f Mev/s, %s" % (R, res["mev_s"], res.get("parity")))
    return res


def thresholds_leg(args, torch, dev, fb, eventsim, oracle, W, H, ev, sched, ops, stream, n):
    """Relative contrast thresholds on the 640x480 sensor: a calibration
    recording (uniform triangle wave, per-pixel thresholds 0.2 +- 0.02)
    counted and turned into C'_i on the device, then the stream reconstructed
    with C'_i multiplying Eq. (6)'s increment (blur on), against the oracle
    with the same multipliers."""
    con, coff = eventsim.pixel_thresholds(W, H, 7)
    cal = eventsim.calibration_stream(W, H, con, coff, periods=1, amplitude=4.0)
    cx = torch.from_numpy(cal.x.view(np.int16)).to(dev)
    cy = torch.from_numpy(cal.y.view(np.int16)).to(dev)
    cp = torch.from_numpy(cal.p).to(dev)
    n_on = torch.zeros(W * H, dtype=torch.int32, device=dev)
    n_off = torch.zeros_like(n_on)
    c_rel = torch.empty(W * H, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert fb.fibar_count_polarities(cx, cy, cp, W, H, n_on, n_off, stream) == 0
    assert fb.fibar_relative_thresholds(n_on, n_off, W, H, c_rel, None, None, stream) == 0
    torch.cuda.synchronize()
    cal_s = time.perf_counter() - t0
    gain = c_rel.cpu().numpy()
    ctx = fb.Context(W, H, stream=stream)
    assert ctx.set_gain(c_rel) == 0
    for _ in range(args.warmup):
        assert ctx.reset() == 0 and ctx.submit(ops) == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        assert ctx.reset() == 0 and ctx.submit(ops) == 0
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    assert ctx.synchronize() == 0
    st = ctx.stats()
    g = ctx.readout_host(int(ev.t[-1]))
    ctx.close()
    orc = oracle.Oracle(W, H)
    assert orc.set_gain(gain.astype(np.float64)) == 0
    for it in sched:
        if it[0] == "push":   # readouts change no state
            assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
    par = final_parity(g, orc.readout(int(ev.t[-1])), True)
    par["window_scalars_equal"] = all(st[f] == orc.stats()[f] for f in ("k", "h", "Q", "P", "T"))
    orc.close()
    res = {"calibration_events": len(cal), "calibration_ms": round(1e3 * cal_s, 3),
           "calibration_mev_s": round(len(cal) / cal_s / 1e6, 1),
           "relative_threshold_spread": round(float(gain.std()), 4),
           "blur_on_mev_s": round(n / el / 1e6, 3), "parity": par}
    log("vga relative thresholds: calibration of %d events in %.2f ms; reconstruction %.1f "
        "Mev/s, parity %s" % (len(cal), 1e3 * cal_s, n / el / 1e6, par))
    return res


def distinct_per_packet(x, y, W, packet, sample_every=16):
    """Mean number of distinct pixels per packet, over every 16th packet."""
    n = x.shape[0]
    tot_d, tot_e = 0, 0
    for a in range(0, n, packet * sample_every):
        b = min(n, a + packet)
        pix = y[a:b].astype(np.int64) * W + x[a:b]
        tot_d += np.unique(pix).size
        tot_e += b - a
    return tot_d / max(tot_e, 1)


def run_batched(args, torch, dev, fb, eventsim):
    """16 streams of uneven resolution and rate, advanced together by one
    group submission (one step = every stream from a reset state)."""
    from concurrent.futures import ThreadPoolExecutor
    wls = eventsim.batched_streams(16, meta_seed=4, scale=args.multi_scale)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, len(os.sched_getaffinity(0)))) as pool:
        evs = list(pool.map(lambda w: eventsim.generate(w.scene), wls))
    total = sum(len(e) for e in evs)
    log("batched streams: %d streams, %d events generated in %.1f s"
        % (len(wls), total, time.time() - t0))
    stream = torch.cuda.current_stream(dev).cuda_stream
    keep, op_lists, ctxs, n_reads = [], [], [], []
    for w, ev in zip(wls, evs):
        W, H = w.scene.width, w.scene.height
        gx = torch.from_numpy(ev.x.view(np.int16)).to(dev)
        gy = torch.from_numpy(ev.y.view(np.int16)).to(dev)
        gp = torch.from_numpy(ev.p).to(dev)
        n = len(ev)
        ro = list(range(2_000_000, n, 2_000_000)) + [n]
        n_reads.append(len(ro))
        frames = torch.empty((len(ro), W * H), dtype=torch.float32, device=dev)
        keep.append((gx, gy, gp, frames))
        ops, r = [], 0
        for it in eventsim.schedule(n, w.packet, ro):
            if it[0] == "push":
                a, bb = it[1], it[2]
                op = fb.fibar_op()
                op.kind = fb.FIBAR_OP_PUSH
                op.packet = fb.fibar_packet(gx.data_ptr() + 2 * a, gy.data_ptr() + 2 * a,
                                            gp.data_ptr() + a, None, bb - a, 1)
            else:
                op = fb.fibar_op()
                op.kind = fb.FIBAR_OP_READOUT
                op.t = int(it[1])
                op.readout = fb.fibar_readout_buf(frames.data_ptr() + 4 * W * H * r, None, None,
                                                  None, None, None, None, None, 1)
                r += 1
            ops.append(op)
        op_lists.append(ops)
        ctxs.append(fb.Context(W, H, max_packet=32768, stream=stream))
    group = fb.Group(ctxs, stream=stream)
    op_lists = fb.OpLists(op_lists)

    def reset_all():
        for c in ctxs:
            assert c.reset() == 0

    # autotuned launch shape on the warm-up submission
    assert group.autotune() == 0
    for _ in range(max(1, args.warmup)):
        reset_all()
        assert group.submit(op_lists) == 0
    torch.cuda.synchronize()
    shape = group.shape()
    config = group.config()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reset_all()
        assert group.submit(op_lists) == 0
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    # the same streams one after another through single contexts
    reset_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lib = fb.load()
    for c, arr, n_ops in zip(ctxs, op_lists.arrays, op_lists.sizes):
        assert lib.fibar_submit(c.handle, arr, n_ops) == 0
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    for c in ctxs:
        assert c.synchronize() == 0
    stale = [c.stats()["total_stale"] for c in ctxs]
    group.close()
    for c in ctxs:
        c.close()
    # algorithmic bytes of every stream, summed (each at its own u, s, R)
    alg = 0.0
    for w, ev, nread, st in zip(wls, evs, n_reads, stale):
        n = len(ev)
        u = distinct_per_packet(ev.x, ev.y, w.scene.width, w.packet)
        alg += n * bytes_per_event(u, st / n, w.scene.width, w.scene.height, n / nread, True)
    achieved = alg / el / 1e9
    res = {"streams": len(wls), "events": total,
           "resolutions": ["%dx%d" % (w.scene.width, w.scene.height) for w in wls],
           "packets": [w.packet for w in wls], "mev_s": round(total / el / 1e6, 2),
           "ms_per_step": round(1e3 * el, 3),
           "one_stream_at_a_time_mev_s": round(total / el_seq / 1e6, 2),
           "launch_shape": {"block": shape[0], "grid": shape[1],
                            "launches": "hip graphs" if config < 5 else "direct",
                            "autotuned": True},
           "roofline": {"bound": "hbm", "kernel": "whole group step (all streams)",
                        "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(achieved / 8000.0, 5), "traffic": None,
                        "algorithmic_bytes": round(alg)}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = batched_oracle(wls, evs)
    log("batched streams: %.1f Mev/s together, %.1f Mev/s one at a time"
        % (res["mev_s"], res["one_stream_at_a_time_mev_s"]))
    return res


def batched_oracle(wls, evs):
    """The FP64 oracle over every stream of the batched workload, one stream
    at a time per thread, min(16, usable CPUs) threads, each pinned to a CPU
    of its own; streams are taken longest first."""
    import queue
    import threading

    import eventsim
    import oracle
    k = min(16, len(os.sched_getaffinity(0)))
    order = sorted(range(len(wls)), key=lambda i: -len(evs[i]))
    q = queue.Queue()
    for i in order:
        q.put(i)
    err = []

    def worker(j):
        try:
            while True:
                try:
                    i = q.get_nowait()
                except queue.Empty:
                    return
                w, ev = wls[i], evs[i]
                n = len(ev)
                ro = list(range(2_000_000, n, 2_000_000)) + [n]
                sched = eventsim.schedule(n, w.packet, ro)
                _, _, orc = time_oracle(oracle, w.scene.width, w.scene.height, ev, sched, True,
                                        cpu=j)
                orc.close()
        except Exception as e:  # reported below
            err.append(e)

    t0 = time.perf_counter()
    threads = [threading.Thread(target=worker, args=(j,)) for j in range(k)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    el = time.perf_counter() - t0
    if err:
        raise err[0]
    total = sum(len(e) for e in evs)
    log("batched streams, oracle: %d events in %.1f s on %d threads (%.1f Mev/s)"
        % (total, el, k, total / el / 1e6))
    out = {"value": round(total / el / 1e6, 3), "unit": "Mev/s", "cores": k, "kind": "oracle",
           "sample": "every stream of the batched workload whole, blur on, FP64, one stream at "
                     "a time per thread, each thread pinned to its own CPU"}
    out.update(host_info())
    return out


def fill_frames(torch, dev, fb, eventsim, seeds, n_events, every, stream, pool):
    """Readouts (L, stale mask, log age) every `every` events of 1280x720
    sequences, reconstructed with blur on, and their calibrated ground-truth
    targets; stacked on the device as [frames, H, W].  The host work
    (simulation, ground-truth frames, target fits) runs on `pool`."""
    def simulate(seed):
        sc = eventsim.fill_scene(seed, n_events)
        ev = eventsim.generate(sc)
        ro = list(range(every, len(ev) + 1, every))
        gt = eventsim.render_frames(sc, [int(ev.t[k - 1]) for k in ro])
        return sc, ev, ro, gt

    def targets(gt, Lh, act):
        return np.stack([eventsim.fill_target(gt[f], Lh[f], act[f]) for f in range(len(gt))])

    sims = [pool.submit(simulate, sd) for sd in seeds]
    Ls, Ss, As, Tf = [], [], [], []
    for fut in sims:
        sc, ev, ro, gt = fut.result()
        W, H = sc.width, sc.height
        gx = torch.from_numpy(ev.x.view(np.int16)).to(dev)
        gy = torch.from_numpy(ev.y.view(np.int16)).to(dev)
        gp = torch.from_numpy(ev.p).to(dev)
        F = len(ro)
        L = torch.empty((F, H, W), dtype=torch.float32, device=dev)
        S = torch.empty((F, H, W), dtype=torch.uint8, device=dev)
        A = torch.empty((F, H, W), dtype=torch.float32, device=dev)
        C = torch.empty((F, H, W), dtype=torch.int32, device=dev)
        ctx = fb.Context(W, H, stream=stream)
        ops, r = [], 0
        for it in eventsim.schedule(len(ev), 16384, ro):
            if it[0] == "push":
                ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
            else:
                ops.append(fb.readout_op(int(ev.t[it[1] - 1]), L[r], stale=S[r], cnt=C[r],
                                         log_age=A[r]))
                r += 1
        assert ctx.submit(ops) == 0 and ctx.synchronize() == 0
        ctx.close()
        Tf.append(pool.submit(targets, gt, L.cpu().numpy(), C.cpu().numpy() > 0))
        del C, gx, gy, gp
        Ls.append(L)
        Ss.append(S)
        As.append(A)
    Ts = [torch.from_numpy(f.result()).to(dev) for f in Tf]
    return torch.cat(Ls), torch.cat(Ss), torch.cat(As), torch.cat(Ts)


def psnr_dev(torch, img, target, mask):
    """PSNR (dB) of img against target over mask, on the device, FP64 sums;
    the peak is the target's range over the frame (as the simulator's
    fill_psnr)."""
    m = mask != 0
    cnt = int(m.sum())
    t = target.double()
    err = (img.double() - t)[m]
    mse = float((err * err).sum()) / cnt if cnt else 0.0
    peak = float(t.max() - t.min())
    if mse == 0.0 or peak == 0.0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)


def tile_sse(torch, img, target, mask, tile):
    """Squared error over mask, summed per tile x tile block (FP64)."""
    H, W = img.shape
    e = (img.double() - target.double()) ** 2 * (mask != 0).double()
    ph, pw = (-H) % tile, (-W) % tile
    if ph or pw:
        e = torch.nn.functional.pad(e, (0, pw, 0, ph))
    return e.reshape((H + ph) // tile, tile, (W + pw) // tile, tile).sum(dim=(1, 3))


FILL_FWD_FLOP_PX = 10368.0      # 2 x (432 + 2304 + 2304 + 144) multiply-adds
FILL_TRAIN_FLOP_PX = 30240.0    # forward, weight gradients, input gradients of layers 2-4


def run_fill(args, torch, dev, fb, eventsim, hd=None):
    """Learned stale fill: train on readouts of seeded 1280x720 sequences,
    choose the per-tile fallback threshold on the training frames, score
    against the Gaussian fill on held-out ones, and time inference, training
    steps and the reconstruction with the fill on every readout."""
    from concurrent.futures import ThreadPoolExecutor
    stream = torch.cuda.current_stream(dev).cuda_stream
    t0 = time.time()
    train_seeds = list(range(5000, 5000 + args.fill_train_seqs))
    eval_seeds = list(range(6000, 6000 + args.fill_eval_seqs))
    with ThreadPoolExecutor(max_workers=min(16, len(os.sched_getaffinity(0)))) as pool:
        Ltr, Str, Atr, Ttr = fill_frames(torch, dev, fb, eventsim, train_seeds,
                                         args.fill_events, 100_000, stream, pool)
        Lev, Sev, Aev, Tev = fill_frames(torch, dev, fb, eventsim, eval_seeds,
                                         args.fill_events, 100_000, stream, pool)
    F, H, W = Ltr.shape
    log("fill: %d training and %d evaluation frames (%d + %d sequences) in %.1f s"
        % (F, Lev.shape[0], len(train_seeds), len(eval_seeds), time.time() - t0))

    rng = np.random.default_rng(args.fill_seed)
    B, TS, TILE = 32, 128, 16
    ar = torch.arange(TS, device=dev)

    def batch():
        f = torch.from_numpy(rng.integers(0, F, B)).to(dev)[:, None, None]
        y = torch.from_numpy(rng.integers(0, H - TS + 1, B)).to(dev)[:, None, None] + ar[None, :, None]
        x = torch.from_numpy(rng.integers(0, W - TS + 1, B)).to(dev)[:, None, None] + ar[None, None, :]
        return [t[f, y, x].contiguous() for t in (Ltr, Str, Atr, Ttr)]

    fill = fb.Fill(eventsim.fill_init_params(args.fill_seed), stream=stream)
    losses = []
    t0 = time.time()
    for step in range(args.fill_steps):
        want = step % 100 == 0 or step == args.fill_steps - 1
        rc, loss = fill.train_step(*batch(), lr=args.fill_lr, want_loss=want)
        assert rc == 0
        if want:
            losses.append((step, round(loss, 5)))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log("fill: %d Adam steps in %.1f s, batch loss %s" % (args.fill_steps, train_s, losses))

    out = torch.empty((H, W), dtype=torch.float32, device=dev)

    def mean_psnr(Ls, Ss, As, Ts, frames, theta):
        v = []
        for k in frames:
            assert fill.apply(Ls[k], Ss[k], As[k], out, tile=TILE, theta=theta)[0] == 0
            v.append(psnr_dev(torch, out, Ts[k], Ss[k]))
        return float(np.mean(v))

    # ---- the fallback threshold, chosen on training frames -----------------
    # theta: the fraction of a tile's pixels that must be stale for the
    # network to fill it (0: every tile with a stale pixel; 1: none)
    grid = [0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.4, 0.5, 0.6, 0.8, 1.0]
    sel = list(range(0, F, max(1, F // args.fill_theta_frames)))
    train_curve = [(th, round(mean_psnr(Ltr, Str, Atr, Ttr, sel, th), 4)) for th in grid]
    theta = max(train_curve, key=lambda c: c[1])[0]
    log("fill: training PSNR by theta %s -> theta %.2f" % (train_curve, theta))

    # ---- quality on held-out frames ---------------------------------------
    psnr_g, psnr_l, psnr_f, psnr_ub, fb_frac = [], [], [], [], []
    pred = torch.empty_like(out)
    tiles = ((H + TILE - 1) // TILE) * ((W + TILE - 1) // TILE)
    for k in range(Lev.shape[0]):
        L, S, A, T = Lev[k], Sev[k], Aev[k], Tev[k]
        psnr_g.append(psnr_dev(torch, L, T, S))
        assert fill.apply(L, S, A, out, tile=TILE, theta=0.0)[0] == 0
        psnr_l.append(psnr_dev(torch, out, T, S))
        rc, nfb = fill.apply(L, S, A, out, tile=TILE, theta=theta)
        assert rc == 0
        psnr_f.append(psnr_dev(torch, out, T, S))
        fb_frac.append(nfb / tiles)
        # per-tile choice with the ground truth in hand: an upper bound of
        # any per-tile rule between the two fills
        assert fill.predict(L[None], S[None], A[None], pred) == 0
        best = torch.minimum(tile_sse(torch, pred, T, S, TILE), tile_sse(torch, L, T, S, TILE))
        cnt = int((S != 0).sum())
        mse = float(best.sum()) / max(cnt, 1)
        peak = float(T.max() - T.min())
        psnr_ub.append(10.0 * np.log10(peak * peak / mse) if mse > 0 and peak > 0 else float("inf"))
    # the same check with the simulator's host scorer on one frame
    assert abs(eventsim.fill_psnr(Lev[0].cpu().numpy(), Tev[0].cpu().numpy(),
                                  Sev[0].cpu().numpy()) - psnr_g[0]) < 1e-6

    # ---- throughput ---------------------------------------------------------
    lib = fb.load()
    reps = 50
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        lib.fibar_fill_apply(fill.handle, Lev[0].data_ptr(), Sev[0].data_ptr(), Aev[0].data_ptr(),
                             H, W, TILE, theta, out.data_ptr(), None)
    ev_a.record()
    for _ in range(reps):
        lib.fibar_fill_apply(fill.handle, Lev[0].data_ptr(), Sev[0].data_ptr(), Aev[0].data_ptr(),
                             H, W, TILE, theta, out.data_ptr(), None)
    ev_b.record()
    torch.cuda.synchronize()
    infer_ms = ev_a.elapsed_time(ev_b) / reps
    # the fused network kernel alone (prediction without the fallback pass)
    ev_a.record()
    for _ in range(reps):
        lib.fibar_fill_predict(fill.handle, Lev[0].data_ptr(), Sev[0].data_ptr(), Aev[0].data_ptr(),
                               1, H, W, pred.data_ptr())
    ev_b.record()
    torch.cuda.synchronize()
    fused_ms = ev_a.elapsed_time(ev_b) / reps
    bt = [batch() for _ in range(4)]
    for b_ in bt:
        fill.train_step(*b_, lr=0.0, want_loss=False)
    ev_a.record()
    for i in range(reps):
        fill.train_step(*bt[i % 4], lr=0.0, want_loss=False)
    ev_b.record()
    torch.cuda.synchronize()
    step_ms = ev_a.elapsed_time(ev_b) / reps
    combined = None
    if hd is not None:
        combined = fill_pipeline(args, torch, dev, fb, fill, hd, theta, stream)
    fill.close()
    del Ltr, Str, Atr, Ttr
    infer_tflops = FILL_FWD_FLOP_PX * H * W / (infer_ms * 1e-3) / 1e12
    fused_tflops = FILL_FWD_FLOP_PX * H * W / (fused_ms * 1e-3) / 1e12
    train_tflops = FILL_TRAIN_FLOP_PX * B * TS * TS / (step_ms * 1e-3) / 1e12
    m = lambda v: round(float(np.mean(v)), 3)   # noqa: E731
    res = {"train_frames": int(F), "eval_frames": int(Lev.shape[0]),
           "train_sequences": len(train_seeds), "eval_sequences": len(eval_seeds),
           "events_per_sequence": args.fill_events, "readout_every": 100_000,
           "steps": args.fill_steps, "batch": "%dx%dx%d" % (B, TS, TS), "lr": args.fill_lr,
           "batch_loss": losses,
           "psnr_db": {"gaussian_fill": m(psnr_g), "learned": m(psnr_l),
                       "learned_with_fallback": m(psnr_f),
                       "per_tile_ground_truth_upper_bound": m(psnr_ub),
                       "gain_db": round(float(np.mean(psnr_l) - np.mean(psnr_g)), 3),
                       "gain_with_fallback_db": round(float(np.mean(psnr_f) - np.mean(psnr_g)), 3)},
           "fallback": {"rule": "the network fills a 16x16 tile when more than a fraction theta "
                                "of its pixels are stale and every stale prediction is finite",
                        "tile": TILE, "theta": theta,
                        "theta_chosen_on": "%d training frames" % len(sel),
                        "training_psnr_by_theta": train_curve,
                        "tiles_fallen_back": round(float(np.mean(fb_frac)), 4)},
           "inference": {"ms_per_frame": round(infer_ms, 4), "tflops": round(infer_tflops, 2),
                         "frac_bf16_peak": round(infer_tflops / 2500.0, 5)},
           "reconstruction_with_fill": combined,
           "training": {"ms_per_step": round(step_ms, 4), "tflops": round(train_tflops, 2),
                        "frac_bf16_peak": round(train_tflops / 2500.0, 5)},
           "roofline": {"bound": "mfma", "kernel": "k_fill_fused", "achieved": round(fused_tflops, 2),
                        "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": round(fused_tflops / 2500.0, 5), "traffic": None,
                        "us_per_launch_back_to_back": round(fused_ms * 1e3, 3),
                        "flops_per_launch": FILL_FWD_FLOP_PX * H * W}}
    log("fill: PSNR gaussian %.2f dB, learned %.2f dB, with fallback (theta %.2f) %.2f dB, "
        "per-tile upper bound %.2f dB; inference %.3f ms per 1280x720 frame (%.1f TFLOP/s), "
        "training step %.3f ms (%.1f TFLOP/s)"
        % (res["psnr_db"]["gaussian_fill"], res["psnr_db"]["learned"], theta,
           res["psnr_db"]["learned_with_fallback"],
           res["psnr_db"]["per_tile_ground_truth_upper_bound"], infer_ms, infer_tflops, step_ms,
           train_tflops))
    return res


def fill_pipeline(args, torch, dev, fb, fill, hd, theta, stream):
    """The hd720 stream reconstructed with the learned fill applied to every
    readout: the stream's pushes and readouts (brightness, stale mask, log
    age into per-readout device buffers) submitted at once, then the fill of
    every readout, all on one stream.  Returns Mev/s of the whole."""
    W, H, n = hd["W"], hd["H"], hd["n"]
    sched = hd["sched"]
    gx, gy, gp = hd["gx"], hd["gy"], hd["gp"]
    n_read = sum(1 for it in sched if it[0] == "read")
    L = torch.empty((n_read, H, W), dtype=torch.float32, device=dev)
    S = torch.empty((n_read, H, W), dtype=torch.uint8, device=dev)
    A = torch.empty((n_read, H, W), dtype=torch.float32, device=dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    ops, r = [], 0
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            ops.append(fb.readout_op(int(hd["ev_t"][it[1] - 1]), L[r], stale=S[r], log_age=A[r]))
            r += 1
    arr = (fb.fibar_op * len(ops))(*ops)
    lib = fb.load()
    ctx = fb.Context(W, H, stream=stream)
    Lp, Sp, Ap = L.data_ptr(), S.data_ptr(), A.data_ptr()
    fsz, ssz = 4 * W * H, W * H

    def step():
        assert ctx.reset() == 0
        assert lib.fibar_submit(ctx.handle, arr, len(ops)) == 0
        for k in range(n_read):
            assert lib.fibar_fill_apply(fill.handle, Lp + k * fsz, Sp + k * ssz, Ap + k * fsz,
                                        H, W, 16, theta, out.data_ptr(), None) == 0

    steps = max(1, min(args.steps, 5))
    for _ in range(max(1, min(args.warmup, 2))):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    assert ctx.synchronize() == 0
    ctx.close()
    res = {"mev_s": round(n / el / 1e6, 2), "ms_per_step": round(1e3 * el, 3),
           "fills_per_step": n_read, "plain_mev_s": round(hd["plain_mev_s"], 2),
           "workload": "the hd720 stream with readouts of brightness, stale mask and log age, "
                       "and the learned fill (theta %.2f) on each" % theta}
    log("fill: hd720 reconstruction with the fill on all %d readouts: %.1f Mev/s (%.1f ms/step)"
        % (n_read, res["mev_s"], 1e3 * el))
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--launch", choices=sorted(LAUNCH_MODES), default="direct",
                    help="how a batch's in-order kernels are issued (spatial filter on)")
    ap.add_argument("--events", type=int, default=100_000_000)
    ap.add_argument("--cpu-sample-events", type=int, default=100_000_000,
                    help="events of the stream the oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nsf", action="store_true", help="skip the blur-off measurement")
    ap.add_argument("--only-nsf", action="store_true",
                    help="measure only the blur-off mode (for profiling)")
    ap.add_argument("--roofline-kernel", default="pop_blur", choices=KERNELS)
    ap.add_argument("--time-every", type=int, default=16,
                    help="time every n-th launch of the roofline kernel (events on its dispatch)")
    ap.add_argument("--no-multi", action="store_true", help="skip the batched-streams measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 64x48 and 640x480 configurations")
    ap.add_argument("--no-tiles", action="store_true",
                    help="skip the per-tile-queue measurement")
    ap.add_argument("--tile", type=int, default=32, help="tile side of the per-tile-queue leg")
    ap.add_argument("--only-configs", action="store_true",
                    help="run only the 64x48 and 640x480 configurations")
    ap.add_argument("--only-multi", action="store_true",
                    help="measure only the batched streams (for profiling)")
    ap.add_argument("--multi-scale", type=float, default=1.0,
                    help="scale of the batched streams' lengths (1.0: 5-40M events each)")
    ap.add_argument("--no-fill", action="store_true", help="skip the learned-fill leg")
    ap.add_argument("--only-fill", action="store_true", help="run only the learned-fill leg")
    ap.add_argument("--fill-train-seqs", type=int, default=200,
                    help="training sequences (seeds 5000...; 200 for the full set)")
    ap.add_argument("--fill-eval-seqs", type=int, default=20,
                    help="held-out sequences (seeds 6000...; 20 for the full set)")
    ap.add_argument("--fill-events", type=int, default=2_000_000)
    ap.add_argument("--fill-steps", type=int, default=1000)
    ap.add_argument("--fill-lr", type=float, default=1e-3)
    ap.add_argument("--fill-theta-frames", type=int, default=400,
                    help="training frames the fallback threshold is chosen on")
    ap.add_argument("--fill-seed", type=int, default=7)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (for scaling the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the FIBAR path keeps one global window per "
              "stream and this build has no multi-GPU path (see the design notes for how it "
              "would shard). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import eventsim
    import paper_2510_20071_amd as fb

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    fb.load()
    if args.only_multi:
        run_batched(args, torch, dev, fb, eventsim)
        return
    if args.only_fill:
        print(json.dumps(run_fill(args, torch, dev, fb, eventsim)))
        return
    if args.only_configs:
        print(json.dumps({name: run_config(args, torch, dev, fb, eventsim, name)
                          for name in ("sensor64x48", "vga")}))
        return

    wl = eventsim.preset("hd720", n_events=args.events)
    W, H = wl.scene.width, wl.scene.height
    npx = W * H
    t0 = time.time()
    ev = eventsim.generate(wl.scene)
    n = len(ev)
    log("generated %d events in %.1f s" % (n, time.time() - t0))
    sched = eventsim.schedule(n, wl.packet, wl.readouts)
    n_push = sum(1 for it in sched if it[0] == "push")
    n_read = sum(1 for it in sched if it[0] == "read")

    gx = torch.from_numpy(ev.x.view(np.int16)).to(dev)
    gy = torch.from_numpy(ev.y.view(np.int16)).to(dev)
    gp = torch.from_numpy(ev.p).to(dev)
    frames = torch.empty((n_read, npx), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    bx, by, bp = gx.data_ptr(), gy.data_ptr(), gp.data_ptr()
    fptr = frames.data_ptr()

    def build_ops():
        ops = []
        r = 0
        for it in sched:
            if it[0] == "push":
                a, b = it[1], it[2]
                op = fb.fibar_op()
                op.kind = fb.FIBAR_OP_PUSH
                op.packet = fb.fibar_packet(bx + 2 * a, by + 2 * a, bp + a, None, b - a, 1)
                ops.append(op)
            else:
                op = fb.fibar_op()
                op.kind = fb.FIBAR_OP_READOUT
                op.t = int(ev.t[it[1] - 1])
                op.readout = fb.fibar_readout_buf(fptr + 4 * npx * r, None, None, None, None,
                                                  None, None, None, 1)
                ops.append(op)
                r += 1
        return (fb.fibar_op * len(ops))(*ops), len(ops)

    ops, n_ops = build_ops()
    lib = fb.load()
    stream = torch.cuda.current_stream(dev).cuda_stream

    def run_mode(spatial, steps, warmup, time_kernel=None):
        ctx = fb.Context(W, H, spatial_filter=spatial, stream=stream)
        if spatial:
            assert fb.fibar_set_launch_mode(ctx.handle, LAUNCH_MODES[args.launch]) == 0
        # timing is on from the warm-up, so that the warm-up already builds
        # every graph the timed steps replay
        if time_kernel is not None:
            fb.fibar_set_kernel_timing(ctx.handle, 1 << KERNELS.index(time_kernel),
                                       args.time_every)
        for _ in range(warmup):
            assert ctx.reset() == 0
            assert lib.fibar_submit(ctx.handle, ops, n_ops) == 0
        torch.cuda.synchronize()
        if time_kernel is not None:
            for kind in range(5):
                fb.fibar_kernel_time(ctx.handle, kind)  # clear the warm-up's
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            assert ctx.reset() == 0
            assert lib.fibar_submit(ctx.handle, ops, n_ops) == 0
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kt = None
        if time_kernel is not None:
            rc, ms, launches = fb.fibar_kernel_time(ctx.handle, KERNELS.index(time_kernel))
            kt = (ms, launches)
            for kind in range(5):
                fb.fibar_kernel_time(ctx.handle, kind)  # the others' events go back to the pool
            fb.fibar_set_kernel_timing(ctx.handle, 0)
        assert ctx.synchronize() == 0
        st = ctx.stats() if spatial else None
        final = ctx.readout_host(int(ev.t[-1]))
        ctx.close()
        return elapsed, kt, st, final

    if args.only_nsf:
        el_off, _, _, _ = run_mode(False, args.steps, args.warmup)
        log("blur off: %.1f ms/step, %.1f Mev/s" % (1e3 * el_off / args.steps,
                                                     n * args.steps / el_off / 1e6))
        return
    el_on, kt, st_on, final_on = run_mode(True, args.steps, args.warmup, args.roofline_kernel)
    mev_on = n * args.steps / el_on / 1e6
    log("blur on : %.1f ms/step, %.1f Mev/s" % (1e3 * el_on / args.steps, mev_on))
    mev_off = None
    if not args.no_nsf:
        el_off, _, _, final_off = run_mode(False, args.steps, args.warmup)
        mev_off = n * args.steps / el_off / 1e6
        log("blur off: %.1f ms/step, %.1f Mev/s" % (1e3 * el_off / args.steps, mev_off))

    # ---- roofline of the timed kernel ------------------------------------
    u = distinct_per_packet(ev.x, ev.y, W, wl.packet)          # distinct pixels / event
    s_per_ev = st_on["total_stale"] / n                         # stale pixels / event
    pops = st_on["h"]                                           # popped events, whole stream
    stale = st_on["total_stale"]
    ms, launches = kt
    avg_s = ms / 1e3 / max(launches, 1)
    if args.roofline_kernel == "pop_blur":
        per_launch = (8.0 * pops + 42.0 * stale) / n_push
    elif args.roofline_kernel == "apply":
        per_launch = ((28.0 * u + 4.0) * n + 2.0 * stale) / n_push
    elif args.roofline_kernel == "group_compose":
        # one launch per batch of up to 256 chunks of 16384 events
        chunks = sum(-(-(b - a) // 16384) for it in sched if it[0] == "push"
                     for a, b in [(it[1], it[2])])
        per_launch = 5.0 * n / -(-chunks // 256)
    elif args.roofline_kernel == "readout":
        per_launch = 8.0 * npx
    else:
        per_launch = 8.0 * npx + (8.0 * pops + 42.0 * stale) / n_push
    achieved = per_launch / avg_s / 1e9
    R = n / n_read
    B_on = bytes_per_event(u, s_per_ev, W, H, R, True)
    B_off = bytes_per_event(u, s_per_ev, W, H, R, False)
    roofline = {"bound": "hbm", "kernel": "k_" + args.roofline_kernel,
                "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 5),
                "traffic": measured_traffic(args.roofline_kernel),
                "avg_launch_us": round(avg_s * 1e6, 3), "timed_launches": launches,
                "timed_every": args.time_every, "bytes_per_launch": round(per_launch, 1),
                "duration": "HIP events on every %d-th dispatch of the kernel in the timed "
                            "steps; they span the dispatch too, so they read above the "
                            "profiler's kernel duration" % args.time_every,
                "frac_end_to_end": {
                    "blur_on": round(B_on * mev_on * 1e6 / 8e12, 5),
                    "blur_off": None if mev_off is None else
                    round(B_off * mev_off * 1e6 / 8e12, 5),
                    "bytes_per_event": {"blur_on": round(B_on, 2), "blur_off": round(B_off, 2)}}}

    # ---- CPU baseline (the FP64 oracle) and parity -------------------------
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        secs, m, orc = time_oracle(oracle, W, H, ev, sched, True, limit=args.cpu_sample_events)
        cpu = {"value": round(m / secs / 1e6, 3), "unit": "Mev/s", "cores": 1, "kind": "oracle",
               "sample": "first %d events of the hd720 stream with their readouts, blur on, "
                         "FP64, one thread pinned to one CPU" % m}
        cpu.update(host_info())
        log("oracle: %d events in %.1f s (%.2f Mev/s)" % (m, secs, m / secs / 1e6))
        if m == n:
            parity = final_parity(final_on, orc.readout(int(ev.t[-1])), True)
            parity["window_scalars_equal"] = all(st_on[f] == orc.stats()[f]
                                                 for f in ("k", "h", "Q", "P", "T"))
            log("parity: %s" % parity)
        orc.close()
        if not args.no_nsf:
            secs, m, orc = time_oracle(oracle, W, H, ev, sched, False,
                                       limit=args.cpu_sample_events)
            cpu["blur_off_value"] = round(m / secs / 1e6, 3)
            log("oracle, blur off: %d events in %.1f s (%.2f Mev/s)"
                % (m, secs, m / secs / 1e6))
            if m == n and parity is not None:
                parity["blur_off"] = final_parity(final_off, orc.readout(int(ev.t[-1])), False)
            orc.close()

    tiles = None
    if not args.no_tiles:
        tiles = tiles_leg(args, torch, dev, fb, W, H, ev, sched, ops, n_ops, stream, n)

    configs = None
    if not args.no_configs:
        configs = {name: run_config(args, torch, dev, fb, eventsim, name)
                   for name in ("sensor64x48", "vga")}
    batched = None
    if not args.no_multi:
        batched = run_batched(args, torch, dev, fb, eventsim)
    learned_fill = None
    if not args.no_fill:
        hd = {"gx": gx, "gy": gy, "gp": gp, "ev_t": ev.t, "sched": sched, "W": W, "H": H,
              "n": n, "plain_mev_s": mev_on}
        learned_fill = run_fill(args, torch, dev, fb, eventsim, hd)

    out = {
        "metric": "Mev/s reconstructed at 1280x720 (blur on)",
        "value": round(mev_on, 2),
        "unit": "Mev/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * el_on / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hd720: 1280x720 sensor, %d events, %d-event packets, %d readouts "
                               "(random indices), T_cut=40, r_fill=1/2, spatial filter on"
                               % (n, wl.packet, n_read),
                   "events": n, "packets": n_push, "readouts": n_read, "launch": args.launch},
        "blur_off_mev_s": None if mev_off is None else round(mev_off, 2),
        "workload_stats": {"distinct_pixels_per_event": round(u, 4),
                           "stale_pixels_per_event": round(s_per_ev, 5),
                           "popped_events": pops,
                           "final_queue_length": st_on["q"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "per_tile_queues": tiles,
        "configs": configs,
        "batched_streams": batched,
        "learned_fill": learned_fill,
        "paper_cpu_context_mev_s": {"blur_on": 42, "blur_off": 140},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
