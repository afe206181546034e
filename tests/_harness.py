"""Shared helpers of the GPU parity tests: run a schedule through libfibar
(C ABI) and through the FP64 oracle, and compare the results."""
import numpy as np

import eventsim
import oracle
import paper_2510_20071_amd as fb

# Brightness tolerance (FP32 device state against the FP64 oracle): per
# pixel |dL| <= REL * max(|L_ref|, 1), and over the frame
# max|dL| <= REL * max(max|L_ref|, 1).  One event moves L by about
# (1 + beta)/2 * alpha ~ 0.8 at T_cut = 40, so the floor of 1 is one
# event's step.
REL = 1e-5


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def to_device(ev):
    torch, dev = torch_dev()
    gx = torch.from_numpy(np.ascontiguousarray(ev.x).view(np.int16)).to(dev)
    gy = torch.from_numpy(np.ascontiguousarray(ev.y).view(np.int16)).to(dev)
    gp = torch.from_numpy(np.ascontiguousarray(ev.p)).to(dev)
    return gx, gy, gp


def make_ctx(W, H, **kw):
    torch, dev = torch_dev()
    stream = torch.cuda.current_stream(dev).cuda_stream
    return fb.Context(W, H, stream=stream, **kw)


def oracle_kw(kw):
    keep = {k: v for k, v in kw.items() if k in ("t_cut", "fill", "q_min", "q_max",
                                                  "spatial_filter", "regulation", "region",
                                                  "age_max")}
    return keep


def compare_state(g, r, spatial, where=""):
    """g: readout_host dict of the GPU; r: oracle readout."""
    assert np.array_equal(g["last"], r["last"]), "last_index " + where
    if "tot" in g:
        assert np.array_equal(g["tot"].astype(np.uint64), r["tot"].astype(np.uint64)), \
            "total_count " + where
    if spatial:
        assert np.array_equal(g["cnt"].astype(np.int64), r["cnt"].astype(np.int64)), "cnt " + where
        assert np.array_equal(g["stale"], r["stale"]), "stale " + where
        assert np.array_equal(g["tcnt"].astype(np.int64), r["tcnt"].astype(np.int64)), "tcnt " + where
    for key in ("L", "pbar"):
        ref = r[key]
        d = np.abs(g[key].astype(np.float64) - ref)
        bound = REL * np.maximum(np.abs(ref), 1.0)
        bad = np.nonzero(d > bound)[0]
        assert bad.size == 0, "%s %s: %d pixels off, worst %.3g at %d (ref %.6g)" % (
            key, where, bad.size, d.max(), int(np.argmax(d)), ref[int(np.argmax(d))])
        assert d.max() <= REL * max(np.abs(ref).max(), 1.0), key + " " + where


def compare_stats(gs, os_, where=""):
    for f in ("k", "h", "Q", "P", "T", "n_regulations", "last_stale", "total_stale"):
        assert gs[f] == os_[f], "%s %s: gpu %d oracle %d" % (f, where, gs[f], os_[f])


def compare_tiles(ctx, orc, where=""):
    """Per-tile scalars of a per-tile-queue context against the oracle's."""
    g, r = ctx.tile_stats(), orc.region_stats()
    for key in ("q", "Q", "P", "T", "front"):
        assert np.array_equal(g[key], r[key]), "tile %s %s" % (key, where)


def oracle_step_record(st, n):
    """The oracle's window scalars after a regulation step, in the field
    order of fibar_step_record."""
    return [st["k"], st["h"], st["q"], st["Q"], st["P"], st["T"], st["last_stale"], n]


def telemetry_buffer(ctx, capacity):
    """A device buffer for `capacity` step records, registered with ctx."""
    torch, dev = torch_dev()
    buf = torch.full((capacity, fb.STEP_RECORD_WORDS), -7, dtype=torch.int64, device=dev)
    assert ctx.set_telemetry(buf, capacity) == fb.FIBAR_OK
    return buf


def compare_telemetry(buf, want, where=""):
    """Records written by the device against the oracle's, bit for bit."""
    got = buf.cpu().numpy()
    want = np.asarray(want, dtype=np.int64).reshape(-1, fb.STEP_RECORD_WORDS)
    n = min(len(want), got.shape[0])
    for i in range(n):
        if not np.array_equal(got[i], want[i]):
            raise AssertionError("step record %d %s: gpu %s oracle %s (fields %s)" % (
                i, where, got[i].tolist(), want[i].tolist(), fb.STEP_RECORD_FIELDS))
    assert np.all(got[n:] == -7), "records written past the regulation steps " + where


def run_pair(ev, W, H, sched, check_every_read=1, check_stats=True, telemetry=True, gain=None,
             **kw):
    """Run `sched` on GPU (device packets) and oracle; compare at readouts,
    and (spatial filter on) every step's window scalars.  `gain`: per-pixel
    multipliers of Eq. (6)'s increment (float32 values, given to both)."""
    ctx = make_ctx(W, H, **kw)
    orc = oracle.Oracle(W, H, **oracle_kw(kw))
    if gain is not None:
        torch, dev = torch_dev()
        g32 = np.ascontiguousarray(gain, np.float32)
        gd = torch.from_numpy(g32).to(dev)
        assert ctx.set_gain(gd) == fb.FIBAR_OK
        assert orc.set_gain(g32.astype(np.float64)) == 0
    gx, gy, gp = to_device(ev)
    spatial = kw.get("spatial_filter", True)
    tel, want = None, []
    if spatial and telemetry:
        tel = telemetry_buffer(ctx, sum(1 for it in sched if it[0] == "push") + 2)
    nread = 0
    for item in sched:
        if item[0] == "push":
            a, b = item[1], item[2]
            assert ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
            assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
            if tel is not None and b > a:
                want.append(oracle_step_record(orc.stats(), b - a))
        else:
            nread += 1
            if (nread - 1) % check_every_read:
                continue
            k = item[1]
            g = ctx.readout_host(0)
            r = orc.readout(0)
            assert isinstance(g, dict), g
            compare_state(g, r, spatial, "at event %d" % k)
            if check_stats and spatial:
                compare_stats(ctx.stats(), orc.stats(), "at event %d" % k)
            if kw.get("region"):
                compare_tiles(ctx, orc, "at event %d" % k)
    g = ctx.readout_host(0)
    r = orc.readout(0)
    compare_state(g, r, spatial, "final")
    if spatial:
        compare_stats(ctx.stats(), orc.stats(), "final")
    if tel is not None:
        compare_telemetry(tel, want, "(%dx%d)" % (W, H))
    ctx.close()
    return g, r
