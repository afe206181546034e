"""GPU parity: libfibar (HIP, through the C ABI) against the FP64 oracle.

Integer state (active counts, last-update indices, stale masks, active
tiles, window scalars) must match bit for bit; brightness and the polarity
average within 1e-5 relative (per pixel, with a floor of one event's step).
"""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import (REL, compare_state, compare_stats, make_ctx, run_pair, to_device,
                      torch_dev)

pytestmark = pytest.mark.gpu


def flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("spatial", [True, False])
def test_sensor64x48_full_stream(spatial):
    w = eventsim.preset("sensor64x48")
    ev = eventsim.generate(w.scene)
    flush("sensor64x48 200k events, spatial=%s" % spatial)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    run_pair(ev, 64, 48, sched, spatial_filter=spatial)


def test_ragged_packets_spanning_chunks():
    w = eventsim.preset("sensor64x48", n_events=150000, seed=7)
    ev = eventsim.generate(w.scene)
    sizes = [1, 2, 3, 17, 1023, 1024, 1025, 16383, 16384, 16385, 40000, 5, 7, 33000]
    sched, a = [], 0
    i = 0
    while a < len(ev):
        b = min(len(ev), a + sizes[i % len(sizes)])
        sched.append(("push", a, b))
        sched.append(("read", b))
        a = b
        i += 1
    flush("ragged packets on 64x48 (%d pushes)" % (len(sched) // 2))
    run_pair(ev, 64, 48, sched, q_min=8)


@pytest.mark.parametrize("W,H", [(1, 1), (2, 2), (4, 2), (3, 3), (5, 4)])
def test_tiny_sensors(W, H):
    rng = np.random.default_rng(W * 10 + H)
    n = 3000
    pix = np.empty(n, np.int64)
    cur = 0
    for e in range(n):
        if rng.random() < 0.35:
            cur = int(rng.integers(0, W * H))
        pix[e] = cur
    ev = eventsim.Events((pix % W).astype(np.uint16), (pix // W).astype(np.uint16),
                         (rng.random(n) < 0.5).astype(np.uint8), np.arange(n, dtype=np.uint64))
    sched, a = [], 0
    while a < n:
        b = min(n, a + int(rng.integers(1, 9)))
        sched.append(("push", a, b))
        sched.append(("read", b))
        a = b
    flush("tiny sensor %dx%d" % (W, H))
    run_pair(ev, W, H, sched, q_min=1)


def test_single_pixel_long_segments_closed_form():
    W, H = 16, 8
    n = 50000
    ev = eventsim.Events(np.full(n, 5, np.uint16), np.full(n, 3, np.uint16),
                         np.ones(n, np.uint8), np.arange(n, dtype=np.uint64))
    sched = [("push", 0, 20000), ("read", 20000), ("push", 20000, 20001), ("read", 20001),
             ("push", 20001, 50000), ("read", 50000)]
    flush("single pixel, segments of 20000 and 29999 events")
    g, r = run_pair(ev, W, H, sched, q_min=1, max_packet=1 << 20)
    a, b = oracle.coefficients(40.0)
    i = 3 * W + 5
    assert abs(g["pbar"][i] - (1.0 - a ** n)) <= REL
    assert abs(g["L"][i]) <= REL   # decayed to zero after 50000 identical events


def test_polarity_flip_is_exact_negation():
    w = eventsim.preset("sensor64x48", n_events=60000, seed=3)
    ev = eventsim.generate(w.scene)
    flip = eventsim.Events(ev.x, ev.y, (1 - ev.p).astype(np.uint8), ev.t)
    outs = []
    for e in (ev, flip):
        ctx = make_ctx(64, 48, q_min=16)
        gx, gy, gp = to_device(e)
        for a in range(0, len(e), 1024):
            assert ctx.push(gx[a:a + 1024], gy[a:a + 1024], gp[a:a + 1024]) == 0
        outs.append(ctx.readout_host(0))
        ctx.close()
    assert np.array_equal(outs[0]["L"], -outs[1]["L"])
    assert np.array_equal(outs[0]["pbar"], -outs[1]["pbar"])
    for key in ("cnt", "stale", "last", "tcnt"):
        assert np.array_equal(outs[0][key], outs[1][key])


def test_same_input_twice_is_bit_identical():
    w = eventsim.preset("vga", n_events=400000, seed=12)
    ev = eventsim.generate(w.scene)
    outs = []
    for _ in range(2):
        ctx = make_ctx(640, 480)
        gx, gy, gp = to_device(ev)
        for a in range(0, len(ev), 8192):
            assert ctx.push(gx[a:a + 8192], gy[a:a + 8192], gp[a:a + 8192]) == 0
        outs.append(ctx.readout_host(0))
        ctx.close()
    for key in outs[0]:
        assert np.array_equal(outs[0][key], outs[1][key]), key


@pytest.mark.parametrize("spatial", [True, False])
def test_vga_two_million_events(spatial):
    w = eventsim.preset("vga", n_events=2_000_000)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    flush("vga 2M events, spatial=%s" % spatial)
    run_pair(ev, 640, 480, sched, check_every_read=8, spatial_filter=spatial)


@pytest.mark.parametrize("spatial", [True, False])
def test_vga_full_stream_as_submitted(spatial):
    """The 640x480 configuration at its full length: 20 M events in
    8192-event packets with a brightness readout every 50 000 events (400),
    all in one submit, blur on and off.  Sampled frames (first, last and
    every 40th) and the final state against the FP64 oracle."""
    torch, dev = torch_dev()
    W, H = 640, 480
    npx = W * H
    w = eventsim.preset("vga")
    ev = eventsim.generate(w.scene)
    assert len(ev) == 20_000_000
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    n_read = sum(1 for it in sched if it[0] == "read")
    flush("vga %d events, %d readouts in one submit, spatial=%s" % (len(ev), n_read, spatial))
    sample = sorted(set(range(0, n_read, 40)) | {1, n_read - 1})
    gx, gy, gp = to_device(ev)
    scratch = torch.empty(npx, dtype=torch.float32, device=dev)
    frames = {i: torch.empty(npx, dtype=torch.float32, device=dev) for i in sample}
    ops, r = [], 0
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            ops.append(fb.readout_op(0, frames.get(r, scratch)))
            r += 1
    ctx = make_ctx(W, H, spatial_filter=spatial)
    assert ctx.submit(ops) == 0
    assert ctx.synchronize() == 0
    got = {i: f.cpu().numpy() for i, f in frames.items()}
    final = ctx.readout_host(0)
    orc = oracle.Oracle(W, H, spatial_filter=spatial)
    r = 0
    for it in sched:
        if it[0] == "push":
            assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
            continue
        if r in got:
            ref = orc.readout(0)["L"]
            d = np.abs(got[r].astype(np.float64) - ref)
            assert np.all(d <= REL * np.maximum(np.abs(ref), 1.0)), \
                "frame %d: worst %.3g" % (r, d.max())
        r += 1
    compare_state(final, orc.readout(0), spatial, "end of the 640x480 stream")
    if spatial:
        compare_stats(ctx.stats(), orc.stats())
    flush("vga full stream: %d sampled frames and the final state match" % len(got))
    ctx.close()


def test_hd720_twenty_million_events():
    w = eventsim.preset("hd720", n_events=20_000_000)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    flush("hd720 20M events, blur on, %d readouts" % len(w.readouts))
    run_pair(ev, 1280, 720, sched, check_every_read=25)


def test_hd720_benchmark_stream_as_submitted():
    """The benchmark's stream as bench.py submits it: 1280x720, 100 M events,
    16384-event packets, 1000 brightness-only device readouts at random event
    indices, all in one submit (so most readouts are written by the pop
    launch of the push before them).  Sampled frames and the final state
    against the FP64 oracle."""
    torch, dev = torch_dev()
    W, H = 1280, 720
    npx = W * H
    w = eventsim.preset("hd720")
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    n_read = sum(1 for it in sched if it[0] == "read")
    flush("hd720 %d events, %d readouts in one submit" % (len(ev), n_read))
    sample = sorted({0, 1, n_read // 3, n_read // 2, n_read - 2, n_read - 1})
    gx, gy, gp = to_device(ev)
    scratch = torch.empty(npx, dtype=torch.float32, device=dev)
    frames = {i: torch.empty(npx, dtype=torch.float32, device=dev) for i in sample}
    ops, r = [], 0
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            ops.append(fb.readout_op(0, frames.get(r, scratch)))
            r += 1
    ctx = make_ctx(W, H, max_packet=w.packet)
    assert ctx.submit(ops) == 0
    assert ctx.synchronize() == 0
    got = {i: f.cpu().numpy() for i, f in frames.items()}
    final = ctx.readout_host(0)
    orc = oracle.Oracle(W, H)
    r = 0
    for it in sched:
        if it[0] == "push":
            assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
            continue
        if r in got:
            ref = orc.readout(0)["L"]
            d = np.abs(got[r].astype(np.float64) - ref)
            assert np.all(d <= REL * np.maximum(np.abs(ref), 1.0)), \
                "frame %d: worst %.3g" % (r, d.max())
        r += 1
    compare_state(final, orc.readout(0), True, "end of the benchmark stream")
    compare_stats(ctx.stats(), orc.stats())
    flush("hd720 benchmark stream: %d sampled frames and the final state match" % len(got))
    ctx.close()


def test_empty_push_and_repeated_readout_change_nothing():
    w = eventsim.preset("sensor64x48", n_events=30000)
    ev = eventsim.generate(w.scene)
    ctx = make_ctx(64, 48)
    gx, gy, gp = to_device(ev)
    for a in range(0, len(ev), 1024):
        assert ctx.push(gx[a:a + 1024], gy[a:a + 1024], gp[a:a + 1024]) == 0
    r1 = ctx.readout_host(0)
    s1 = ctx.stats()
    assert ctx.push(gx[:0], gy[:0], gp[:0]) == 0
    r2 = ctx.readout_host(0)
    assert ctx.stats() == s1
    for key in r1:
        assert np.array_equal(r1[key], r2[key])
    ctx.close()


def test_device_packet_rejection_changes_nothing():
    torch, dev = torch_dev()
    w = eventsim.preset("sensor64x48", n_events=20000)
    ev = eventsim.generate(w.scene)
    ctx = make_ctx(64, 48)
    orc = oracle.Oracle(64, 48)
    gx, gy, gp = to_device(ev)
    assert ctx.push(gx[:5000], gy[:5000], gp[:5000]) == 0
    orc.push(ev.x[:5000], ev.y[:5000], ev.p[:5000])
    before = ctx.readout_host(0)
    bx = gx[5000:6000].clone()
    bx[17] = 64                       # x == width
    assert ctx.push(bx, gy[5000:6000], gp[5000:6000]) == 0   # checked on the device
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    assert ctx.synchronize() == 0     # reported once
    bp = gp[5000:6000].clone()
    bp[3] = 2
    assert ctx.push(gx[5000:6000], gy[5000:6000], bp) == 0
    assert ctx.synchronize() == fb.FIBAR_E_POLARITY
    after = ctx.readout_host(0)
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    # the stream continues normally
    assert ctx.push(gx[5000:], gy[5000:], gp[5000:]) == 0
    orc.push(ev.x[5000:], ev.y[5000:], ev.p[5000:])
    compare_state(ctx.readout_host(0), orc.readout(0), True, "after rejection")
    compare_stats(ctx.stats(), orc.stats())
    ctx.close()


def test_host_packets_and_errors():
    w = eventsim.preset("sensor64x48", n_events=20000)
    ev = eventsim.generate(w.scene)
    ctx = make_ctx(64, 48)
    orc = oracle.Oracle(64, 48)
    for a in range(0, len(ev), 3000):
        sl = slice(a, a + 3000)
        assert ctx.push(ev.x[sl], ev.y[sl], ev.p[sl], ev.t[sl]) == 0
        orc.push(ev.x[sl], ev.y[sl], ev.p[sl], ev.t[sl])
    x = ev.x[:10].copy()
    x[2] = 999
    assert ctx.push(x, ev.y[:10], ev.p[:10]) == fb.FIBAR_E_RANGE
    p = ev.p[:10].copy()
    p[0] = 7
    assert ctx.push(ev.x[:10], ev.y[:10], p) == fb.FIBAR_E_POLARITY
    assert ctx.readout_host(int(ev.t[-1]) - 1) == fb.FIBAR_E_TIME
    compare_state(ctx.readout_host(int(ev.t[-1])), orc.readout(int(ev.t[-1])), True)
    big = np.zeros(70000, np.uint16)
    assert ctx.push(big, big, big.astype(np.uint8)) == fb.FIBAR_E_INVALID_ARG
    ctx.close()


def test_submit_equals_single_calls_and_device_readouts():
    torch, dev = torch_dev()
    w = eventsim.preset("vga", n_events=600000, seed=4)
    ev = eventsim.generate(w.scene)
    gx, gy, gp = to_device(ev)
    ro = [100000, 250001, 400000, 600000]
    sched = eventsim.schedule(len(ev), w.packet, ro)
    # one call per op
    c1 = make_ctx(640, 480)
    res1 = []
    for it in sched:
        if it[0] == "push":
            assert c1.push(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]) == 0
        else:
            res1.append(c1.readout_host(0))
    # one submit of the whole schedule, readouts into device buffers
    c2 = make_ctx(640, 480)
    npx = 640 * 480
    bufs = []
    ops = []
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            b = dict(L=torch.empty(npx, dtype=torch.float32, device=dev),
                     stale=torch.empty(npx, dtype=torch.uint8, device=dev),
                     cnt=torch.empty(npx, dtype=torch.int32, device=dev),
                     last=torch.empty(npx, dtype=torch.int64, device=dev),
                     log_age=torch.empty(npx, dtype=torch.float32, device=dev))
            bufs.append(b)
            ops.append(fb.readout_op(0, b["L"], stale=b["stale"], cnt=b["cnt"], last=b["last"],
                                     log_age=b["log_age"]))
    assert c2.submit(ops) == 0
    torch.cuda.synchronize()
    for r, b in zip(res1, bufs):
        assert np.array_equal(r["L"], b["L"].cpu().numpy())
        assert np.array_equal(r["stale"], b["stale"].cpu().numpy())
        assert np.array_equal(r["cnt"].view(np.int32), b["cnt"].cpu().numpy())
        assert np.array_equal(r["last"], b["last"].cpu().numpy())
        assert np.array_equal(r["log_age"], b["log_age"].cpu().numpy())
    # log age definition
    k = len(ev) - 1
    last = bufs[-1]["last"].cpu().numpy()
    want = np.log1p((k - last).astype(np.float64))
    assert np.allclose(bufs[-1]["log_age"].cpu().numpy(), want, rtol=1e-6, atol=1e-6)
    c1.close()
    c2.close()


def test_readouts_taken_by_the_pop_launch():
    """Blur on: a device readout right after a push, without the window count,
    is written by the pop launch of that push (its own workgroups compute the
    blurred value of pixels going stale in the step).  It must equal a
    separate readout bit for bit and match the oracle; a second readout right
    after the first takes the separate kernel."""
    torch, dev = torch_dev()
    W, H = 640, 480
    npx, ntiles = W * H, ((W + 1) // 2) * ((H + 1) // 2)
    w = eventsim.preset("vga", n_events=400_000, seed=11)
    ev = eventsim.generate(w.scene)
    gx, gy, gp = to_device(ev)
    ro = [1, 4096, 50_001, 123_456, 250_000, 400_000]
    sched = eventsim.schedule(len(ev), w.packet, ro)
    # per-call pushes and host readouts (the separate readout kernel)
    c1 = make_ctx(W, H)
    ref = []
    for it in sched:
        if it[0] == "push":
            assert c1.push(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]) == 0
        else:
            ref.append((it[1], c1.readout_host(0)))
    # one submit; every readout doubled: the first of a pair is fused
    c2 = make_ctx(W, H)
    ops, bufs = [], []
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
            continue
        for _ in range(2):
            b = dict(L=torch.empty(npx, dtype=torch.float32, device=dev),
                     pbar=torch.empty(npx, dtype=torch.float32, device=dev),
                     stale=torch.empty(npx, dtype=torch.uint8, device=dev),
                     last=torch.empty(npx, dtype=torch.int64, device=dev),
                     log_age=torch.empty(npx, dtype=torch.float32, device=dev),
                     tcnt=torch.empty(ntiles, dtype=torch.int32, device=dev))
            bufs.append(b)
            ops.append(fb.readout_op(0, b["L"], pbar=b["pbar"], stale=b["stale"], last=b["last"],
                                     log_age=b["log_age"], tcnt=b["tcnt"]))
    assert c2.submit(ops) == 0
    torch.cuda.synchronize()
    assert len(bufs) == 2 * len(ref)
    orc = oracle.Oracle(W, H)
    n = 0
    for it in sched:
        if it[0] == "push":
            assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
            continue
        k, r = ref[n]
        for b in bufs[2 * n:2 * n + 2]:
            g = {key: v.cpu().numpy() for key, v in b.items()}
            for key in ("L", "pbar", "stale", "last", "log_age"):
                assert np.array_equal(g[key], r[key]), "%s at %d" % (key, k)
            assert np.array_equal(g["tcnt"].view(np.uint32), r["tcnt"]), "tcnt at %d" % k
        o = orc.readout(0)
        compare_state(r, o, True, "readout at %d" % k)
        assert np.array_equal(g["stale"], o["stale"]) and np.array_equal(g["last"], o["last"])
        n += 1
    assert c2.stats()["k"] == len(ev) - 1
    c1.close()
    c2.close()


def test_pop_launch_readouts_after_rejected_and_multi_chunk_packets():
    """Readouts written by the pop launch after (i) a packet of several
    chunks (its pops take pixels from the ring), (ii) a rejected packet (it
    pops nothing and must leave the readout equal to the one before)."""
    torch, dev = torch_dev()
    W, H = 640, 480
    npx, ntiles = W * H, (W // 2) * (H // 2)
    w = eventsim.preset("vga", n_events=120_000, seed=13)
    ev = eventsim.generate(w.scene)
    gx, gy, gp = to_device(ev)
    bad = gx[100_000:101_000].clone()
    bad[5] = W                              # x == width: the packet is rejected
    ctx = make_ctx(W, H)
    ops, bufs = [], []

    def readout():
        b = dict(L=torch.empty(npx, dtype=torch.float32, device=dev),
                 pbar=torch.empty(npx, dtype=torch.float32, device=dev),
                 stale=torch.empty(npx, dtype=torch.uint8, device=dev),
                 last=torch.empty(npx, dtype=torch.int64, device=dev),
                 tcnt=torch.empty(ntiles, dtype=torch.int32, device=dev))
        bufs.append(b)
        ops.append(fb.readout_op(0, b["L"], pbar=b["pbar"], stale=b["stale"], last=b["last"],
                                 tcnt=b["tcnt"]))

    ops.append(fb.push_op(gx[:50_000], gy[:50_000], gp[:50_000]))        # four chunks
    readout()
    ops.append(fb.push_op(gx[50_000:100_000], gy[50_000:100_000], gp[50_000:100_000]))
    readout()
    ops.append(fb.push_op(bad, gy[100_000:101_000], gp[100_000:101_000]))
    readout()
    ops.append(fb.push_op(gx[100_000:], gy[100_000:], gp[100_000:]))
    readout()
    assert ctx.submit(ops) == 0
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    g = [{k: v.cpu().numpy() for k, v in b.items()} for b in bufs]
    for key in g[1]:
        assert np.array_equal(g[1][key], g[2][key]), "rejected packet changed " + key
    orc = oracle.Oracle(W, H)
    want = []
    for a, b in ((0, 50_000), (50_000, 100_000), (100_000, len(ev))):
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        want.append(orc.readout(0))
    for gi, r in zip((g[0], g[1], g[3]), want):
        assert np.array_equal(gi["last"], r["last"])
        assert np.array_equal(gi["stale"], r["stale"])
        assert np.array_equal(gi["tcnt"].view(np.uint32), r["tcnt"])
        for key in ("L", "pbar"):
            d = np.abs(gi[key].astype(np.float64) - r[key])
            assert np.all(d <= REL * np.maximum(np.abs(r[key]), 1.0)), key
    ctx.close()


@pytest.mark.parametrize("W,H", [(346, 260), (3, 3), (5, 4), (17, 9)])
def test_pop_launch_readouts_on_ragged_pixel_counts(W, H):
    """Readouts written by the pop launch when the pixel count is not a
    multiple of its 128-thread workgroups (346 x 260, 17 x 9) or is below
    one workgroup (3 x 3, 5 x 4), with a small target length so that pixels
    go stale in most steps: every output equals the separate readout kernel
    of the same state (a readout following another readout) bit for bit."""
    torch, dev = torch_dev()
    npx, ntiles = W * H, ((W + 1) // 2) * ((H + 1) // 2)
    rng = np.random.default_rng(W * 1000 + H)
    n = 40_000
    pix = np.empty(n, np.int64)
    cur = 0
    for e in range(n):
        if rng.random() < 0.3:
            cur = int(rng.integers(0, npx))
        pix[e] = cur
    ev = eventsim.Events((pix % W).astype(np.uint16), (pix // W).astype(np.uint16),
                         (rng.random(n) < 0.5).astype(np.uint8), np.arange(n, dtype=np.uint64))
    gx, gy, gp = to_device(ev)
    ctx = make_ctx(W, H, q_min=1, q_max=max(64, npx // 2))
    ops, bufs, packets = [], [], []
    a = 0
    flush("pop-launch readouts %dx%d" % (W, H))
    while a < n:
        b = min(n, a + int(rng.integers(1, 3000)))
        packets.append((a, b))
        ops.append(fb.push_op(gx[a:b], gy[a:b], gp[a:b]))
        for _ in range(2):   # the first is taken by the pop launch, the second is separate
            d = dict(L=torch.empty(npx, dtype=torch.float32, device=dev),
                     pbar=torch.empty(npx, dtype=torch.float32, device=dev),
                     stale=torch.empty(npx, dtype=torch.uint8, device=dev),
                     last=torch.empty(npx, dtype=torch.int64, device=dev),
                     log_age=torch.empty(npx, dtype=torch.float32, device=dev),
                     tcnt=torch.empty(ntiles, dtype=torch.int32, device=dev))
            bufs.append(d)
            ops.append(fb.readout_op(int(ev.t[b - 1]), d["L"], pbar=d["pbar"], stale=d["stale"],
                                     last=d["last"], log_age=d["log_age"], tcnt=d["tcnt"]))
        a = b
    assert ctx.submit(ops) == 0
    torch.cuda.synchronize()
    assert ctx.stats()["total_stale"] > 0
    for j in range(0, len(bufs), 2):
        f = {k: v.cpu().numpy() for k, v in bufs[j].items()}
        r = {k: v.cpu().numpy() for k, v in bufs[j + 1].items()}
        for key in f:
            assert np.array_equal(f[key].view(np.uint8), r[key].view(np.uint8)), \
                "%s after push %d" % (key, j // 2)
    orc = oracle.Oracle(W, H, q_min=1, q_max=max(64, npx // 2))
    for a, b in packets:   # the target is regulated once per packet
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
    o = orc.readout(0)
    g = {k: v.cpu().numpy() for k, v in bufs[-1].items()}
    assert np.array_equal(g["last"], o["last"]) and np.array_equal(g["stale"], o["stale"])
    assert np.array_equal(g["tcnt"].view(np.uint32), o["tcnt"])
    d = np.abs(g["L"].astype(np.float64) - o["L"])
    assert np.all(d <= REL * np.maximum(np.abs(o["L"]), 1.0))
    ctx.close()


def test_nsf_rejects_spatial_outputs():
    ctx = make_ctx(32, 16, spatial_filter=False, q_min=1)
    npx = 32 * 16
    L = np.empty(npx, np.float32)
    st = np.empty(npx, np.uint8)
    buf = fb.fibar_readout_buf(L.ctypes.data, None, st.ctypes.data, None, None, None, None, None,
                               0)
    assert fb.fibar_readout(ctx.handle, 0, buf) == fb.FIBAR_E_UNSUPPORTED
    ctx.close()


def _submit_with_device_readouts(ctx, ev, sched, gx, gy, gp, npx, with_extras=True):
    torch, dev = torch_dev()
    ops, bufs = [], []
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
        else:
            b = dict(k=it[1], L=torch.empty(npx, dtype=torch.float32, device=dev))
            if with_extras:
                b.update(pbar=torch.empty(npx, dtype=torch.float32, device=dev),
                         last=torch.empty(npx, dtype=torch.int64, device=dev),
                         log_age=torch.empty(npx, dtype=torch.float32, device=dev))
            bufs.append(b)
            ops.append(fb.readout_op(0, b["L"], pbar=b.get("pbar"), last=b.get("last"),
                                     log_age=b.get("log_age")))
    assert ctx.submit(ops) == 0
    torch.cuda.synchronize()
    return bufs


def test_nsf_batched_readouts_match_oracle():
    """Blur off: one submit of pushes and device readouts (the batched path
    writes every readout when its events are applied) against the oracle."""
    w = eventsim.preset("vga", n_events=900_000, seed=8)
    ev = eventsim.generate(w.scene)
    ro = [1, 8191, 8192, 100_000, 123_457, 500_000, 900_000]
    sched = eventsim.schedule(len(ev), w.packet, ro)
    gx, gy, gp = to_device(ev)
    ctx = make_ctx(640, 480, spatial_filter=False)
    bufs = _submit_with_device_readouts(ctx, ev, sched, gx, gy, gp, 640 * 480)
    orc = oracle.Oracle(640, 480, spatial_filter=False)
    done = 0
    for b in bufs:
        k = b["k"]
        orc.push(ev.x[done:k], ev.y[done:k], ev.p[done:k])
        done = k
        r = orc.readout(0)
        g = {"L": b["L"].cpu().numpy(), "pbar": b["pbar"].cpu().numpy(),
             "last": b["last"].cpu().numpy()}
        compare_state(g, r, False, "readout at %d" % k)
        want = np.log1p((k - 1 - r["last"]).astype(np.float64))
        assert np.allclose(b["log_age"].cpu().numpy(), want, rtol=1e-6, atol=1e-6)
    assert ctx.stats()["k"] == len(ev) - 1
    ctx.close()


def _hot_pixel_stream(W, H, n, share, seed):
    """Uniform events with random polarity, of which about `share` go to one
    pixel: the blur-off counting sorts then hold buckets of thousands of one
    key's events, and an event out of time order would change that pixel's
    brightness and last index."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, W, n).astype(np.uint16)
    y = rng.integers(0, H, n).astype(np.uint16)
    hot = rng.random(n) < share
    x[hot] = W // 3
    y[hot] = (2 * H) // 3
    p = rng.integers(0, 2, n).astype(np.uint8)
    return eventsim.Events(x, y, p, np.arange(n, dtype=np.uint64))


@pytest.mark.parametrize("W,H,n,extras", [(64, 48, 600_000, False), (64, 48, 600_000, True),
                                          (1280, 1024, 400_000, False)])
def test_nsf_hot_pixel_batched(W, H, n, extras):
    """Blur off, one submit of 16384-event packets and device readouts, half of
    the events on one pixel; 1280x1024 has 1280 regions, beyond the scatter's
    counting sort (its radix sort runs).  Brightness-only readouts and readouts
    with every output take the two variants of the apply kernel."""
    ev = _hot_pixel_stream(W, H, n, 0.5, seed=W + n)
    sched = eventsim.schedule(n, 16384, [50_000, 333_333, n])
    gx, gy, gp = to_device(ev)
    flush("blur off, hot pixel, %dx%d, %d events, extras=%s" % (W, H, n, extras))
    ctx = make_ctx(W, H, spatial_filter=False)
    bufs = _submit_with_device_readouts(ctx, ev, sched, gx, gy, gp, W * H, with_extras=extras)
    orc = oracle.Oracle(W, H, spatial_filter=False)
    done = 0
    for b in bufs:
        k = b["k"]
        orc.push(ev.x[done:k], ev.y[done:k], ev.p[done:k])
        done = k
        r = orc.readout(0)
        if extras:
            g = {"L": b["L"].cpu().numpy(), "pbar": b["pbar"].cpu().numpy(),
                 "last": b["last"].cpu().numpy()}
            compare_state(g, r, False, "readout at %d" % k)
        else:
            d = np.abs(b["L"].cpu().numpy().astype(np.float64) - r["L"])
            assert d.max() <= REL * max(np.abs(r["L"]).max(), 1.0), "L at %d" % k
    compare_state(ctx.readout_host(0), orc.readout(0), False, "final")
    ctx.close()
    orc.close()


def test_nsf_many_batches_and_host_readouts():
    """More events than one batch holds, host readouts in between."""
    w = eventsim.preset("hd720", n_events=9_000_000, seed=5)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, [4_200_000, 8_999_999])
    flush("hd720 9M events blur off, host readouts")
    run_pair(ev, 1280, 720, sched, spatial_filter=False)


def test_nsf_back_to_back_submits_reuse_the_descriptor_buffer():
    """Blur off, ~40 submits in a row with no wait between them.  Each submit
    is one batch whose chunk and readout descriptors the host writes into the
    one host buffer that the batch's first kernel reads in place, so the host
    has to wait until the batch before has read it; every fifth submit is a
    readout alone (its descriptors go by copy instead).  Every readout must see
    exactly the events submitted before it."""
    W, H = 640, 480
    w = eventsim.preset("vga", n_events=600_000, seed=21)
    ev = eventsim.generate(w.scene)
    n = len(ev)
    gx, gy, gp = to_device(ev)
    torch, dev = torch_dev()
    rng = np.random.default_rng(3)
    flush("blur off, back-to-back submits, 640x480, %d events" % n)
    ctx = make_ctx(W, H, spatial_filter=False)
    bufs, k, sub = [], 0, 0

    def readout(ops):
        b = dict(k=k, L=torch.empty(W * H, dtype=torch.float32, device=dev))
        bufs.append(b)
        ops.append(fb.readout_op(0, b["L"]))

    while k < n:
        ops = []
        if sub % 5 == 4:
            readout(ops)
        else:
            for _ in range(int(rng.integers(1, 4))):
                m = int(min(n - k, rng.integers(1, 16385)))
                ops.append(fb.push_op(gx[k:k + m], gy[k:k + m], gp[k:k + m]))
                k += m
                if rng.random() < 0.5 or k == n:
                    readout(ops)
                if k == n:
                    break
        assert ctx.submit(ops) == 0
        sub += 1
    torch.cuda.synchronize()
    assert sub >= 30 and len(bufs) >= 30
    orc = oracle.Oracle(W, H, spatial_filter=False)
    done = 0
    for b in bufs:
        orc.push(ev.x[done:b["k"]], ev.y[done:b["k"]], ev.p[done:b["k"]])
        done = b["k"]
        r = orc.readout(0)
        d = np.abs(b["L"].cpu().numpy().astype(np.float64) - r["L"])
        assert d.max() <= REL * max(np.abs(r["L"]).max(), 1.0), "L at %d" % b["k"]
    compare_state(ctx.readout_host(0), orc.readout(0), False, "final")
    ctx.close()
    orc.close()


def test_nsf_device_packet_rejection():
    w = eventsim.preset("sensor64x48", n_events=20000)
    ev = eventsim.generate(w.scene)
    ctx = make_ctx(64, 48, spatial_filter=False)
    orc = oracle.Oracle(64, 48, spatial_filter=False)
    gx, gy, gp = to_device(ev)
    bx = gx[5000:6000].clone()
    bx[999] = 100
    ops = [fb.push_op(gx[:5000], gy[:5000], gp[:5000]),
           fb.push_op(bx, gy[5000:6000], gp[5000:6000]),
           fb.push_op(gx[6000:], gy[6000:], gp[6000:])]
    assert ctx.submit(ops) == 0
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    orc.push(ev.x[:5000], ev.y[:5000], ev.p[:5000])
    orc.push(ev.x[6000:], ev.y[6000:], ev.p[6000:])
    compare_state(ctx.readout_host(0), orc.readout(0), False, "after rejected packet")
    assert ctx.stats()["k"] == len(ev) - 1000 - 1
    ctx.close()


def test_telemetry_skips_rejected_and_empty_pushes():
    # one record per regulation step: a rejected device packet and an empty
    # push make no step, and records past the buffer are not written
    from _harness import compare_telemetry, oracle_step_record, telemetry_buffer
    w = eventsim.preset("sensor64x48", n_events=30000, seed=5)
    ev = eventsim.generate(w.scene)
    ctx = make_ctx(64, 48, q_min=16)
    orc = oracle.Oracle(64, 48, q_min=16)
    gx, gy, gp = to_device(ev)
    cap = 20
    tel = telemetry_buffer(ctx, cap)
    want = []
    bounds = list(range(0, len(ev), 1500)) + [len(ev)]
    for i, (a, b) in enumerate(zip(bounds[:-1], bounds[1:])):
        if i == 3:
            bx = gx[a:b].clone()
            bx[5] = 64                       # rejected on the device
            assert ctx.push(bx, gy[a:b], gp[a:b]) == 0
        if i == 5:
            assert ctx.push(gx[a:a], gy[a:a], gp[a:a]) == 0   # empty: no step
        assert ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        want.append(oracle_step_record(orc.stats(), b - a))
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    assert len(want) == 20 == cap
    compare_telemetry(tel, want, "with a rejected and an empty push")
    compare_stats(ctx.stats(), orc.stats(), "after telemetry")
    compare_state(ctx.readout_host(0), orc.readout(0), True, "after telemetry")
    ctx.close()


def test_total_count_blur_off_region_path():
    # the blur-off batch path keeps the per-pixel event total too
    w = eventsim.preset("vga", n_events=400000, seed=9)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, [150000, 400000])
    g, r = run_pair(ev, 640, 480, sched, spatial_filter=False)
    assert np.array_equal(g["tot"], r["tot"])
    assert int(g["tot"].sum()) == len(ev)


def test_host_packets_through_the_pinned_ring():
    """Host packets are copied into a pinned ring and on to the device without
    waiting for the stream; the ring (4M events) wraps here.  The result is
    bit-identical to the same packets given as device arrays, with host
    readouts and device packets interleaved."""
    torch, dev = torch_dev()
    W, H = 346, 260
    sc = eventsim.Scene(W, H, 5_000_000, 71, n_blobs=150, checker_cell=16.0,
                        checker_contrast=0.5, speed_px_s=200.0, noise_frac=0.01)
    ev = eventsim.generate(sc)
    n = len(ev)
    gx, gy, gp = to_device(ev)
    flush("346x260, %d events, host packets through the pinned ring" % n)
    a_ctx = make_ctx(W, H, max_packet=131072)
    b_ctx = make_ctx(W, H, max_packet=131072)
    sizes = [100_000, 3, 77_777, 131_072, 12_345]
    a, r, reads = 0, 0, []
    while a < n:
        b = min(n, a + sizes[r % len(sizes)])
        if r % 7 == 3:   # a device packet among the host ones
            assert a_ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
        else:
            assert a_ctx.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        assert b_ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
        if r % 11 == 10:
            reads.append((a_ctx.readout_host(0), b_ctx.readout_host(0)))
        a, r = b, r + 1
    reads.append((a_ctx.readout_host(0), b_ctx.readout_host(0)))
    for ga, gb in reads:
        for key in ga:
            assert np.array_equal(ga[key], gb[key]), key
    assert a_ctx.stats() == b_ctx.stats()
    orc = oracle.Oracle(W, H)
    a, r = 0, 0
    while a < n:
        b = min(n, a + sizes[r % len(sizes)])
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        a, r = b, r + 1
    compare_state(reads[-1][0], orc.readout(0), True, "after the host packets")
    a_ctx.close()
    b_ctx.close()
