"""GPU: per-tile event queues (the paper's Limitations: event queues operated
separately for each tile of the image; params.region, params.age_max)
against the FP64 oracle's per-tile queues: every tile's window, counts and
target, the integer state bit for bit and brightness within the FP32
tolerance."""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import compare_state, compare_stats, compare_tiles, make_ctx, run_pair, to_device

pytestmark = pytest.mark.gpu


def flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("R", [16, 8, 32])
def test_sensor64x48_stream_with_tiles(R):
    w = eventsim.preset("sensor64x48")
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    flush("64x48, %d events, tiles of %d" % (len(ev), R))
    run_pair(ev, 64, 48, sched, telemetry=False, region=R, q_min=16)


def test_short_age_limit_and_cut_tiles():
    """Tiles cut by the image (70 x 50 in tiles of 16) and an age limit short
    enough that tiles empty out between their events."""
    W, H = 70, 50
    sc = eventsim.Scene(W, H, 120_000, 61, n_blobs=32, speed_px_s=40.0, noise_frac=0.01)
    ev = eventsim.generate(sc)
    ro = list(range(7000, len(ev), 13000))
    sched = eventsim.schedule(len(ev), 1500, ro)
    flush("70x50, tiles of 16, age limit 3000")
    run_pair(ev, W, H, sched, telemetry=False, region=16, q_min=8, age_max=3000)


def test_vga_packets_of_several_chunks_with_tiles():
    """640x480 in tiles of 32, packets from 1 to 40000 events (several
    16384-event chunks), readouts in between."""
    w = eventsim.preset("vga", n_events=1_200_000, seed=23)
    ev = eventsim.generate(w.scene)
    n = len(ev)
    sizes = [40000, 1, 7, 16384, 16385, 3000, 32768]
    sched, a, r = [], 0, 0
    while a < n:
        b = min(n, a + sizes[r % len(sizes)])
        sched.append(("push", a, b))
        if r % 6 == 5:
            sched.append(("read", b))
        a, r = b, r + 1
    flush("640x480, tiles of 32, %d pushes" % sum(1 for it in sched if it[0] == "push"))
    run_pair(ev, 640, 480, sched, telemetry=False, region=32)


@pytest.mark.parametrize("R", [8, 32])
def test_hot_tile_with_thousands_of_events_per_packet(R):
    """About half of every 8192-event packet on one pixel, random polarity:
    its tile takes ~4000 of a packet's events (the step kernel's pieces of 512
    events) and, with a window of at most R^2 events, pops nearly all of them
    in the same step (entries past those the kernel keeps in LDS are read back
    from the ring)."""
    W, H, n = 64, 48, 300_000
    rng = np.random.default_rng(31 + R)
    x = rng.integers(0, W, n).astype(np.uint16)
    y = rng.integers(0, H, n).astype(np.uint16)
    hot = rng.random(n) < 0.5
    x[hot] = 20
    y[hot] = 13
    p = rng.integers(0, 2, n).astype(np.uint8)
    ev = eventsim.Events(x, y, p, np.arange(n, dtype=np.uint64))
    sched = eventsim.schedule(n, 8192, list(range(20_000, n, 40_000)) + [n])
    flush("64x48, hot tile, tiles of %d" % R)
    run_pair(ev, W, H, sched, telemetry=False, region=R, q_min=16)


def test_rejected_packet_changes_nothing_with_tiles():
    W, H = 64, 48
    w = eventsim.preset("sensor64x48", n_events=30000)
    ev = eventsim.generate(w.scene)
    gx, gy, gp = to_device(ev)
    ctx = make_ctx(W, H, region=16, q_min=16)
    assert ctx.push(gx[:20000], gy[:20000], gp[:20000]) == 0
    before, st, tiles = ctx.readout_host(0), ctx.stats(), ctx.tile_stats()
    bad = gx[20000:].clone()
    bad[5] = W
    assert ctx.push(bad, gy[20000:], gp[20000:]) == 0
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    after = ctx.readout_host(0)
    assert ctx.stats() == st
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    for key, v in ctx.tile_stats().items():
        assert np.array_equal(v, tiles[key]), key
    assert ctx.push(gx[20000:], gy[20000:], gp[20000:]) == 0
    orc = oracle.Oracle(W, H, region=16, q_min=16)
    assert orc.push(ev.x[:20000], ev.y[:20000], ev.p[:20000]) == 0
    assert orc.push(ev.x[20000:], ev.y[20000:], ev.p[20000:]) == 0
    compare_state(ctx.readout_host(0), orc.readout(0), True, "after a rejected packet")
    compare_stats(ctx.stats(), orc.stats())
    compare_tiles(ctx, orc)
    ctx.close()


def test_tile_contexts_refuse_telemetry_and_groups():
    torch, dev = __import__("_harness").torch_dev()
    ctx = make_ctx(64, 48, region=16)
    buf = torch.zeros((4, fb.STEP_RECORD_WORDS), dtype=torch.int64, device=dev)
    assert ctx.set_telemetry(buf, 4) == fb.FIBAR_E_UNSUPPORTED
    assert fb.fibar_multi_create([ctx.handle])[0] == fb.FIBAR_E_UNSUPPORTED
    ctx.close()
    one = make_ctx(64, 48)
    assert fb.fibar_tile_stats(one.handle, 12)[0] == fb.FIBAR_E_UNSUPPORTED
    one.close()
