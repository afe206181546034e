"""GPU: per-event regulation (FIBAR_REG_EVENT, the paper's literal
procedure; Method, "Spatial filtering", steps 1-3 with Eq. (20) after every
event) against the FP64 oracle's per-event mode: integer state and window
scalars bit for bit, brightness within the FP32 tolerance."""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import compare_state, compare_stats, make_ctx, run_pair, to_device

pytestmark = pytest.mark.gpu


def flush(msg):
    print(msg, flush=True)


def test_sensor64x48_full_stream_event_regulation():
    """The 64x48 configuration whole: 200 000 events in 1024-event packets,
    a readout every 10 000 events, each compared with the oracle."""
    w = eventsim.preset("sensor64x48")
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    flush("64x48, %d events, per-event regulation" % len(ev))
    run_pair(ev, 64, 48, sched, telemetry=False, regulation="event")


def random_stream(W, H, n, seed, cluster=0.3):
    """Pixels that repeat in runs, so that pixels go active and stale often."""
    rng = np.random.default_rng(seed)
    pix = np.empty(n, np.int64)
    cur = 0
    for e in range(n):
        if rng.random() < cluster:
            cur = int(rng.integers(0, W * H))
        pix[e] = cur
    x = (pix % W).astype(np.uint16)
    y = (pix // W).astype(np.uint16)
    p = rng.integers(0, 2, n).astype(np.uint8)
    return x, y, p


class Ev:
    def __init__(self, x, y, p):
        self.x, self.y, self.p = x, y, p
        self.t = np.arange(1, len(x) + 1, dtype=np.uint64)

    def __len__(self):
        return len(self.x)


@pytest.mark.parametrize("W,H,q_min,q_max", [(1, 1, 1, 0), (3, 2, 1, 0), (5, 7, 2, 9),
                                             (33, 17, 4, 0), (64, 48, 64, 200)])
def test_small_sensors_against_oracle(W, H, q_min, q_max):
    n = 20000
    x, y, p = random_stream(W, H, n, seed=W * 100 + H)
    ev = Ev(x, y, p)
    sizes = [1, 2, 3, 50, 1000, 333]
    sched, a, r = [], 0, 0
    while a < n:
        b = min(n, a + sizes[r % len(sizes)])
        sched.append(("push", a, b))
        if r % 5 == 4:
            sched.append(("read", b))
        a, r = b, r + 1
    flush("%dx%d, q_min %d, q_max %d, per-event regulation" % (W, H, q_min, q_max))
    run_pair(ev, W, H, sched, telemetry=False, regulation="event", q_min=q_min, q_max=q_max)


def test_result_does_not_depend_on_packet_sizes():
    """Per-event regulation makes the packet boundaries irrelevant: the same
    events in packets of 1, 7, 1000 and all at once give identical state."""
    W, H = 64, 48
    w = eventsim.preset("sensor64x48", n_events=4000)
    ev = eventsim.generate(w.scene)
    gx, gy, gp = to_device(ev)
    outs = []
    for size in (1, 7, 1000, len(ev)):
        ctx = make_ctx(W, H, regulation="event")
        for a in range(0, len(ev), size):
            assert ctx.push(gx[a:a + size], gy[a:a + size], gp[a:a + size]) == 0
        outs.append((ctx.readout_host(0), ctx.stats()))
        ctx.close()
    for g, st in outs[1:]:
        assert st == outs[0][1]
        for key in g:
            assert np.array_equal(g[key], outs[0][0][key]), key
    orc = oracle.Oracle(W, H, regulation="event")
    assert orc.push(ev.x, ev.y, ev.p) == 0
    compare_state(outs[0][0], orc.readout(0), True, "per-event regulation")
    compare_stats(outs[0][1], orc.stats(), "per-event regulation")


def test_largest_sensor_and_window():
    """128 x 64 pixels (the limit) with the default window limit of one
    event per pixel: the state needs more than 64 KiB of LDS."""
    W, H = 128, 64
    x, y, p = random_stream(W, H, 60000, seed=5, cluster=0.05)
    ev = Ev(x, y, p)
    sched = [("push", a, min(a + 4096, 60000)) for a in range(0, 60000, 4096)]
    sched.insert(5, ("read", sched[4][2]))
    flush("128x64, per-event regulation")
    run_pair(ev, W, H, sched, telemetry=False, regulation="event", q_min=16)


def test_rejected_packet_changes_nothing():
    torch, dev = __import__("_harness").torch_dev()
    W, H = 16, 12
    x, y, p = random_stream(W, H, 3000, seed=3)
    gx, gy, gp = to_device(Ev(x, y, p))
    ctx = make_ctx(W, H, regulation="event", q_min=4)
    assert ctx.push(gx[:2000], gy[:2000], gp[:2000]) == 0
    before, st = ctx.readout_host(0), ctx.stats()
    bad_x = gx[2000:].clone()
    bad_x[17] = W
    assert ctx.push(bad_x, gy[2000:], gp[2000:]) == 0
    assert ctx.synchronize() == fb.FIBAR_E_RANGE
    bad_p = gp[2000:].clone()
    bad_p[3] = 2
    assert ctx.push(gx[2000:], gy[2000:], bad_p) == 0
    assert ctx.synchronize() == fb.FIBAR_E_POLARITY
    after = ctx.readout_host(0)
    assert ctx.stats() == st
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    # and the stream goes on as if the bad packets had never come
    assert ctx.push(gx[2000:], gy[2000:], gp[2000:]) == 0
    orc = oracle.Oracle(W, H, regulation="event", q_min=4)
    assert orc.push(x, y, p) == 0
    compare_state(ctx.readout_host(0), orc.readout(0), True, "after rejected packets")
    ctx.close()


def test_event_contexts_refuse_telemetry_and_groups():
    ctx = make_ctx(64, 48, regulation="event")
    torch, dev = __import__("_harness").torch_dev()
    buf = torch.zeros((4, fb.STEP_RECORD_WORDS), dtype=torch.int64, device=dev)
    assert ctx.set_telemetry(buf, 4) == fb.FIBAR_E_UNSUPPORTED
    rc, _ = fb.fibar_multi_create([ctx.handle])
    assert rc == fb.FIBAR_E_UNSUPPORTED
    ctx.close()
