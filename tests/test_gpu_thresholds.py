"""GPU: relative contrast thresholds (Experiments, "Inter-pixel threshold
variation"; threshold appendix, Eq. (21)-(30)): per-pixel event counts and
relative thresholds of a calibration recording against the oracle's, and
reconstructions with the per-pixel multiplier of Eq. (6) on every path
against the oracle with the same multipliers."""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import compare_state, compare_stats, make_ctx, run_pair, to_device, torch_dev

pytestmark = pytest.mark.gpu


def calibration(W, H, seed=7, periods=5, amplitude=40.0):
    con, coff = eventsim.pixel_thresholds(W, H, seed)
    return eventsim.calibration_stream(W, H, con, coff, periods=periods, amplitude=amplitude)


def device_thresholds(ev, W, H, splits=3):
    torch, dev = torch_dev()
    gx, gy, gp = to_device(ev)
    n_on = torch.zeros(W * H, dtype=torch.int32, device=dev)
    n_off = torch.zeros(W * H, dtype=torch.int32, device=dev)
    n = len(ev)
    cuts = [n * k // splits for k in range(splits + 1)]
    for a, b in zip(cuts[:-1], cuts[1:]):
        assert fb.fibar_count_polarities(gx[a:b], gy[a:b], gp[a:b], W, H, n_on, n_off) == 0
    c = torch.empty(W * H, dtype=torch.float32, device=dev)
    c_on, c_off = torch.empty_like(c), torch.empty_like(c)
    assert fb.fibar_relative_thresholds(n_on, n_off, W, H, c, c_on, c_off) == 0
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (c, c_on, c_off, n_on, n_off)]


@pytest.mark.parametrize("W,H", [(64, 48), (37, 11)])
def test_counts_and_relative_thresholds_match_oracle(W, H):
    ev = calibration(W, H)
    # one pixel silent, one with ON events only
    keep = ~((ev.x == 3) & (ev.y == 2)) & ~((ev.x == 5) & (ev.y == 1) & (ev.p == 0))
    ev = eventsim.Events(ev.x[keep], ev.y[keep], ev.p[keep], ev.t[keep])
    got = device_thresholds(ev, W, H)
    want = oracle.relative_thresholds(ev.x, ev.y, ev.p, W, H)
    assert np.array_equal(got[3].astype(np.int64), want[3])
    assert np.array_equal(got[4].astype(np.int64), want[4])
    for g, w in zip(got[:3], want[:3]):
        # double precision on both sides, rounded once to float
        assert np.array_equal(g, w.astype(np.float32))
    assert got[0][2 * W + 3] == 1.0 and got[2][1 * W + 5] == 1.0


def test_rejected_calibration_packet_adds_nothing():
    torch, dev = torch_dev()
    W, H = 16, 8
    ev = calibration(W, H, periods=1, amplitude=4.0)
    gx, gy, gp = to_device(ev)
    n_on = torch.zeros(W * H, dtype=torch.int32, device=dev)
    n_off = torch.zeros(W * H, dtype=torch.int32, device=dev)
    bad = gx.clone()
    bad[10] = W
    assert fb.fibar_count_polarities(bad, gy, gp, W, H, n_on, n_off) == fb.FIBAR_E_RANGE
    badp = gp.clone()
    badp[7] = 3
    assert fb.fibar_count_polarities(gx, gy, badp, W, H, n_on, n_off) == fb.FIBAR_E_POLARITY
    assert int(n_on.sum()) == 0 and int(n_off.sum()) == 0


def gains_for(W, H):
    """The relative thresholds of a calibration of this sensor."""
    return device_thresholds(calibration(W, H, periods=1, amplitude=4.0), W, H)[0]


@pytest.mark.parametrize("spatial", [True, False])
def test_packet_regulation_with_relative_thresholds(spatial):
    W, H = 640, 480
    w = eventsim.preset("vga", n_events=600_000, seed=21)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    g = gains_for(W, H)
    assert g.std() > 0.02
    run_pair(ev, W, H, sched, gain=g, spatial_filter=spatial)


def test_event_regulation_with_relative_thresholds():
    W, H = 64, 48
    w = eventsim.preset("sensor64x48", n_events=60_000)
    ev = eventsim.generate(w.scene)
    sched = eventsim.schedule(len(ev), w.packet, w.readouts)
    run_pair(ev, W, H, sched, gain=gains_for(W, H), telemetry=False, regulation="event")


def test_gain_can_be_replaced_and_removed():
    """Multipliers apply to pushes after the call: a stream half with gains,
    half without, matches the oracle switched at the same point."""
    torch, dev = torch_dev()
    W, H = 346, 260
    sc = eventsim.Scene(W, H, 300_000, 77, n_blobs=150, checker_cell=16.0,
                        checker_contrast=0.5, speed_px_s=200.0, noise_frac=0.01)
    ev = eventsim.generate(sc)
    gx, gy, gp = to_device(ev)
    g = gains_for(W, H)
    ctx = make_ctx(W, H)
    orc = oracle.Oracle(W, H)
    gd = torch.from_numpy(g).to(dev)
    assert ctx.set_gain(gd) == 0 and orc.set_gain(g.astype(np.float64)) == 0
    gd.fill_(7.0)   # the context holds its own copy
    for a in range(0, 150_000, 4096):
        b = min(a + 4096, 150_000)
        assert ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
    assert ctx.set_gain(None) == 0 and orc.set_gain(None) == 0
    for a in range(150_000, len(ev), 4096):
        b = min(a + 4096, len(ev))
        assert ctx.push(gx[a:b], gy[a:b], gp[a:b]) == 0
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
    compare_state(ctx.readout_host(0), orc.readout(0), True, "gain set, then removed")
    compare_stats(ctx.stats(), orc.stats())
    ctx.close()


def test_group_applies_each_contexts_gains():
    """Two contexts with different multipliers advanced as one group."""
    torch, dev = torch_dev()
    specs = [(64, 48, 60_000, 1024, 1), (346, 260, 200_000, 4096, 2)]
    ctxs, orcs, keep, op_lists = [], [], [], []
    for W, H, n, packet, seed in specs:
        sc = eventsim.Scene(W, H, n, 950 + seed, n_blobs=max(32, W * H // 600),
                            checker_cell=16.0, checker_contrast=0.5, speed_px_s=200.0,
                            noise_frac=0.01)
        ev = eventsim.generate(sc)
        g = gains_for(W, H)
        ctx = make_ctx(W, H, max_packet=32768)
        orc = oracle.Oracle(W, H)
        assert ctx.set_gain(torch.from_numpy(g).to(dev)) == 0
        assert orc.set_gain(g.astype(np.float64)) == 0
        gx, gy, gp = to_device(ev)
        keep.append((gx, gy, gp))
        ops = []
        for a in range(0, n, packet):
            b = min(a + packet, n)
            ops.append(fb.push_op(gx[a:b], gy[a:b], gp[a:b]))
            assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        ctxs.append(ctx)
        orcs.append(orc)
        op_lists.append(ops)
    group = fb.Group(ctxs)
    assert group.submit(op_lists) == 0
    torch.cuda.synchronize()
    for ctx, orc in zip(ctxs, orcs):
        compare_state(ctx.readout_host(0), orc.readout(0), True, "group with gains")
        compare_stats(ctx.stats(), orc.stats())
    group.close()
    for c in ctxs:
        c.close()
