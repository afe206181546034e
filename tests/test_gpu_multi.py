"""GPU: several streams advanced together (fibar_multi_*) give exactly what
each stream gives alone, for every launch shape, and match the oracle."""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import compare_state, compare_stats, make_ctx, to_device, torch_dev

pytestmark = pytest.mark.gpu


def make_streams():
    specs = [((64, 48), 60_000, 1024, 1), ((346, 260), 300_000, 4096, 2),
             ((640, 480), 400_000, 16384, 3), ((1280, 720), 500_000, 32768, 4),
             ((346, 260), 50_000, 2048, 5)]
    out = []
    for (W, H), n, packet, seed in specs:
        sc = eventsim.Scene(W, H, n, 900 + seed, n_blobs=max(32, W * H // 600),
                            checker_cell=16.0, checker_contrast=0.5, speed_px_s=200.0,
                            noise_frac=0.01)
        ev = eventsim.generate(sc)
        ro = sorted(set(int(v) for v in np.random.default_rng(seed).integers(1, n, 5))) + [n]
        out.append((W, H, ev, eventsim.schedule(n, packet, ro)))
    return out


def run_group(streams, shape=None, autotune=False):
    torch, dev = torch_dev()
    ctxs = [make_ctx(W, H, max_packet=32768) for W, H, _, _ in streams]
    group = fb.Group(ctxs)
    if shape is not None:
        assert group.set_shape(shape) == 0
    if autotune:
        assert group.autotune() == 0
    op_lists, bufs = [], []
    keep = []
    for (W, H, ev, sched), ctx in zip(streams, ctxs):
        gx, gy, gp = to_device(ev)
        keep.append((gx, gy, gp))
        ops, b = [], []
        for it in sched:
            if it[0] == "push":
                ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
            else:
                d = dict(k=it[1], L=torch.empty(W * H, dtype=torch.float32, device=dev),
                         stale=torch.empty(W * H, dtype=torch.uint8, device=dev),
                         cnt=torch.empty(W * H, dtype=torch.int32, device=dev),
                         last=torch.empty(W * H, dtype=torch.int64, device=dev))
                b.append(d)
                ops.append(fb.readout_op(it[1], d["L"], stale=d["stale"], cnt=d["cnt"],
                                         last=d["last"]))
        op_lists.append(ops)
        bufs.append(b)
    assert group.submit(op_lists) == 0
    torch.cuda.synchronize()
    res = [[{k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()} for d in b]
           for b in bufs]
    finals = [c.readout_host(10 ** 12) for c in ctxs]
    stats = [c.stats() for c in ctxs]
    shape_used = group.shape()
    group.close()
    for c in ctxs:
        c.close()
    return res, finals, stats, shape_used


def run_alone(W, H, ev, sched):
    torch, dev = torch_dev()
    ctx = make_ctx(W, H, max_packet=32768)
    gx, gy, gp = to_device(ev)
    out = []
    for it in sched:
        if it[0] == "push":
            assert ctx.push(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]) == 0
        else:
            out.append(ctx.readout_host(it[1]))
    final = ctx.readout_host(10 ** 12)
    stats = ctx.stats()
    ctx.close()
    return out, final, stats


def test_group_equals_each_stream_alone_and_oracle():
    streams = make_streams()
    print("group of %d streams" % len(streams), flush=True)
    res, finals, stats, _ = run_group(streams)
    for si, (W, H, ev, sched) in enumerate(streams):
        alone, final, st = run_alone(W, H, ev, sched)
        assert st == stats[si]
        for key in final:
            assert np.array_equal(final[key], finals[si][key]), (si, key)
        for a, g in zip(alone, res[si]):
            assert np.array_equal(a["L"], g["L"]), si
            assert np.array_equal(a["stale"], g["stale"]), si
            assert np.array_equal(a["cnt"].view(np.int32), g["cnt"]), si
            assert np.array_equal(a["last"], g["last"]), si
        orc = oracle.Oracle(W, H)
        for it in sched:
            if it[0] == "push":
                orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]])
        compare_state(finals[si], orc.readout(10 ** 12), True, "stream %d" % si)
        compare_stats(stats[si], orc.stats(), "stream %d" % si)


def test_launch_shape_never_changes_results():
    streams = make_streams()[:3]
    ref = None
    for shape in range(fb.MULTI_CONFIGS):
        print("shape %d" % shape, flush=True)
        res, finals, stats, used = run_group(streams, shape=shape)
        if ref is None:
            ref = (res, finals, stats)
            continue
        assert stats == ref[2]
        for a, b in zip(finals, ref[1]):
            for key in a:
                assert np.array_equal(a[key], b[key]), key
        for ra, rb in zip(res, ref[0]):
            for da, db in zip(ra, rb):
                for key in ("L", "stale", "cnt", "last"):
                    assert np.array_equal(da[key], db[key]), key


def test_autotune_picks_a_shape_and_keeps_results():
    streams = make_streams()[1:4]
    res0, finals0, stats0, _ = run_group(streams, shape=0)
    res1, finals1, stats1, used = run_group(streams, autotune=True)
    assert used[0] in (64, 128, 256)
    assert stats0 == stats1
    for a, b in zip(finals0, finals1):
        for key in a:
            assert np.array_equal(a[key], b[key]), key


def test_group_reports_rejected_packet_of_one_stream():
    torch, dev = torch_dev()
    streams = make_streams()[:2]
    ctxs = [make_ctx(W, H, max_packet=32768) for W, H, _, _ in streams]
    group = fb.Group(ctxs)
    op_lists, keep = [], []
    for si, (W, H, ev, sched) in enumerate(streams):
        gx, gy, gp = to_device(ev)
        if si == 1:
            gx = gx.clone()
            gx[sched[0][2] + 5] = W        # second packet of stream 1 is out of range
        keep.append((gx, gy, gp))
        op_lists.append([fb.push_op(gx[a:b], gy[a:b], gp[a:b])
                         for it in sched if it[0] == "push" for a, b in [it[1:]]])
    assert group.submit(op_lists) == 0
    assert ctxs[0].synchronize() == 0
    assert ctxs[1].synchronize() == fb.FIBAR_E_RANGE
    W, H, ev, sched = streams[1]
    orc = oracle.Oracle(W, H)
    pushes = [it for it in sched if it[0] == "push"]
    for j, it in enumerate(pushes):
        if j != 1:
            orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]])
    compare_state(ctxs[1].readout_host(10 ** 12), orc.readout(10 ** 12), True, "after rejection")
    group.close()


def test_group_argument_checks():
    a = make_ctx(64, 48)
    nsf = make_ctx(64, 48, spatial_filter=False)
    rc, _ = fb.fibar_multi_create([a.handle, a.handle])
    assert rc == fb.FIBAR_E_INVALID_ARG
    rc, _ = fb.fibar_multi_create([a.handle, nsf.handle])
    assert rc == fb.FIBAR_E_UNSUPPORTED
    g = fb.Group([a])
    x = np.zeros(10, np.uint16)
    assert g.submit([[fb.push_op(x, x, x.astype(np.uint8))]]) == fb.FIBAR_E_INVALID_ARG
    assert g.set_shape(fb.MULTI_CONFIGS) == fb.FIBAR_E_INVALID_ARG
    assert g.set_shape(7) == 0 and g.config() == 7 and g.shape() == (128, 1024)
    g.close()


@pytest.mark.parametrize("config", [0, 5])
def test_group_spanning_many_batches_equals_streams_alone(config):
    """More rounds and more chunks than one batch of the group holds: the
    pending commits and staged descriptors at batch boundaries keep every
    stream exact (tiny packets give thousands of rounds)."""
    specs = [((64, 48), 2500 * 64, 64, 11), ((346, 260), 1200 * 512, 512, 12),
             ((640, 480), 40 * 32768, 32768, 13)]
    streams = []
    for (W, H), n, packet, seed in specs:
        sc = eventsim.Scene(W, H, n, 900 + seed, n_blobs=max(32, W * H // 600),
                            checker_cell=16.0, checker_contrast=0.5, speed_px_s=200.0,
                            noise_frac=0.01)
        ev = eventsim.generate(sc)
        n = len(ev)
        ro = list(range(n // 7, n, n // 7)) + [n]
        streams.append((W, H, ev, eventsim.schedule(n, packet, ro)))
    print("rounds per stream:", [sum(1 for it in s[3] if it[0] == "push") for s in streams],
          flush=True)
    res, finals, stats, _ = run_group(streams, shape=config)
    for si, (W, H, ev, sched) in enumerate(streams):
        alone, final, st = run_alone(W, H, ev, sched)
        assert st == stats[si], si
        for key in final:
            assert np.array_equal(final[key], finals[si][key]), (si, key)
        assert len(alone) == len(res[si])
        for a, g in zip(alone, res[si]):
            assert np.array_equal(a["L"], g["L"]), si
            assert np.array_equal(a["stale"], g["stale"]), si
            assert np.array_equal(a["last"], g["last"]), si
        orc = oracle.Oracle(W, H)
        for it in sched:
            if it[0] == "push":
                orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]])
        compare_state(finals[si], orc.readout(10 ** 12), True, "stream %d" % si)
        compare_stats(stats[si], orc.stats(), "stream %d" % si)
