"""GPU: graph launches (fibar_set_launch_mode) give exactly the results of
direct launches, batch after batch, including the graphs' parameter updates
and their timing (fibar_set_kernel_timing)."""
import numpy as np
import pytest

import eventsim
import oracle
import paper_2510_20071_amd as fb
from _harness import compare_state, make_ctx, to_device, torch_dev

pytestmark = pytest.mark.gpu

W, H = 64, 48
NPX = W * H
NTILES = ((W + 1) // 2) * ((H + 1) // 2)


def flush(msg):
    print(msg, flush=True)


def _stream(n_events=150_000, packet=500, seed=21):
    w = eventsim.preset("sensor64x48", n_events=n_events, seed=seed)
    ev = eventsim.generate(w.scene)
    # readouts right after pushes (taken by the pop launch), one right after
    # another readout, and one before any push
    ro = [0, 1, 777, 20_000, 20_000, 64_123, 99_999, 128_001, 150_000]
    return ev, eventsim.schedule(len(ev), packet, ro)


def _ops(sched, g, kinds):
    """The schedule as one op list; readout j takes kinds[j % len(kinds)]:
    'dev' (device, no window count), 'cnt' (device with the window count:
    the separate readout kernel), 'host' (host arrays: the batch runs on
    direct launches).  Returns (ops, outputs)."""
    torch, dev = torch_dev()
    gx, gy, gp = g
    ops, outs, j = [], [], 0
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
            continue
        kind = kinds[j % len(kinds)]
        j += 1
        if kind == "host":
            b = dict(L=np.empty(NPX, np.float32), pbar=np.empty(NPX, np.float32),
                     stale=np.empty(NPX, np.uint8), last=np.empty(NPX, np.int64),
                     log_age=np.empty(NPX, np.float32), tcnt=np.empty(NTILES, np.uint32))
            ops.append(fb.readout_op(0, b["L"], pbar=b["pbar"], stale=b["stale"], last=b["last"],
                                     log_age=b["log_age"], tcnt=b["tcnt"], on_device=0))
        else:
            b = dict(L=torch.empty(NPX, dtype=torch.float32, device=dev),
                     pbar=torch.empty(NPX, dtype=torch.float32, device=dev),
                     stale=torch.empty(NPX, dtype=torch.uint8, device=dev),
                     last=torch.empty(NPX, dtype=torch.int64, device=dev),
                     log_age=torch.empty(NPX, dtype=torch.float32, device=dev),
                     tcnt=torch.empty(NTILES, dtype=torch.int32, device=dev))
            cnt = None
            if kind == "cnt":
                b["cnt"] = torch.empty(NPX, dtype=torch.int32, device=dev)
                cnt = b["cnt"]
            ops.append(fb.readout_op(0, b["L"], pbar=b["pbar"], stale=b["stale"], cnt=cnt,
                                     last=b["last"], log_age=b["log_age"], tcnt=b["tcnt"]))
        outs.append(b)
    return ops, outs


def _host(b):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v.copy()) for k, v in b.items()}


def _run(mode, sched, g, kinds, repeats):
    """Submit the schedule `repeats` times (reset in between); returns the
    outputs and final stats of every submission."""
    import torch
    ctx = make_ctx(W, H)
    assert fb.fibar_set_launch_mode(ctx.handle, mode) == fb.FIBAR_OK
    res = []
    for r in range(repeats):
        assert ctx.reset() == 0
        ops, outs = _ops(sched, g, kinds)
        assert ctx.submit(ops) == 0
        torch.cuda.synchronize()
        res.append(([_host(b) for b in outs], ctx.stats(), ctx.readout_host(0)))
    ctx.close()
    return res


def _same(a, b, where):
    outs_a, st_a, fin_a = a
    outs_b, st_b, fin_b = b
    assert len(outs_a) == len(outs_b)
    for j, (x, y) in enumerate(zip(outs_a, outs_b)):
        assert x.keys() == y.keys()
        for key in x:
            assert np.array_equal(x[key].view(np.uint8), y[key].view(np.uint8)), \
                "%s of readout %d, %s" % (key, j, where)
    for f in ("k", "h", "Q", "P", "T", "n_regulations", "last_stale", "total_stale"):
        assert st_a[f] == st_b[f], "%s %s" % (f, where)
    for key in fin_a:
        assert np.array_equal(fin_a[key], fin_b[key]), "final %s %s" % (key, where)


@pytest.mark.parametrize("kinds", [("dev",), ("dev", "cnt"), ("dev", "host", "cnt")])
def test_graph_launches_equal_direct_launches(kinds):
    """305 packets (two batches: 256 and 49 packets) submitted three times:
    the first graph copy runs as instantiated, then both copies are updated
    and reused.  Every readout and the final state equal direct launches bit
    for bit, and the oracle within the parity tolerance."""
    ev, sched = _stream()
    g = to_device(ev)
    flush("graph vs direct, readout kinds %s" % (kinds,))
    direct = _run(fb.FIBAR_LAUNCH_DIRECT, sched, g, kinds, 1)[0]
    graph = _run(fb.FIBAR_LAUNCH_GRAPH, sched, g, kinds, 3)
    for r, res in enumerate(graph):
        _same(direct, res, "submission %d" % r)
    orc = oracle.Oracle(W, H)
    for it in sched:
        if it[0] == "push":
            assert orc.push(ev.x[it[1]:it[2]], ev.y[it[1]:it[2]], ev.p[it[1]:it[2]]) == 0
    compare_state(graph[-1][2], orc.readout(0), True, "final state, graph launches")


def test_graph_launches_multi_chunk_packets_and_mode_switch():
    """Packets of several chunks, switching between the modes between
    submissions of one stream: the same results as direct launches."""
    torch, dev = torch_dev()
    ev, _ = _stream(n_events=130_000, seed=23)
    sizes = [1, 16384, 16385, 40_000, 3, 33_000, 20_000]
    bounds = np.cumsum([0] + sizes)
    assert bounds[-1] <= len(ev)
    gx, gy, gp = to_device(ev)
    ctxs = [make_ctx(W, H) for _ in range(2)]
    frames = []
    for mode_seq, ctx in zip(([0, 0, 0], [1, 0, 1]), ctxs):
        out = []
        for part in range(3):
            assert fb.fibar_set_launch_mode(ctx.handle, mode_seq[part]) == fb.FIBAR_OK
            ops = []
            for i in range(len(sizes)):
                if i % 3 != part:
                    continue
                a, b = int(bounds[i]), int(bounds[i + 1])
                ops.append(fb.push_op(gx[a:b], gy[a:b], gp[a:b]))
            L = torch.empty(NPX, dtype=torch.float32, device=dev)
            ops.append(fb.readout_op(0, L))
            assert ctx.submit(ops) == 0
            torch.cuda.synchronize()
            out.append((L.cpu().numpy(), ctx.stats()))
        frames.append(out)
    for (La, sa), (Lb, sb) in zip(*frames):
        assert np.array_equal(La.view(np.uint32), Lb.view(np.uint32))
        for f in ("k", "h", "Q", "P", "T", "total_stale"):
            assert sa[f] == sb[f], f
    for c in ctxs:
        c.close()


def test_graph_launch_timing_counts_per_batch():
    """With graph launches the timed count restarts with every batch and pop
    launches that also write a readout count as pops (kept under kernel 3):
    batches of 256 and 49 packets timed every 16th pop give 16 + 4 timed pop
    (and apply) launches per submission, with positive durations."""
    torch, dev = torch_dev()
    ev, sched = _stream()
    g = to_device(ev)
    ctx = make_ctx(W, H)
    assert fb.fibar_set_launch_mode(ctx.handle, fb.FIBAR_LAUNCH_GRAPH) == fb.FIBAR_OK
    assert fb.fibar_set_kernel_timing(ctx.handle, (1 << 1) | (1 << 2), 16) == fb.FIBAR_OK
    n_push = sum(1 for it in sched if it[0] == "push")
    batches = [256, n_push - 256]            # one chunk per packet, 256 chunks per batch
    assert 0 < batches[1] <= 256
    expect = sum((b + 15) // 16 for b in batches)
    for rep in range(2):
        assert ctx.reset() == 0
        ops, _ = _ops(sched, g, ("dev",))
        assert ctx.submit(ops) == 0
        rc2, ms2, n2 = fb.fibar_kernel_time(ctx.handle, 2)
        rc3, ms3, n3 = fb.fibar_kernel_time(ctx.handle, 3)
        rc1, ms1, n1 = fb.fibar_kernel_time(ctx.handle, 1)
        assert rc1 == rc2 == rc3 == fb.FIBAR_OK
        assert n2 + n3 == expect, (n2, n3, expect)
        assert n1 == expect, (n1, expect)
        assert n2 > 0 and 0.0 < ms2 / n2 < 1.0, (ms2, n2)
        assert n1 > 0 and 0.0 < ms1 / n1 < 1.0, (ms1, n1)
    ctx.close()


def test_set_launch_mode_rejects_unknown_modes():
    ctx = make_ctx(W, H)
    for mode in (-1, 2, 7):
        assert fb.fibar_set_launch_mode(ctx.handle, mode) == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_set_launch_mode(None, fb.FIBAR_LAUNCH_GRAPH) == fb.FIBAR_E_INVALID_ARG
    ctx.close()
