"""GPU: per-kernel timing (fibar_set_kernel_timing / fibar_kernel_time)
times every launch, or every n-th, of the selected kernels, reports
positive device time, and leaves the results unchanged."""
import numpy as np
import pytest

import eventsim
import paper_2510_20071_amd as fb
from _harness import make_ctx, to_device

pytestmark = pytest.mark.gpu


def run(timed_mask, every=1):
    sc = eventsim.Scene(346, 260, 200_000, 77, n_blobs=128, checker_cell=16.0,
                        checker_contrast=0.5, speed_px_s=200.0, noise_frac=0.01)
    ev = eventsim.generate(sc)
    n = len(ev)
    sched = eventsim.schedule(n, 4096, [n // 3, n])
    gx, gy, gp = to_device(ev)
    ctx = make_ctx(346, 260)
    assert fb.fibar_set_kernel_timing(ctx.handle, timed_mask, every) == 0
    ops = []
    for it in sched:
        if it[0] == "push":
            ops.append(fb.push_op(gx[it[1]:it[2]], gy[it[1]:it[2]], gp[it[1]:it[2]]))
    assert ctx.submit(ops) == 0
    times = [fb.fibar_kernel_time(ctx.handle, k) for k in range(len(fb.KERNEL_NAMES))]
    final = ctx.readout_host(10 ** 12)
    stats = ctx.stats()
    ctx.close()
    return len(ops), times, final, stats


def test_kernel_timing_counts_launches_and_keeps_results():
    n_push, times, final, stats = run((1 << 1) | (1 << 2))
    kinds = {name: t for name, t in zip(fb.KERNEL_NAMES, times)}
    for k, (rc, ms, launches) in enumerate(times):
        assert rc == 0
        if k in (1, 2):
            assert launches == n_push, (k, launches)   # one apply and one pop per packet
            assert ms > 0.0
        else:
            assert launches == 0 and ms == 0.0
    _, times0, final0, stats0 = run(0)
    assert all(t[2] == 0 for t in times0)
    assert stats == stats0
    for key in final:
        assert np.array_equal(final[key], final0[key]), key
    print(kinds)


def test_kernel_timing_samples_every_nth_launch():
    n_push, times, _, _ = run(1 << 2, every=4)
    rc, ms, launches = times[2]
    assert rc == 0 and launches == (n_push + 3) // 4 and ms > 0.0


def test_kernel_timing_argument_checks():
    ctx = make_ctx(64, 48)
    assert fb.fibar_set_kernel_timing(ctx.handle, 1 << 5) == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_set_kernel_timing(ctx.handle, 1, 0) == fb.FIBAR_E_INVALID_ARG
    rc, _, _ = fb.fibar_kernel_time(ctx.handle, 5)
    assert rc == fb.FIBAR_E_INVALID_ARG
    ctx.close()
