"""fibar_fill_apply_noalloc (the entry point for callers that cannot
allocate) against fibar_fill_apply: the same filled image bit for bit and
the same count of tiles that kept L, on two calls in a row (the second
smaller, so the library's fixed scratch still holds the first call's values),
and the size limit of that scratch."""
import numpy as np
import pytest

import eventsim
import paper_2510_20071_amd as fb

pytestmark = pytest.mark.gpu


def frame(seed, H, W):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, 2, (H, W)).astype(np.float32)
    stale = (rng.random((H, W)) < rng.uniform(0.05, 0.6, (H, 1))).astype(np.uint8)
    age = rng.uniform(0, 12, (H, W)).astype(np.float32)
    return L, stale, age


def test_noalloc_apply_equals_apply_on_two_calls():
    import torch
    d = torch.device("cuda:0")
    stream = torch.cuda.current_stream(d).cuda_stream
    prm = eventsim.fill_init_params(21, zero_last=False)
    f = fb.Fill(prm, stream=stream)
    for call, (H, W, tile, theta) in enumerate([(720, 1280, 16, 0.25), (37, 45, 8, 0.4)]):
        print("noalloc call %d: %dx%d tile %d theta %.2f" % (call, H, W, tile, theta), flush=True)
        L, stale, age = frame(30 + call, H, W)
        gL, gS, gA = (torch.from_numpy(a).to(d) for a in (L, stale, age))
        want = torch.full((H, W), -1.0, dtype=torch.float32, device=d)
        got = torch.full((H, W), -2.0, dtype=torch.float32, device=d)
        rc1, n1 = f.apply(gL, gS, gA, want, tile=tile, theta=theta)
        rc2, n2 = f.apply_noalloc(gL, gS, gA, got, tile=tile, theta=theta)
        assert rc1 == 0 and rc2 == 0
        assert n1 == n2
        assert 0 < n1
        assert torch.equal(want, got)
    f.close()


def test_noalloc_apply_rejects_frames_beyond_its_scratch():
    import torch
    d = torch.device("cuda:0")
    f = fb.Fill(eventsim.fill_init_params(22), stream=torch.cuda.current_stream(d).cuda_stream)
    small = torch.zeros(16, dtype=torch.float32, device=d)
    st = torch.zeros(16, dtype=torch.uint8, device=d)
    H, W = 1025, 1024
    assert H * W > fb.FILL_NOALLOC_MAX_PIXELS
    rc, _ = fb.fibar_fill_apply_noalloc(f.handle, small, st, small, H, W, 16, 0.0, small)
    assert rc == fb.FIBAR_E_INVALID_ARG
    f.close()
