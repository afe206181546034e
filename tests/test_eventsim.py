"""The seeded input generator: known answers, determinism and the event model."""
import numpy as np
import pytest

import eventsim


def test_philox_known_answers():
    # Known-answer vectors published with the Philox4x32-10 definition
    # (Salmon et al., SC'11, Random123 distribution).
    assert list(eventsim.philox4x32_10([0, 0, 0, 0], [0, 0])) == \
        [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert list(eventsim.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)) == \
        [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert list(eventsim.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                       [0xA4093822, 0x299F31D0])) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_deterministic_per_seed():
    w = eventsim.preset("sensor64x48", n_events=20000)
    a = eventsim.generate(w.scene)
    b = eventsim.generate(w.scene)
    for f in "xypt":
        assert np.array_equal(getattr(a, f), getattr(b, f))
    w2 = eventsim.preset("sensor64x48", n_events=20000, seed=99)
    c = eventsim.generate(w2.scene)
    assert not np.array_equal(a.x, c.x)


@pytest.mark.parametrize("name,n", [("sensor64x48", 50000), ("vga", 300000)])
def test_stream_shape(name, n):
    w = eventsim.preset(name, n_events=n)
    ev = eventsim.generate(w.scene)
    assert len(ev) == n
    assert ev.x.max() < w.scene.width and ev.y.max() < w.scene.height
    assert set(np.unique(ev.p)) <= {0, 1}
    assert np.all(np.diff(ev.t.astype(np.int64)) >= 0)
    assert 0.4 < ev.p.mean() < 0.6


def test_events_follow_threshold_crossings():
    """Without noise, the signed event count at a pixel times C equals the
    ground-truth change of log intensity, to within one threshold."""
    sc = eventsim.Scene(64, 48, 40000, 5, n_blobs=32, speed_px_s=30.0, noise_frac=0.0,
                        thr_on=0.2, thr_off=0.2)
    ev = eventsim.generate(sc)
    g = eventsim.render_frames(sc, [0, int(ev.t[-1])])
    pix = ev.y.astype(np.int64) * 64 + ev.x
    net = np.bincount(pix, weights=np.where(ev.p == 1, 1.0, -1.0), minlength=64 * 48)
    d = (g[1] - g[0]).reshape(-1)
    # the last step's crossings may be cut off at n_events; allow 2 thresholds
    assert np.max(np.abs(net * 0.2 - d)) <= 2 * 0.2 + 1e-6


def test_schedule_splits_packets_at_readouts():
    s = eventsim.schedule(10, 4, [2, 4, 9, 10])
    assert s == [("push", 0, 2), ("read", 2), ("push", 2, 4), ("read", 4),
                 ("push", 4, 8), ("push", 8, 9), ("read", 9), ("push", 9, 10), ("read", 10)]
    pushes = [(a, b) for it in s if it[0] == "push" for a, b in [it[1:]]]
    assert sum(b - a for a, b in pushes) == 10
