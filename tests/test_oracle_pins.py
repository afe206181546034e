"""Pins of the FP64 oracle against facts fixed by the paper and mathematics.

None of these retype the oracle's own update rules: each compares the oracle
with a closed form, a library routine, a transfer function, a brute-force
recount or an invariant the paper states.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

import eventsim
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_pixel_stream(W, H, x, y, pols):
    n = len(pols)
    return (np.full(n, x, np.uint16), np.full(n, y, np.uint16),
            np.asarray(pols, np.uint8), np.arange(n, dtype=np.uint64))


# ---------------------------------------------------------------------------
# Filter coefficients: Eq. (17)-(18) against the transfer functions Eq. (12)
# ---------------------------------------------------------------------------
def H_alpha(z, a):
    return a * (z - 1.0) / (z - a)


def H_beta(z, b):
    return z * (1.0 + b) / (2.0 * (z - b))


@pytest.mark.parametrize("t_cut", [5.0, 10.0, 20.0, 40.0, 100.0, 1000.0])
def test_half_power_at_cutoff(t_cut):
    a, b = oracle.coefficients(t_cut)
    assert 0.0 < a < 1.0 and 0.0 < b < 1.0
    w = 2 * np.pi / t_cut
    z = np.exp(1j * w)
    # H_alpha is a high pass: its maximum magnitude is at omega = pi (z = -1)
    ra = abs(H_alpha(z, a)) ** 2 / abs(H_alpha(-1.0, a)) ** 2
    # H_beta is a low pass: its maximum magnitude is at omega = 0 (z = 1)
    rb = abs(H_beta(z, b)) ** 2 / abs(H_beta(1.0, b)) ** 2
    # Eq. (18) subtracts nearly equal numbers for long cutoffs; the rounding
    # error of beta grows like 1 / (1 - beta), so the bound widens with T_cut
    tol = 1e-12 if t_cut <= 100 else 1e-9
    assert ra == pytest.approx(0.5, abs=tol)
    assert rb == pytest.approx(0.5, abs=tol)


@pytest.mark.parametrize("t_cut", [200.0, 1000.0, 10000.0])
def test_taylor_second_order(t_cut):
    # both coefficients share the expansion 1 - w + w^2/2 + O(w^3)
    a, b = oracle.coefficients(t_cut)
    w = 2 * np.pi / t_cut
    approx = 1.0 - w + 0.5 * w * w
    assert abs(a - approx) <= 1.0 * w ** 3
    assert abs(b - approx) <= 1.0 * w ** 3


def test_paper_facts_golden():
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        facts = json.load(f)
    # Fig. 2 caption: omega_cut = 0.02 pi corresponds to T_cut = 100 events
    w = 2 * np.pi / facts["fig2_t_cut"]
    assert w == pytest.approx(facts["fig2_omega_cut_over_pi"] * np.pi, rel=1e-15)
    a, b = oracle.coefficients(facts["fig2_t_cut"])
    z = np.exp(1j * w)
    assert abs(H_alpha(z, a)) ** 2 / abs(H_alpha(-1, a)) ** 2 == pytest.approx(0.5, abs=1e-12)
    # Eq. (19): the observed fill ratio lies in [1/A, 1] for 2x2 tiles
    assert facts["fill_ratio_min"] == pytest.approx(1.0 / facts["tile_area"])


# ---------------------------------------------------------------------------
# Temporal filter: closed form for k identical events at one pixel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t_cut", [40.0, 100.0, 7.0])
@pytest.mark.parametrize("pol", [0, 1])
@pytest.mark.parametrize("spatial", [False, True])
def test_closed_form_identical_events(t_cut, pol, spatial):
    W, H = 8, 6
    kmax = 400
    a, b = oracle.coefficients(t_cut)
    c = 0.5 * (1.0 + b)
    p = 1.0 if pol else -1.0
    orc = oracle.Oracle(W, H, t_cut=t_cut, spatial_filter=spatial, q_min=1, q_max=0)
    x, y, pp, t = one_pixel_stream(W, H, 3, 2, [pol] * kmax)
    for k in range(1, kmax + 1):
        assert orc.push(x[k - 1:k], y[k - 1:k], pp[k - 1:k], t[k - 1:k]) == 0
        if k in (1, 2, 3, 6, 17, 100, 400):
            r = orc.readout(k)
            i = 2 * W + 3
            # pbar_k = p (1 - a^k); L_k = c p a sum_{j=0}^{k-1} b^{k-1-j} a^j
            pb = p * (1.0 - a ** k)
            geo = sum(b ** (k - 1 - j) * a ** j for j in range(k))
            Lk = c * p * a * geo
            # once pbar ~ p, the increment p - pbar carries an absolute
            # rounding error ~ eps that L accumulates with gain c/(1-beta)
            atol = 1e-13
            assert r["pbar"][i] == pytest.approx(pb, rel=1e-12, abs=atol)
            assert r["L"][i] == pytest.approx(Lk, rel=1e-12, abs=atol)
            others = np.ones(W * H, bool)
            others[i] = False
            assert np.all(r["L"][others] == 0.0) and np.all(r["pbar"][others] == 0.0)
            if spatial:
                assert r["stale"][i] == 0 and r["cnt"][i] >= 1


# ---------------------------------------------------------------------------
# Temporal filter: Eq. (15) as a library IIR with zero initial conditions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t_cut", [40.0, 100.0])
def test_nsf_matches_lfilter(t_cut):
    rng = np.random.default_rng(7)
    W, H = 16, 8
    n = 20000
    # a few busy pixels plus random others, interleaved
    pix = rng.integers(0, W * H, size=n)
    busy = rng.random(n) < 0.5
    pix[busy] = rng.integers(0, 4, size=busy.sum())
    pol = (rng.random(n) < 0.45).astype(np.uint8)   # ON/OFF imbalance
    orc = oracle.Oracle(W, H, t_cut=t_cut, spatial_filter=False)
    for a0 in range(0, n, 777):
        a1 = min(n, a0 + 777)
        assert orc.push(pix[a0:a1] % W, pix[a0:a1] // W, pol[a0:a1]) == 0
    r = orc.readout(0)
    a, b = oracle.coefficients(t_cut)
    c = 0.5 * (1.0 + b)
    for i in range(W * H):
        seq = np.where(pol[pix == i] == 1, 1.0, -1.0)
        if seq.size == 0:
            assert r["L"][i] == 0.0
            continue
        Lf = scipy.signal.lfilter([c * a, -c * a], [1.0, -(a + b), a * b], seq)
        pf = scipy.signal.lfilter([1.0 - a], [1.0, -a], seq)
        assert r["L"][i] == pytest.approx(Lf[-1], rel=1e-10, abs=1e-12)
        assert r["pbar"][i] == pytest.approx(pf[-1], rel=1e-10, abs=1e-12)
        assert r["tot"][i] == seq.size
        assert r["last"][i] == np.nonzero(pix == i)[0][-1]


def test_frequency_response_of_impulse():
    """The oracle's impulse response has the spectrum H_alpha * H_beta."""
    t_cut = 40.0
    a, b = oracle.coefficients(t_cut)
    K = 4000
    seq = (np.arange(K) % 3 == 0).astype(np.uint8)
    flip = seq.copy()
    flip[0] ^= 1
    Ls = []
    for s in (seq, flip):
        orc = oracle.Oracle(1, 1, t_cut=t_cut, spatial_filter=False, q_min=1)
        out = np.empty(K)
        for k in range(K):
            orc.push(np.zeros(1, np.uint16), np.zeros(1, np.uint16), s[k:k + 1])
            out[k] = orc.readout(0)["L"][0]
        Ls.append(out)
    # the filter is linear in p, so half the difference is the response to
    # a unit impulse at k = 0 (p changes by 2 there)
    sign = 1.0 if seq[0] == 1 else -1.0
    h = sign * (Ls[0] - Ls[1]) / 2.0
    ws = np.linspace(0.01, np.pi, 57)
    kk = np.arange(K)
    for w in list(ws) + [2 * np.pi / t_cut]:
        Hm = np.sum(h * np.exp(-1j * w * kk))
        z = np.exp(1j * w)
        Hr = H_alpha(z, a) * H_beta(z, b)
        assert abs(Hm - Hr) <= 1e-9 * max(1.0, abs(Hr))
    # |H|^2 at the cutoff = (1/2 of H_alpha's peak) * (1/2 of H_beta's peak)
    wc = 2 * np.pi / t_cut
    Hc = np.sum(h * np.exp(-1j * wc * kk))
    peak = abs(H_alpha(-1.0, a)) ** 2 * abs(H_beta(1.0, b)) ** 2
    assert abs(Hc) ** 2 == pytest.approx(0.25 * peak, rel=1e-9)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def small_stream(n=30000, seed=11, W=64, H=48):
    sc = eventsim.Scene(W, H, n, seed, n_blobs=32, speed_px_s=30.0, noise_frac=0.01)
    return sc, eventsim.generate(sc)


def run(ev, W, H, packet, **kw):
    orc = oracle.Oracle(W, H, **kw)
    sched = eventsim.schedule(len(ev), packet, [])
    oracle.run_schedule(orc, ev, sched)
    return orc, orc.readout(int(ev.t[-1]))


def test_readout_and_empty_push_do_not_change_state():
    sc, ev = small_stream(8000)
    orc, r1 = run(ev, 64, 48, 1024)
    r2 = orc.readout(int(ev.t[-1]))
    assert orc.push(ev.x[:0], ev.y[:0], ev.p[:0], ev.t[:0]) == 0
    s_before = orc.stats()
    r3 = orc.readout(int(ev.t[-1]))
    assert orc.stats() == s_before
    for key in r1:
        assert np.array_equal(r1[key], r2[key]) and np.array_equal(r1[key], r3[key])


@pytest.mark.parametrize("mode", ["packet", "event"])
def test_timestamp_rescaling_invariance(mode):
    sc, ev = small_stream(12000)
    o1 = oracle.Oracle(64, 48, regulation=mode)
    o2 = oracle.Oracle(64, 48, regulation=mode)
    t2 = ev.t * np.uint64(3) + np.uint64(12345)
    for a in range(0, len(ev), 1000):
        b = min(len(ev), a + 1000)
        o1.push(ev.x[a:b], ev.y[a:b], ev.p[a:b], ev.t[a:b])
        o2.push(ev.x[a:b], ev.y[a:b], ev.p[a:b], t2[a:b])
    r1 = o1.readout(int(ev.t[-1]))
    r2 = o2.readout(int(t2[-1]))
    for key in r1:
        assert np.array_equal(r1[key], r2[key]), key


@pytest.mark.parametrize("mode", ["packet", "event"])
@pytest.mark.parametrize("spatial", [True, False])
def test_polarity_flip_negates_exactly(mode, spatial):
    sc, ev = small_stream(12000)
    o1 = oracle.Oracle(64, 48, regulation=mode, spatial_filter=spatial)
    o2 = oracle.Oracle(64, 48, regulation=mode, spatial_filter=spatial)
    for a in range(0, len(ev), 1024):
        b = min(len(ev), a + 1024)
        o1.push(ev.x[a:b], ev.y[a:b], ev.p[a:b])
        o2.push(ev.x[a:b], ev.y[a:b], 1 - ev.p[a:b])
    r1, r2 = o1.readout(0), o2.readout(0)
    assert np.array_equal(r1["L"], -r2["L"])
    assert np.array_equal(r1["pbar"], -r2["pbar"])
    for key in ("cnt", "tot", "last", "tcnt", "stale"):
        assert np.array_equal(r1[key], r2[key])
    assert o1.stats() == o2.stats()


def test_nsf_cross_pixel_reordering_is_bit_identical():
    sc, ev = small_stream(20000)
    pix = ev.y.astype(np.int64) * 64 + ev.x
    # stable sort by pixel keeps each pixel's own order
    order = np.argsort(pix, kind="stable")
    o1 = oracle.Oracle(64, 48, spatial_filter=False)
    o2 = oracle.Oracle(64, 48, spatial_filter=False)
    o1.push(ev.x, ev.y, ev.p)
    o2.push(ev.x[order], ev.y[order], ev.p[order])
    r1, r2 = o1.readout(0), o2.readout(0)
    assert np.array_equal(r1["L"], r2["L"]) and np.array_equal(r1["pbar"], r2["pbar"])
    assert np.array_equal(r1["tot"], r2["tot"])


@pytest.mark.parametrize("mode,packet", [("packet", 1024), ("packet", 97), ("event", 1000)])
def test_window_invariants(mode, packet):
    sc, ev = small_stream(40000, seed=5)
    W, H = 64, 48
    orc = oracle.Oracle(W, H, regulation=mode, q_min=16)
    tw = (W + 1) // 2
    npx = W * H
    tile = (np.arange(npx) // W // 2) * tw + (np.arange(npx) % W) // 2
    for a in range(0, len(ev), packet):
        b = min(len(ev), a + packet)
        assert orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        if (a // packet) % 7:
            continue
        s = orc.stats()
        r = orc.readout(0)
        cnt = r["cnt"].astype(np.int64)
        assert cnt.sum() == s["q"] == s["k"] - s["h"] + 1
        assert (cnt > 0).sum() == s["P"]
        assert (r["tcnt"] > 0).sum() == s["T"]
        # per-tile active-pixel count matches the pixel counters
        tc = np.bincount(tile[cnt > 0], minlength=r["tcnt"].size)
        assert np.array_equal(tc, r["tcnt"])
        # window is the newest events: active <=> last index inside [h, k]
        assert np.array_equal(cnt > 0, r["last"] >= s["h"])
        # fill ratio bounds of Eq. (19): 1/4 <= P / (4 T) <= 1
        assert s["T"] <= s["P"] <= 4 * s["T"]
        assert 16 <= s["Q"] <= npx
        # stale = seen and not active
        assert np.array_equal(r["stale"] == 1, (r["tot"] > 0) & (cnt == 0))
        # never-seen pixels keep their initial value (never blurred: no
        # event ever made them active)
        never = r["tot"] == 0
        assert np.all(r["L"][never] == 0.0) and np.all(r["pbar"][never] == 0.0)


# ---------------------------------------------------------------------------
# Special cases that reduce to simpler methods
# ---------------------------------------------------------------------------
def test_no_pops_equals_nsf():
    sc, ev = small_stream(20000)
    n = len(ev)
    _, r1 = run(ev, 64, 48, 1024, q_min=3072, q_max=3072)
    _, r2 = run(ev, 64, 48, 1024, spatial_filter=False)
    # q_max = W*H < n, so pops do happen here; use a bigger window instead
    o3 = oracle.Oracle(64, 48, q_min=3072, q_max=3072)
    o3.push(ev.x[:3000], ev.y[:3000], ev.p[:3000])
    o4 = oracle.Oracle(64, 48, spatial_filter=False)
    o4.push(ev.x[:3000], ev.y[:3000], ev.p[:3000])
    r3, r4 = o3.readout(0), o4.readout(0)
    assert o3.stats()["h"] == 0
    assert np.array_equal(r3["L"], r4["L"]) and np.array_equal(r3["pbar"], r4["pbar"])
    assert n > 3072 and not np.array_equal(r1["L"], r2["L"])


def test_first_blur_step_is_binomial_correlation():
    """At the first step with stale pixels, every stale pixel takes the 3x3
    binomial average (clamp-to-edge) of the pre-blur image, which equals the
    blur-off image up to that step."""
    sc, ev = small_stream(60000, seed=3)
    W, H = 64, 48
    fib = oracle.Oracle(W, H, q_min=8)
    nsf = oracle.Oracle(W, H, spatial_filter=False)
    k3 = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    packet = 256
    for a in range(0, len(ev), packet):
        b = min(len(ev), a + packet)
        fib.push(ev.x[a:b], ev.y[a:b], ev.p[a:b])
        nsf.push(ev.x[a:b], ev.y[a:b], ev.p[a:b])
        if fib.stats()["total_stale"] > 0:
            break
    else:
        pytest.fail("no pixel went stale")
    rf, rn = fib.readout(0), nsf.readout(0)
    ref = scipy.ndimage.correlate(rn["L"].reshape(H, W), k3, mode="nearest").reshape(-1)
    st = rf["stale"] == 1
    assert st.sum() == fib.stats()["last_stale"] > 0
    assert np.allclose(rf["L"][st], ref[st], rtol=0, atol=1e-14)
    assert np.array_equal(rf["L"][~st], rn["L"][~st])
    assert np.array_equal(rf["pbar"], rn["pbar"])


def test_edge_pixel_blur_uses_clamped_border():
    """A corner pixel going stale takes the clamp-to-edge binomial average.

    4x4 sensor, window of two events (q_min = 1, q_max = 2), one-event
    packets: (0,0) ON, (1,0) OFF, (0,1) ON.  The third push makes the queue
    three long, so the event of (0,0) leaves it and (0,0) goes stale."""
    W, H = 4, 4
    orc = oracle.Oracle(W, H, q_min=1, q_max=2)
    nsf = oracle.Oracle(W, H, spatial_filter=False, q_min=1)
    seq = [(0, 0, 1), (1, 0, 0), (0, 1, 1)]
    for x, y, p in seq:
        for o in (orc, nsf):
            o.push(np.array([x], np.uint16), np.array([y], np.uint16), np.array([p], np.uint8))
    r, rn = orc.readout(0), nsf.readout(0)
    assert np.nonzero(r["stale"])[0].tolist() == [0]
    k3 = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    img = rn["L"].reshape(H, W)
    want = scipy.ndimage.correlate(img, k3, mode="nearest")[0, 0]
    zero_pad = scipy.ndimage.correlate(img, k3, mode="constant")[0, 0]
    assert r["L"][0] == pytest.approx(want, rel=0, abs=1e-15)
    assert abs(want - zero_pad) > 1e-3
    assert np.array_equal(r["L"][1:], rn["L"][1:])
    s = orc.stats()
    assert (s["h"], s["q"], s["P"], s["T"]) == (1, 2, 2, 1)


def test_event_mode_equals_packet_mode_for_single_events():
    """With one-event packets the two regulation modes agree whenever no step
    stales more than one pixel (only the blur order inside a burst differs)."""
    sc, ev = small_stream(6000, seed=9)
    W, H = 64, 48
    oe = oracle.Oracle(W, H, regulation="event", q_min=64)
    op = oracle.Oracle(W, H, regulation="packet", q_min=64)
    multi = 0
    for k in range(len(ev)):
        sl = slice(k, k + 1)
        oe.push(ev.x[sl], ev.y[sl], ev.p[sl])
        op.push(ev.x[sl], ev.y[sl], ev.p[sl])
        multi += op.stats()["last_stale"] > 1
        if multi == 0:
            assert oe.stats() == op.stats()
    assert oe.stats()["k"] == op.stats()["k"]
    if multi == 0:
        re, rp = oe.readout(0), op.readout(0)
        for key in re:
            assert np.array_equal(re[key], rp[key])


def brute_event_mode(W, H, xs, ys, ps, t_cut, q_min, q_max, fill):
    """The per-event procedure written out with Python lists: after each
    event (temporal filter, then the event joins the window) events leave
    from the front while the window is longer than Q; a pixel with no event
    left in the window is blurred right away from the image as it is at that
    moment (3x3 binomial, borders clamped); Q is then recomputed from the
    distinct pixels and 2x2 tiles of the window.  Yields (L, stats) after
    every event."""
    a, b = oracle.coefficients(t_cut)
    L = [0.0] * (W * H)
    pbar = [0.0] * (W * H)
    ev, h, Q = [], 0, q_max
    wts = (0.25, 0.5, 0.25)
    for x, y, p in zip(xs, ys, ps):
        i = int(y) * W + int(x)
        pk = 1.0 if p else -1.0
        pbar[i] = a * pbar[i] + (1.0 - a) * pk
        L[i] = b * L[i] + 0.5 * (1.0 + b) * (pk - pbar[i])
        ev.append(i)
        stale = 0
        while len(ev) - h > Q:
            j = ev[h]
            h += 1
            if j not in ev[h:]:
                jx, jy = j % W, j // W
                acc = 0.0
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        xx = min(max(jx + dx, 0), W - 1)
                        yy = min(max(jy + dy, 0), H - 1)
                        acc += wts[dy + 1] * wts[dx + 1] * L[yy * W + xx]
                L[j] = acc
                stale += 1
        win = ev[h:]
        P = len(set(win))
        T = len(set((k // W // 2) * ((W + 1) // 2) + (k % W) // 2 for k in win))
        if P:
            Q = max(q_min, min(q_max, (len(win) * fill[0] * 4 * T) // (fill[1] * P)))
        yield list(L), {"h": h, "Q": Q, "P": P, "T": T, "last_stale": stale}


def test_event_mode_sequential_blurs_against_brute_force():
    """Per-event regulation blurs the pixels that go stale in one step one
    after another, each from the image with the earlier blurs in it.  On a
    5x4 sensor with bursts of several stale pixels per step the oracle
    follows the list-based procedure after every event; packet regulation
    (simultaneous blurs) ends up elsewhere on the same events."""
    W, H = 5, 4
    rng = np.random.default_rng(17)
    n = 1500
    pix, cur = [], 0
    for _ in range(n):
        if rng.random() < 0.5:
            cur = int(rng.integers(0, W * H))
        pix.append(cur)
    xs = np.array([q % W for q in pix], np.uint16)
    ys = np.array([q // W for q in pix], np.uint16)
    ps = rng.integers(0, 2, n).astype(np.uint8)
    q_min, q_max, fill = 1, W * H, (1, 2)
    orc = oracle.Oracle(W, H, q_min=q_min, q_max=q_max, fill=fill, regulation="event")
    bursts = 0
    for e, (Lb, sb) in enumerate(brute_event_mode(W, H, xs, ys, ps, 40.0, q_min, q_max, fill)):
        assert orc.push(xs[e:e + 1], ys[e:e + 1], ps[e:e + 1]) == 0
        s = orc.stats()
        assert {k: s[k] for k in sb} == sb, e
        assert np.allclose(orc.readout(0)["L"], Lb, rtol=0, atol=1e-12), e
        bursts += sb["last_stale"] > 1
    assert bursts > 20
    pk = oracle.Oracle(W, H, q_min=q_min, q_max=q_max, fill=fill)
    for e in range(n):
        pk.push(xs[e:e + 1], ys[e:e + 1], ps[e:e + 1])
    assert not np.allclose(pk.readout(0)["L"], orc.readout(0)["L"], rtol=0, atol=1e-9)


# ---------------------------------------------------------------------------
# Brute force on tiny sensors: recount the window from scratch
# ---------------------------------------------------------------------------
class BruteWindow:
    """Recounts the active-event window from the event list after each step."""

    def __init__(self, W, H, q_min, q_max, num, den):
        self.W, self.H = W, H
        self.q_min, self.q_max, self.num, self.den = q_min, q_max, num, den
        self.events = []   # pixel ids of all events, in order
        self.h = 0
        self.Q = q_max

    def tile(self, i):
        return (i // self.W // 2) * ((self.W + 1) // 2) + (i % self.W) // 2

    def push(self, pixels):
        self.events.extend(pixels)

    def regulate(self):
        k = len(self.events) - 1
        while k - self.h + 1 > self.Q:
            self.h += 1
        win = self.events[self.h:]
        P = len(set(win))
        T = len(set(self.tile(i) for i in win))
        if P > 0:
            v = (len(win) * self.num * 4 * T) // (self.den * P)
            self.Q = max(self.q_min, min(self.q_max, v))
        return P, T

    def cnt(self):
        c = np.zeros(self.W * self.H, np.int64)
        for i in self.events[self.h:]:
            c[i] += 1
        return c


def check_against_brute(W, H, pix_seq, packets, mode, q_min=1, fill=(1, 2)):
    q_max = W * H
    orc = oracle.Oracle(W, H, q_min=q_min, q_max=q_max, fill=fill, regulation=mode)
    bw = BruteWindow(W, H, q_min, q_max, fill[0], fill[1])
    pos = 0
    seen = np.zeros(W * H, bool)
    for n in packets:
        chunk = pix_seq[pos:pos + n]
        pos += n
        xs = np.array([i % W for i in chunk], np.uint16)
        ys = np.array([i // W for i in chunk], np.uint16)
        assert orc.push(xs, ys, np.ones(len(chunk), np.uint8)) == 0
        if mode == "event":
            for i in chunk:
                bw.push([i])
                P, T = bw.regulate()
        else:
            bw.push(list(chunk))
            P, T = bw.regulate()
        seen[list(chunk)] = True
        s = orc.stats()
        assert (s["h"], s["Q"], s["P"], s["T"]) == (bw.h, bw.Q, P, T)
        r = orc.readout(0)
        c = bw.cnt()
        assert np.array_equal(r["cnt"].astype(np.int64), c)
        assert np.array_equal(r["stale"] == 1, seen & (c == 0))


@pytest.mark.parametrize("W,H,length", [(2, 2, 6), (4, 2, 4)])
def test_bruteforce_exhaustive_single_event_packets(W, H, length):
    for seq in itertools.product(range(W * H), repeat=length):
        check_against_brute(W, H, list(seq), [1] * length, "event")
        check_against_brute(W, H, list(seq), [1] * length, "packet")


def test_bruteforce_exhaustive_two_packets():
    W, H = 2, 2
    for seq in itertools.product(range(4), repeat=6):
        for split in (1, 3, 5):
            check_against_brute(W, H, list(seq), [split, 6 - split], "packet")


@pytest.mark.parametrize("fill", [(1, 2), (3, 10), (7, 10), (1, 1)])
def test_bruteforce_random_long(fill):
    rng = np.random.default_rng(fill[0] * 31 + fill[1])
    W, H = 4, 4
    n = 3000
    # mildly clustered sequence so pixels go active and stale repeatedly
    pix = []
    cur = 0
    for _ in range(n):
        if rng.random() < 0.3:
            cur = int(rng.integers(0, W * H))
        pix.append(cur)
    sizes = []
    left = n
    while left:
        s = int(min(left, rng.integers(1, 40)))
        sizes.append(s)
        left -= s
    check_against_brute(W, H, pix, sizes, "packet", q_min=2, fill=fill)
    check_against_brute(W, H, pix[:600], [1] * 600, "event", q_min=2, fill=fill)


# ---------------------------------------------------------------------------
# Controller behaviour described in the paper (Spatial filtering, Fig. 4)
# ---------------------------------------------------------------------------
def test_queue_length_grows_with_fill_ratio():
    sc, ev = small_stream(150000, seed=21)
    W, H = 64, 48
    means = []
    fills = []
    for fill in [(3, 10), (1, 2), (7, 10)]:
        orc = oracle.Oracle(W, H, fill=fill, q_min=16)
        qs, rs = [], []
        for a in range(0, len(ev), 1024):
            orc.push(ev.x[a:a + 1024], ev.y[a:a + 1024], ev.p[a:a + 1024])
            if a > 30000:
                s = orc.stats()
                qs.append(s["q"])
                rs.append(s["P"] / (4.0 * s["T"]))
        means.append(np.mean(qs))
        fills.append(np.mean(rs))
    # longer queues for larger target fill ratios (paper, Fig. 4 caption)
    assert means[0] < means[1] < means[2]
    # and the observed fill ratio tracks the target
    for f, tgt in zip(fills, [0.3, 0.5, 0.7]):
        assert abs(f - tgt) < 0.12


def test_invalid_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.Oracle(0, 4)
    with pytest.raises(ValueError):
        oracle.Oracle(4, 4, t_cut=3.0)
    with pytest.raises(ValueError):
        oracle.Oracle(4, 4, fill=(3, 2))
    with pytest.raises(ValueError):
        oracle.Oracle(4, 4, q_min=100)   # q_min above q_max = 16
    orc = oracle.Oracle(4, 4, q_min=1)
    x = np.array([1, 4], np.uint16)
    y = np.array([1, 1], np.uint16)
    p = np.array([1, 1], np.uint8)
    before = orc.readout(0)
    assert orc.push(x, y, p) == oracle.E_RANGE
    assert orc.push(np.array([1, 2], np.uint16), y, np.array([1, 2], np.uint8)) == oracle.E_POLARITY
    after = orc.readout(0)
    for key in before:
        assert np.array_equal(before[key], after[key])
    assert orc.stats()["k"] == -1
    assert orc.push(np.array([1], np.uint16), np.array([1], np.uint16), p[:1],
                    np.array([100], np.uint64)) == 0
    assert orc.readout(99) == oracle.E_TIME
    assert isinstance(orc.readout(100), dict)


# ---------------------------------------------------------------------------
# Relative-threshold variant (Experiments, "Inter-pixel threshold variation";
# threshold appendix, Eq. (21)-(30))
# ---------------------------------------------------------------------------
def test_relative_thresholds_recover_the_pixels_own_thresholds():
    """A uniform triangle wave seen by pixels with thresholds of their own:
    the estimate from event counts matches C_i / C with C_i the harmonic mean
    of the pixel's ON and OFF thresholds and C the harmonic mean of all C_i
    (Eq. (23), (28)), within what one lost threshold per ramp (a reference
    level never reaches the wave's extremes exactly) and the count
    granularity allow; the spread of the true values is ten times that."""
    W, H, A, periods = 32, 24, 40.0, 5
    con, coff = eventsim.pixel_thresholds(W, H, 7)
    ev = eventsim.calibration_stream(W, H, con, coff, periods=periods, amplitude=A)
    c, c_on, c_off, n_on, n_off = oracle.relative_thresholds(ev.x, ev.y, ev.p, W, H)
    Ci = 2 * con * coff / (con + coff)
    C = 1.0 / np.mean(1.0 / Ci)
    tol = max(con.max(), coff.max()) / A + 2.0 / (n_on + n_off).min()
    assert np.abs(c / (Ci / C) - 1).max() <= tol
    assert np.abs(c_on / (con / C) - 1).max() <= tol
    assert np.abs(c_off / (coff / C) - 1).max() <= tol
    assert np.std(Ci / C) > 5 * tol
    # by construction the relative thresholds have a harmonic mean of one
    assert np.mean(1.0 / c) == pytest.approx(1.0, rel=1e-14, abs=0)


def test_relative_thresholds_of_pixels_without_events():
    x = np.array([0, 0, 1, 1, 1], np.uint16)
    y = np.array([0, 0, 0, 0, 0], np.uint16)
    p = np.array([1, 0, 1, 1, 0], np.uint8)
    c, c_on, c_off, n_on, n_off = oracle.relative_thresholds(x, y, p, 3, 1)
    mean = 5.0 / 3.0
    assert c.tolist() == [mean / 2, mean / 3, 1.0]
    assert c_on.tolist() == [0.5 * mean, 0.5 * mean / 2, 1.0]
    assert c_off.tolist() == [0.5 * mean, 0.5 * mean, 1.0]


def test_gain_multiplies_the_detrended_increment():
    """The variant multiplies the right-hand side of Eq. (6) by C'_i: pbar is
    untouched, and since L is linear in the increments and starts at zero,
    one pixel's brightness scales by its gain (temporal filter alone, and
    with the spatial filter a uniform gain scales the whole image, blurs
    included, while the window state stays the same)."""
    sc, ev = small_stream(20000, seed=31)
    W, H = 64, 48
    gain = np.full(W * H, 1.0)
    gain[5 * W + 7] = 1.7
    for spatial in (False, True):
        ref = oracle.Oracle(W, H, spatial_filter=spatial)
        one = oracle.Oracle(W, H, spatial_filter=spatial)
        var = oracle.Oracle(W, H, spatial_filter=spatial)
        assert one.set_gain(np.ones(W * H)) == 0
        assert var.set_gain(gain if not spatial else np.full(W * H, 0.8)) == 0
        for o in (ref, one, var):
            assert o.push(ev.x, ev.y, ev.p) == 0
        r, r1, rv = ref.readout(0), one.readout(0), var.readout(0)
        for key in r:
            assert np.array_equal(r[key], r1[key]), key
        assert np.array_equal(r["pbar"], rv["pbar"])
        for key in ("cnt", "last", "stale", "tcnt", "tot"):
            assert np.array_equal(r[key], rv[key]), key
        want = r["L"] * (gain if not spatial else 0.8)
        assert np.allclose(rv["L"], want, rtol=1e-12, atol=1e-14)
        assert np.abs(rv["L"] - r["L"]).max() > 1e-3


# ---------------------------------------------------------------------------
# Per-tile queues (Limitations: event queues operated separately per tile)
# ---------------------------------------------------------------------------
def test_one_tile_covering_the_sensor_is_the_single_queue():
    """A tile that covers the whole sensor, with an age limit never reached,
    is exactly FIBAR's single queue: every output after every packet."""
    sc, ev = small_stream(30000, seed=41)
    W, H = 64, 48
    one = oracle.Oracle(W, H)
    til = oracle.Oracle(W, H, region=64, age_max=1 << 62)
    for a in range(0, len(ev), 777):
        b = min(len(ev), a + 777)
        for o in (one, til):
            assert o.push(ev.x[a:b], ev.y[a:b], ev.p[a:b]) == 0
        assert til.stats() == one.stats()
        if a % (777 * 8) == 0:
            r1, r2 = one.readout(0), til.readout(0)
            for key in r1:
                assert np.array_equal(r1[key], r2[key]), key
    assert one.stats()["total_stale"] > 1000


class BruteTiles:
    """Each tile's window recounted from the list of its events after every
    packet: events leave from the front while the window is longer than the
    tile's target or its oldest event is age_max or more events old."""

    def __init__(self, W, H, R, q_min, age_max, num, den):
        self.W, self.H, self.R = W, H, R
        self.RW, self.RH = -(-W // R), -(-H // R)
        self.q_min, self.age_max, self.num, self.den = q_min, age_max, num, den
        self.win = [[] for _ in range(self.RW * self.RH)]   # (global index, pixel)
        self.npix = []
        for ry in range(self.RH):
            for rx in range(self.RW):
                self.npix.append(min(R, W - rx * R) * min(R, H - ry * R))
        self.Q = list(self.npix)
        self.k = -1

    def region(self, i):
        return (i // self.W // self.R) * self.RW + (i % self.W) // self.R

    def push(self, pixels):
        for i in pixels:
            self.k += 1
            self.win[self.region(i)].append((self.k, i))
        for r, w in enumerate(self.win):
            while w and (len(w) > self.Q[r] or self.k - w[0][0] >= self.age_max):
                w.pop(0)
            P = len(set(i for _, i in w))
            T = len(set((i // self.W // 2, (i % self.W) // 2) for _, i in w))
            if P:
                v = (len(w) * self.num * 4 * T) // (self.den * P)
                self.Q[r] = max(min(self.q_min, self.npix[r]), min(self.npix[r], v))

    def stats(self):
        q = [len(w) for w in self.win]
        P = [len(set(i for _, i in w)) for w in self.win]
        T = [len(set((i // self.W // 2, (i % self.W) // 2) for _, i in w)) for w in self.win]
        front = [w[0][0] if w else self.k + 1 for w in self.win]
        return q, list(self.Q), P, T, front

    def cnt(self):
        c = np.zeros(self.W * self.H, np.int64)
        for w in self.win:
            for _, i in w:
                c[i] += 1
        return c


@pytest.mark.parametrize("W,H,R,age", [(6, 6, 2, 40), (8, 4, 4, 1000), (7, 5, 4, 25)])
def test_tiles_against_brute_force(W, H, R, age):
    rng = np.random.default_rng(W * 10 + H + R)
    n = 2500
    pix, cur = [], 0
    for _ in range(n):
        if rng.random() < 0.3:
            cur = int(rng.integers(0, W * H))
        pix.append(cur)
    q_min = 2
    orc = oracle.Oracle(W, H, q_min=q_min, region=R, age_max=age)
    bt = BruteTiles(W, H, R, q_min, age, 1, 2)
    seen = np.zeros(W * H, bool)
    pos = 0
    while pos < n:
        m = int(min(n - pos, rng.integers(1, 30)))
        chunk = pix[pos:pos + m]
        pos += m
        xs = np.array([i % W for i in chunk], np.uint16)
        ys = np.array([i // W for i in chunk], np.uint16)
        assert orc.push(xs, ys, np.ones(m, np.uint8)) == 0
        bt.push(chunk)
        seen[chunk] = True
        rs = orc.region_stats()
        q, Q, P, T, front = bt.stats()
        assert rs["q"].tolist() == q and rs["Q"].tolist() == Q
        assert rs["P"].tolist() == P and rs["T"].tolist() == T
        assert rs["front"].tolist() == front
        r = orc.readout(0)
        c = bt.cnt()
        assert np.array_equal(r["cnt"].astype(np.int64), c)
        assert np.array_equal(r["stale"] == 1, seen & (c == 0))
        s = orc.stats()
        assert (s["q"], s["P"], s["T"]) == (sum(q), sum(P), sum(T))


def test_slow_feature_keeps_its_events_in_its_own_tile():
    """The paper's example: with one queue, a slowly moving feature's events
    are pushed out by a fast one's and it is blurred early; with a queue per
    tile the slow pixel stays active as long as its events are younger than
    the age limit."""
    W, H = 8, 8
    seq = []
    fast = [0, 1, 9, 10, 8, 2]            # a few pixels of the top-left 4x4 tile
    for e in range(6000):
        seq.append(fast[e % len(fast)] if e % 50 else 6)   # pixel (6, 0): top-right tile
    xs = np.array([i % W for i in seq], np.uint16)
    ys = np.array([i // W for i in seq], np.uint16)
    ps = np.ones(len(seq), np.uint8)
    blurred = {}
    for name, kw in (("single", {}), ("tiles", {"region": 4})):
        o = oracle.Oracle(W, H, q_min=4, **kw)
        stale_slow = 0
        for a in range(0, len(seq), 10):
            assert o.push(xs[a:a + 10], ys[a:a + 10], ps[a:a + 10]) == 0
            stale_slow += int(o.readout(0)["stale"][6])
        blurred[name] = stale_slow
    assert blurred["single"] > 100
    assert blurred["tiles"] == 0
