"""Seeded synthetic event streams with ground truth (input generator only).

This module produces the inputs that both the oracle and the GPU library are
fed: events (x uint16, y uint16, polarity uint8, t uint64 ns), ground-truth
log-intensity frames, and the push/readout schedule a harness follows.  It
holds none of the reconstruction method's arithmetic.

The event model is the paper's (Notation section, Eq. (1)-(3)): an event is
emitted whenever a pixel's log intensity crosses its ON/OFF contrast
threshold.  The recorded datasets the paper measures on are not available, so
these seeded scenes stand in for them (see `preset`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eventsim.c")
_LIB = os.path.join(_HERE, "libeventsim.so")


def build(force: bool = False) -> str:
    """Compile the simulator with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class SimParams(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("n_events", ctypes.c_uint64), ("seed", ctypes.c_uint64),
        ("n_blobs", ctypes.c_int32),
        ("amp_lo", ctypes.c_double), ("amp_hi", ctypes.c_double),
        ("sig_lo", ctypes.c_double), ("sig_hi", ctypes.c_double),
        ("checker_cell", ctypes.c_double), ("checker_contrast", ctypes.c_double),
        ("speed_px_s", ctypes.c_double), ("rot_rad_s", ctypes.c_double),
        ("thr_on", ctypes.c_double), ("thr_off", ctypes.c_double),
        ("thr_jitter", ctypes.c_double), ("noise_frac", ctypes.c_double),
        ("step_px", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.sim_generate.restype = ctypes.c_int64
        lib.sim_generate.argtypes = [ctypes.POINTER(SimParams), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_uint64)]
        lib.sim_render_frames.restype = ctypes.c_int
        lib.sim_render_frames.argtypes = [ctypes.POINTER(SimParams), ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]
        lib.sim_step_seconds.restype = ctypes.c_double
        lib.sim_step_seconds.argtypes = [ctypes.POINTER(SimParams)]
        lib.sim_philox4x32_10.restype = None
        lib.sim_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (exposed for its known-answer test)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    _load().sim_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


@dataclass
class Scene:
    width: int
    height: int
    n_events: int
    seed: int
    n_blobs: int = 32
    amp: tuple = (-1.0, 1.0)
    sigma: tuple = (2.0, 8.0)
    checker_cell: float = 0.0
    checker_contrast: float = 0.0
    speed_px_s: float = 30.0
    rot_rad_s: float = 0.0
    thr_on: float = 0.2
    thr_off: float = 0.2
    thr_jitter: float = 0.0
    noise_frac: float = 0.01
    step_px: float = 0.25

    def c_params(self) -> SimParams:
        return SimParams(self.width, self.height, self.n_events, self.seed, self.n_blobs,
                         self.amp[0], self.amp[1], self.sigma[0], self.sigma[1],
                         self.checker_cell, self.checker_contrast, self.speed_px_s,
                         self.rot_rad_s, self.thr_on, self.thr_off, self.thr_jitter,
                         self.noise_frac, self.step_px)


@dataclass
class Events:
    x: np.ndarray
    y: np.ndarray
    p: np.ndarray
    t: np.ndarray
    steps: int = 0

    def __len__(self):
        return int(self.x.shape[0])

    def slice(self, a: int, b: int) -> "Events":
        return Events(self.x[a:b], self.y[a:b], self.p[a:b], self.t[a:b])


def generate(scene: Scene, max_steps: int = 1 << 40) -> Events:
    n = int(scene.n_events)
    x = np.empty(n, np.uint16)
    y = np.empty(n, np.uint16)
    p = np.empty(n, np.uint8)
    t = np.empty(n, np.uint64)
    steps = ctypes.c_uint64(0)
    prm = scene.c_params()
    got = _load().sim_generate(ctypes.byref(prm), x.ctypes.data, y.ctypes.data, p.ctypes.data,
                               t.ctypes.data, max_steps, ctypes.byref(steps))
    if got < 0:
        raise MemoryError("event simulator failed")
    return Events(x[:got], y[:got], p[:got], t[:got], int(steps.value))


def render_frames(scene: Scene, t_ns) -> np.ndarray:
    """Ground-truth log intensity, shape (len(t_ns), H, W), float32."""
    t = np.ascontiguousarray(np.asarray(t_ns, dtype=np.uint64).reshape(-1))
    out = np.empty((t.shape[0], scene.height, scene.width), np.float32)
    prm = scene.c_params()
    if _load().sim_render_frames(ctypes.byref(prm), t.ctypes.data, t.shape[0], out.ctypes.data) != 0:
        raise MemoryError("render failed")
    return out


# --------------------------------------------------------------------------
# Workload presets.  Each stands in for a recorded dataset of the paper's
# kind (moving camera, 640x480 sensor in the paper's runtime section); the
# numbers below are the workload definitions, not measurements.
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    scene: Scene
    packet: int
    readouts: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))


def preset(name: str, n_events: int | None = None, seed: int | None = None) -> Workload:
    """Named synthetic workloads.

    sensor64x48  : 64x48, 32 blobs, 30 px/s, C=0.2, 1% noise, 1024-event
                   packets, readout every 10 000 events (200 000 events).
    vga          : 640x480, 512 blobs + 16 px checkerboard (contrast 0.5),
                   200 px/s, C = 0.2 +- 0.02 per pixel, 1% noise, 8192-event
                   packets, readout every 50 000 events (20 M events).
    hd720        : 1280x720, 2048 blobs, 0.5 rad/s rotation + 300 px/s,
                   C=0.15, 2% noise, 16384-event packets, readouts at random
                   indices with mean spacing 100 000 (100 M events).  Time
                   steps of at most 1 texel of motion keep generation of the
                   100 M-event stream to well under a minute.
    """
    if name == "sensor64x48":
        n = 200_000 if n_events is None else n_events
        sc = Scene(64, 48, n, 1 if seed is None else seed, n_blobs=32, speed_px_s=30.0,
                   thr_on=0.2, thr_off=0.2, noise_frac=0.01)
        ro = np.arange(10_000, n + 1, 10_000, dtype=np.int64)
        return Workload(name, sc, 1024, ro)
    if name == "vga":
        n = 20_000_000 if n_events is None else n_events
        sc = Scene(640, 480, n, 2 if seed is None else seed, n_blobs=512, checker_cell=16.0,
                   checker_contrast=0.5, speed_px_s=200.0, thr_on=0.2, thr_off=0.2,
                   thr_jitter=0.02, noise_frac=0.01)
        ro = np.arange(50_000, n + 1, 50_000, dtype=np.int64)
        return Workload(name, sc, 8192, ro)
    if name == "hd720":
        n = 100_000_000 if n_events is None else n_events
        sd = 3 if seed is None else seed
        sc = Scene(1280, 720, n, sd, n_blobs=2048, speed_px_s=300.0, rot_rad_s=0.5,
                   thr_on=0.15, thr_off=0.15, noise_frac=0.02, step_px=1.0)
        nro = max(1, n // 100_000)
        rng = np.random.default_rng(1000 + sd)
        ro = np.sort(rng.choice(np.arange(1, n, dtype=np.int64), size=min(nro, n - 1),
                                replace=False)) if n > 1 else np.zeros(0, np.int64)
        return Workload(name, sc, 16384, ro)
    raise KeyError(name)


def schedule(n_events: int, packet: int, readouts) -> list:
    """Push/readout schedule: a list of ("push", a, b) and ("read", k) items.

    Packets are consecutive runs of `packet` events; a readout index r (the
    number of events applied before the readout) that falls inside a packet
    splits that packet in two, so every consumer sees the same pushes.
    """
    ro = sorted(set(int(r) for r in readouts if 0 < int(r) <= n_events))
    out = []
    ri = 0
    a = 0
    while a < n_events:
        b = min(a + packet, n_events)
        while ri < len(ro) and ro[ri] <= b:
            r = ro[ri]
            if r > a:
                out.append(("push", a, r))
                a = r
            out.append(("read", r))
            ri += 1
        if b > a:
            out.append(("push", a, b))
        a = b
    return out


# --------------------------------------------------------------------------
# Calibration recording for relative contrast thresholds: a spatially uniform
# screen whose log brightness is a triangle wave (the threshold appendix's
# set-up), seen by pixels with thresholds of their own.
# --------------------------------------------------------------------------
def pixel_thresholds(width: int, height: int, seed: int, thr: float = 0.2, jitter: float = 0.02):
    """Per-pixel ON and OFF thresholds, uniform over [thr - jitter, thr + jitter],
    drawn independently (FP64, [H * W] each)."""
    rng = np.random.default_rng(seed)
    n = width * height
    return (rng.uniform(thr - jitter, thr + jitter, n), rng.uniform(thr - jitter, thr + jitter, n))


def calibration_stream(width: int, height: int, c_on, c_off, periods: int = 20,
                       amplitude: float = 2.0, period_ns: int = 1_000_000_000) -> Events:
    """Events of `periods` periods of a uniform triangle wave of log brightness
    (0 -> amplitude -> 0, one period per `period_ns`): each pixel emits an ON
    event when the brightness has risen by its c_on above its reference
    level and an OFF event when it has fallen by its c_off below it, the
    reference moving by one threshold per event.  Event times are the exact
    crossing times; events are ordered by (time, pixel)."""
    npx = width * height
    c_on = np.asarray(c_on, np.float64)
    c_off = np.asarray(c_off, np.float64)
    ref = np.zeros(npx)
    half = period_ns / 2.0
    slope = amplitude / half
    pix_all, t_all, p_all = [], [], []
    idx = np.arange(npx)
    for per in range(periods):
        t0 = per * period_ns
        for rising in (True, False):
            c = c_on if rising else c_off
            nmax = int(np.ceil(amplitude / c.min())) + 2
            m = np.arange(1, nmax + 1)[None, :]
            if rising:
                lvl = ref[:, None] + m * c[:, None]
                ok = lvl <= amplitude
                tt = t0 + lvl / slope
            else:
                lvl = ref[:, None] - m * c[:, None]
                ok = lvl >= 0.0
                tt = t0 + half + (amplitude - lvl) / slope
            cnt = ok.sum(axis=1)
            ref = ref + (cnt * c if rising else -cnt * c)
            pix_all.append(np.broadcast_to(idx[:, None], ok.shape)[ok])
            t_all.append(tt[ok])
            p_all.append(np.full(int(cnt.sum()), 1 if rising else 0, np.uint8))
    pix = np.concatenate(pix_all)
    t = np.round(np.concatenate(t_all)).astype(np.uint64)
    p = np.concatenate(p_all)
    order = np.lexsort((pix, t))
    pix, t, p = pix[order], t[order], p[order]
    return Events((pix % width).astype(np.uint16), (pix // width).astype(np.uint16), p, t)


# --------------------------------------------------------------------------
# Many streams of uneven resolution and rate.
# --------------------------------------------------------------------------
RESOLUTIONS = ((346, 260), (640, 480), (1280, 720))


def batched_streams(n_streams: int = 16, meta_seed: int = 4, scale: float = 1.0):
    """Workloads of `n_streams` independent streams (meta seed 4, stream
    seeds 400 + i): resolution uniform over 346x260 / 640x480 / 1280x720,
    event rate log-uniform over 1-50 Mev/s, length uniform over 5-40 M
    events (times `scale`), scene as the vga preset, packet size
    clamp(nextpow2(rate x 1 ms), 1024, 32768)."""
    rng = np.random.default_rng(meta_seed)
    out = []
    for i in range(n_streams):
        W, H = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        rate = float(np.exp(rng.uniform(np.log(1e6), np.log(50e6))))
        length = int(rng.integers(5_000_000, 40_000_001) * scale)
        packet = 1 << int(np.ceil(np.log2(max(rate * 1e-3, 1.0))))
        packet = int(min(max(packet, 1024), 32768))
        n_blobs = max(32, int(512 * W * H / (640 * 480)))
        sc = Scene(W, H, max(length, 1), 400 + i, n_blobs=n_blobs, checker_cell=16.0,
                   checker_contrast=0.5, speed_px_s=200.0, thr_on=0.2, thr_off=0.2,
                   thr_jitter=0.02, noise_frac=0.01)
        out.append(Workload("stream%02d_%dx%d" % (i, W, H), sc, packet,
                            np.zeros(0, np.int64)))
        out[-1].rate = rate
    return out


# --------------------------------------------------------------------------
# Inputs of the learned stale fill: seeded initial parameters, the training
# target and the quality score.  None of this is the fill's arithmetic (the
# network lives in the library and in the oracle); these are the random draws
# and the evaluation protocol both sides are given.
# --------------------------------------------------------------------------
FILL_CHANNELS = (3, 16, 16, 16, 1)


def fill_init_params(seed: int, zero_last: bool = True) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / (9 Cin))), zero biases, as one
    flat FP32 vector in layer order, w in [Cout][Cin][3][3] then b.  With
    zero_last the last layer starts at zero, so the untrained fill is the
    Gaussian fill itself."""
    rng = np.random.default_rng(seed)
    parts = []
    layers = list(zip(FILL_CHANNELS[:-1], FILL_CHANNELS[1:]))
    for k, (cin, cout) in enumerate(layers):
        std = np.sqrt(2.0 / (9 * cin))
        w = rng.normal(0.0, std, size=cout * cin * 9)
        if zero_last and k == len(layers) - 1:
            w[:] = 0.0
        parts.append(w)
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def fill_scene(seed: int, n_events: int = 2_000_000) -> Scene:
    """A 1280x720 training / evaluation sequence of the learned fill: the hd720
    preset's scene (2048 blobs, 0.5 rad/s + 300 px/s, C = 0.15, 2 % noise)
    with its own seed (training seeds 5000-5199, evaluation 6000-6019)."""
    return Scene(1280, 720, n_events, seed, n_blobs=2048, speed_px_s=300.0, rot_rad_s=0.5,
                 thr_on=0.15, thr_off=0.15, noise_frac=0.02, step_px=1.0)


def fill_target(gt, L, active):
    """Ground truth in the units of the reconstruction: the least-squares
    affine map of a frame's ground-truth log intensity onto its brightness L,
    fitted on the frame's active pixels (there the reconstruction follows the
    scene), applied to the whole frame.  gt, L: [H, W]; active: bool [H, W]."""
    g = np.asarray(gt, np.float64)[active]
    l = np.asarray(L, np.float64)[active]
    if g.size < 2 or np.var(g) == 0:
        return np.zeros_like(np.asarray(gt, np.float32))
    a = np.cov(g, l, bias=True)[0, 1] / np.var(g)
    b = l.mean() - a * g.mean()
    return (a * np.asarray(gt, np.float64) + b).astype(np.float32)


def fill_psnr(img, target, mask):
    """PSNR (dB) of img against target over mask; the peak is the target's
    range over the frame."""
    m = np.asarray(mask) != 0
    t = np.asarray(target, np.float64)
    err = np.asarray(img, np.float64)[m] - t[m]
    mse = float(np.mean(err * err)) if err.size else 0.0
    peak = float(t.max() - t.min())
    if mse == 0.0 or peak == 0.0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)
