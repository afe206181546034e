"""FP64 CPU oracle of FIBAR (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the GPU path: it is a separate C file compiled with
gcc, driven through ctypes.

``Oracle`` wraps one reconstruction context; ``run_schedule`` feeds it the
push/readout schedule a harness uses so that the GPU path and the oracle see
identical packet boundaries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fibar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID_ARG, E_RANGE, E_POLARITY, E_TIME, E_NOMEM = 0, -1, -2, -3, -4, -5
REG_PACKET, REG_EVENT = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle: -O2, no fast-math, single thread."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math",
                               "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class RefParams(ctypes.Structure):
    _fields_ = [("t_cut", ctypes.c_double), ("fill_num", ctypes.c_uint32),
                ("fill_den", ctypes.c_uint32), ("q_min", ctypes.c_uint32),
                ("q_max", ctypes.c_uint32), ("spatial_filter", ctypes.c_uint32),
                ("regulation", ctypes.c_uint32), ("region", ctypes.c_uint32),
                ("age_max", ctypes.c_uint64)]


class RefStats(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("h", ctypes.c_uint64), ("q", ctypes.c_uint64),
                ("Q", ctypes.c_uint64), ("P", ctypes.c_uint64), ("T", ctypes.c_uint64),
                ("n_regulations", ctypes.c_uint64), ("last_stale", ctypes.c_uint64),
                ("total_stale", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp = ctypes.c_void_p
        lib.fibar_ref_default_params.argtypes = [ctypes.POINTER(RefParams)]
        lib.fibar_ref_create.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.POINTER(RefParams), ctypes.POINTER(vp)]
        lib.fibar_ref_push_events.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t]
        lib.fibar_ref_readout.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, vp, vp]
        lib.fibar_ref_get_stats.argtypes = [vp, ctypes.POINTER(RefStats)]
        lib.fibar_ref_destroy.argtypes = [vp]
        lib.fibar_ref_destroy.restype = None
        lib.fibar_ref_coefficients.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]
        lib.fibar_ref_coefficients.restype = None
        lib.fibar_ref_set_gain.argtypes = [vp, vp]
        lib.fibar_ref_region_stats.argtypes = [vp, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def coefficients(t_cut: float):
    """(alpha, beta) of Eq. (17)-(18) as the oracle computes them."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().fibar_ref_coefficients(float(t_cut), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def _ptr(a):
    return None if a is None else a.ctypes.data


class Oracle:
    """One FP64 reconstruction context."""

    def __init__(self, width, height, t_cut=40.0, fill=(1, 2), q_min=64, q_max=0,
                 spatial_filter=True, regulation="packet", region=0, age_max=0):
        lib = _load()
        prm = RefParams()
        lib.fibar_ref_default_params(ctypes.byref(prm))
        prm.t_cut = float(t_cut)
        prm.fill_num, prm.fill_den = int(fill[0]), int(fill[1])
        prm.q_min = int(q_min)
        prm.q_max = int(q_max)
        prm.spatial_filter = 1 if spatial_filter else 0
        prm.regulation = REG_EVENT if regulation == "event" else REG_PACKET
        prm.region = int(region)
        prm.age_max = int(age_max)
        h = ctypes.c_void_p()
        rc = lib.fibar_ref_create(int(width), int(height), ctypes.byref(prm), ctypes.byref(h))
        if rc != OK:
            raise ValueError("fibar_ref_create failed: %d" % rc)
        self._h = h
        self.width, self.height = int(width), int(height)
        self.tiles_w, self.tiles_h = (self.width + 1) // 2, (self.height + 1) // 2
        self.spatial_filter = bool(spatial_filter)
        self.region = int(region)
        if self.region:
            self.regions_w = (self.width + self.region - 1) // self.region
            self.regions_h = (self.height + self.region - 1) // self.region

    def close(self):
        if self._h:
            _load().fibar_ref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, x, y, p, t=None) -> int:
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        p = np.ascontiguousarray(p, np.uint8)
        t = None if t is None else np.ascontiguousarray(t, np.uint64)
        n = int(x.shape[0])
        if y.shape[0] != n or p.shape[0] != n or (t is not None and t.shape[0] != n):
            raise ValueError("ragged packet")
        return _load().fibar_ref_push_events(self._h, _ptr(x), _ptr(y), _ptr(p), _ptr(t), n)

    def readout(self, t: int = 0):
        npx = self.width * self.height
        out = {
            "L": np.empty(npx, np.float64), "pbar": np.empty(npx, np.float64),
            "cnt": np.empty(npx, np.uint32), "tot": np.empty(npx, np.uint64),
            "last": np.empty(npx, np.int64),
            "tcnt": np.empty(self.tiles_w * self.tiles_h, np.uint32),
            "stale": np.empty(npx, np.uint8),
        }
        rc = _load().fibar_ref_readout(self._h, int(t), _ptr(out["L"]), _ptr(out["pbar"]),
                                       _ptr(out["cnt"]), _ptr(out["tot"]), _ptr(out["last"]),
                                       _ptr(out["tcnt"]), _ptr(out["stale"]))
        if rc != OK:
            return rc
        return out

    def set_gain(self, gain) -> int:
        """Per-pixel multipliers of Eq. (6) (the relative thresholds C'_i);
        None removes them."""
        if gain is None:
            return _load().fibar_ref_set_gain(self._h, None)
        g = np.ascontiguousarray(gain, np.float64).reshape(-1)
        if g.shape[0] != self.width * self.height:
            raise ValueError("one gain per pixel")
        return _load().fibar_ref_set_gain(self._h, g.ctypes.data)

    def region_stats(self) -> dict:
        """Per-tile scalars (per-tile queues): q, Q, P, T and the global index
        of each tile's oldest window event (k + 1 if empty), row-major."""
        n = self.regions_w * self.regions_h
        out = {k: np.empty(n, np.uint64) for k in ("q", "Q", "P", "T", "front")}
        rc = _load().fibar_ref_region_stats(self._h, *(out[k].ctypes.data for k in
                                                         ("q", "Q", "P", "T", "front")))
        if rc != OK:
            raise ValueError("not a per-tile-queue oracle")
        return out

    def stats(self) -> dict:
        s = RefStats()
        _load().fibar_ref_get_stats(self._h, ctypes.byref(s))
        return s.as_dict()


def relative_thresholds(x, y, p, width, height):
    """Relative contrast thresholds from the events of a calibration recording
    (threshold appendix, Eq. (21)-(30)): with N_on_i, N_off_i the ON and OFF
    events of pixel i and N_tot the mean over all pixels of N_on_i + N_off_i,
    C'_i = N_tot / (N_on_i + N_off_i) and C'_on_i = N_tot / (2 N_on_i),
    C'_off_i = N_tot / (2 N_off_i).  Reading: a pixel without events of a
    kind gets 1 for the ratios that would divide by zero.  FP64.  Returns
    (c_rel, c_on_rel, c_off_rel, n_on, n_off)."""
    npx = int(width) * int(height)
    pix = np.asarray(y, np.int64) * int(width) + np.asarray(x, np.int64)
    on = np.asarray(p) != 0
    n_on = np.bincount(pix[on], minlength=npx).astype(np.int64)
    n_off = np.bincount(pix[~on], minlength=npx).astype(np.int64)
    n_tot = n_on + n_off
    mean = n_tot.sum() / npx
    with np.errstate(divide="ignore"):
        c = np.where(n_tot > 0, mean / np.maximum(n_tot, 1), 1.0)
        c_on = np.where(n_on > 0, 0.5 * mean / np.maximum(n_on, 1), 1.0)
        c_off = np.where(n_off > 0, 0.5 * mean / np.maximum(n_off, 1), 1.0)
    return c, c_on, c_off, n_on, n_off


def run_schedule(orc: Oracle, ev, sched, on_read=None, on_push=None):
    """Feed `sched` (from eventsim.schedule) to `orc`.

    on_push(item, status) is called after each push, on_read(k, readout)
    at each readout.  Returns the list of readouts.
    """
    reads = []
    for item in sched:
        if item[0] == "push":
            a, b = item[1], item[2]
            rc = orc.push(ev.x[a:b], ev.y[a:b], ev.p[a:b], ev.t[a:b])
            if rc != OK:
                raise RuntimeError("oracle push failed: %d" % rc)
            if on_push is not None:
                on_push(item, orc)
        else:
            k = item[1]
            tt = int(ev.t[k - 1]) if k > 0 else 0
            r = orc.readout(tt)
            if on_read is not None:
                on_read(k, r)
            else:
                reads.append((k, r))
    return reads
