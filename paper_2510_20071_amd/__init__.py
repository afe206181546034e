"""Python binding of libfibar (FIBAR event-camera reconstruction on MI355X).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``libfibar.so`` behind the C ABI of ``include/fibar.h``.  The
functions below carry the C names.  Device buffers are passed as raw
pointers (for example ``tensor.data_ptr()`` of a torch tensor on the GPU);
host buffers as numpy arrays.

Importing this package does not need a GPU.  Using it does: if the library
has not been built, ``load()`` raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfibar.so")

FIBAR_OK = 0
FIBAR_E_INVALID_ARG = -1
FIBAR_E_RANGE = -2
FIBAR_E_POLARITY = -3
FIBAR_E_TIME = -4
FIBAR_E_NOMEM = -5
FIBAR_E_DEVICE = -6
FIBAR_E_UNSUPPORTED = -7
FIBAR_REG_PACKET = 0
FIBAR_REG_EVENT = 1
FIBAR_OP_PUSH = 0
FIBAR_LAUNCH_DIRECT = 0
FIBAR_LAUNCH_GRAPH = 1
FIBAR_OP_READOUT = 1


class FibarError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what or "fibar", _status_text(status), status))


class fibar_params(ctypes.Structure):
    _fields_ = [("t_cut", ctypes.c_double), ("fill_num", ctypes.c_uint32),
                ("fill_den", ctypes.c_uint32), ("q_min", ctypes.c_uint32),
                ("q_max", ctypes.c_uint32), ("spatial_filter", ctypes.c_uint32),
                ("regulation", ctypes.c_uint32), ("max_packet", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("region", ctypes.c_uint32),
                ("age_max", ctypes.c_uint64)]


class fibar_packet(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("p", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("n", ctypes.c_size_t), ("on_device", ctypes.c_int)]


class fibar_readout_buf(ctypes.Structure):
    _fields_ = [("brightness", ctypes.c_void_p), ("pbar", ctypes.c_void_p),
                ("stale_mask", ctypes.c_void_p), ("active_count", ctypes.c_void_p),
                ("last_index", ctypes.c_void_p), ("log_age", ctypes.c_void_p),
                ("tile_count", ctypes.c_void_p), ("total_count", ctypes.c_void_p),
                ("on_device", ctypes.c_int)]


class fibar_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("packet", fibar_packet), ("t", ctypes.c_uint64),
                ("readout", fibar_readout_buf)]


class fibar_stats(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("h", ctypes.c_uint64), ("q", ctypes.c_uint64),
                ("Q", ctypes.c_uint64), ("P", ctypes.c_uint64), ("T", ctypes.c_uint64),
                ("n_regulations", ctypes.c_uint64), ("last_stale", ctypes.c_uint64),
                ("total_stale", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


# name -> (restype, argtypes); every function declared in include/fibar.h
_SIGNATURES = {
    "fibar_default_params": (None, [ctypes.POINTER(fibar_params)]),
    "fibar_create": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(fibar_params),
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "fibar_push_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(fibar_packet)]),
    "fibar_readout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.POINTER(fibar_readout_buf)]),
    "fibar_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(fibar_op), ctypes.c_size_t]),
    "fibar_destroy": (None, [ctypes.c_void_p]),
    "fibar_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(fibar_stats)]),
    "fibar_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "fibar_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fibar_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "fibar_set_kernel_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "fibar_kernel_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "fibar_set_launch_mode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fibar_set_telemetry": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "fibar_count_polarities": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fibar_relative_thresholds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                                 ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p]),
    "fibar_set_pixel_gain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fibar_tile_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

_SIGNATURES.update({
    "fibar_multi_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "fibar_multi_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.POINTER(fibar_op)),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "fibar_multi_autotune": (ctypes.c_int, [ctypes.c_void_p]),
    "fibar_multi_get_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32)]),
    "fibar_multi_get_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "fibar_multi_set_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fibar_multi_destroy": (None, [ctypes.c_void_p]),
})

# include/fibar_fill.h
FILL_PARAMS = 5233
_FP = ctypes.POINTER(ctypes.c_float)
_SIGNATURES.update({
    "fibar_fill_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "fibar_fill_set_params": (ctypes.c_int, [ctypes.c_void_p, _FP]),
    "fibar_fill_get_params": (ctypes.c_int, [ctypes.c_void_p, _FP]),
    "fibar_fill_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_void_p]),
    "fibar_fill_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_uint32, _FP, _FP]),
    "fibar_fill_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_float,
                                             _FP]),
    "fibar_fill_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "fibar_fill_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_uint32, ctypes.c_float,
                                                ctypes.c_void_p,
                                                ctypes.POINTER(ctypes.c_uint32)]),
    "fibar_fill_destroy": (None, [ctypes.c_void_p]),
})
FILL_NOALLOC_MAX_PIXELS = 1 << 20

KERNEL_NAMES = ("group_compose", "apply", "pop_blur", "pop_blur_readout", "readout")

_lib = None


def load():
    """Load libfibar.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfibar.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2510_20071_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_text(status: int) -> str:
    try:
        return load().fibar_status_string(int(status)).decode()
    except Exception:
        return "status"


# ---- same-name wrappers of the C ABI ---------------------------------------
def fibar_default_params() -> fibar_params:
    p = fibar_params()
    load().fibar_default_params(ctypes.byref(p))
    return p


def fibar_create(width: int, height: int, params: fibar_params | None = None):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    rc = load().fibar_create(int(width), int(height),
                             None if params is None else ctypes.byref(params), ctypes.byref(h))
    return rc, h


def fibar_push_events(handle, packet: fibar_packet) -> int:
    return load().fibar_push_events(handle, ctypes.byref(packet))


def fibar_readout(handle, t: int, buf: fibar_readout_buf) -> int:
    return load().fibar_readout(handle, int(t), ctypes.byref(buf))


def fibar_submit(handle, ops) -> int:
    arr = (fibar_op * len(ops))(*ops)
    return load().fibar_submit(handle, arr, len(ops))


def fibar_destroy(handle) -> None:
    load().fibar_destroy(handle)


def fibar_get_stats(handle):
    """Returns (status, stats dict)."""
    s = fibar_stats()
    rc = load().fibar_get_stats(handle, ctypes.byref(s))
    return rc, s.as_dict()


def fibar_synchronize(handle) -> int:
    return load().fibar_synchronize(handle)


def fibar_status_string(status: int) -> str:
    return _status_text(status)


def fibar_reset(handle) -> int:
    return load().fibar_reset(handle)


def fibar_set_kernel_timing(handle, kernel_mask: int, every: int = 1) -> int:
    return load().fibar_set_kernel_timing(handle, int(kernel_mask), int(every))


def fibar_set_telemetry(handle, records, capacity: int) -> int:
    """records: a device buffer of capacity * STEP_RECORD_WORDS int64 (or None)."""
    return load().fibar_set_telemetry(handle, _addr(records), int(capacity))


def fibar_count_polarities(x, y, p, width, height, n_on, n_off, stream=None) -> int:
    """Device arrays: events x, y (uint16 / int16), p (uint8); counters n_on,
    n_off (int32 / uint32, width*height each), which receive the counts."""
    return load().fibar_count_polarities(_addr(x), _addr(y), _addr(p), int(x.shape[0]),
                                         int(width), int(height), _addr(n_on), _addr(n_off),
                                         stream)


def fibar_relative_thresholds(n_on, n_off, width, height, c_rel, c_on_rel=None, c_off_rel=None,
                              stream=None) -> int:
    return load().fibar_relative_thresholds(_addr(n_on), _addr(n_off), int(width), int(height),
                                            _addr(c_rel), _addr(c_on_rel), _addr(c_off_rel),
                                            stream)


def fibar_tile_stats(handle, n_tiles):
    """Per-tile scalars of a per-tile-queue context: (status, dict of q, Q, P,
    T, front arrays)."""
    out = {k: np.empty(int(n_tiles), np.uint64) for k in ("q", "Q", "P", "T", "front")}
    rc = load().fibar_tile_stats(handle, *(out[k].ctypes.data for k in ("q", "Q", "P", "T",
                                                                          "front")))
    return rc, out


def fibar_set_pixel_gain(handle, gain) -> int:
    """gain: a device float buffer of width*height values, or None."""
    return load().fibar_set_pixel_gain(handle, _addr(gain))


STEP_RECORD_FIELDS = ("k", "h", "q", "Q", "P", "T", "stale", "n")
STEP_RECORD_WORDS = len(STEP_RECORD_FIELDS)


def fibar_set_launch_mode(handle, mode: int) -> int:
    return load().fibar_set_launch_mode(handle, int(mode))


def fibar_kernel_time(handle, kernel: int):
    """Returns (status, total_ms, launches)."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    rc = load().fibar_kernel_time(handle, int(kernel), ctypes.byref(ms), ctypes.byref(n))
    return rc, ms.value, int(n.value)


def fibar_multi_create(handles, stream=None):
    """Returns (status, group handle)."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    out = ctypes.c_void_p()
    rc = load().fibar_multi_create(arr, len(handles), stream, ctypes.byref(out))
    return rc, out


class OpLists:
    """Op lists marshalled once for repeated fibar_multi_submit calls."""

    def __init__(self, op_lists):
        self.arrays = [(fibar_op * len(ops))(*ops) for ops in op_lists]
        self.ptrs = (ctypes.POINTER(fibar_op) * len(self.arrays))(
            *[ctypes.cast(a, ctypes.POINTER(fibar_op)) for a in self.arrays])
        self.sizes = (ctypes.c_size_t * len(self.arrays))(*[len(ops) for ops in op_lists])


def fibar_multi_submit(group, op_lists) -> int:
    """op_lists: one list of fibar_op per context of the group, or OpLists."""
    if not isinstance(op_lists, OpLists):
        op_lists = OpLists(op_lists)
    return load().fibar_multi_submit(group, op_lists.ptrs, op_lists.sizes)


def fibar_multi_autotune(group) -> int:
    return load().fibar_multi_autotune(group)


def fibar_multi_get_shape(group):
    """Returns (status, block, grid)."""
    b, g = ctypes.c_uint32(), ctypes.c_uint32()
    rc = load().fibar_multi_get_shape(group, ctypes.byref(b), ctypes.byref(g))
    return rc, int(b.value), int(g.value)


def fibar_multi_get_config(group):
    """Returns (status, candidate index)."""
    i = ctypes.c_uint32()
    rc = load().fibar_multi_get_config(group, ctypes.byref(i))
    return rc, i.value


MULTI_CONFIGS = 10   # launch configurations of a group (see fibar_multi_set_shape)


def fibar_multi_set_shape(group, index: int) -> int:
    return load().fibar_multi_set_shape(group, int(index))


def fibar_multi_destroy(group) -> None:
    load().fibar_multi_destroy(group)


# ---- convenience layer used by the tests and the benchmark -----------------
def _addr(a):
    """Pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())


def make_packet(x, y, p, t=None, on_device=None) -> fibar_packet:
    n = int(x.shape[0])
    if on_device is None:
        on_device = 0 if isinstance(x, np.ndarray) else 1
    return fibar_packet(_addr(x), _addr(y), _addr(p), _addr(t), n, int(on_device))


class Context:
    """One reconstruction context (owns its device state)."""

    def __init__(self, width, height, t_cut=40.0, fill=(1, 2), q_min=64, q_max=0,
                 spatial_filter=True, max_packet=65536, stream=None, regulation="packet",
                 region=0, age_max=0):
        prm = fibar_default_params()
        prm.region = int(region)
        prm.age_max = int(age_max)
        prm.regulation = FIBAR_REG_EVENT if regulation == "event" else FIBAR_REG_PACKET
        prm.t_cut = float(t_cut)
        prm.fill_num, prm.fill_den = int(fill[0]), int(fill[1])
        prm.q_min = int(q_min)
        prm.q_max = int(q_max)
        prm.spatial_filter = 1 if spatial_filter else 0
        prm.max_packet = int(max_packet)
        prm.stream = stream
        rc, h = fibar_create(width, height, prm)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_create")
        self.handle = h
        self.width, self.height = int(width), int(height)
        self.tiles = ((self.width + 1) // 2) * ((self.height + 1) // 2)
        self.spatial_filter = bool(spatial_filter)
        self.region = int(region)
        if self.region:
            self.tiles_x = -(-self.width // self.region)
            self.tiles_y = -(-self.height // self.region)

    def tile_stats(self):
        """Per-tile q, Q, P, T and window fronts (per-tile queues)."""
        rc, out = fibar_tile_stats(self.handle, self.tiles_x * self.tiles_y)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_tile_stats")
        return out

    def close(self):
        if getattr(self, "handle", None):
            fibar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, x, y, p, t=None) -> int:
        return fibar_push_events(self.handle, make_packet(x, y, p, t))

    def readout_host(self, t=0, spatial_outputs=None):
        """Read everything into numpy arrays (synchronises); returns dict or status."""
        npx = self.width * self.height
        sp = self.spatial_filter if spatial_outputs is None else spatial_outputs
        out = {"L": np.empty(npx, np.float32), "pbar": np.empty(npx, np.float32),
               "last": np.empty(npx, np.int64), "log_age": np.empty(npx, np.float32)}
        out["tot"] = np.empty(npx, np.uint64)
        if sp:
            out.update(stale=np.empty(npx, np.uint8), cnt=np.empty(npx, np.uint32),
                       tcnt=np.empty(self.tiles, np.uint32))
        buf = fibar_readout_buf(_addr(out["L"]), _addr(out["pbar"]), _addr(out.get("stale")),
                                _addr(out.get("cnt")), _addr(out["last"]),
                                _addr(out["log_age"]), _addr(out.get("tcnt")),
                                _addr(out["tot"]), 0)
        rc = fibar_readout(self.handle, t, buf)
        if rc != FIBAR_OK:
            return rc
        return out

    def readout_device(self, t, L, pbar=None, stale=None, cnt=None, last=None, log_age=None,
                       tcnt=None, tot=None) -> int:
        buf = fibar_readout_buf(_addr(L), _addr(pbar), _addr(stale), _addr(cnt), _addr(last),
                                _addr(log_age), _addr(tcnt), _addr(tot), 1)
        return fibar_readout(self.handle, t, buf)

    def set_gain(self, gain) -> int:
        return fibar_set_pixel_gain(self.handle, gain)

    def set_telemetry(self, records, capacity: int) -> int:
        return fibar_set_telemetry(self.handle, records, capacity)

    def stats(self):
        rc, s = fibar_get_stats(self.handle)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_get_stats")
        return s

    def synchronize(self) -> int:
        return fibar_synchronize(self.handle)

    def submit(self, ops) -> int:
        return fibar_submit(self.handle, ops)

    def reset(self) -> int:
        return fibar_reset(self.handle)


def push_op(x, y, p, t=None, on_device=None) -> fibar_op:
    op = fibar_op()
    op.kind = FIBAR_OP_PUSH
    op.packet = make_packet(x, y, p, t, on_device)
    return op


def readout_op(t, L, pbar=None, stale=None, cnt=None, last=None, log_age=None, tcnt=None,
               on_device=1, tot=None) -> fibar_op:
    op = fibar_op()
    op.kind = FIBAR_OP_READOUT
    op.t = int(t)
    op.readout = fibar_readout_buf(_addr(L), _addr(pbar), _addr(stale), _addr(cnt), _addr(last),
                                   _addr(log_age), _addr(tcnt), _addr(tot), int(on_device))
    return op


class Group:
    """Several contexts advanced together (fibar_multi_*)."""

    def __init__(self, contexts, stream=None):
        rc, h = fibar_multi_create([c.handle for c in contexts], stream)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_multi_create")
        self.handle = h
        self.contexts = list(contexts)

    def submit(self, op_lists) -> int:
        return fibar_multi_submit(self.handle, op_lists)

    def autotune(self) -> int:
        return fibar_multi_autotune(self.handle)

    def shape(self):
        rc, b, g = fibar_multi_get_shape(self.handle)
        return b, g

    def config(self) -> int:
        rc, i = fibar_multi_get_config(self.handle)
        return i

    def set_shape(self, index) -> int:
        return fibar_multi_set_shape(self.handle, index)

    def close(self):
        if getattr(self, "handle", None):
            fibar_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fibar_fill_create(stream=None):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    rc = load().fibar_fill_create(stream, ctypes.byref(h))
    return rc, h


def fibar_fill_set_params(handle, params) -> int:
    a = np.ascontiguousarray(params, dtype=np.float32)
    return load().fibar_fill_set_params(handle, a.ctypes.data_as(_FP))


def fibar_fill_get_params(handle):
    """Returns (status, params)."""
    a = np.empty(FILL_PARAMS, np.float32)
    rc = load().fibar_fill_get_params(handle, a.ctypes.data_as(_FP))
    return rc, a


def fibar_fill_predict(handle, L, stale, log_age, n, H, W, pred) -> int:
    return load().fibar_fill_predict(handle, _addr(L), _addr(stale), _addr(log_age), n, H, W,
                                     _addr(pred))


def fibar_fill_loss_grad(handle, L, stale, log_age, target, n, H, W, want_grad=True):
    """Returns (status, loss, grad or None)."""
    loss = ctypes.c_float()
    g = np.empty(FILL_PARAMS, np.float32) if want_grad else None
    rc = load().fibar_fill_loss_grad(handle, _addr(L), _addr(stale), _addr(log_age),
                                     _addr(target), n, H, W, ctypes.byref(loss),
                                     g.ctypes.data_as(_FP) if g is not None else None)
    return rc, float(loss.value), g


def fibar_fill_train_step(handle, L, stale, log_age, target, n, H, W, lr, want_loss=True):
    """Returns (status, loss before the step or None)."""
    loss = ctypes.c_float()
    rc = load().fibar_fill_train_step(handle, _addr(L), _addr(stale), _addr(log_age),
                                      _addr(target), n, H, W, float(lr),
                                      ctypes.byref(loss) if want_loss else None)
    return rc, (float(loss.value) if want_loss else None)


def fibar_fill_apply(handle, L, stale, log_age, H, W, tile, theta, out):
    """Returns (status, tiles with stale pixels that kept L)."""
    fb = ctypes.c_uint32()
    rc = load().fibar_fill_apply(handle, _addr(L), _addr(stale), _addr(log_age), H, W, int(tile),
                                 float(theta), _addr(out), ctypes.byref(fb))
    return rc, int(fb.value)


def fibar_fill_apply_noalloc(handle, L, stale, log_age, H, W, tile, theta, out):
    """Returns (status, tiles with stale pixels that kept L)."""
    fb = ctypes.c_uint32()
    rc = load().fibar_fill_apply_noalloc(handle, _addr(L), _addr(stale), _addr(log_age), H, W,
                                         int(tile), float(theta), _addr(out), ctypes.byref(fb))
    return rc, int(fb.value)


def fibar_fill_destroy(handle) -> None:
    load().fibar_fill_destroy(handle)


class Fill:
    """Learned stale fill (fibar_fill_*).  Image arguments are device tensors
    of [n,] H x W (float32 L, log_age, target and outputs; uint8 stale)."""

    def __init__(self, params=None, stream=None):
        rc, h = fibar_fill_create(stream)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_fill_create")
        self.handle = h
        if params is not None:
            rc = self.set_params(params)
            if rc != FIBAR_OK:
                raise FibarError(rc, "fibar_fill_set_params")

    def set_params(self, params) -> int:
        assert np.asarray(params).shape == (FILL_PARAMS,)
        return fibar_fill_set_params(self.handle, params)

    def get_params(self):
        rc, a = fibar_fill_get_params(self.handle)
        if rc != FIBAR_OK:
            raise FibarError(rc, "fibar_fill_get_params")
        return a

    @staticmethod
    def _dims(L):
        shp = tuple(L.shape)
        return (1,) + shp if len(shp) == 2 else shp

    def predict(self, L, stale, log_age, out) -> int:
        return fibar_fill_predict(self.handle, L, stale, log_age, *self._dims(L), out)

    def loss_grad(self, L, stale, log_age, target, want_grad=True):
        return fibar_fill_loss_grad(self.handle, L, stale, log_age, target, *self._dims(L),
                                    want_grad=want_grad)

    def train_step(self, L, stale, log_age, target, lr, want_loss=True):
        return fibar_fill_train_step(self.handle, L, stale, log_age, target, *self._dims(L), lr,
                                     want_loss=want_loss)

    def apply(self, L, stale, log_age, out, tile=16, theta=0.0):
        _, H, W = self._dims(L)
        return fibar_fill_apply(self.handle, L, stale, log_age, H, W, tile, theta, out)

    def apply_noalloc(self, L, stale, log_age, out, tile=16, theta=0.0):
        _, H, W = self._dims(L)
        return fibar_fill_apply_noalloc(self.handle, L, stale, log_age, H, W, tile, theta, out)

    def close(self):
        if getattr(self, "handle", None):
            fibar_fill_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
