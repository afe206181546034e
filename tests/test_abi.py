"""The C-ABI library: it is built, loads, and exports every declared symbol.

No compute call is made here (no GPU in this environment)."""
import ctypes
import os
import re

import pytest

import paper_2510_20071_amd as fb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(inc, fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(fibar_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fibar_create", "fibar_push_events", "fibar_readout", "fibar_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fb.LIB_PATH):
        pytest.fail("libfibar.so is not built")
    lib = ctypes.CDLL(fb.LIB_PATH)
    for name in sorted(declared_functions()):
        assert hasattr(lib, name), name
    # and the binding wraps every one of them under the same name
    for name in declared_functions():
        assert name in fb._SIGNATURES, name
        assert callable(getattr(fb, name)), name


def test_binding_structs_match_header_sizes():
    # x86-64 SysV layout of the public structs
    assert ctypes.sizeof(fb.fibar_params) == 8 + 7 * 4 + 4 + 8 + 4 + 4 + 8
    assert ctypes.sizeof(fb.fibar_packet) == 4 * 8 + 8 + 8
    assert ctypes.sizeof(fb.fibar_readout_buf) == 8 * 8 + 8
    assert fb.STEP_RECORD_WORDS * 8 == 64   # fibar_step_record: one int64 and seven uint64
    assert ctypes.sizeof(fb.fibar_stats) == 9 * 8


def test_status_strings_and_defaults_without_gpu():
    lib = fb.load()
    assert fb.fibar_status_string(fb.FIBAR_E_RANGE).startswith("event coordinate")
    p = fb.fibar_default_params()
    assert p.t_cut == 40.0 and (p.fill_num, p.fill_den) == (1, 2)
    assert p.spatial_filter == 1 and p.q_min == 64 and p.q_max == 0
    # argument validation happens before any device call
    assert fb.fibar_create(0, 10, p)[0] == fb.FIBAR_E_INVALID_ARG
    bad = fb.fibar_default_params()
    bad.t_cut = 4.0
    assert fb.fibar_create(10, 10, bad)[0] == fb.FIBAR_E_INVALID_ARG
    bad = fb.fibar_default_params()
    bad.fill_num, bad.fill_den = 3, 2
    assert fb.fibar_create(10, 10, bad)[0] == fb.FIBAR_E_INVALID_ARG
    bad = fb.fibar_default_params()
    bad.q_min = 1000
    assert fb.fibar_create(10, 10, bad)[0] == fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_push_events(None, None) == fb.FIBAR_E_INVALID_ARG
    lib.fibar_destroy(None)


def test_fill_entry_points_reject_null_handles_without_gpu():
    lib = fb.load()
    assert lib.fibar_fill_create(None, None) == fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_fill_set_params(None, None) == fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_fill_get_params(None, None) == fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_fill_predict(None, None, None, None, 1, 1, 1, None) == fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_fill_apply(None, None, None, None, 1, 1, 16, 1.0, None, None) == \
        fb.FIBAR_E_INVALID_ARG
    lib.fibar_fill_destroy(None)
    assert fb.FILL_PARAMS == 5233


def test_sensor_size_limit_of_the_sort_key_without_gpu():
    # an event's sort key is (tile-major pixel key << 1) | polarity in 32 bits,
    # four keys per 2x2 tile: sensors above 2^29 tiles are rejected before any
    # device call (at 65535 x 65535 the key would lose its top bit)
    p = fb.fibar_default_params()
    for w, h in ((65535, 65535), (46341, 46341), (65535, 32769), (32769, 65535)):
        tiles = ((w + 1) // 2) * ((h + 1) // 2)
        assert 4 * tiles > 2 ** 31
        assert fb.fibar_create(w, h, p)[0] == fb.FIBAR_E_INVALID_ARG, (w, h)


def test_telemetry_rejects_bad_arguments_without_gpu():
    lib = fb.load()
    assert lib.fibar_set_telemetry(None, None, 0) == fb.FIBAR_E_INVALID_ARG


def test_event_regulation_limits_without_gpu():
    # per-event regulation keeps the state of a packet in one workgroup's
    # local memory: at most 8192 pixels and windows of at most 16382 events
    p = fb.fibar_default_params()
    p.regulation = fb.FIBAR_REG_EVENT
    assert fb.fibar_create(128, 65, p)[0] == fb.FIBAR_E_INVALID_ARG      # 8320 pixels
    p.q_max = 16383
    assert fb.fibar_create(64, 48, p)[0] == fb.FIBAR_E_INVALID_ARG
    p = fb.fibar_default_params()
    p.regulation = 2
    assert fb.fibar_create(64, 48, p)[0] == fb.FIBAR_E_INVALID_ARG


def test_threshold_entry_points_reject_bad_arguments_without_gpu():
    lib = fb.load()
    assert lib.fibar_count_polarities(None, None, None, 0, 4, 4, None, None, None) == \
        fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_count_polarities(None, None, None, 0, 0, 4, 8, 8, None) == \
        fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_relative_thresholds(None, None, 4, 4, None, None, None, None) == \
        fb.FIBAR_E_INVALID_ARG
    assert lib.fibar_set_pixel_gain(None, None) == fb.FIBAR_E_INVALID_ARG


def test_per_tile_queue_parameters_without_gpu():
    p = fb.fibar_default_params()
    assert p.region == 0 and p.age_max == 0
    for bad in (3, 34, 64):                 # odd, or more than 32
        p = fb.fibar_default_params()
        p.region = bad
        assert fb.fibar_create(64, 48, p)[0] == fb.FIBAR_E_INVALID_ARG
    p = fb.fibar_default_params()
    p.region = 8
    p.spatial_filter = 0
    assert fb.fibar_create(64, 48, p)[0] == fb.FIBAR_E_INVALID_ARG
    p = fb.fibar_default_params()
    p.region = 8
    p.regulation = fb.FIBAR_REG_EVENT
    assert fb.fibar_create(64, 48, p)[0] == fb.FIBAR_E_INVALID_ARG
    p = fb.fibar_default_params()
    p.region = 2                             # 640 x 360 = 230400 tiles > 16384
    assert fb.fibar_create(1280, 720, p)[0] == fb.FIBAR_E_INVALID_ARG
    assert fb.load().fibar_tile_stats(None, None, None, None, None, None) == fb.FIBAR_E_INVALID_ARG
