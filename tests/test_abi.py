"""CPU checks of the C ABI: the library loads, exports every declared entry point, and rejects
bad arguments before touching a device."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2303_15762_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "grwave.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(gr_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in L.SIGNATURES}
    assert set(declared) <= bound


def test_struct_layouts_match_header_sizes():
    assert C.sizeof(L.GrMaterial) == 28
    assert C.sizeof(L.GrSensor) == 64
    assert C.sizeof(L.GrSource) == 60
    assert C.sizeof(L.GrTraceOpts) == 56
    assert C.sizeof(L.GrStats) == 120
    assert C.sizeof(L.GrSceneInfo) == 40


@pytest.fixture
def ctx():
    lib = L.load()
    h = C.c_void_p()
    assert lib.gr_create(C.byref(h), 0, None) == 0
    yield lib, h
    lib.gr_destroy(h)


def test_null_and_range_errors(ctx):
    lib, h = ctx
    assert lib.gr_create(None, 0, None) == -1
    hh = C.c_void_p()
    assert lib.gr_create(C.byref(hh), -1, None) == -1
    assert lib.gr_set_sensor(h, None) == -1
    s = L.GrSensor()
    s.axis_u = (C.c_float * 3)(1, 0, 0)
    s.axis_v = (C.c_float * 3)(0, 1, 0)
    s.dir = (C.c_float * 3)(0, 0, 2)          # not a unit vector
    s.width = s.height = 4
    s.pitch_m = s.sigma_m = 1e-4
    assert lib.gr_set_sensor(h, C.byref(s)) == -1
    assert b"unit" in lib.gr_last_error(h)
    s.dir = (C.c_float * 3)(0, 0, -1)
    s.width = 0
    assert lib.gr_set_sensor(h, C.byref(s)) == -1
    s.width = 4
    assert lib.gr_set_sensor(h, C.byref(s)) == 0
    src = (L.GrSource * 1)()
    src[0].kind = 7
    assert lib.gr_set_sources(h, src, 1) == -1
    assert lib.gr_set_sources(h, src, 17) == -1
    assert lib.gr_set_sources(h, None, 0) == 0


def test_trace_rejects_before_device_use(ctx):
    lib, h = ctx
    lam = (C.c_float * 1)(0.55)
    o = L.GrTraceOpts(spp_begin=0, spp_count=1, spp_norm=1, max_depth=1)
    dummy = C.cast(C.c_void_p(16), C.POINTER(C.c_float))
    # no scene yet
    assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -2
    o.max_depth = 0
    assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -1
    o.max_depth = 1
    o.bsdf_mode = 5
    assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -1
    bad = (C.c_float * 1)(-1.0)
    o.bsdf_mode = 0
    assert lib.gr_trace(h, bad, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -1
    # flags: unknown bits, and hero-wavelength paths or anisotropic rays outside what they support
    for bad_flag in (4, 64):
        o.flags = bad_flag
        assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -1
    for mode in (1, 2):
        o.flags = L.GR_TRACE_ANISO
        o.bsdf_mode = mode
        assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -5
        assert b"anisotropic" in lib.gr_last_error(h)
    o.bsdf_mode = 0
    o.flags = L.GR_TRACE_ANISO
    assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -2
    o.flags = L.GR_TRACE_HERO
    assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -1
    assert b"n_lambda" in lib.gr_last_error(h)
    lam4 = (C.c_float * 4)(0.45, 0.5, 0.55, 0.6)
    o.flags = L.GR_TRACE_HERO
    o.bsdf_mode = 1
    assert lib.gr_trace(h, lam4, 4, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -5
    o.bsdf_mode = 0
    assert lib.gr_trace(h, lam4, 4, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -2
    o.flags = L.GR_TRACE_HERO | L.GR_TRACE_ANISO
    assert lib.gr_trace(h, lam4, 4, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -5
    # composite interactions (scalar, anisotropic or hero-wavelength rays, closed-form or
    # learned p_w where the rays allow it) only after gr_scene_boundaries
    o.flags, o.bsdf_mode = L.GR_TRACE_COMPOSITE | L.GR_TRACE_HERO, 1     # hero paths: closed form only
    assert lib.gr_trace(h, lam4, 4, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -5
    o.bsdf_mode = 0
    assert lib.gr_trace(h, lam4, 4, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -2
    for flags, mode in ((L.GR_TRACE_COMPOSITE, 0), (L.GR_TRACE_COMPOSITE, 1),
                        (L.GR_TRACE_COMPOSITE | L.GR_TRACE_ANISO, 0)):
        o.flags, o.bsdf_mode = flags, mode
        assert lib.gr_trace(h, lam, 1, C.byref(o), C.c_void_p(4096), 1 << 20, dummy, None) == -2
    o.flags, o.bsdf_mode = L.GR_TRACE_COMPOSITE, 0
    n = C.c_int64(0)
    assert lib.gr_scene_boundaries(h, 2e-3, C.byref(n)) == -2
    assert lib.gr_scene_boundaries(h, 0.0, C.byref(n)) == -1
    assert lib.gr_scene_boundaries(h, 2.0, C.byref(n)) == -1
    assert lib.gr_pw_composite_eval(h, None, 4, None) == -1


def test_scene_validation(ctx):
    lib, h = ctx
    v = np.zeros((3, 3), np.float32)
    v[1, 0] = 1
    v[2, 1] = 1
    t = np.array([[0, 1, 5]], np.int32)          # index out of range
    tm = np.zeros(1, np.int32)
    mats = (L.GrMaterial * 1)()
    mats[0].kind = 0
    mats[0].reflectance = 1.0
    fp = C.POINTER(C.c_float)
    ip = C.POINTER(C.c_int32)
    rc = lib.gr_scene_upload(h, v.ctypes.data_as(fp), 3, None, t.ctypes.data_as(ip), 1,
                             tm.ctypes.data_as(ip), mats, 1)
    assert rc == -1
    t[0, 2] = 2
    tm[0] = 3                                     # material out of range
    rc = lib.gr_scene_upload(h, v.ctypes.data_as(fp), 3, None, t.ctypes.data_as(ip), 1,
                             tm.ctypes.data_as(ip), mats, 1)
    assert rc == -1
    tm[0] = 0
    mats[0].kind = 2
    mats[0].length_um = 1.0
    mats[0].gdir = (C.c_float * 3)(0, 0, 0)      # grating without a direction
    rc = lib.gr_scene_upload(h, v.ctypes.data_as(fp), 3, None, t.ctypes.data_as(ip), 1,
                             tm.ctypes.data_as(ip), mats, 1)
    assert rc == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        L.load()
