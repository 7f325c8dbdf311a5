"""ctypes binding of libgrwave.so (argument marshalling only).

The structures mirror include/grwave.h field by field.  Loading fails loudly when the HIP
library has not been built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrwave.so")

GR_OK = 0
ERRORS = {-1: "GR_E_INVALID", -2: "GR_E_NO_SCENE", -3: "GR_E_DEVICE", -4: "GR_E_OOM",
          -5: "GR_E_UNSUPPORTED", -6: "GR_E_WORKSPACE"}
GR_BSDF_PLAIN, GR_BSDF_SURROGATE_BF16, GR_BSDF_SURROGATE_FP8 = 0, 1, 2
GR_TRACE_KEEP_PATHS = 1
GR_TRACE_SHORT_LDS_STACK = 2
GR_TRACE_HERO = 8
GR_TRACE_ANISO = 16
GR_TRACE_COMPOSITE = 32
GR_MLP_PARAMS = 13249


class GrMaterial(C.Structure):
    _fields_ = [("kind", C.c_int32), ("height_um", C.c_float), ("length_um", C.c_float),
                ("gdir", C.c_float * 3), ("reflectance", C.c_float)]


class GrSensor(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("axis_u", C.c_float * 3), ("axis_v", C.c_float * 3),
                ("dir", C.c_float * 3), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_m", C.c_float), ("sigma_m", C.c_float)]


class GrSource(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_float * 3), ("pos", C.c_float * 3),
                ("eu", C.c_float * 3), ("ev", C.c_float * 3),
                ("coherence_radius_um", C.c_float), ("power", C.c_float)]


class GrTraceOpts(C.Structure):
    _fields_ = [("spp_begin", C.c_int64), ("spp_count", C.c_int64), ("spp_norm", C.c_int64),
                ("max_depth", C.c_int32), ("bsdf_mode", C.c_int32), ("rr_enable", C.c_int32),
                ("rr_p", C.c_float), ("seed", C.c_uint64), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


class GrStats(C.Structure):
    _fields_ = [("paths", C.c_uint64), ("segments", C.c_uint64), ("shadow_rays", C.c_uint64),
                ("surrogate_evals", C.c_uint64), ("fallbacks", C.c_uint64),
                ("evanescent", C.c_uint64), ("backfacing", C.c_uint64),
                ("nonfinite", C.c_uint64), ("node_visits", C.c_uint64),
                ("tri_tests", C.c_uint64), ("composite", C.c_uint64),
                ("measured_smooth", C.c_uint64), ("measured_rough", C.c_uint64),
                ("measured_grating", C.c_uint64), ("ms", C.c_float), ("ms_reduce", C.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class GrSceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32),
                ("max_leaf", C.c_int32), ("device_bytes", C.c_int64), ("build_ms", C.c_float),
                ("reserved", C.c_float)]


class GrCoherentDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_slits", C.c_int32), ("centre_um", C.c_double * 8),
                ("width_um", C.c_double), ("nodes_per_slit", C.c_int32),
                ("phase_mode", C.c_int32), ("z_um", C.c_double), ("lambda_um", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("pitch_um", C.c_double),
                ("sigma_um", C.c_double), ("spp", C.c_int64), ("seed", C.c_uint64)]


# (name, restype, argtypes) of every exported entry point declared in include/grwave.h
_vp = C.c_void_p
_fp = C.POINTER(C.c_float)
SIGNATURES = [
    ("gr_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int, _vp]),
    ("gr_destroy", None, [_vp]),
    ("gr_last_error", C.c_char_p, [_vp]),
    ("gr_scene_upload", C.c_int, [_vp, _fp, C.c_int64, _fp, C.POINTER(C.c_int32), C.c_int64,
                                  C.POINTER(C.c_int32), C.POINTER(GrMaterial), C.c_int32]),
    ("gr_scene_info_get", C.c_int, [_vp, C.POINTER(GrSceneInfo)]),
    ("gr_scene_boundaries", C.c_int, [_vp, C.c_float, C.POINTER(C.c_int64)]),
    ("gr_set_sensor", C.c_int, [_vp, C.POINTER(GrSensor)]),
    ("gr_set_sources", C.c_int, [_vp, C.POINTER(GrSource), C.c_int32]),
    ("gr_workspace_size", C.c_int, [_vp, C.POINTER(GrTraceOpts), C.c_int32,
                                    C.POINTER(C.c_size_t)]),
    ("gr_workspace_paths", C.c_int, [_vp, _vp, C.POINTER(_fp)]),
    ("gr_trace", C.c_int, [_vp, _fp, C.c_int32, C.POINTER(GrTraceOpts), _vp, C.c_size_t, _fp,
                           C.POINTER(GrStats)]),
    ("gr_trace_noalloc", C.c_int, [_vp, _fp, C.c_int32, C.POINTER(GrTraceOpts), _fp]),
    ("gr_bsdf_eval", C.c_int, [_vp, _fp, C.c_int64, C.c_int32, _fp]),
    ("gr_pw_composite_eval", C.c_int, [_vp, _fp, C.c_int64, _fp]),
    ("gr_surrogate_samples", C.c_int, [_vp, C.c_int64, C.c_uint64, _fp, _fp, _fp, _fp]),
    ("gr_mlp_workspace_size", C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
    ("gr_mlp_forward", C.c_int, [_vp, _fp, _fp, C.c_int64, C.c_int32, _vp, _fp]),
    ("gr_mlp_backward", C.c_int, [_vp, _fp, _fp, _fp, C.c_int64, _vp, _fp, _fp]),
    ("gr_mlp_activation", C.c_int, [_vp, _fp, C.c_int64, _fp, _fp]),
    ("gr_adam_step", C.c_int, [_vp, _fp, _fp, _fp, _fp, C.c_int32, C.c_float, C.c_float,
                               C.c_float, C.c_float]),
    ("gr_set_surrogate", C.c_int, [_vp, _fp, _fp]),
    ("gr_coherent_measure", C.c_int, [_vp, C.POINTER(GrCoherentDesc), _fp, _fp]),
]

_lib = None


class GrError(RuntimeError):
    pass


def load():
    """Load libgrwave.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_15762_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc, ctx=None, what=""):
    if rc != GR_OK:
        msg = ""
        if ctx is not None:
            m = load().gr_last_error(ctx)
            msg = m.decode() if m else ""
        raise GrError(f"{what}: {ERRORS.get(rc, rc)} {msg}")
