"""Python front end of libgrwave: marshals workloads into the C ABI.

PyTorch provides device memory and the stream; every step of the tracing runs in the HIP
kernels of libgrwave.so.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


def _fptr(t):
    return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_float))


def _f3(v):
    return (C.c_float * 3)(*[float(x) for x in np.asarray(v, np.float64)])


def material_struct(m) -> L.GrMaterial:
    s = L.GrMaterial()
    s.kind = int(m.kind)
    s.height_um = float(m.height_um)
    s.length_um = float(m.length_um)
    g = np.asarray(m.gdir, np.float64)
    g = g / np.linalg.norm(g)
    s.gdir = _f3(g)
    s.reflectance = float(m.reflectance)
    return s


def sensor_struct(sen) -> L.GrSensor:
    s = L.GrSensor()
    s.origin = _f3(sen.origin)
    s.axis_u = _f3(sen.axis_u)
    s.axis_v = _f3(sen.axis_v)
    s.dir = _f3(sen.dir)
    s.width = int(sen.width)
    s.height = int(sen.height)
    s.pitch_m = float(sen.pitch_m)
    s.sigma_m = float(sen.sigma_m)
    return s


def source_struct(src) -> L.GrSource:
    s = L.GrSource()
    s.kind = int(src.kind)
    s.dir = _f3(src.dir)
    s.pos = _f3(src.pos)
    s.eu = _f3(src.eu)
    s.ev = _f3(src.ev)
    s.coherence_radius_um = float(src.coherence_radius_um)
    s.power = float(src.power)
    return s


class Renderer:
    """One libgrwave context on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.lib = L.load()
        self.dev = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.dev) if stream is None else stream
        h = C.c_void_p()
        rc = self.lib.gr_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        L.check(rc, None, "gr_create")
        self.h = h
        self._ws = None
        self.sensor = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.gr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        L.check(rc, self.h, what)

    # -- scene / sensor / sources ------------------------------------------------------
    def upload_scene(self, scene):
        verts = np.ascontiguousarray(scene.verts, np.float32)
        tris = np.ascontiguousarray(scene.tris, np.int32)
        tm = np.ascontiguousarray(scene.tri_mat, np.int32)
        mats = (L.GrMaterial * len(scene.materials))(*[material_struct(m) for m in scene.materials])
        nrm = None
        if scene.normals is not None:
            nrm = np.ascontiguousarray(scene.normals, np.float32)
        fp = C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int32)
        rc = self.lib.gr_scene_upload(self.h, verts.ctypes.data_as(fp), verts.shape[0],
                                      nrm.ctypes.data_as(fp) if nrm is not None else None,
                                      tris.ctypes.data_as(ip), tris.shape[0],
                                      tm.ctypes.data_as(ip), mats, len(scene.materials))
        self._check(rc, "gr_scene_upload")
        return self.scene_info()

    def scene_info(self):
        info = L.GrSceneInfo()
        self._check(self.lib.gr_scene_info_get(self.h, C.byref(info)), "gr_scene_info_get")
        return {name: getattr(info, name) for name, _ in info._fields_ if name != "reserved"}

    def set_sensor(self, sensor):
        s = sensor_struct(sensor)
        self._check(self.lib.gr_set_sensor(self.h, C.byref(s)), "gr_set_sensor")
        self.sensor = sensor

    def set_sources(self, sources: Sequence):
        arr = (L.GrSource * max(1, len(sources)))(*[source_struct(s) for s in sources])
        self._check(self.lib.gr_set_sources(self.h, arr, len(sources)), "gr_set_sources")

    def boundaries(self, reach_m=2e-3):
        """Find the uploaded scene's material boundaries (gr_scene_boundaries) for composite
        interactions; returns the number of boundary edges."""
        n = C.c_int64(0)
        self._check(self.lib.gr_scene_boundaries(self.h, float(reach_m), C.byref(n)), "gr_scene_boundaries")
        return int(n.value)

    def load_workload(self, wl):
        info = self.upload_scene(wl.scene)
        self.set_sensor(wl.sensor)
        self.set_sources(wl.sources)
        return info

    # -- trace -----------------------------------------------------------------------------
    def opts(self, spp_begin=0, spp_count=1, spp_norm=None, max_depth=1, bsdf_mode=0,
             rr_enable=False, rr_p=0.8, seed=0, keep_paths=False,
             short_lds_stack=False, hero=False, aniso=False, composite=False) -> L.GrTraceOpts:
        o = L.GrTraceOpts()
        o.spp_begin = int(spp_begin)
        o.spp_count = int(spp_count)
        o.spp_norm = int(spp_count if spp_norm is None else spp_norm)
        o.max_depth = int(max_depth)
        o.bsdf_mode = int(bsdf_mode)
        o.rr_enable = int(bool(rr_enable))
        o.rr_p = float(rr_p)
        o.seed = int(seed)
        o.flags = (L.GR_TRACE_KEEP_PATHS if keep_paths else 0) | \
            (L.GR_TRACE_SHORT_LDS_STACK if short_lds_stack else 0) | \
            (L.GR_TRACE_HERO if hero else 0) | (L.GR_TRACE_ANISO if aniso else 0) | \
            (L.GR_TRACE_COMPOSITE if composite else 0)
        return o

    def workspace(self, opts: L.GrTraceOpts, n_lambda: int):
        n = C.c_size_t()
        self._check(self.lib.gr_workspace_size(self.h, C.byref(opts), n_lambda, C.byref(n)),
                    "gr_workspace_size")
        need = int(n.value)
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.dev)
        return self._ws, need

    def trace(self, lambdas_um, opts: L.GrTraceOpts, image=None, stats=True):
        """Returns (image [n_lambda, H, W] float32 tensor, stats dict or None)."""
        lam = np.ascontiguousarray(np.asarray(lambdas_um, np.float32))
        nl = lam.shape[0]
        ws, need = self.workspace(opts, nl)
        if image is None:
            image = self.torch.zeros((nl, self.sensor.height, self.sensor.width),
                                     dtype=self.torch.float32, device=self.dev)
        st = L.GrStats() if stats else None
        rc = self.lib.gr_trace(self.h, lam.ctypes.data_as(C.POINTER(C.c_float)), nl, C.byref(opts),
                               C.c_void_p(ws.data_ptr()), ws.numel(), _fptr(image),
                               C.byref(st) if st is not None else None)
        self._check(rc, "gr_trace")
        return image, (st.as_dict() if st is not None else None)

    def trace_noalloc(self, lambdas_um, opts: L.GrTraceOpts, image):
        """gr_trace_noalloc: the same trace in the library's static device workspace; adds to the
        caller's image [n_lambda, H, W] float32 tensor.  No allocation, no synchronisation."""
        lam = np.ascontiguousarray(np.asarray(lambdas_um, np.float32))
        rc = self.lib.gr_trace_noalloc(self.h, lam.ctypes.data_as(C.POINTER(C.c_float)), lam.shape[0],
                                       C.byref(opts), _fptr(image))
        self._check(rc, "gr_trace_noalloc")
        return image

    def path_records(self, opts: L.GrTraceOpts, n_lambda: int):
        """Per-path contributions kept by the last trace with keep_paths: a tensor view
        [spp_count, H, W, n_lambda] of the workspace."""
        ws, need = self.workspace(opts, n_lambda)
        p = C.POINTER(C.c_float)()
        self._check(self.lib.gr_workspace_paths(self.h, C.c_void_p(ws.data_ptr()), C.byref(p)),
                    "gr_workspace_paths")
        off = C.cast(p, C.c_void_p).value - ws.data_ptr()
        n = opts.spp_count * self.sensor.height * self.sensor.width * n_lambda
        return ws[off:off + 4 * n].view(self.torch.float32).view(
            opts.spp_count, self.sensor.height, self.sensor.width, n_lambda)

    def render_workload(self, wl, spp_begin=0, spp_count=None, bsdf_mode=0, stats=True,
                        keep_paths=False, hero=False, aniso=False, composite=False):
        spp_count = wl.spp if spp_count is None else spp_count
        o = self.opts(spp_begin=spp_begin, spp_count=spp_count, spp_norm=wl.spp,
                      max_depth=wl.max_depth, bsdf_mode=bsdf_mode, rr_enable=wl.rr_enable,
                      rr_p=wl.rr_p, seed=wl.seed, keep_paths=keep_paths, hero=hero, aniso=aniso,
                      composite=composite)
        return self.trace(wl.lambdas_um, o, stats=stats)

    # -- scattering kernels ---------------------------------------------------------------
    def bsdf_eval(self, queries, mode=0):
        """queries: float32 device tensor [n, 14] (see gr_bsdf_eval); returns [n]."""
        q = queries.contiguous()
        out = self.torch.empty(q.shape[0], dtype=self.torch.float32, device=self.dev)
        self._check(self.lib.gr_bsdf_eval(self.h, _fptr(q), q.shape[0], int(mode), _fptr(out)),
                    "gr_bsdf_eval")
        return out

    def pw_composite_eval(self, queries):
        """queries: float32 device tensor [n, 23] (see gr_pw_composite_eval); returns [n]."""
        q = queries.contiguous()
        out = self.torch.empty(q.shape[0], dtype=self.torch.float32, device=self.dev)
        self._check(self.lib.gr_pw_composite_eval(self.h, _fptr(q), q.shape[0], _fptr(out)),
                    "gr_pw_composite_eval")
        return out

    # -- coherent measurement -------------------------------------------------------------
    def coherent(self, case, phase_mode=1, nodes_per_slit=16, timing=False):
        """Coherent measurement of a two-point / double-slit case (workloads.CoherentCase).
        phase_mode: 0 FP32, 1 FP64, 2 two-float.  Returns (image [H, W] tensor, ms or None)."""
        d = L.GrCoherentDesc()
        d.kind = 0 if case.kind == "points" else 1
        c = list(np.asarray(case.centres_um, np.float64))
        d.n_slits = len(c)
        d.centre_um = (C.c_double * 8)(*(c + [0.0] * (8 - len(c))))
        d.width_um = float(case.width_um)
        d.nodes_per_slit = int(nodes_per_slit)
        d.phase_mode = int(phase_mode)
        d.z_um = float(case.z_m * 1e6)
        d.lambda_um = float(case.lambda_um)
        d.width = int(case.width)
        d.height = int(case.height)
        d.pitch_um = float(case.pitch_um)
        d.sigma_um = float(case.sigma_um)
        d.spp = int(case.spp)
        d.seed = int(case.seed)
        img = self.torch.empty((case.height, case.width), dtype=self.torch.float32, device=self.dev)
        ms = C.c_float(0.0)
        rc = self.lib.gr_coherent_measure(self.h, C.byref(d), _fptr(img), C.byref(ms) if timing else None)
        self._check(rc, "gr_coherent_measure")
        return img, (ms.value if timing else None)
