"""FP64 CPU oracle of the backward generalized-ray path tracer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``.  The product package never imports it.

The oracle is a plain double-precision C++ program (``oracle.cpp``) plus this ctypes
binding, and a NumPy FP64 multilayer perceptron (``mlp.py``).  It shares no code with the
HIP path; only the seeded input generators in ``workloads`` feed both.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC, "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


class OrMaterial(C.Structure):
    _fields_ = [("kind", C.c_int32), ("height_um", C.c_double), ("length_um", C.c_double),
                ("gdir", C.c_double * 3), ("reflectance", C.c_double)]


class OrSensor(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("axis_u", C.c_double * 3),
                ("axis_v", C.c_double * 3), ("dir", C.c_double * 3),
                ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_m", C.c_double), ("sigma_m", C.c_double)]


class OrSource(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_double * 3), ("pos", C.c_double * 3),
                ("eu", C.c_double * 3), ("ev", C.c_double * 3),
                ("rc_um", C.c_double), ("power", C.c_double)]


class OrOpts(C.Structure):
    _fields_ = [("spp_begin", C.c_int64), ("spp_count", C.c_int64), ("spp_norm", C.c_double),
                ("max_depth", C.c_int32), ("rr_enable", C.c_int32),
                ("rr_threshold24", C.c_uint32), ("rr_p", C.c_double), ("seed", C.c_uint64),
                ("use_bvh", C.c_int32), ("n_threads", C.c_int32), ("hero", C.c_int32),
                ("aniso", C.c_int32), ("composite", C.c_int32), ("reach_m", C.c_double)]


class OrCoherent(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_nodes", C.c_int32),
                ("xs", C.POINTER(C.c_double)), ("ws", C.POINTER(C.c_double)),
                ("z_um", C.c_double), ("lambda_um", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_um", C.c_double), ("sigma_um", C.c_double),
                ("spp", C.c_int64), ("seed", C.c_uint64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build(force=True)
            L = C.CDLL(_SO)
            dp = C.POINTER(C.c_double)
            L.or_philox.argtypes = [C.POINTER(C.c_uint32)] * 3
            L.or_philox_batch.argtypes = [C.POINTER(C.c_uint32), C.c_int64,
                                          C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
            L.or_besselj.argtypes = [C.c_int, C.c_double]
            L.or_besselj.restype = C.c_double
            L.or_propagate.argtypes = [C.c_double] * 4 + [dp]
            L.or_pw.argtypes = [C.c_int] + [C.c_double] * 13
            L.or_pw.restype = C.c_double
            L.or_pw_batch.argtypes = [dp, C.c_int64, dp]
            L.or_sample.argtypes = [C.c_int] + [C.c_double] * 12 + [dp]
            L.or_sample.restype = C.c_int
            L.or_hero_step_batch.argtypes = [C.c_int] + [C.c_double] * 10 + [dp, C.c_int64, dp]
            L.or_hero_composite_step_batch.argtypes = [dp, dp] + [C.c_double] * 7 + [dp, C.c_int64, dp]
            L.or_scene_create.argtypes = [dp, C.c_int64, dp, C.POINTER(C.c_int32), C.c_int64,
                                          C.POINTER(C.c_int32), C.POINTER(OrMaterial), C.c_int32]
            L.or_scene_create.restype = C.c_void_p
            L.or_scene_destroy.argtypes = [C.c_void_p]
            L.or_intersect.argtypes = [C.c_void_p, dp, C.c_int64, C.c_double, C.c_int, dp]
            L.or_interaction.argtypes = [C.c_void_p, dp, C.c_double, dp, dp]
            L.or_trace.argtypes = [C.c_void_p, C.POINTER(OrSensor), C.POINTER(OrSource),
                                   C.c_int32, dp, C.c_int32, C.POINTER(OrOpts),
                                   C.POINTER(C.c_int32), C.c_int64, dp, dp,
                                   C.POINTER(C.c_uint64)]
            L.or_trace.restype = C.c_int
            L.or_coherent_mc.argtypes = [C.POINTER(OrCoherent), dp, C.c_int32, C.c_int32]
            L.or_coherent_exact.argtypes = [C.POINTER(OrCoherent), C.POINTER(C.c_int32),
                                            C.c_int64, dp, dp, C.c_int32, dp, dp, C.c_int32, dp]
            L.or_hankel1_re.argtypes = [C.c_double]
            L.or_hankel1_re.restype = C.c_double
            L.or_hankel1_im.argtypes = [C.c_double]
            L.or_hankel1_im.restype = C.c_double
            L.or_transverse_frame.argtypes = [dp, dp, dp]
            L.or_aniso_free.argtypes = [C.c_double, C.c_double, dp]
            L.or_aniso_interact.argtypes = [dp, dp, dp, dp]
            L.or_aniso_footprint.argtypes = [dp, dp, dp, dp, dp, dp]
            L.or_scene_boundaries.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int64, C.c_double]
            L.or_scene_boundaries.restype = C.c_int64
            L.or_boundary_edge.argtypes = [C.c_void_p, C.c_int64, dp]
            L.or_nearest_boundary.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64, C.c_double, dp]
            L.or_faddeeva.argtypes = [C.c_double, C.c_double, dp]
            L.or_halfplane_field.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, C.c_int64, dp]
            L.or_pw_composite_batch.argtypes = [dp, C.c_int64, dp]
            L.or_path_vertices.argtypes = [C.c_void_p, C.POINTER(OrSensor), C.POINTER(OrSource), C.c_int32, dp,
                                           C.c_int32, C.POINTER(OrOpts), C.c_int32, C.c_int32, C.c_int64,
                                           C.c_int32, dp, C.c_int32, dp]
            L.or_path_vertices.restype = C.c_int32
            L.or_interaction_composite.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, dp, C.c_double, dp]
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _v3(x):
    return (C.c_double * 3)(*[float(v) for v in np.asarray(x, np.float64)])


# ------------------------------------------------------------------------------------------
# Random numbers
# ------------------------------------------------------------------------------------------

def philox(counters, key):
    """Philox4x32-10 of an [n, 4] uint32 counter array under a 2-word key."""
    ctr = np.ascontiguousarray(np.asarray(counters, np.uint32).reshape(-1, 4))
    k = np.ascontiguousarray(np.asarray(key, np.uint32).reshape(2))
    out = np.empty_like(ctr)
    u32p = C.POINTER(C.c_uint32)
    lib().or_philox_batch(ctr.ctypes.data_as(u32p), ctr.shape[0], k.ctypes.data_as(u32p),
                          out.ctypes.data_as(u32p))
    return out


def besselj(n, x):
    return lib().or_besselj(int(n), float(x))


def propagate(beta2, rho, z_um, k):
    """Generalized-ray parameters after free-space propagation over z_um: (beta^2, rho)."""
    out = np.zeros(2)
    lib().or_propagate(float(beta2), float(rho), float(z_um), float(k), _dp(out))
    return out[0], out[1]


# ------------------------------------------------------------------------------------------
# Scattering kernels
# ------------------------------------------------------------------------------------------

def pw(kind, h, L, k, kit, kot, S, g=(1.0, 0.0), refl=1.0):
    """Windowed diffraction density p_w(kit -> kot) (um^2) for one query.  S = (sxx, syy, sxy)
    footprint covariance (um^2), g = grating direction in the frame."""
    return lib().or_pw(int(kind), float(h), float(L), float(refl), float(k), float(kit[0]),
                       float(kit[1]), float(kot[0]), float(kot[1]), float(S[0]), float(S[1]),
                       float(S[2]), float(g[0]), float(g[1]))


def pw_batch(q):
    """q: [n, 14] rows (kind, h, L, refl, k, kix, kiy, kox, koy, sxx, syy, sxy, gx, gy)."""
    q = np.ascontiguousarray(np.asarray(q, np.float64))
    out = np.empty(q.shape[0])
    lib().or_pw_batch(_dp(q), q.shape[0], _dp(out))
    return out


def faddeeva(z):
    """Faddeeva function w(z) = exp(-z^2) erfc(-i z) for Im z >= 0 (array)."""
    z = np.asarray(z, np.complex128)
    out = np.empty(z.shape, np.complex128)
    buf = np.zeros(2)
    for i, v in enumerate(z.ravel()):
        lib().or_faddeeva(float(v.real), float(v.imag), _dp(buf))
        out.flat[i] = complex(buf[0], buf[1])
    return out


def halfplane_field(S, n, c, v):
    """Normalised window fields at transfers v [m][2]: (whole plane (real), far half-plane
    n.x > c (complex)).  S = (sxx, syy, sxy) intensity footprint covariance (um^2)."""
    v = np.ascontiguousarray(np.asarray(v, np.float64).reshape(-1, 2))
    out = np.zeros((v.shape[0], 3))
    lib().or_halfplane_field(_dp(np.ascontiguousarray(S, np.float64)), float(n[0]), float(n[1]), float(c),
                             _dp(v), v.shape[0], _dp(out))
    return out[:, 0], out[:, 1] + 1j * out[:, 2]


def pw_composite_batch(q):
    """Composite p_w for rows q [n][23] (see or_pw_composite_batch)."""
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros(q.shape[0])
    lib().or_pw_composite_batch(_dp(q), q.shape[0], _dp(out))
    return out


def sample_continuation(kind, h, L, k, kit, ci, u, g=(1.0, 0.0), refl=1.0):
    """Continuation sample from the unwindowed kernel.  Returns (kot_x, kot_y, weight) or
    None when the path ends (evanescent)."""
    out = np.zeros(3)
    ok = lib().or_sample(int(kind), float(h), float(L), float(refl), float(k), float(kit[0]),
                         float(kit[1]), float(ci), float(u[0]), float(u[1]), float(u[2]),
                         float(g[0]), float(g[1]), _dp(out))
    return (out[0], out[1], out[2]) if ok else None


def hero_step(kind, h, L, kh, kc, ui, ci, U, g=(1.0, 0.0), refl=1.0):
    """Hero-wavelength continuation step for uniforms U [n, 3]: the hero's sample at
    wavenumber kh from incident tangential direction ui, and a companion's ratios at kc.
    Returns [n, 5]: (kox, koy, hero weight, f_c / p_h, p_c / p_h); NaN rows end the path."""
    U = np.ascontiguousarray(U, np.float64).reshape(-1, 3)
    out = np.empty((U.shape[0], 5))
    lib().or_hero_step_batch(int(kind), float(h), float(L), float(refl), float(kh), float(kc),
                             float(ui[0]), float(ui[1]), float(ci), float(g[0]), float(g[1]),
                             _dp(U), U.shape[0], _dp(out))
    return out


def hero_composite_step(near, far, mass_h, mass_c, kh, kc, ui, ci, U):
    """Hero-wavelength continuation step at a composite interaction for uniforms U [n, 4] (the
    sampler's three and the side choice).  near / far: (kind, h, L, refl, gx, gy) with the
    grating direction in the frame; mass_h, mass_c: the hero's and the companion's far masses.
    Returns [n, 6]: (kox, koy, f_h / p_h, f_c / p_h, p_c / p_h, class of the sampled direction:
    0 specular, 1 rough lobe, 2 dispersive grating order); NaN rows end the path."""
    U = np.ascontiguousarray(U, np.float64).reshape(-1, 4)
    out = np.empty((U.shape[0], 6))
    nm = np.ascontiguousarray(near, np.float64)
    fm = np.ascontiguousarray(far, np.float64)
    lib().or_hero_composite_step_batch(_dp(nm), _dp(fm), float(mass_h), float(mass_c), float(kh), float(kc),
                                       float(ui[0]), float(ui[1]), float(ci), _dp(U), U.shape[0], _dp(out))
    return out


def _vec3(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).reshape(3))


def transverse_frame(d):
    """Orthonormal basis (e1, e2) of the plane normal to the unit vector d."""
    e1, e2 = np.zeros(3), np.zeros(3)
    lib().or_transverse_frame(_dp(_vec3(d)), _dp(e1), _dp(e2))
    return e1, e2


def _pack(S):
    S = np.asarray(S, np.float64)
    return np.ascontiguousarray(np.concatenate([S[:2, :2].ravel(), S[:2, 2:].ravel(), S[2:, 2:].ravel()]))


def _unpack(st):
    S = np.zeros((4, 4))
    S[:2, :2] = st[0:4].reshape(2, 2)
    S[:2, 2:] = st[4:8].reshape(2, 2)
    S[2:, :2] = st[4:8].reshape(2, 2).T
    S[2:, 2:] = st[8:12].reshape(2, 2)
    return S


def aniso_free(S, z_um, k):
    """Free-space step of an anisotropic generalized ray.  S: 4x4 second moments
    [[Srr, Srk], [Srk^T, Skk]] in the transverse frame of its direction."""
    st = _pack(S)
    lib().or_aniso_free(float(z_um), float(k), _dp(st))
    return _unpack(st)


def aniso_interact(S, di, do, n):
    """Interaction map from mean direction di to do at a surface of normal n."""
    st = _pack(S)
    lib().or_aniso_interact(_dp(_vec3(di)), _dp(_vec3(do)), _dp(_vec3(n)), _dp(st))
    return _unpack(st)


def aniso_footprint(S, d, n, xa, ya):
    """(sxx, syy, sxy) footprint covariance on the surface frame (xa, ya)."""
    out = np.zeros(3)
    lib().or_aniso_footprint(_dp(_vec3(d)), _dp(_vec3(n)), _dp(_vec3(xa)), _dp(_vec3(ya)), _dp(_pack(S)), _dp(out))
    return out


# ------------------------------------------------------------------------------------------
# Scenes and rendering
# ------------------------------------------------------------------------------------------

class OracleScene:
    def __init__(self, scene):
        L = lib()
        verts = np.ascontiguousarray(scene.verts, np.float64)
        tris = np.ascontiguousarray(scene.tris, np.int32)
        tm = np.ascontiguousarray(scene.tri_mat, np.int32)
        mats = (OrMaterial * len(scene.materials))()
        for i, m in enumerate(scene.materials):
            mats[i].kind = m.kind
            mats[i].height_um = m.height_um
            mats[i].length_um = m.length_um
            mats[i].gdir = _v3(m.gdir)
            mats[i].reflectance = m.reflectance
        nrm = None
        if scene.normals is not None:
            nrm = np.ascontiguousarray(scene.normals, np.float64)
        i32p = C.POINTER(C.c_int32)
        self._keep = (verts, tris, tm, mats, nrm)
        self.n_boundaries = None
        self.h = L.or_scene_create(_dp(verts), verts.shape[0],
                                   _dp(nrm) if nrm is not None else None,
                                   tris.ctypes.data_as(i32p), tris.shape[0],
                                   tm.ctypes.data_as(i32p), mats, len(scene.materials))
        if not self.h:
            raise ValueError("oracle rejected the scene")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_scene_destroy(self.h)
            self.h = None

    def boundaries(self, reach_m=2e-3):
        """Find the material-boundary edges (once) and grid them for searches within reach_m;
        returns their number."""
        tris = self._keep[1]
        n = lib().or_scene_boundaries(self.h, tris.ctypes.data_as(C.POINTER(C.c_int32)), tris.shape[0],
                                      float(reach_m))
        if n < 0:
            raise RuntimeError("oracle boundary search failed")
        self.n_boundaries = int(n)
        return self.n_boundaries

    def boundary_edges(self):
        """[n][14]: p0 (3), p1 (3), the two materials, the two triangles' third vertices (6)."""
        n = self.boundaries() if self.n_boundaries is None else self.n_boundaries
        out = np.zeros((n, 14))
        row = np.zeros(14)
        for i in range(n):
            lib().or_boundary_edge(self.h, i, _dp(row))
            out[i] = row
        return out

    def nearest_boundary(self, mat, points, reach_m):
        """Nearest boundary edge of material mat within reach of each point: [n][2] (index or
        -1, distance)."""
        if self.n_boundaries is None:
            self.boundaries()
        P = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, 3))
        out = np.zeros((P.shape[0], 2))
        lib().or_nearest_boundary(self.h, int(mat), _dp(P), P.shape[0], float(reach_m), _dp(out))
        return out

    def interaction_composite(self, origin, direction, k, beta2, u, reach_m=2e-3):
        """One interaction with composite interactions: dict with composite, c (um), n, the
        far side's window mass, the side chosen by u[3], weight, direction and ended."""
        self.boundaries(reach_m)
        ray = np.ascontiguousarray(np.concatenate([np.asarray(origin, np.float64).ravel(),
                                                   np.asarray(direction, np.float64).ravel()]))
        out = np.zeros(11)
        lib().or_interaction_composite(self.h, _dp(ray), float(k), float(beta2),
                                       _dp(np.ascontiguousarray(u, np.float64)), float(reach_m), _dp(out))
        return {"composite": bool(out[0]), "c": out[1], "n": out[2:4], "mass_far": out[4],
                "far": bool(out[5]), "weight": out[6], "dir": out[7:10], "ended": bool(out[10])}

    def interaction(self, origin, direction, k, u=(0.5, 0.5, 0.5)):
        """One interaction of the path loop: dict with hit, ns, ng, ci, the continuation
        direction sampled with uniforms u at wavenumber k (um^-1), its weight, and ended."""
        ray = np.ascontiguousarray(np.concatenate([np.asarray(origin, np.float64).ravel(),
                                                   np.asarray(direction, np.float64).ravel()]))
        out = np.zeros(13)
        lib().or_interaction(self.h, _dp(ray), float(k), _dp(np.ascontiguousarray(u, np.float64)), _dp(out))
        return {"hit": bool(out[0]), "ns": out[1:4], "ng": out[4:7], "ci": out[7],
                "dir": out[8:11], "weight": out[11], "ended": bool(out[12])}

    def intersect(self, origins, dirs, tmin=-1.0, use_bvh=True):
        rays = np.ascontiguousarray(np.concatenate([origins, dirs], 1), np.float64)
        out = np.empty((rays.shape[0], 4))
        lib().or_intersect(self.h, _dp(rays), rays.shape[0], float(tmin), int(use_bvh), _dp(out))
        return out


def _sensor_struct(s):
    st = OrSensor()
    st.origin = _v3(s.origin)
    st.axis_u = _v3(s.axis_u)
    st.axis_v = _v3(s.axis_v)
    st.dir = _v3(s.dir)
    st.width = s.width
    st.height = s.height
    st.pitch_m = s.pitch_m
    st.sigma_m = s.sigma_m
    return st


def _sources_struct(srcs):
    arr = (OrSource * max(1, len(srcs)))()
    for i, s in enumerate(srcs):
        arr[i].kind = s.kind
        arr[i].dir = _v3(s.dir)
        arr[i].pos = _v3(s.pos)
        arr[i].eu = _v3(s.eu)
        arr[i].ev = _v3(s.ev)
        arr[i].rc_um = s.coherence_radius_um
        arr[i].power = s.power
    return arr


def rr_threshold24(p: float) -> int:
    return int(min(1 << 24, max(0, round(float(np.float32(p)) * (1 << 24)))))


def render(wl, oscene=None, pixels=None, spp_begin=0, spp_count=None, spp_norm=None,
           use_bvh=True, n_threads=0, keep_paths=False, lambdas=None, hero=False, aniso=False,
           composite=False, reach_m=2e-3):
    """Render a workload (or a pixel subset of it).  Returns (image, stats[, paths]).

    image: [n_lambda, H, W] when pixels is None, else [n_lambda, n_pixels].
    hero: one path per (pixel, sample, rotation group of four wavelengths), sampled at a hero
    wavelength drawn from its group (n_lambda must be a multiple of 4).
    aniso: anisotropic generalized rays (matrix beta, rho; not with hero).
    composite: composite interactions where a material boundary lies within the footprint
    (at most reach_m metres from the hit; scalar one-wavelength paths only)."""
    L = lib()
    oscene = OracleScene(wl.scene) if oscene is None else oscene
    if composite:
        oscene.boundaries(reach_m)
    lam = np.ascontiguousarray(wl.lambdas_um if lambdas is None else lambdas, np.float64)
    nl = lam.shape[0]
    spp_count = wl.spp if spp_count is None else spp_count
    spp_norm = float(wl.spp if spp_norm is None else spp_norm)
    op = OrOpts(spp_begin=spp_begin, spp_count=spp_count, spp_norm=spp_norm,
                max_depth=wl.max_depth, rr_enable=int(wl.rr_enable),
                rr_threshold24=rr_threshold24(wl.rr_p), rr_p=float(np.float32(wl.rr_p)),
                seed=wl.seed, use_bvh=int(use_bvh), n_threads=n_threads, hero=int(hero),
                aniso=int(aniso), composite=int(composite), reach_m=float(reach_m))
    sen = _sensor_struct(wl.sensor)
    srcs = _sources_struct(wl.sources)
    if pixels is None:
        npix = wl.sensor.width * wl.sensor.height
        pix = None
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, np.int32).reshape(-1, 2))
        npix = pix.shape[0]
    img = np.zeros((nl, npix))
    paths = np.zeros((spp_count, npix, nl)) if keep_paths else None
    stats = (C.c_uint64 * 8)()
    i32p = C.POINTER(C.c_int32)
    rc = L.or_trace(oscene.h, C.byref(sen), srcs, len(wl.sources), _dp(lam), nl, C.byref(op),
                    pix.ctypes.data_as(i32p) if pix is not None else None, npix, _dp(img),
                    _dp(paths) if paths is not None else None, stats)
    if rc != 0:
        raise RuntimeError("oracle trace failed")
    st = dict(segments=stats[0], shadow_rays=stats[1], evanescent=stats[2], backfacing=stats[3],
              composite=stats[4], measured_smooth=stats[5], measured_rough=stats[6],
              measured_grating=stats[7])
    if pixels is None:
        img = img.reshape(nl, wl.sensor.height, wl.sensor.width)
    if keep_paths:
        return img, st, paths
    return img, st


def path_vertices(wl, px, py, s, w, oscene=None, composite=False, reach_m=2e-3, aniso=False):
    """The interactions of one path of a render: (contribution, rows [n][12] = depth,
    triangle, hit point (3), composite, c (um), boundary normal (2), far mass, measurement,
    continuation side (0 near, 1 far, -1 none))."""
    oscene = OracleScene(wl.scene) if oscene is None else oscene
    if composite:
        oscene.boundaries(reach_m)
    lam = np.ascontiguousarray(wl.lambdas_um, np.float64)
    op = OrOpts(spp_begin=0, spp_count=wl.spp, spp_norm=float(wl.spp), max_depth=wl.max_depth,
                rr_enable=int(wl.rr_enable), rr_threshold24=rr_threshold24(wl.rr_p),
                rr_p=float(np.float32(wl.rr_p)), seed=wl.seed, use_bvh=1, n_threads=1, hero=0, aniso=int(aniso),
                composite=int(composite), reach_m=float(reach_m))
    sen = _sensor_struct(wl.sensor)
    srcs = _sources_struct(wl.sources)
    out = np.zeros((64, 12))
    val = np.zeros(1)
    n = lib().or_path_vertices(oscene.h, C.byref(sen), srcs, len(wl.sources), _dp(lam), lam.shape[0],
                               C.byref(op), int(px), int(py), int(s), int(w), _dp(out), 64, _dp(val))
    return float(val[0]), out[:n]


# ------------------------------------------------------------------------------------------
# Coherent measurement
# ------------------------------------------------------------------------------------------

def coherent_nodes(case, n_per_slit=16):
    """Emitter nodes: points as given; slits by Gauss-Legendre quadrature over each width
    (numpy's leggauss)."""
    if case.kind == "points":
        xs = np.asarray(case.centres_um, np.float64)
        return xs, np.ones_like(xs)
    t, w = np.polynomial.legendre.leggauss(n_per_slit)
    xs = np.concatenate([c + 0.5 * case.width_um * t for c in case.centres_um])
    ws = np.concatenate([0.5 * case.width_um * w for _ in case.centres_um])
    return xs, ws


def _coh_struct(case, xs, ws, spp=None):
    st = OrCoherent()
    st.kind = 0 if case.kind == "points" else 1
    st.n_nodes = xs.shape[0]
    st.xs = _dp(xs)
    st.ws = _dp(ws)
    st.z_um = case.z_m * 1e6
    st.lambda_um = case.lambda_um
    st.width = case.width
    st.height = case.height
    st.pitch_um = case.pitch_um
    st.sigma_um = case.sigma_um
    st.spp = case.spp if spp is None else spp
    st.seed = case.seed
    return st


def coherent_mc(case, n_per_slit=16, n_threads=0, rows=None):
    """Per-sample estimator of the coherent measurement, [rows, width] (the leading rows of
    the case's sensor; sample streams use its full height)."""
    xs, ws = coherent_nodes(case, n_per_slit)
    xs = np.ascontiguousarray(xs)
    ws = np.ascontiguousarray(ws)
    st = _coh_struct(case, xs, ws)
    rows = case.height if rows is None else rows
    out = np.empty((rows, case.width))
    lib().or_coherent_mc(C.byref(st), _dp(out), n_threads, rows)
    return out


def coherent_exact(case, xpix, n_per_slit=16, n_gh=48, n_gl=16):
    """Expectation of the coherent measurement at the given pixel columns (row 0)."""
    xs, ws = coherent_nodes(case, n_per_slit)
    xs = np.ascontiguousarray(xs)
    ws = np.ascontiguousarray(ws)
    st = _coh_struct(case, xs, ws)
    ghx, ghw = np.polynomial.hermite.hermgauss(n_gh)
    glx, glw = np.polynomial.legendre.leggauss(n_gl)
    xp = np.ascontiguousarray(np.asarray(xpix, np.int32))
    out = np.empty(xp.shape[0])
    lib().or_coherent_exact(C.byref(st), xp.ctypes.data_as(C.POINTER(C.c_int32)), xp.shape[0],
                            _dp(np.ascontiguousarray(ghx)), _dp(np.ascontiguousarray(ghw)), n_gh,
                            _dp(np.ascontiguousarray(glx)), _dp(np.ascontiguousarray(glw)), n_gl,
                            _dp(out))
    return out


def hankel1(x):
    return complex(lib().or_hankel1_re(float(x)), lib().or_hankel1_im(float(x)))
