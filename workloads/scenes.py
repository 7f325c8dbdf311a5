"""Seeded scene, sensor and source generators.

Units: geometry, sensor pitch and sensor window in metres; surface heights,
correlation lengths, grating pitches, coherence radii and wavelengths in
micrometres.

Every generator is deterministic in its seed.  The functions here only lay out
data; the renderer and the oracle each interpret it with their own code.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SMOOTH, ROUGH, GRATING = 0, 1, 2
PLANE_WAVE, GSM_AREA = 0, 1


@dataclass
class Material:
    kind: int                 # SMOOTH, ROUGH (gaussian random) or GRATING (1-D sinusoid)
    height_um: float = 0.0    # rough: RMS height s; grating: amplitude A (half the peak-to-valley depth)
    length_um: float = 1.0    # rough: 1/e correlation length; grating: pitch
    gdir: tuple = (1.0, 0.0, 0.0)   # grating vector direction in world space
    reflectance: float = 1.0


@dataclass
class Sensor:
    origin: np.ndarray        # corner of pixel (0, 0), metres
    axis_u: np.ndarray        # unit vector along +x pixels
    axis_v: np.ndarray        # unit vector along +y pixels
    dir: np.ndarray           # unit viewing direction (into the scene)
    width: int
    height: int
    pitch_m: float
    sigma_m: float            # intensity standard deviation of a detection state


@dataclass
class Source:
    kind: int                 # PLANE_WAVE or GSM_AREA
    dir: np.ndarray           # plane wave: travel direction; area: emission axis (unit)
    pos: np.ndarray = field(default_factory=lambda: np.zeros(3))   # area: emitter centre
    eu: np.ndarray = field(default_factory=lambda: np.zeros(3))    # area: half-extent vector 1
    ev: np.ndarray = field(default_factory=lambda: np.zeros(3))    # area: half-extent vector 2
    coherence_radius_um: float = 0.0
    power: float = 1.0


@dataclass
class Scene:
    verts: np.ndarray                 # float64 [nv, 3]
    tris: np.ndarray                  # int32 [nt, 3]
    tri_mat: np.ndarray               # int32 [nt]
    materials: List[Material]
    normals: Optional[np.ndarray] = None   # float64 [nv, 3] per-vertex shading normals

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


@dataclass
class Workload:
    name: str
    scene: Scene
    sensor: Sensor
    sources: List[Source]
    lambdas_um: np.ndarray
    spp: int
    max_depth: int
    seed: int
    rr_enable: bool = False
    rr_p: float = 0.8

    @property
    def n_paths(self) -> int:
        return self.sensor.width * self.sensor.height * self.spp * len(self.lambdas_um)


def wavelength_bins(n: int, lo_nm: float = 400.0, hi_nm: float = 700.0) -> np.ndarray:
    """Bin centres of n equal bins over [lo, hi] nm, returned in micrometres."""
    i = np.arange(n, dtype=np.float64)
    return (lo_nm + (i + 0.5) * (hi_nm - lo_nm) / n) * 1e-3


def _unit(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _ortho_sensor(centre, view_dir, up_hint, width, height, pitch, sigma) -> Sensor:
    d = _unit(view_dir)
    u = np.cross(up_hint, d)
    u = _unit(u)
    v = _unit(np.cross(d, u))
    origin = np.asarray(centre, np.float64) - 0.5 * width * pitch * u - 0.5 * height * pitch * v
    return Sensor(origin=origin, axis_u=u, axis_v=v, dir=d, width=width, height=height,
                  pitch_m=pitch, sigma_m=sigma)


# --------------------------------------------------------------------------------------
# Tiny: one grating quad under a plane wave
# --------------------------------------------------------------------------------------

def tiny_grating(width: int = 32, height: int = 32, spp: int = 8, seed: int = 1) -> Workload:
    """1 mm square quad in z=0 with h(x) = 0.1 sin(2 pi x / 2) um, lit by a plane wave at
    30 degrees in the x-z plane, lambda = 0.55 um, seen by an orthographic 32x32 sensor 1 cm
    away whose axis is the reversed +1 diffraction order (sin(theta) = 0.5 - 0.55/2)."""
    half = 0.5e-3
    verts = np.array([[-half, -half, 0.0], [half, -half, 0.0], [half, half, 0.0],
                      [-half, half, 0.0]], np.float64)
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    mats = [Material(GRATING, height_um=0.1, length_um=2.0, gdir=(1.0, 0.0, 0.0))]
    scene = Scene(verts=verts, tris=tris, tri_mat=np.zeros(2, np.int32), materials=mats,
                  normals=None)
    s_o = 0.5 - 0.55 / 2.0
    out_dir = np.array([s_o, 0.0, math.sqrt(1.0 - s_o * s_o)])   # +1 order, leaving the quad
    view = -out_dir
    pitch = 1e-3 / 32.0
    centre = 0.01 * out_dir
    sensor = _ortho_sensor(centre, view, np.array([0.0, 1.0, 0.0]), width, height, pitch, 20e-6)
    th = math.radians(30.0)
    src = Source(PLANE_WAVE, dir=np.array([math.sin(th), 0.0, -math.cos(th)]), power=1.0)
    return Workload("tiny-grating", scene, sensor, [src], np.array([0.55]), spp=spp,
                    max_depth=1, seed=seed)


def parallel_mirror(width: int = 16, height: int = 16, spp: int = 4, n_lambda: int = 8,
                    seed: int = 5) -> Workload:
    """1 mm square smooth quad in z=0 under a plane wave travelling along -z, seen at normal
    incidence by an orthographic sensor 1 cm above it (its axis along -z): every path meets
    the quad at the same distance and is lit at the mirror direction, so each path of a given
    wavelength contributes the same value, whatever its random numbers."""
    half = 0.5e-3
    verts = np.array([[-half, -half, 0.0], [half, -half, 0.0], [half, half, 0.0],
                      [-half, half, 0.0]], np.float64)
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    scene = Scene(verts=verts, tris=tris, tri_mat=np.zeros(2, np.int32),
                  materials=[Material(SMOOTH, reflectance=0.9)], normals=None)
    pitch = 0.5e-3 / width
    sensor = _ortho_sensor(np.array([0.0, 0.0, 0.01]), np.array([0.0, 0.0, -1.0]),
                           np.array([0.0, 1.0, 0.0]), width, height, pitch, 20e-6)
    src = Source(PLANE_WAVE, dir=np.array([0.0, 0.0, -1.0]), power=1.0)
    return Workload("parallel-mirror", scene, sensor, [src], wavelength_bins(n_lambda), spp=spp,
                    max_depth=2, seed=seed)


def grating_relay(width: int = 16, height: int = 16, spp: int = 8, seed: int = 9,
                  height_m: float = 2e-3) -> Workload:
    """A grating relayed by a mirror.  A 0.5 mm square grating quad in z=0 (pitch 1 um,
    amplitude 0.1 um, grooves across x) is seen at normal incidence by an orthographic sensor
    1 cm above it, lambda = 0.55 um.  Its -1 order (sin(o) = 0.55, towards +x) meets a smooth
    mirror (reflectance 0.9) in the plane z = height_m, facing down and off to the side of the
    sensor's view, and a plane wave travelling along (-sin(o), 0, cos(o)) reaches that mirror at
    the specular direction of the relayed beam.  Light reaches the sensor only through the -1
    order and the mirror: the other propagating orders miss the mirror, and the grating cannot
    see the source.  Every such path has the same geometry, so its contribution depends only on
    the ray's footprint on the mirror."""
    lam = 0.55
    s_o = lam / 1.0
    c_o = math.sqrt(1.0 - s_o * s_o)
    half = 0.25e-3
    xm = height_m * s_o / c_o                        # where the beam from x = 0 meets the mirror
    verts = np.array([[-half, -half, 0.0], [half, -half, 0.0], [half, half, 0.0], [-half, half, 0.0],
                      [xm - 0.3e-3, -0.3e-3, height_m], [xm + 0.3e-3, -0.3e-3, height_m],
                      [xm + 0.3e-3, 0.3e-3, height_m], [xm - 0.3e-3, 0.3e-3, height_m]], np.float64)
    tris = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7]], np.int32)
    mats = [Material(GRATING, height_um=0.1, length_um=1.0, gdir=(1.0, 0.0, 0.0)),
            Material(SMOOTH, reflectance=0.9)]
    scene = Scene(verts=verts, tris=tris, tri_mat=np.array([0, 0, 1, 1], np.int32), materials=mats,
                  normals=None)
    pitch = 0.4e-3 / width
    sensor = _ortho_sensor(np.array([0.0, 0.0, 0.01]), np.array([0.0, 0.0, -1.0]),
                           np.array([0.0, 1.0, 0.0]), width, height, pitch, 20e-6)
    src = Source(PLANE_WAVE, dir=np.array([-s_o, 0.0, c_o]), power=1.0)
    return Workload("grating-relay", scene, sensor, [src], np.array([lam]), spp=spp, max_depth=2,
                    seed=seed)


def split_mirror(width: int = 64, height: int = 4, spp: int = 4, seed: int = 11,
                 left: Optional[Material] = None, right: Optional[Material] = None,
                 pitch: float = 6e-6, sigma: float = 10e-6, n_lambda: int = 1) -> Workload:
    """A 2 mm square in z=0 made of two 1 mm x 2 mm halves of different materials (x < 0:
    `left`, default smooth with reflectance 1; x > 0: `right`, default smooth with reflectance
    0.25), meshed as two quads that share the boundary edge x = 0 (6 vertices, 4 triangles).
    A plane wave travels along -z; an orthographic sensor 1 cm above looks straight down, its
    rows across the boundary (pixel x grows with world x, the sensor centred on the boundary),
    so every path meets the surface at normal incidence at the mirror direction of the light."""
    h = 1e-3
    verts = np.array([[-h, -h, 0.0], [0.0, -h, 0.0], [h, -h, 0.0],
                      [-h, h, 0.0], [0.0, h, 0.0], [h, h, 0.0]], np.float64)
    tris = np.array([[0, 1, 4], [0, 4, 3], [1, 2, 5], [1, 5, 4]], np.int32)
    mats = [left if left is not None else Material(SMOOTH, reflectance=1.0),
            right if right is not None else Material(SMOOTH, reflectance=0.25)]
    scene = Scene(verts=verts, tris=tris, tri_mat=np.array([0, 0, 1, 1], np.int32), materials=mats,
                  normals=None)
    sensor = _ortho_sensor(np.array([0.0, 0.0, 0.01]), np.array([0.0, 0.0, -1.0]),
                           np.array([0.0, -1.0, 0.0]), width, height, pitch, sigma)
    src = Source(PLANE_WAVE, dir=np.array([0.0, 0.0, -1.0]), power=1.0)
    lam = np.array([0.55]) if n_lambda == 1 else wavelength_bins(n_lambda)
    return Workload("split-mirror", scene, sensor, [src], lam, spp=spp, max_depth=1, seed=seed)


def rough_box(width: int = 16, height: int = 16, spp: int = 4, max_depth: int = 64, seed: int = 13,
              reflectance: float = 0.9) -> Workload:
    """A closed 1 cm cube of Gaussian rough walls (RMS 0.05 um, correlation length 2 um,
    reflectance 0.9) with a partially coherent 4 mm emitter inside, 4 mm above the centre and
    facing down, seen by an orthographic sensor inside the cube looking down at 30 degrees:
    no path escapes, so every path runs to the depth limit unless it ends evanescently, and
    its measurements spread over all depths."""
    h = 5e-3
    c = np.array([[-h, -h, -h], [h, -h, -h], [h, h, -h], [-h, h, -h],
                  [-h, -h, h], [h, -h, h], [h, h, h], [-h, h, h]], np.float64)
    quads = [(0, 1, 2, 3), (4, 7, 6, 5), (0, 4, 5, 1), (1, 5, 6, 2), (2, 6, 7, 3), (3, 7, 4, 0)]
    tris = np.array([t for a, b, cc, d in quads for t in ((a, b, cc), (a, cc, d))], np.int32)
    mats = [Material(ROUGH, height_um=0.05, length_um=2.0, reflectance=reflectance)]
    scene = Scene(verts=c, tris=tris, tri_mat=np.zeros(len(tris), np.int32), materials=mats, normals=None)
    th = math.radians(30.0)
    view = np.array([math.sin(th), 0.0, -math.cos(th)])
    pitch = 2e-3 / max(width, height)
    sensor = _ortho_sensor(np.array([-1e-3, 0.0, 3e-3]), view, np.array([0.0, 1.0, 0.0]), width, height,
                           pitch, pitch / 4.0)
    src = Source(GSM_AREA, dir=np.array([0.0, 0.0, -1.0]), pos=np.array([0.0, 0.0, 4e-3]),
                 eu=np.array([2e-3, 0.0, 0.0]), ev=np.array([0.0, 2e-3, 0.0]),
                 coherence_radius_um=5.0, power=1.0)
    return Workload("rough-box", scene, sensor, [src], np.array([0.55]), spp=spp, max_depth=max_depth,
                    seed=seed)


# --------------------------------------------------------------------------------------
# Terrain: value-noise heightfield with per-tile materials
# --------------------------------------------------------------------------------------

def _value_noise(x, y, rng, octaves, base_lattice, amplitude, extent):
    h = np.zeros_like(x)
    for o in range(octaves):
        lat = base_lattice / (2 ** o)
        amp = amplitude / (2 ** o)
        n = int(math.ceil(extent / lat)) + 2
        vals = rng.uniform(-1.0, 1.0, size=(n + 1, n + 1))
        gx = x / lat
        gy = y / lat
        ix = np.floor(gx).astype(np.int64)
        iy = np.floor(gy).astype(np.int64)
        fx = gx - ix
        fy = gy - iy
        sx = fx * fx * fx * (fx * (fx * 6 - 15) + 10)
        sy = fy * fy * fy * (fy * (fy * 6 - 15) + 10)
        v00 = vals[iy, ix]
        v10 = vals[iy, ix + 1]
        v01 = vals[iy + 1, ix]
        v11 = vals[iy + 1, ix + 1]
        h += amp * ((v00 * (1 - sx) + v10 * sx) * (1 - sy) + (v01 * (1 - sx) + v11 * sx) * sy)
    return h


def _grid_mesh(nx, ny, extent_x, extent_y, heights):
    xs = np.linspace(0.0, extent_x, nx + 1)
    ys = np.linspace(0.0, extent_y, ny + 1)
    X, Y = np.meshgrid(xs, ys)
    verts = np.stack([X.ravel(), Y.ravel(), heights.ravel()], axis=1)
    i = np.arange(nx)
    j = np.arange(ny)
    I, J = np.meshgrid(i, j)
    v00 = (J * (nx + 1) + I).ravel()
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    t0 = np.stack([v00, v10, v11], 1)
    t1 = np.stack([v00, v11, v01], 1)
    tris = np.empty((2 * nx * ny, 3), np.int64)
    tris[0::2] = t0
    tris[1::2] = t1
    quad_i = np.repeat(I.ravel(), 2)
    quad_j = np.repeat(J.ravel(), 2)
    return verts, tris.astype(np.int32), quad_i, quad_j


def _vertex_normals(verts, tris):
    p0 = verts[tris[:, 0]]
    p1 = verts[tris[:, 1]]
    p2 = verts[tris[:, 2]]
    fn = np.cross(p1 - p0, p2 - p0)          # area-weighted face normals
    n = np.zeros_like(verts)
    for c in range(3):
        np.add.at(n, tris[:, c], fn)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return n


def _draw_material(rng) -> Material:
    kind = int(rng.integers(0, 3))
    if kind == SMOOTH:
        return Material(SMOOTH)
    if kind == ROUGH:
        return Material(ROUGH, height_um=float(rng.uniform(0.05, 0.5)),
                        length_um=float(rng.uniform(0.5, 5.0)))
    pitch = float(rng.uniform(0.8, 4.0))
    depth = float(rng.uniform(0.05, 0.3))      # peak-to-valley
    ang = float(rng.uniform(0.0, math.pi))
    return Material(GRATING, height_um=0.5 * depth, length_um=pitch,
                    gdir=(math.cos(ang), math.sin(ang), 0.0))


def terrain_scene(nx=256, ny=128, extent=0.1, seed=2, tiles=16, octaves=4,
                  base_lattice=0.0125, amplitude=0.005, material_seed=None) -> Scene:
    """Value-noise terrain of 2*nx*ny triangles over an extent x extent metre square, with
    one material per tile of a tiles x tiles partition."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, extent, nx + 1)
    ys = np.linspace(0.0, extent, ny + 1)
    X, Y = np.meshgrid(xs, ys)
    H = _value_noise(X, Y, rng, octaves, base_lattice, amplitude, extent)
    verts, tris, qi, qj = _grid_mesh(nx, ny, extent, extent, H)
    normals = _vertex_normals(verts, tris)
    mrng = np.random.default_rng(seed + 1000 if material_seed is None else material_seed)
    mats = [_draw_material(mrng) for _ in range(tiles * tiles)]
    tx = (qi * tiles) // nx
    ty = (qj * tiles) // ny
    tri_mat = (ty * tiles + tx).astype(np.int32)
    return Scene(verts=verts, tris=tris, tri_mat=tri_mat, materials=mats, normals=normals)


def _gsm_emitter(target, azimuth_deg, elevation_deg, dist, size, rc_um, power=1.0) -> Source:
    az = math.radians(azimuth_deg)
    el = math.radians(elevation_deg)
    # emission axis points down onto the target
    axis = _unit([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), -math.sin(el)])
    pos = np.asarray(target, np.float64) - dist * axis
    side = _unit(np.cross(axis, [0.0, 0.0, 1.0]))
    other = _unit(np.cross(side, axis))
    return Source(GSM_AREA, dir=axis, pos=pos, eu=0.5 * size * side, ev=0.5 * size * other,
                  coherence_radius_um=rc_um, power=power)


def mid_terrain(width=512, height=512, spp=16, n_lambda=8, max_depth=4, seed=3,
                window=None) -> Workload:
    """The mid-size plain-method workload: 65,536-triangle terrain (10 cm, 16x16 material
    tiles), one partially coherent 4x4 cm emitter 10 cm up with its axis 45 degrees down
    onto the terrain, an orthographic sensor whose axis is 30 degrees off vertical.

    ``window`` = (x0, y0, w, h) keeps the full-resolution pixel grid but renders only that
    sub-rectangle (the sensor origin moves; pitch and sigma are unchanged)."""
    scene = terrain_scene(seed=2)
    srng = np.random.default_rng(seed)
    rc = float(srng.uniform(5.0, 50.0))
    centre = np.array([0.05, 0.05, 0.0])
    # emitter 10 cm above the terrain plane, axis 45 degrees down through the terrain centre
    src = _gsm_emitter(centre, azimuth_deg=0.0, elevation_deg=45.0, dist=0.1 * math.sqrt(2.0),
                       size=0.04, rc_um=rc)
    pitch = 0.1 / 512.0
    th = math.radians(30.0)
    view = np.array([-math.sin(th), 0.0, -math.cos(th)])
    sens_centre = centre - 0.2 * view
    sensor = _ortho_sensor(sens_centre, view, np.array([0.0, 0.0, 1.0]), 512, 512, pitch,
                           pitch / 4.0)
    if width != 512 or height != 512 or window is not None:
        if window is None:
            # same field of view at lower resolution
            pitch_w = 0.1 / width
            pitch_h = 0.1 / height
            pitch = max(pitch_w, pitch_h)
            sensor = _ortho_sensor(sens_centre, view, np.array([0.0, 0.0, 1.0]), width, height,
                                   pitch, pitch / 4.0)
        else:
            x0, y0, w, h = window
            sensor = Sensor(origin=sensor.origin + x0 * pitch * sensor.axis_u
                            + y0 * pitch * sensor.axis_v,
                            axis_u=sensor.axis_u, axis_v=sensor.axis_v, dir=sensor.dir,
                            width=w, height=h, pitch_m=pitch, sigma_m=pitch / 4.0)
    return Workload("mid-terrain", scene, sensor, [src], wavelength_bins(n_lambda), spp=spp,
                    max_depth=max_depth, seed=seed)


# --------------------------------------------------------------------------------------
# Large: instanced displaced tiles plus random boxes
# --------------------------------------------------------------------------------------

def _box_tris(lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    f = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]], np.int64)
    return v, f


def large_scene(n_inst_x=10, n_inst_y=6, n_boxes=21845, seed=6, tile_nx=256, tile_ny=128):
    """60 instances of one 65,536-triangle displaced terrain tile (random rotation by multiples
    of 90 degrees and a per-instance height offset), flattened, plus n_boxes random boxes of
    12 triangles each."""
    rng = np.random.default_rng(seed)
    tile = terrain_scene(nx=tile_nx, ny=tile_ny, seed=seed + 1)
    n_mat_tile = len(tile.materials)
    mrng = np.random.default_rng(seed + 2000)
    extra = [_draw_material(mrng) for _ in range(256)]
    materials = list(tile.materials) + extra
    verts_l, norms_l, tris_l, mats_l = [], [], [], []
    nv = 0
    ext = 0.1
    for iy in range(n_inst_y):
        for ix in range(n_inst_x):
            k = int(rng.integers(0, 4))
            c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][k]
            R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], np.float64)
            p = tile.verts - np.array([ext / 2, ext / 2, 0.0])
            p = p @ R.T + np.array([ix * ext + ext / 2, iy * ext + ext / 2,
                                    float(rng.uniform(-0.002, 0.002))])
            verts_l.append(p)
            norms_l.append(tile.normals @ R.T)
            tris_l.append(tile.tris.astype(np.int64) + nv)
            shift = int(rng.integers(0, n_mat_tile))
            mats_l.append(((tile.tri_mat + shift) % n_mat_tile).astype(np.int32))
            nv += p.shape[0]
    W = n_inst_x * ext
    Hh = n_inst_y * ext
    bx = rng.uniform(0.0, W, n_boxes)
    by = rng.uniform(0.0, Hh, n_boxes)
    sx = rng.uniform(0.002, 0.02, n_boxes)
    sy = rng.uniform(0.002, 0.02, n_boxes)
    sz = rng.uniform(0.002, 0.03, n_boxes)
    bz = rng.uniform(-0.004, 0.004, n_boxes)
    bm = rng.integers(n_mat_tile, n_mat_tile + 256, n_boxes)
    _, f = _box_tris((0, 0, 0), (1, 1, 1))
    unit_v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                       [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], np.float64)
    lo = np.stack([bx - sx / 2, by - sy / 2, bz], 1)
    size = np.stack([sx, sy, sz], 1)
    bv = lo[:, None, :] + unit_v[None, :, :] * size[:, None, :]     # [n, 8, 3]
    bt = f[None, :, :] + (nv + 8 * np.arange(n_boxes))[:, None, None]
    verts_l.append(bv.reshape(-1, 3))
    # boxes are faceted: their vertex normals are left to the geometric normal (marked by 0)
    norms_l.append(np.zeros((8 * n_boxes, 3)))
    tris_l.append(bt.reshape(-1, 3))
    mats_l.append(np.repeat(bm, 12).astype(np.int32))
    verts = np.concatenate(verts_l)
    normals = np.concatenate(norms_l)
    tris = np.concatenate(tris_l).astype(np.int32)
    tri_mat = np.concatenate(mats_l).astype(np.int32)
    return Scene(verts=verts, tris=tris, tri_mat=tri_mat, materials=materials, normals=normals)


def large_workload(width=1920, height=1080, spp=64, n_lambda=16, max_depth=6, seed=6,
                   scene=None) -> Workload:
    scene = large_scene(seed=seed) if scene is None else scene
    rng = np.random.default_rng(seed + 1)
    W, H = 1.0, 0.6
    n_src = int(rng.integers(1, 4))
    sources = []
    for _ in range(n_src):
        tgt = np.array([rng.uniform(0.2, 0.8) * W, rng.uniform(0.2, 0.8) * H, 0.0])
        sources.append(_gsm_emitter(tgt, azimuth_deg=float(rng.uniform(0, 360)),
                                    elevation_deg=float(rng.uniform(35, 70)), dist=0.3,
                                    size=0.3, rc_um=float(rng.uniform(5.0, 200.0))))
    pitch = W / width
    th = math.radians(25.0)
    view = np.array([-math.sin(th), 0.0, -math.cos(th)])
    centre = np.array([W / 2, H / 2, 0.0]) - 0.8 * view
    sensor = _ortho_sensor(centre, view, np.array([0.0, 0.0, 1.0]), width, height, pitch,
                           pitch / 4.0)
    return Workload("large-instanced", scene, sensor, sources, wavelength_bins(n_lambda),
                    spp=spp, max_depth=max_depth, seed=seed, rr_enable=True, rr_p=0.8)


def as_float32_inputs(wl: Workload) -> Workload:
    """The same workload with every real-valued input rounded to float32: the values a float32
    interface (the GPU library's scene, sensor and source structures) actually receives, so that
    a float64 consumer of the returned workload sees identical geometry."""
    def r(x):
        return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)

    def rf(x):
        return float(np.float32(x))

    sc = wl.scene
    scene = Scene(verts=r(sc.verts), tris=sc.tris, tri_mat=sc.tri_mat,
                  materials=[Material(m.kind, rf(m.height_um), rf(m.length_um),
                                      tuple(float(v) for v in r(m.gdir)), rf(m.reflectance))
                             for m in sc.materials],
                  normals=None if sc.normals is None else r(sc.normals))
    sn = wl.sensor
    sensor = Sensor(origin=r(sn.origin), axis_u=r(sn.axis_u), axis_v=r(sn.axis_v), dir=r(sn.dir),
                    width=sn.width, height=sn.height, pitch_m=rf(sn.pitch_m),
                    sigma_m=rf(sn.sigma_m))
    sources = [Source(kind=q.kind, dir=r(q.dir), pos=r(q.pos), eu=r(q.eu), ev=r(q.ev),
                      coherence_radius_um=rf(q.coherence_radius_um), power=rf(q.power))
               for q in wl.sources]
    return Workload(wl.name, scene, sensor, sources, r(wl.lambdas_um), spp=wl.spp,
                    max_depth=wl.max_depth, seed=wl.seed, rr_enable=wl.rr_enable, rr_p=wl.rr_p)


# --------------------------------------------------------------------------------------
# Coherent double-slit / two-point cases
# --------------------------------------------------------------------------------------

@dataclass
class CoherentCase:
    """Apertures in the plane z = 0 lit by a normal plane wave (slits) or two mutually
    coherent point emitters (points); a 1-D row of pixels (width) repeated over height rows
    at distance z_m.  Slits are infinitely long along y, so the field is y-independent."""
    kind: str                   # "slits" or "points"
    centres_um: np.ndarray      # x centres of the slits / points (um)
    width_um: float             # slit width b (unused for points)
    z_m: float
    lambda_um: float
    width: int
    height: int
    pitch_um: float
    sigma_um: float
    spp: int
    seed: int


def coherent_case(kind="slits", z_m=1.0, lambda_um=0.55, sigma_mode="pitch", width=1024,
                  height=64, spp=64, seed=5, separation_um=50.0, slit_um=10.0) -> CoherentCase:
    """Double slit (b = 10 um, d = 50 um) or two points 50 um apart.  The sensor pitch shows
    8 fringes of the mid wavelength (0.55 um) across the row; sigma is one pitch, or a quarter
    of the fringe period of this case's wavelength ("quarter")."""
    pitch_um = 8.0 * 0.55 * (z_m * 1e6) / (separation_um * width)
    period_um = lambda_um * (z_m * 1e6) / separation_um
    sigma_um = pitch_um if sigma_mode == "pitch" else period_um / 4.0
    c = np.array([-separation_um / 2.0, separation_um / 2.0])
    return CoherentCase(kind, c, slit_um, z_m, lambda_um, width, height, pitch_um, sigma_um,
                        spp, seed)


def surrogate_query_box():
    """Parameter ranges of the terrain material mix (um) that a learned scattering model
    is trained over."""
    return {
        "lambda_um": (0.4, 0.7),
        "rough_s_um": (0.05, 0.5),
        "rough_ell_um": (0.5, 5.0),
        "grating_pitch_um": (0.8, 4.0),
        "grating_amp_um": (0.025, 0.15),
    }
