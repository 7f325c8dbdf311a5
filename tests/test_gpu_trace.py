"""GPU parity of the HIP tracer against the FP64 oracle, through the C ABI.

Tolerance: relative L2 error of the image <= 1e-3 for the plain (closed-form) scattering path,
the bound stated for FP32 geometry and scattering arithmetic against the FP64 oracle.
"""

import math

import numpy as np
import pytest

import oracle
from workloads import scenes as W

pytestmark = pytest.mark.gpu

RTOL_IMAGE = 1e-3


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2303_15762_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


def _gpu_image(R, wl, **kw):
    R.load_workload(wl)
    img, st = R.render_workload(wl, **kw)
    return img.cpu().numpy().astype(np.float64), st


def test_tiny_grating_matches_oracle(R):
    wl = W.tiny_grating()
    g, st = _gpu_image(R, wl)
    o, ost = oracle.render(wl)
    print("tiny: rel L2", rel_l2(g, o), st)
    assert st["paths"] == 32 * 32 * 8
    assert st["segments"] == ost["segments"]
    assert st["shadow_rays"] == ost["shadow_rays"]
    # one grating: every measurement is counted in its class
    assert st["measured_grating"] == ost["measured_grating"] == st["shadow_rays"] > 0
    assert st["measured_smooth"] == st["measured_rough"] == 0
    assert rel_l2(g, o) <= 1e-5
    # interior pixel values agree one by one
    np.testing.assert_allclose(g[0, 4:28, 4:28], o[0, 4:28, 4:28], rtol=1e-5)


def test_tiny_grating_path_records(R):
    wl = W.tiny_grating(width=8, height=8, spp=4)
    R.load_workload(wl)
    opts = R.opts(spp_count=4, spp_norm=4, max_depth=1, seed=wl.seed, keep_paths=True)
    R.trace(wl.lambdas_um, opts)
    rec = R.path_records(opts, 1).cpu().numpy().astype(np.float64)   # [s, H, W, nl]
    _, _, paths = oracle.render(wl, keep_paths=True)                   # [s, npix, nl]
    np.testing.assert_allclose(rec.reshape(4, 64, 1), paths, rtol=1e-5, atol=1e-9)


def _random_queries(n, seed):
    rng = np.random.default_rng(seed)
    q = np.zeros((n, 14))
    q[:, 0] = rng.integers(0, 3, n)
    lam = rng.uniform(0.4, 0.7, n)
    k = 2 * np.pi / lam
    q[:, 4] = k
    rough = q[:, 0] == 1
    grat = q[:, 0] == 2
    q[:, 1] = np.where(rough, rng.uniform(0.05, 0.5, n), rng.uniform(0.025, 0.15, n))
    q[:, 2] = np.where(rough, rng.uniform(0.5, 5.0, n), rng.uniform(0.8, 4.0, n))
    q[:, 3] = 1.0
    th = rng.uniform(0, 1.2, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    q[:, 5] = k * np.sin(th) * np.cos(ph)
    q[:, 6] = k * np.sin(th) * np.sin(ph)
    sx = np.exp(rng.uniform(np.log(3), np.log(200), n))
    sy = np.exp(rng.uniform(np.log(3), np.log(200), n))
    rho = rng.uniform(-0.8, 0.8, n)
    q[:, 9] = sx * sx
    q[:, 10] = sy * sy
    q[:, 11] = rho * sx * sy
    # outgoing: near a lobe of the material (specular or a grating order) plus a spread
    K = 2 * np.pi / q[:, 2]
    j = np.where(grat, rng.integers(-2, 3, n), 0)
    spread = np.where(rough, rng.normal(0, 1.0, n), rng.normal(0, 1.0, n) / np.maximum(sx, sy))
    q[:, 7] = q[:, 5] - j * K + spread
    q[:, 8] = q[:, 6] + np.where(rough, rng.normal(0, 1.0, n), rng.normal(0, 1, n) / np.maximum(sx, sy))
    q[:, 12] = 1.0
    q[:, 13] = 0.0
    keep = (q[:, 7] ** 2 + q[:, 8] ** 2) < 0.98 * k * k
    return q[keep]


def test_bsdf_eval_matches_oracle(R):
    import torch
    # both sides evaluate the same query: the kernel reads FP32, so the oracle gets the
    # FP32-rounded values (the rounding alone moves p_w by ~1e-5 at narrow lobes)
    q = _random_queries(4000, 7).astype(np.float32).astype(np.float64)
    ref = oracle.pw_batch(q)
    got = R.bsdf_eval(torch.tensor(q, dtype=torch.float32, device=R.dev)).cpu().numpy()
    for kind in range(3):
        m = q[:, 0] == kind
        r, g = ref[m], got[m]
        big = r > 1e-4 * r.max()
        err = np.abs(g[big] - r[big]) / r[big]
        print("kind", kind, "n", big.sum(), "max rel err", err.max(), "median", np.median(err))
        assert np.median(err) < 1e-5
        assert np.quantile(err, 0.99) < 2e-3
        assert np.abs(g - r).max() <= 1e-3 * r.max()


def test_terrain_small_ragged_matches_oracle(R):
    """The mid workload's scene, samples per pixel, wavelengths and depth on a 41 x 29 sensor
    (a ragged tail of paths in the last wave)."""
    wl = W.mid_terrain(width=41, height=29, spp=16, n_lambda=8)
    g, st = _gpu_image(R, wl)
    o, ost = oracle.render(wl)
    e = rel_l2(g, o)
    print("terrain 41x29: rel L2", e, st, ost)
    assert st["paths"] == 41 * 29 * 16 * 8
    assert abs(st["segments"] - ost["segments"]) <= 1e-3 * ost["segments"]
    # measurements per material class (smooth, rough and grating tiles)
    for kind in ("smooth", "rough", "grating"):
        key = "measured_" + kind
        assert ost[key] > 0 and abs(st[key] - ost[key]) <= 1e-3 * ost[key] + 2, (key, st[key], ost[key])
    assert st["measured_smooth"] + st["measured_rough"] + st["measured_grating"] == st["shadow_rays"]
    assert e <= RTOL_IMAGE


def test_terrain_full_size_sampled_pixels(R):
    """The mid workload at its full size (512 x 512, 16 samples, 8 wavelengths, depth 4) in the
    launch configuration the benchmark times; the oracle computes a random subset of pixels
    one by one and the GPU image must match it there."""
    wl = W.mid_terrain()
    g, st = _gpu_image(R, wl)
    rng = np.random.default_rng(0)
    # oversample the lit region so that the check is not dominated by black pixels
    lit = np.argwhere(g.sum(0) > 0)
    pick_lit = lit[rng.choice(len(lit), size=min(400, len(lit)), replace=False)]
    pick_any = np.stack([rng.integers(0, 512, 200), rng.integers(0, 512, 200)], 1)
    pix_yx = np.concatenate([pick_lit, pick_any])
    pix = np.stack([pix_yx[:, 1], pix_yx[:, 0]], 1)
    o, _ = oracle.render(wl, pixels=pix)
    gs = g[:, pix_yx[:, 0], pix_yx[:, 1]]
    e = rel_l2(gs, o)
    print("terrain full: rel L2 on", len(pix), "pixels:", e, st)
    assert st["paths"] == 512 * 512 * 16 * 8
    assert e <= RTOL_IMAGE


def test_deterministic_and_spp_split(R):
    wl = W.mid_terrain(width=40, height=32, spp=6, n_lambda=3)
    R.load_workload(wl)
    a, _ = R.render_workload(wl)
    b, _ = R.render_workload(wl)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    p1, _ = R.render_workload(wl, spp_begin=0, spp_count=2)
    p2, _ = R.render_workload(wl, spp_begin=2, spp_count=4)
    np.testing.assert_allclose((p1 + p2).cpu().numpy(), a.cpu().numpy(), rtol=1e-5, atol=1e-9)


def test_traversal_stack_overflow_path(R):
    """With only 4 traversal-stack entries per lane in LDS, most of the stack of the terrain's
    BVH (depth 8: up to 27 entries) lives in the workspace's overflow region; the image and the
    path counters are unchanged.  The work counters agree to 0.1 %: shadow rays run in waves
    of whichever rays the queue holds together, and an any-hit query ends at the first hit its
    wave's traversal order reaches, so its node count depends on its neighbours."""
    wl = W.mid_terrain(width=41, height=29, spp=4, n_lambda=8)
    R.load_workload(wl)
    o = dict(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed)
    a, sa = R.trace(wl.lambdas_um, R.opts(**o))
    b, sb = R.trace(wl.lambdas_um, R.opts(short_lds_stack=True, **o))
    print("LDS stack 14:", sa, "LDS stack 4:", sb)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    for key in ("paths", "segments", "shadow_rays"):
        assert sa[key] == sb[key]
    for key in ("node_visits", "tri_tests"):
        assert abs(sa[key] - sb[key]) <= 1e-3 * sa[key]


def _terrain_variant(name):
    """The small terrain with rough surfaces on every tile (the Poisson-series p_w and its
    sampler everywhere), or with a second, plane-wave source, Russian roulette and paths of up
    to 6 interactions.  (Tiles of smooth or grating material alone leave the small sensor dark:
    their lobes are far narrower than the spread of terrain normals.)"""
    import dataclasses
    wl = W.mid_terrain(width=41, height=29, spp=8, n_lambda=8)
    rng = np.random.default_rng(17)
    sc = wl.scene
    if name == "rough":
        mats = [W.Material(W.ROUGH, height_um=float(rng.uniform(0.05, 0.5)),
                           length_um=float(rng.uniform(0.5, 5.0))) for _ in range(len(sc.materials))]
        return dataclasses.replace(wl, scene=dataclasses.replace(sc, materials=mats))
    th = math.radians(40.0)
    d = np.array([0.3 * math.sin(th), math.sin(th), -math.cos(th)])
    pw = W.Source(W.PLANE_WAVE, dir=d / np.linalg.norm(d), power=0.7)
    return dataclasses.replace(wl, sources=list(wl.sources) + [pw], max_depth=6, rr_enable=True,
                               rr_p=0.8)


@pytest.mark.parametrize("name", ["rough", "two_sources_rr"])
def test_terrain_variants_match_oracle(R, name):
    """The oracle gets the float32-rounded inputs the library receives: in the rough variant
    one path's narrow lobe moves its value 50-fold with the input rounding alone (2.2e-5 per
    path with equal inputs, 4e-2 without)."""
    wl = W.as_float32_inputs(_terrain_variant(name))
    g, st = _gpu_image(R, wl)
    o, ost = oracle.render(wl)
    e = rel_l2(g, o)
    print("terrain variant", name, ": rel L2", e, st, ost)
    assert o.sum() > 0 and st["nonfinite"] == 0 and st["shadow_rays"] > 0
    assert abs(st["segments"] - ost["segments"]) <= 1e-3 * ost["segments"]
    assert e <= RTOL_IMAGE


def test_edge_cases(R):
    import torch
    wl = W.mid_terrain(width=1, height=1, spp=3, n_lambda=1)
    g, st = _gpu_image(R, wl)
    o, _ = oracle.render(wl)
    assert st["paths"] == 3
    np.testing.assert_allclose(g, o, rtol=1e-4, atol=1e-12)
    # zero samples: the image is left untouched
    img = torch.full((1, 1, 1), 7.0, device=R.dev)
    out, st = R.trace(wl.lambdas_um, R.opts(spp_count=0, spp_norm=1, max_depth=4, seed=3), image=img)
    assert float(out[0, 0, 0]) == 7.0 and st["paths"] == 0


def test_no_sources_leave_the_image(R):
    """Without sources no vertex measures anything: every record is zero, so an image that
    already holds values keeps them exactly (the measurement slots of each vertex are still
    stored and merged)."""
    import torch
    wl = W.mid_terrain(width=24, height=16, spp=2, n_lambda=2)
    R.load_workload(wl)
    R.set_sources([])
    img = torch.full((2, 16, 24), 0.25, device=R.dev)
    out, st = R.trace(wl.lambdas_um, R.opts(spp_count=2, spp_norm=2, max_depth=4, seed=wl.seed), image=img)
    assert st["paths"] == 24 * 16 * 2 * 2 and st["segments"] >= st["paths"] and st["shadow_rays"] == 0
    assert bool((out == 0.25).all())
    R.set_sources(wl.sources)


@pytest.mark.parametrize("depth", [1, 9, 64])
def test_depth_limits_match_oracle(R, depth):
    """Path depth 1 (one slot per path), 9 and 64 (the largest allowed): the merge sums the
    slots each path stored, in depth order; terrain crop against the oracle."""
    import dataclasses
    wl = dataclasses.replace(W.mid_terrain(width=33, height=21, spp=3, n_lambda=2), max_depth=depth)
    g, st = _gpu_image(R, wl)
    o, ost = oracle.render(wl)
    err = rel_l2(g, o)
    print("depth", depth, "rel L2", err, "segments", st["segments"], ost["segments"])
    assert abs(st["segments"] - ost["segments"]) <= 1e-3 * ost["segments"]
    assert err <= RTOL_IMAGE


@pytest.mark.parametrize("depth", [9, 64])
def test_rough_box_deep_paths_match_oracle(R, depth):
    """A closed cube of rough walls with the emitter inside: no path escapes, so depth 64 runs
    every path to 64 interactions (6x the segments of depth 9) with measurements at all
    depths.  Compared path by path: a path whose record differs by more than 1 % has taken
    another discrete decision somewhere (an evanescent draw, a Poisson term, a grazing hit)
    because the decision's inputs carry the float rounding of dozens of earlier interactions;
    from there on its contributions are another path's.  Such paths must stay below 1e-3 of
    the paths (measured: 0 at depth 9, 2 of 8,192 at depth 64), and the image of the others
    within the plain path's 1e-3."""
    wl = W.rough_box(width=32, height=32, spp=8, max_depth=depth)
    R.load_workload(wl)
    opts = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed, keep_paths=True)
    img, st = R.trace(wl.lambdas_um, opts)
    rec = R.path_records(opts, 1).cpu().numpy().astype(np.float64).reshape(wl.spp, -1)
    o, ost, paths = oracle.render(wl, keep_paths=True)
    paths = paths[:, :, 0]
    err = rel_l2(img.cpu().numpy(), o)
    scale = np.abs(paths).max()
    flipped = np.abs(rec - paths) > 1e-2 * np.maximum(np.abs(paths), 1e-6 * scale)
    keep = ~flipped
    e_keep = rel_l2((rec * keep).sum(0), (paths * keep).sum(0))
    print("rough box depth", depth, "image rel L2", err, "paths with another decision", int(flipped.sum()), "of",
          flipped.size, "image of the others", e_keep, "segments", st["segments"], ost["segments"])
    assert ost["segments"] > (5 * 32 * 32 * 8 if depth == 64 else 0)
    assert abs(st["segments"] - ost["segments"]) <= 1e-3 * ost["segments"]
    assert flipped.sum() <= 1e-3 * flipped.size
    assert e_keep <= RTOL_IMAGE
    if depth <= 9:
        assert err <= RTOL_IMAGE


def test_terrain_full_frame_matches_oracle(R):
    """The mid workload's whole 512 x 512 x 8 image (16 samples, depth 4) against the oracle's
    whole image, in the launch configuration the benchmark times."""
    wl = W.as_float32_inputs(W.mid_terrain())
    g, st = _gpu_image(R, wl)
    o, ost = oracle.render(wl)
    err = rel_l2(g, o)
    d2 = ((g - o) ** 2).sum(0)
    y, x = np.unravel_index(int(np.argmax(d2)), d2.shape)
    print("mid full frame: rel L2", err, "segments", st["segments"], ost["segments"], "worst pixel", (x, y),
          "share of squared error", d2[y, x] / d2.sum())
    assert st["nonfinite"] == 0
    assert abs(st["segments"] - ost["segments"]) <= 1e-4 * ost["segments"]
    assert err <= RTOL_IMAGE
