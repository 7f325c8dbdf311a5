"""GPU parity of anisotropic generalized rays (GR_TRACE_ANISO) against the oracle's, through the
C ABI.  Both sides draw the same Philox streams as the scalar rays, so images are compared
element by element at the plain path's bound, rel. L2 <= 1e-3; the grating relay is also held
to its closed-form image ratio.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2303_15762_amd._lib import GrError
from workloads import scenes as W

pytestmark = pytest.mark.gpu

RTOL_IMAGE = 1e-3


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def relay_ratio(height_m):
    # the closed form of tests/test_oracle_aniso.py (Gaussian-beam law per axis, in-plane
    # magnification cos(o) at the grating)
    lam, sig, L1 = 0.55, 20.0, 1e4
    k = 2.0 * math.pi / lam
    b0 = 2.0 * sig * sig
    co = math.sqrt(1.0 - lam * lam)
    z1, z2 = L1 / k, height_m * 1e6 / co / k
    b1, r1, a = b0 + z1 * z1 / b0, z1 / b0, 1.0 / b0
    along = co * co * b1 + 2.0 * z2 * r1 + z2 * z2 * a / (co * co)
    return math.sqrt(along / (b0 + (z1 + z2) ** 2 / b0))


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2303_15762_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


@pytest.mark.parametrize("height_m", [2e-3, 5e-3])
def test_aniso_grating_relay_ratio_and_oracle(R, height_m):
    wl = W.grating_relay(height_m=height_m)
    R.load_workload(wl)
    a, st = R.render_workload(wl, aniso=True)
    s, _ = R.render_workload(wl)
    a = a.cpu().numpy().astype(np.float64)
    s = s.cpu().numpy().astype(np.float64)
    lit = s[0] > 0
    print("relay", height_m, st, "lit", int(lit.sum()))
    assert lit.sum() > 200 and st["nonfinite"] == 0
    r = a[0][lit] / s[0][lit]
    print("relay ratio", r.min(), r.max(), "closed form", relay_ratio(height_m))
    np.testing.assert_allclose(r, relay_ratio(height_m), rtol=2e-5)
    o, _ = oracle.render(wl, aniso=True)
    e = rel_l2(a, o)
    print("relay vs oracle: rel L2", e)
    assert e <= RTOL_IMAGE


def test_aniso_parallel_mirror_equals_scalar(R):
    wl = W.parallel_mirror()
    R.load_workload(wl)
    a, _ = R.render_workload(wl, aniso=True)
    s, _ = R.render_workload(wl)
    np.testing.assert_allclose(a.cpu().numpy(), s.cpu().numpy(), rtol=2e-6)


def test_aniso_terrain_small_ragged_matches_oracle(R):
    """The mid workload's scene, samples, wavelengths and depth on a 41 x 29 sensor, with
    per-path records."""
    wl = W.mid_terrain(width=41, height=29, spp=16, n_lambda=8)
    R.load_workload(wl)
    img, st = R.render_workload(wl, aniso=True, keep_paths=True)
    g = img.cpu().numpy().astype(np.float64)
    o, ost, op = oracle.render(wl, aniso=True, keep_paths=True)
    e = rel_l2(g, o)
    print("aniso terrain 41x29: rel L2", e, st, ost)
    assert st["nonfinite"] == 0
    assert abs(st["segments"] - ost["segments"]) <= 1e-3 * ost["segments"]
    assert e <= RTOL_IMAGE
    opts = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
                  keep_paths=True, aniso=True)
    rec = R.path_records(opts, 8).cpu().numpy().astype(np.float64).reshape(16, 41 * 29, 8)
    er = rel_l2(rec, op)
    print("aniso terrain 41x29 records: rel L2", er)
    assert er <= RTOL_IMAGE


def test_aniso_two_sources_roulette_depth6(R):
    import dataclasses
    wl = W.mid_terrain(width=41, height=29, spp=8, n_lambda=8)
    th = math.radians(40.0)
    d = np.array([0.3 * math.sin(th), math.sin(th), -math.cos(th)])
    pw = W.Source(W.PLANE_WAVE, dir=d / np.linalg.norm(d), power=0.7)
    wl = W.as_float32_inputs(dataclasses.replace(wl, sources=list(wl.sources) + [pw], max_depth=6,
                                                 rr_enable=True, rr_p=0.8))
    R.load_workload(wl)
    img, st = R.render_workload(wl, aniso=True)
    g = img.cpu().numpy().astype(np.float64)
    o, ost = oracle.render(wl, aniso=True)
    e = rel_l2(g, o)
    print("aniso two sources, RR, depth 6: rel L2", e, st, ost)
    assert o.sum() > 0 and st["nonfinite"] == 0
    assert e <= RTOL_IMAGE


def test_aniso_terrain_full_size_sampled_pixels(R):
    wl = W.as_float32_inputs(W.mid_terrain())
    R.load_workload(wl)
    img, st = R.render_workload(wl, aniso=True)
    g = img.cpu().numpy().astype(np.float64)
    assert st["paths"] == 512 * 512 * 16 * 8 and st["nonfinite"] == 0
    rng = np.random.default_rng(6)
    lit = np.argwhere(g.sum(0) > 0)
    pick_lit = lit[rng.choice(len(lit), size=min(400, len(lit)), replace=False)]
    pick_any = np.stack([rng.integers(0, 512, 200), rng.integers(0, 512, 200)], 1)
    pix_yx = np.concatenate([pick_lit, pick_any])
    pix = np.stack([pix_yx[:, 1], pix_yx[:, 0]], 1)
    o, _ = oracle.render(wl, pixels=pix, aniso=True)
    e = rel_l2(g[:, pix_yx[:, 0], pix_yx[:, 1]], o)
    print("aniso terrain full: rel L2 on", len(pix), "pixels:", e, st)
    assert e <= RTOL_IMAGE


def test_aniso_rejected_where_unsupported(R):
    wl = W.mid_terrain(width=8, height=8, spp=1, n_lambda=4)
    R.load_workload(wl)
    for kw in (dict(hero=True), dict(bsdf_mode=1)):
        o = R.opts(spp_count=1, max_depth=2, seed=1, aniso=True, **kw)
        with pytest.raises(GrError):
            R.trace(wl.lambdas_um, o)
