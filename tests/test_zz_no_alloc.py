"""gr_trace_noalloc (the trace in the library's static device workspace) against gr_trace.

Two calls in a row through the C ABI, the second with a smaller input, each compared bit for
bit with gr_trace on the same options (same kernels, same launches, deterministic records),
plus the rejection of a trace whose workspace exceeds the static array."""

import numpy as np
import pytest

from paper_2303_15762_amd import Renderer
from paper_2303_15762_amd._lib import GrError
from workloads import scenes as W

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


@pytest.fixture(scope="module")
def R():
    r = Renderer(0)
    yield r
    r.close()


def _both(R, wl, spp, **kw):
    import torch
    o = R.opts(spp_count=spp, spp_norm=spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p, **kw)
    ws, need = R.workspace(o, len(wl.lambdas_um))
    assert need <= STATIC_BYTES, need
    ref, _ = R.trace(wl.lambdas_um, o, stats=False)
    img = torch.zeros_like(ref)
    R.trace_noalloc(wl.lambdas_um, o, img)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), img.cpu().numpy(), need


def test_noalloc_matches_trace_twice_then_smaller(R):
    wl = W.mid_terrain(width=41, height=29, spp=16, n_lambda=8)
    R.load_workload(wl)
    print("noalloc: mid terrain 41x29, 16 spp, 8 wavelengths, depth 4", flush=True)
    ref1, img1, need1 = _both(R, wl, 16)
    assert np.array_equal(ref1, img1)
    assert float(np.abs(ref1).sum()) > 0.0
    # a smaller input next: fewer samples, a smaller sensor; stale scratch contents must not
    # leak into it
    wl2 = W.mid_terrain(width=23, height=17, spp=4, n_lambda=8)
    R.load_workload(wl2)
    print("noalloc: mid terrain 23x17, 4 spp", flush=True)
    ref2, img2, need2 = _both(R, wl2, 4)
    assert need2 < need1
    assert np.array_equal(ref2, img2)
    assert float(np.abs(ref2).sum()) > 0.0


def test_noalloc_hero_and_accumulation(R):
    import torch
    wl = W.mid_terrain(width=24, height=16, spp=8, n_lambda=8)
    R.load_workload(wl)
    print("noalloc: hero-wavelength paths 24x16, 8 spp", flush=True)
    ref, img, _ = _both(R, wl, 8, hero=True)
    assert np.array_equal(ref, img)
    # contributions add to the caller's image: two half-sample renders sum to the full one
    o = dict(spp_norm=8, max_depth=wl.max_depth, seed=wl.seed, rr_enable=wl.rr_enable, rr_p=wl.rr_p)
    acc = torch.zeros((8, wl.sensor.height, wl.sensor.width), device=R.dev)
    R.trace_noalloc(wl.lambdas_um, R.opts(spp_begin=0, spp_count=4, **o), acc)
    R.trace_noalloc(wl.lambdas_um, R.opts(spp_begin=4, spp_count=4, **o), acc)
    full, _ = R.trace(wl.lambdas_um, R.opts(spp_begin=0, spp_count=8, **o), stats=False)
    torch.cuda.synchronize()
    a, f = acc.cpu().numpy().astype(np.float64), full.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(a - f) <= 1e-5 * np.linalg.norm(f)


@pytest.mark.parametrize("mode", ["scalar", "hero", "aniso"])
def test_noalloc_composite_interactions(R, mode):
    """Composite interactions (the scene's material boundaries read by the kernels) through the
    static workspace, scalar, hero-wavelength and anisotropic rays, bit for bit against
    gr_trace."""
    wl = W.mid_terrain(width=24, height=16, spp=8, n_lambda=8)
    R.load_workload(wl)
    R.boundaries(2e-3)
    print("noalloc: composite interactions 24x16, 8 spp,", mode, flush=True)
    ref, img, _ = _both(R, wl, 8, composite=True, hero=mode == "hero", aniso=mode == "aniso")
    assert np.array_equal(ref, img)
    assert float(np.abs(ref).sum()) > 0.0


def test_noalloc_rejects_oversized(R):
    import torch
    wl = W.mid_terrain(width=256, height=256, spp=16, n_lambda=8)
    R.load_workload(wl)
    o = R.opts(spp_count=16, spp_norm=16, max_depth=wl.max_depth, seed=wl.seed)
    _, need = R.workspace(o, 8)
    assert need > STATIC_BYTES
    img = torch.zeros((8, 256, 256), device=R.dev)
    with pytest.raises(GrError, match="static scratch"):
        R.trace_noalloc(wl.lambdas_um, o, img)
    torch.cuda.synchronize()
    assert float(img.abs().sum()) == 0.0
