"""Pins of the oracle's hero-wavelength paths (one path sampled at a hero wavelength carries
the four wavelengths of a rotation group, combined by the one-sample balance heuristic over
the four choices of hero).

Each check compares the oracle with something other than itself:
- a closed form: at normal incidence on a smooth mirror every path contributes the mirror's
  Gaussian-beam value refl * beta^2 / pi, beta^2 from the free-space law;
- the importance-sampling identity of one continuation step: a companion's ratios f_c / p_h
  and p_c / p_h, averaged over the hero's samples, must reproduce averages over the
  companion's own sampler (rough surfaces), or the order-0 closed form (gratings, whose other
  orders are dispersive deltas no companion shares);
- unbiasedness: the hero image and the one-wavelength-per-path image estimate the same
  integral, so on the terrain workload their per-wavelength totals agree within their
  statistical errors.
"""

import math

import numpy as np
import pytest
from scipy import special

import oracle
from workloads import mid_terrain, parallel_mirror


def test_hero_equals_closed_form_and_per_wavelength_paths_on_a_parallel_mirror():
    wl = parallel_mirror()
    hero, st_h = oracle.render(wl, hero=True)
    per, st_p = oracle.render(wl)
    # one path per rotation group: a quarter of the paths, each meeting the mirror once
    assert st_h["segments"] * 4 == st_p["segments"]
    sig = wl.sensor.sigma_m * 1e6
    b0 = 2.0 * sig * sig
    z = 0.01 * 1e6
    for w, lam in enumerate(wl.lambdas_um):
        k = 2.0 * math.pi / lam
        beta2 = b0 + (z / k) ** 2 / b0          # rho = 0 at the sensor
        ref = 0.9 * beta2 / math.pi             # refl N(0; Sigma_k) with Sigma_k = I / (2 beta^2)
        np.testing.assert_allclose(hero[w], ref, rtol=1e-9)
        np.testing.assert_allclose(per[w], ref, rtol=1e-9)


@pytest.mark.parametrize("h,L", [(0.05, 2.0), (0.1, 1.0), (0.3, 3.0), (0.02, 0.8)])
def test_hero_rough_step_importance_identity(h, L):
    rng = np.random.default_rng(int(h * 1000) + int(L * 10))
    n = 100000
    kh, kc = 2 * math.pi / 0.45, 2 * math.pi / 0.65
    th = 0.5
    ui, ci = (math.sin(th), 0.0), math.cos(th)
    a = oracle.hero_step(1, h, L, kh, kc, ui, ci, rng.random((n, 3)), refl=0.8)
    b = oracle.hero_step(1, h, L, kc, kc, ui, ci, rng.random((n, 3)), refl=0.8)
    ma, mb = np.isfinite(a[:, 0]), np.isfinite(b[:, 0])
    for cx, w in [(0.0, 0.05), (0.1, 0.1), (0.3, 0.2), (0.0, 1e-3)]:
        def phi(r, k, m):
            ux = np.where(m, r[:, 0], 0.0) / k - ui[0] - cx
            uy = np.where(m, r[:, 1], 0.0) / k
            return np.where(m, np.exp(-(ux ** 2 + uy ** 2) / (2 * w * w)), 0.0)
        pa, pb = phi(a, kh, ma), phi(b, kc, mb)
        for xa, xb in ((np.where(ma, a[:, 3], 0) * pa, np.where(mb, b[:, 2], 0) * pb),    # f
                       (np.where(ma, a[:, 4], 0) * pa, pb)):                               # p
            se = math.hypot(xa.std(), xb.std()) / math.sqrt(n)
            z = (xa.mean() - xb.mean()) / se
            assert abs(z) < 5.0, (cx, w, xa.mean(), xb.mean(), z)


@pytest.mark.parametrize("A,pitch,th", [(0.1, 2.0, 0.3), (0.05, 1.0, 0.6), (0.25, 3.5, 0.1)])
def test_hero_grating_step_shares_only_order_zero(A, pitch, th):
    rng = np.random.default_rng(7)
    n = 40000
    lh, lc = 0.42, 0.68
    kh, kc = 2 * math.pi / lh, 2 * math.pi / lc
    ui, ci = (math.sin(th), 0.0), math.cos(th)
    a = oracle.hero_step(2, A, pitch, kh, kc, ui, ci, rng.random((n, 3)), refl=0.7)
    ok = np.isfinite(a[:, 0])
    order0 = ok & (np.abs(a[:, 0] / kh - ui[0]) < 1e-12) & (np.abs(a[:, 1]) < 1e-12)
    assert np.all(a[ok & ~order0, 3] == 0.0) and np.all(a[ok & ~order0, 4] == 0.0)

    def weights(k):
        K = 2 * math.pi / pitch
        W, w0 = 0.0, 0.0
        for j in range(-60, 61):
            ox = k * ui[0] - j * K
            no = (ox / k) ** 2
            if no >= 1.0:
                continue
            bj = special.jv(j, k * A * (ci + math.sqrt(1.0 - no))) ** 2
            W += bj
            w0 += bj if j == 0 else 0.0
        return W, w0

    Wh, w0h = weights(kh)
    Wc, w0c = weights(kc)
    # the hero draws order 0 with probability J0^2 / W at its own wavelength
    frac = order0.mean()
    assert abs(frac - w0h / Wh) < 5 * math.sqrt(w0h / Wh * (1 - w0h / Wh) / n) + 1e-12
    # on order 0 the ratios are constants fixed by both wavelengths' order weights
    if order0.any():
        np.testing.assert_allclose(a[order0, 3], 0.7 * w0c / (w0h / Wh), rtol=1e-10)
        np.testing.assert_allclose(a[order0, 4], (w0c / Wc) / (w0h / Wh), rtol=1e-10)


def test_hero_image_unbiased_on_terrain():
    wl = mid_terrain()
    rng = np.random.default_rng(11)
    npx, spp = 2000, 48
    pix = np.stack([rng.integers(0, 512, npx), rng.integers(0, 512, npx)], 1)
    sc = oracle.OracleScene(wl.scene)
    _, _, pa = oracle.render(wl, oscene=sc, pixels=pix, spp_count=spp, keep_paths=True)
    _, sh, pb = oracle.render(wl, oscene=sc, pixels=pix, spp_count=spp, keep_paths=True, hero=True)
    assert sh["shadow_rays"] > 0
    zs = []
    for w in range(len(wl.lambdas_um)):
        xa, xb = pa[:, :, w].sum(1), pb[:, :, w].sum(1)      # per-sample totals (independent)
        se = math.sqrt(spp * (xa.var(ddof=1) + xb.var(ddof=1)))
        zs.append((xb.sum() - xa.sum()) / se)
    print("hero vs per-wavelength paths, z per wavelength:", np.round(zs, 2))
    # (the four members of a rotation group share their paths, so the eight z are not
    # independent; each is tested on its own)
    assert np.all(np.abs(zs) < 4.5)
