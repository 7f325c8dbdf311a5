"""More pins of the FP64 oracle: parts of the path loop and of the learned model's training that
nothing else checks independently.

- Russian roulette (Sec. "Interactive Rendering", implementation details): the exact weighting
  of each path that survives, the depth at which the roulette starts, and unbiasedness.
- Shading-normal interpolation at a hit (barycentric weights) against a hand-computed mirror.
- Adam against PyTorch's own implementation in double precision.
- Rayleigh-Sommerfeld slit quadrature of the coherent measurement: converged.
- Grating order sampler in the ray-optics limit (large phase amplitude, pitch >> wavelength):
  the order histogram approaches the arcsine law of the sinusoid's slopes.
- Gaussian rough p_w (Sec. "Interaction Kernels", ensemble-averaged scatter) against a Monte
  Carlo average over synthesised Gaussian random surfaces of the defining integral.
"""

import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from workloads import scenes as W


# --------------------------------------------------------------------------------------
# Russian roulette
# --------------------------------------------------------------------------------------

def _terrain(max_depth, rr, rr_p=0.5, width=24, height=16, spp=8, n_lambda=4):
    wl = W.as_float32_inputs(W.mid_terrain(width=width, height=height, spp=spp, n_lambda=n_lambda))
    return dataclasses.replace(wl, max_depth=max_depth, rr_enable=rr, rr_p=rr_p)


def test_russian_roulette_weights_survivors_from_the_third_segment_on():
    """Per path: the roulette never acts on the first two segments (depth-2 renders equal with
    and without it), and from the third segment on a path either ends there or carries its
    later measurements divided by the survival probability."""
    p = 0.5
    sz = dict(width=128, height=96, spp=16)
    osc = oracle.OracleScene(_terrain(2, False, **sz).scene)
    _, _, d2 = oracle.render(_terrain(2, False, **sz), osc, keep_paths=True)
    _, _, r2 = oracle.render(_terrain(2, True, p, **sz), osc, keep_paths=True)
    _, _, d3 = oracle.render(_terrain(3, False, **sz), osc, keep_paths=True)
    _, _, r3 = oracle.render(_terrain(3, True, p, **sz), osc, keep_paths=True)
    assert np.array_equal(d2, r2)
    third = d3 - d2                      # the third vertex's measurement of each path
    got = r3 - d2
    scale = np.maximum(np.abs(d3), np.abs(r3))
    has = np.abs(third) > 1e-10 * scale
    n = int(has.sum())
    assert n > 200, n
    killed = got == 0.0
    survived = np.abs(got - third / p) <= 1e-9 * np.abs(third / p) + 1e-13 * scale
    assert np.all(killed | survived)
    kill_frac = (killed & has).sum() / n
    assert abs(kill_frac - (1 - p)) <= 4.5 * math.sqrt(p * (1 - p) / n), kill_frac
    assert (survived & has).sum() > 0


def test_russian_roulette_is_unbiased_on_terrain():
    """Same paths with and without roulette (its decision uses a draw nothing else uses): the
    per-wavelength totals differ by no more than their Monte Carlo error."""
    wl0 = _terrain(6, False, width=32, height=24, spp=16)
    wl1 = _terrain(6, True, 0.5, width=32, height=24, spp=16)
    osc = oracle.OracleScene(wl0.scene)
    _, _, a = oracle.render(wl0, osc, keep_paths=True)
    _, _, b = oracle.render(wl1, osc, keep_paths=True)
    assert not np.array_equal(a, b)
    for w in range(a.shape[2]):
        diff = (b[:, :, w] - a[:, :, w]).ravel()
        se = diff.std() * math.sqrt(diff.size)
        assert abs(diff.sum()) <= 4.5 * se + 1e-12 * abs(a[:, :, w].sum()), (w, diff.sum(), se)


# --------------------------------------------------------------------------------------
# Shading normals
# --------------------------------------------------------------------------------------

def _one_triangle_scene(p, n, kind=0):
    mats = [W.Material(kind=kind, height_um=0.0, length_um=1.0, gdir=(1.0, 0.0, 0.0), reflectance=1.0)]
    return W.Scene(verts=np.asarray(p, np.float64), tris=np.array([[0, 1, 2]], np.int32),
                   tri_mat=np.zeros(1, np.int32), materials=mats, normals=np.asarray(n, np.float64))


@pytest.mark.parametrize("bary", [(0.2, 0.3), (0.6, 0.1), (0.05, 0.9), (1 / 3, 1 / 3)])
def test_shading_normal_is_the_barycentric_interpolation(bary):
    """A smooth mirror triangle with three different vertex normals: at the hit with
    barycentrics (u, v) the shading normal is normalize((1-u-v) n0 + u n1 + v n2) and the
    continuation is the mirror of the ray about it."""
    p = np.array([[0.0, 0.0, 0.0], [1e-3, 0.0, 0.0], [0.0, 1e-3, 0.0]])
    n = np.array([[0.3, -0.2, 1.0], [-0.25, 0.1, 1.0], [0.05, 0.35, 1.0]])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    osc = oracle.OracleScene(_one_triangle_scene(p, n))
    u, v = bary
    P = (1 - u - v) * p[0] + u * p[1] + v * p[2]
    d = np.array([0.2, -0.1, -1.0])
    d /= np.linalg.norm(d)
    r = osc.interaction(P - 0.01 * d, d, k=2 * math.pi / 0.55)
    assert r["hit"] and not r["ended"]
    ns = (1 - u - v) * n[0] + u * n[1] + v * n[2]
    ns /= np.linalg.norm(ns)
    np.testing.assert_allclose(r["ns"], ns, atol=1e-12)
    np.testing.assert_allclose(r["ng"], [0, 0, 1], atol=1e-15)
    assert r["ci"] == pytest.approx(-d @ ns, rel=1e-12)
    np.testing.assert_allclose(r["dir"], d - 2 * (d @ ns) * ns, atol=1e-12)
    assert r["weight"] == 1.0


def test_shading_normal_orientation_follows_the_geometric_side():
    """Hit from below: the geometric normal faces the ray, the interpolated normal is flipped
    to the same side, and a ray grazing the shading normal from behind ends the path."""
    p = np.array([[0.0, 0.0, 0.0], [1e-3, 0.0, 0.0], [0.0, 1e-3, 0.0]])
    n = np.array([[0.0, 0.0, 1.0]] * 3)
    osc = oracle.OracleScene(_one_triangle_scene(p, n))
    P = np.array([2e-4, 3e-4, 0.0])
    d = np.array([0.1, 0.0, 1.0]) / math.hypot(0.1, 1.0)
    r = osc.interaction(P - 0.01 * d, d, k=10.0)
    np.testing.assert_allclose(r["ng"], [0, 0, -1], atol=1e-15)
    np.testing.assert_allclose(r["ns"], [0, 0, -1], atol=1e-15)
    np.testing.assert_allclose(r["dir"], [d[0], d[1], -d[2]], atol=1e-12)
    # strongly tilted vertex normals: the ray meets the shading normal from behind
    n2 = np.array([[1.0, 0.0, 0.05]] * 3)
    n2 /= np.linalg.norm(n2, axis=1, keepdims=True)
    osc2 = oracle.OracleScene(_one_triangle_scene(p, n2))
    d2 = np.array([0.5, 0.0, -1.0]) / math.hypot(0.5, 1.0)
    r2 = osc2.interaction(P - 0.01 * d2, d2, k=10.0)
    assert r2["hit"] and r2["ended"] and r2["ci"] <= 0.0


# --------------------------------------------------------------------------------------
# Adam
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("lr,b1,b2,eps", [(1e-3, 0.9, 0.999, 1e-8), (3e-2, 0.8, 0.99, 1e-6)])
def test_adam_matches_torch(lr, b1, b2, eps):
    import torch
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=257)
    grads = [rng.normal(size=257) * (10.0 ** rng.uniform(-4, 1)) for _ in range(12)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step, g in enumerate(grads, 1):
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, step, lr=lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------------------
# Coherent measurement: slit quadrature
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("z_m", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("lam", [0.40, 0.70])
def test_slit_quadrature_is_converged(z_m, lam):
    """The Rayleigh-Sommerfeld integral over each slit by 16 Gauss-Legendre nodes agrees with
    64 nodes to 1e-9 across the sensor (the precision-stress cases)."""
    case = W.coherent_case("slits", z_m=z_m, lambda_um=lam, width=1024, height=1)
    xp = np.array([0, 137, 300, 511, 512, 700, 901, 1023])
    a = oracle.coherent_exact(case, xp, n_per_slit=16, n_gh=16, n_gl=8)
    b = oracle.coherent_exact(case, xp, n_per_slit=64, n_gh=16, n_gl=8)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-9 * b.max())


# --------------------------------------------------------------------------------------
# Grating sampler: ray-optics limit
# --------------------------------------------------------------------------------------

def test_grating_order_histogram_approaches_the_arcsine_law():
    """h = A sin(K x) with q_z A = m >> 1 and pitch >> wavelength: the orders sampled by the
    inverse CDF of J_j(m_j)^2 follow the density of the sinusoid's slopes, the arcsine law
    1 / (pi sqrt(m^2 - j^2)), to 1e-2 in every bin."""
    lam, A, pitch = 0.55, 10.0, 1000.0
    k = 2 * math.pi / lam
    K = 2 * math.pi / pitch
    m = 2 * k * A
    n = 400
    orders = []
    for i in range(n):
        u = (i + 0.5) / n          # stratified: the samples trace the quantile function
        r = oracle.sample_continuation(2, A, pitch, k, (0.0, 0.0), 1.0, (u, 0.5, 0.5))
        assert r is not None
        orders.append(-r[0] / K)
    orders = np.round(np.array(orders)).astype(int)
    assert np.all(np.diff(orders) >= 0)
    assert abs(orders).max() <= m + 20
    edges = m * np.sin(np.pi * (np.linspace(0.0, 1.0, 11) - 0.5))
    edges = np.round(edges[1:-1]) + 0.5
    inner = np.concatenate([[-np.inf], edges, [np.inf]])
    emp = np.histogram(orders, bins=inner)[0] / n
    F = lambda j: 0.5 + np.arcsin(np.clip(j / m, -1, 1)) / np.pi  # noqa: E731
    law = np.diff(np.concatenate([[0.0], F(edges), [1.0]]))
    np.testing.assert_allclose(emp, law, atol=1e-2)


# --------------------------------------------------------------------------------------
# Rough p_w against Monte Carlo over synthesised surfaces
# --------------------------------------------------------------------------------------

def _gaussian_surfaces(rng, n, N, dx, s, ell):
    """n periodic Gaussian random surfaces on an N x N grid of spacing dx with autocovariance
    s^2 exp(-|tau|^2 / l^2) (the discrete spectrum of the sampled covariance filters white
    noise)."""
    idx = np.minimum(np.arange(N), N - np.arange(N)) * dx
    TX, TY = np.meshgrid(idx, idx, indexing="ij")
    C = s * s * np.exp(-(TX * TX + TY * TY) / ell ** 2)
    S = np.clip(np.fft.fft2(C).real, 0.0, None)
    noise = rng.standard_normal((n, N, N))
    return np.fft.ifft2(np.sqrt(S)[None] * np.fft.fft2(noise, axes=(1, 2)), axes=(1, 2)).real


def test_rough_pw_matches_monte_carlo_over_surfaces():
    """Ensemble average of |int w exp(i (kappa.x + q_z h(x))) dx|^2 / ((2 pi)^2 int |w|^2) over
    synthesised Gaussian surfaces (RMS s, Gaussian autocorrelation of 1/e length l) against the
    oracle's series, at normal incidence, inside the specular peak and across the diffuse
    lobe."""
    rng = np.random.default_rng(11)
    N, dx = 256, 0.15
    s_um, ell = 0.08, 1.0
    lam = 0.6
    k = 2 * math.pi / lam
    S = (6.25, 6.25, 0.0)
    xs = (np.arange(N) - N // 2) * dx
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    w = np.exp(-(X * X + Y * Y) / (4.0 * S[0]))
    norm = (2 * np.pi) ** 2 * np.sum(w * w) * dx * dx
    kappas = [0.0, 0.6, 1.2, 2.0, 3.0]
    qz = [k * (1.0 + math.sqrt(1.0 - (kx / k) ** 2)) for kx in kappas]
    n_real, batch = 1200, 100
    acc = np.zeros((len(kappas), n_real))
    ph = [np.exp(1j * kx * X) for kx in kappas]
    for b0 in range(0, n_real, batch):
        h = _gaussian_surfaces(rng, batch, N, dx, s_um, ell)
        if b0 == 0:
            # the synthesised surfaces have the intended statistics
            assert h.std() == pytest.approx(s_um, rel=0.03)
            lag = int(round(ell / dx))
            c1 = np.mean(h * np.roll(h, lag, axis=1)) / np.mean(h * h)
            assert c1 == pytest.approx(math.exp(-(lag * dx / ell) ** 2), abs=0.03)
        for i, (q, p) in enumerate(zip(qz, ph)):
            F = np.sum(w[None] * p[None] * np.exp(1j * q * h), axis=(1, 2)) * dx * dx
            acc[i, b0:b0 + batch] = np.abs(F) ** 2 / norm
    for i, kx in enumerate(kappas):
        mc = acc[i].mean()
        se = acc[i].std() / math.sqrt(n_real)
        ref = oracle.pw(1, s_um, ell, k, (0.0, 0.0), (kx, 0.0), S)
        assert se < 0.06 * ref
        assert abs(mc - ref) <= 4.0 * se, (kx, mc, ref, se)


# --------------------------------------------------------------------------------------
# Measurements counted per material class
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("left,right", [(W.SMOOTH, W.ROUGH), (W.GRATING, W.SMOOTH), (W.ROUGH, W.GRATING)])
def test_measurements_are_counted_by_the_material_hit(left, right):
    """Split mirror: every path meets the surface once at normal incidence and measures the
    plane wave there, so the count of each class is the number of paths landing on its half:
    pixels 0-31 of each 64-pixel row see x < 0, pixels 32-63 see x > 0."""
    def mat(kind):
        return W.Material(kind, height_um=0.05 if kind != W.SMOOTH else 0.0, length_um=2.0,
                          gdir=(0.0, 1.0, 0.0), reflectance=0.5)
    wl = W.split_mirror(width=64, height=4, spp=4, left=mat(left), right=mat(right))
    _, st = oracle.render(wl)
    names = {W.SMOOTH: "measured_smooth", W.ROUGH: "measured_rough", W.GRATING: "measured_grating"}
    half = 32 * 4 * 4
    assert st[names[left]] == half and st[names[right]] == half
    assert sum(st[n] for n in names.values()) == 2 * half == st["shadow_rays"]


def test_measurement_classes_add_up_on_terrain():
    wl = _terrain(4, False, width=24, height=16, spp=4)
    _, st = oracle.render(wl)
    parts = [st["measured_smooth"], st["measured_rough"], st["measured_grating"]]
    print("terrain measurements by class", parts, st["shadow_rays"])
    assert sum(parts) == st["shadow_rays"] and min(parts) > 0
