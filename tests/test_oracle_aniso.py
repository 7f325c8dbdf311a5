"""Pins of the oracle's anisotropic generalized rays (matrix beta, rho).

The state is the 4x4 second-moment matrix [[Srr, Srk], [Srk^T, Skk]] of the ray's phase-space
Gaussian over the two axes transverse to its mean direction.  Each check compares the oracle
with something other than itself:
- the scalar free-space law (pinned by its own closed forms elsewhere) for isotropic states,
  and the Gaussian-beam law of each principal axis for an astigmatic start;
- the group property of free space and the invariance of det S (a pure state stays pure)
  under free space and interactions;
- mirror reflection as an isometry: an isotropic ray stays isotropic with its widths;
- the anamorphic beam magnification of an in-plane direction change, widths times
  cos(o) / cos(i) along the plane of scattering and unchanged across it;
- the projected-area ratio |n.o| / |n.i| for any direction change;
- the scalar footprint (variance beta^2 / 2 stretched by 1 / cos along the plane of incidence);
- on an all-smooth scene the anisotropic render equals the scalar one;
- a grating relayed by a mirror: the image ratio between anisotropic and scalar rays is the
  square root of the ratio of the in-plane beam variances on the mirror, from the Gaussian-beam
  law per axis with the grating's anamorphic magnification in between.
"""

import math

import numpy as np
import pytest

import oracle
from workloads import grating_relay, parallel_mirror


def iso(beta2, rho=0.0):
    S = np.zeros((4, 4))
    a = (1.0 + rho * rho) / beta2
    S[0, 0] = S[1, 1] = beta2
    S[0, 2] = S[1, 3] = S[2, 0] = S[3, 1] = rho
    S[2, 2] = S[3, 3] = a
    return S


def unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def reflect(d, n):
    return d - 2.0 * np.dot(d, n) * n


@pytest.mark.parametrize("d", [[0, 0, 1], [0, 0, -1], [0.3, -0.4, 0.866], [-0.6, 0.1, -0.79],
                               [1, 0, 0], [0, 1, 1e-9], [0.2, 0.1, -0.9999]])
def test_transverse_frame_is_orthonormal_and_normal_to_d(d):
    d = unit(d)
    e1, e2 = oracle.transverse_frame(d)
    B = np.stack([e1, e2, d])
    np.testing.assert_allclose(B @ B.T, np.eye(3), atol=1e-12)


@pytest.mark.parametrize("beta2,rho,z,k", [(2.0, 0.0, 10.0, 11.0), (0.7, 0.3, 250.0, 16.5),
                                            (800.0, 2.0, 1e5, 8.0)])
def test_isotropic_free_space_is_the_scalar_law(beta2, rho, z, k):
    S = oracle.aniso_free(iso(beta2, rho), z, k)
    b_o, r_o = oracle.propagate(beta2, rho, z, k)
    np.testing.assert_allclose(S, iso(b_o, r_o), rtol=1e-12, atol=1e-14 * b_o)


def test_astigmatic_start_follows_the_gaussian_beam_law_per_axis():
    # waist widths b1, b2 on the two axes: Srr_ii(z) = b_i + zbar^2 / b_i, Srk_ii = zbar / b_i
    b1, b2, k = 3.0, 40.0, 12.0
    S = np.diag([b1, b2, 1.0 / b1, 1.0 / b2])
    for z in (0.0, 5.0, 120.0, 3e4):
        T = oracle.aniso_free(S, z, k)
        zb = z / k
        np.testing.assert_allclose(np.diag(T), [b1 + zb * zb / b1, b2 + zb * zb / b2, 1.0 / b1, 1.0 / b2], rtol=1e-12)
        np.testing.assert_allclose([T[0, 2], T[1, 3], T[0, 1], T[0, 3]], [zb / b1, zb / b2, 0.0, 0.0], atol=1e-12)


def test_free_space_composes_and_keeps_the_state_pure():
    rng = np.random.default_rng(3)
    S = oracle.aniso_free(iso(1.5, 0.0), 40.0, 10.0)
    d = np.array([0.3, 0.2, 0.933]); d /= np.linalg.norm(d)
    S = oracle.aniso_interact(S, d, unit([0.1, -0.5, 0.86]), unit([0.0, -0.2, 1.0]))
    for _ in range(5):
        z1, z2 = rng.uniform(0, 300, 2)
        A = oracle.aniso_free(oracle.aniso_free(S, z1, 9.0), z2, 9.0)
        B = oracle.aniso_free(S, z1 + z2, 9.0)
        np.testing.assert_allclose(A, B, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(np.linalg.det(A), np.linalg.det(S), rtol=1e-9)


def frame_matrix(d):
    e1, e2 = oracle.transverse_frame(d)
    return np.stack([e1, e2])


def world_rr(S, d):
    E = frame_matrix(d)
    return E.T @ S[:2, :2] @ E     # 3x3 spatial covariance in world coordinates


@pytest.mark.parametrize("ti", [0.0, 0.3, 1.0, 1.4])
def test_mirror_reflection_is_an_isometry(ti):
    n = np.array([0.0, 0.0, 1.0])
    di = np.array([math.sin(ti), 0.0, -math.cos(ti)])
    do = reflect(di, n)
    S0 = oracle.aniso_free(iso(2.0), 500.0, 11.0)
    S1 = oracle.aniso_interact(S0, di, do, n)
    np.testing.assert_allclose(S1, S0, rtol=1e-12, atol=1e-12)   # isotropic: frame-independent
    # an anisotropic state keeps its widths (eigenvalues) through the mirror
    A = np.diag([1.0, 9.0, 1.0, 1.0 / 9.0])
    B = oracle.aniso_interact(A, di, do, n)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(B[:2, :2])), [1.0, 9.0], rtol=1e-12)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(B[2:, 2:])), [1.0 / 9.0, 1.0], rtol=1e-12)


@pytest.mark.parametrize("ti,to", [(0.0, 0.5), (0.5236, -0.9), (1.2, 0.2), (0.3, 1.45)])
def test_in_plane_direction_change_gives_the_anamorphic_magnification(ti, to):
    # a grating order leaving at angle to: widths along the plane of scattering scale by
    # cos(to) / cos(ti), widths across it are unchanged; wavevector spreads scale inversely
    n = np.array([0.0, 0.0, 1.0])
    di = np.array([math.sin(ti), 0.0, -math.cos(ti)])
    do = np.array([math.sin(to), 0.0, math.cos(to)])
    b = 2.5
    S = oracle.aniso_interact(iso(b), di, do, n)
    m = math.cos(to) / math.cos(ti)
    R = world_rr(S, do)
    np.testing.assert_allclose(R[1, 1], b, rtol=1e-12)              # across (world y)
    ex = np.array([math.cos(to), 0.0, -math.sin(to)])              # along, normal to do
    np.testing.assert_allclose(ex @ R @ ex, b * m * m, rtol=1e-12)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(S[2:, 2:])), np.sort([1.0 / b, 1.0 / (b * m * m)]),
                               rtol=1e-12)
    np.testing.assert_allclose(np.linalg.det(S), 1.0, rtol=1e-11)


def test_any_direction_change_scales_the_area_by_the_projection_ratio():
    rng = np.random.default_rng(11)
    for _ in range(50):
        n = unit(rng.normal(size=3))
        di = unit(rng.normal(size=3))
        if np.dot(di, n) > -0.05:
            di = reflect(di, n) if np.dot(di, n) > 0.05 else unit(di - 0.5 * n)
        if np.dot(di, n) > -0.05:
            continue
        do = unit(rng.normal(size=3))
        if np.dot(do, n) < 0.05:
            do = reflect(do, n) if np.dot(do, n) < -0.05 else unit(do + 0.5 * n)
        if np.dot(do, n) < 0.05:
            continue
        S0 = oracle.aniso_free(iso(rng.uniform(0.5, 5.0)), rng.uniform(0, 400), 10.0)
        S1 = oracle.aniso_interact(S0, di, do, n)
        ratio = abs(np.dot(do, n)) / abs(np.dot(di, n))
        np.testing.assert_allclose(np.linalg.det(S1[:2, :2]), np.linalg.det(S0[:2, :2]) * ratio ** 2, rtol=1e-9)
        np.testing.assert_allclose(np.linalg.det(S1[2:, 2:]), np.linalg.det(S0[2:, 2:]) / ratio ** 2, rtol=1e-9)
        np.testing.assert_allclose(np.linalg.det(S1), np.linalg.det(S0), rtol=1e-9)
        # the window on the surface is the same from both sides: the outgoing ray's spatial
        # moments carried back onto the surface along do give the incoming ray's footprint
        xa = unit(np.cross(n, [0.3, 0.7, 0.1]))
        ya = np.cross(n, xa)
        f_in = oracle.aniso_footprint(S0, di, n, xa, ya)
        f_out = oracle.aniso_footprint(S1, do, n, xa, ya)
        np.testing.assert_allclose(f_out, f_in, rtol=1e-9, atol=1e-12 * abs(f_in).max())


@pytest.mark.parametrize("ti,phi", [(0.0, 0.0), (0.6, 0.3), (1.3, 2.0)])
def test_isotropic_footprint_is_the_scalar_footprint(ti, phi):
    n = np.array([0.0, 0.0, 1.0])
    xa, ya = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    d = np.array([math.sin(ti) * math.cos(phi), math.sin(ti) * math.sin(phi), -math.cos(ti)])
    b = 3.0
    sxx, syy, sxy = oracle.aniso_footprint(iso(b), d, n, xa, ya)
    ci = math.cos(ti)
    dx, dy = d[0], d[1]
    np.testing.assert_allclose([sxx, syy, sxy], [0.5 * b * (1 + dx * dx / ci ** 2), 0.5 * b * (1 + dy * dy / ci ** 2),
                                                 0.5 * b * dx * dy / ci ** 2], rtol=1e-12, atol=1e-14)


def test_all_smooth_scene_renders_as_the_scalar_rays():
    wl = parallel_mirror()
    a, st_a = oracle.render(wl, aniso=True)
    s, st_s = oracle.render(wl)
    assert st_a == st_s
    np.testing.assert_allclose(a, s, rtol=1e-12)


def test_anisotropic_rays_are_rejected_with_hero_paths():
    wl = parallel_mirror()
    with pytest.raises(RuntimeError):
        oracle.render(wl, aniso=True, hero=True)


def relay_ratio(height_m):
    """Closed form of the anisotropic / scalar image ratio of grating_relay: paths leave the
    sensor (beta0^2 = 2 sigma^2, rho = 0) at normal incidence, travel L1 to the grating, leave
    it in the -1 order at angle o (in-plane magnification m = cos(o)), travel D = H / cos(o) to
    the mirror, where p_w at the specular direction is proportional to sqrt(det S_fp).  The
    axis across the plane of scattering follows the scalar law in both cases."""
    lam, sig, L1 = 0.55, 20.0, 1e4
    k = 2.0 * math.pi / lam
    b0 = 2.0 * sig * sig
    so = lam / 1.0
    co = math.sqrt(1.0 - so * so)
    z1, z2 = L1 / k, height_m * 1e6 / co / k
    b1, r1, a = b0 + z1 * z1 / b0, z1 / b0, 1.0 / b0
    m = co
    along = m * m * b1 + 2.0 * z2 * r1 + z2 * z2 * a / (m * m)
    scalar = b0 + (z1 + z2) ** 2 / b0
    return math.sqrt(along / scalar)


@pytest.mark.parametrize("height_m", [2e-3, 5e-3])
def test_grating_relay_image_ratio_is_the_footprint_ratio(height_m):
    wl = grating_relay(height_m=height_m)
    a, st_a = oracle.render(wl, aniso=True)
    s, st_s = oracle.render(wl)
    assert st_a == st_s
    lit = s[0] > 0
    assert lit.sum() > 200                      # most pixels see the relayed order
    assert np.all((a[0] > 0) == lit)
    np.testing.assert_allclose(a[0][lit] / s[0][lit], relay_ratio(height_m), rtol=1e-12)


def test_continuation_along_the_surface_leaves_the_moments():
    # cos(o) -> 0: the map from the surface onto the outgoing transverse plane is singular
    n = np.array([0.0, 0.0, 1.0])
    di = unit([0.3, 0.0, -1.0])
    do = unit([1.0, 0.0, 1e-9])
    S0 = oracle.aniso_free(iso(2.0), 300.0, 11.0)
    S1 = oracle.aniso_interact(S0, di, do, n)
    np.testing.assert_array_equal(S1, S0)
    assert np.all(np.isfinite(S1))
