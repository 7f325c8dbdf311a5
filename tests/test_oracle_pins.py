"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every check here compares the oracle with something other than itself: a library routine
(rocRAND's Philox engine, scipy's Bessel and Hankel functions), a brute-force quadrature of a
defining integral, a closed form, or values derived from the paper's formulas and stored with
their citation under tests/golden/.
"""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import special

import oracle
from workloads import scenes as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


# --------------------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------------------

def _rocrand_ref_binary():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND reference")
    out = os.path.join("/tmp", "grwave_rocrand_philox_ref")
    src = os.path.join(GOLD, "rocrand_philox_ref.cpp")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.check_call([hipcc, "-O1", "-o", out, src], cwd="/tmp",
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


def test_philox_matches_rocrand_engine():
    """Library pin: rocRAND's Philox4x32-10 engine, positioned at an arbitrary counter."""
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2 ** 32, size=(500, 4), dtype=np.uint64)
    ctr[:4] = [[0, 0, 0, 0], [1, 0, 0, 0], [0xFFFFFFFF, 0xFFFFFFFF, 7, 3], [5, 0, 2, 1]]
    keys = rng.integers(0, 2 ** 32, size=(500, 2), dtype=np.uint64)
    keys[0] = [0, 0]
    ref_bin = _rocrand_ref_binary()
    inp = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, keys))
    res = subprocess.run([ref_bin], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    got = np.stack([oracle.philox(c[None, :], k)[0] for c, k in zip(ctr, keys)]).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_philox_uniform_statistics():
    n = 200_000
    ctr = np.zeros((n // 4, 4), np.uint32)
    ctr[:, 0] = np.arange(n // 4)
    ctr[:, 2] = 3
    x = oracle.philox(ctr, [12345, 678]).ravel()
    u = (x >> 8).astype(np.float64) / 2 ** 24
    # 24-bit uniforms are exact in float32
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = ((hist - n / 64) ** 2 / (n / 64)).sum()
    from scipy.stats import chi2 as chi2d
    assert chi2d.sf(chi2, 63) > 1e-4
    # neighbouring counters are uncorrelated
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.01


# --------------------------------------------------------------------------------------
# Generalized ray: free-space propagation, footprint reading
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("beta,rho,z", [(20.0, 0.0, 2000.0), (10.0, 0.7, 500.0),
                                        (28.2843, 0.0, 1.0e4)])
def test_free_space_law_against_fft_propagation(beta, rho, z):
    """The propagation law (eq. K_free_space_propagation) against paraxial FFT propagation
    of the generalized-ray wave function (eq. def_gen_ray), 1-D factor: intensity variance
    beta^2/2 and wavefront curvature rho/(2 beta^2) after propagation."""
    lam = 0.55
    k = 2 * math.pi / lam
    b2o, rho_o = oracle.propagate(beta * beta, rho, z, k)
    L = 40.0 * math.sqrt(b2o) + 40.0 * beta
    n = 1 << 16
    x = (np.arange(n) - n / 2) * (L / n)
    psi = np.exp(-(1 - 1j * rho) * x * x / (2 * beta * beta))
    kx = 2 * np.pi * np.fft.fftfreq(n, d=L / n)
    psi_z = np.fft.ifft(np.fft.fft(psi) * np.exp(-1j * kx * kx * z / (2 * k)))
    I = np.abs(psi_z) ** 2
    var = np.sum(x * x * I) / np.sum(I)
    assert var == pytest.approx(0.5 * b2o, rel=1e-6)
    # curvature: phase is (rho_o / (2 beta_o^2)) x^2 + const inside the beam
    m = np.abs(x) < 1.5 * math.sqrt(b2o)
    ph = np.unwrap(np.angle(psi_z[m]))
    c2 = np.polyfit(x[m], ph, 2)[0]
    assert c2 == pytest.approx(rho_o / (2 * b2o), rel=1e-5, abs=1e-12)


def test_sigma_k_invariant_under_propagation():
    """sigma_k^2 = (1 + rho^2) / (2 beta^2) is conserved by free-space propagation."""
    k = 2 * math.pi / 0.4
    b2, rho = 37.0, 0.0
    inv0 = (1 + rho * rho) / b2
    for z in [10.0, 1e3, 3e5, 1e7]:
        b2, rho = oracle.propagate(b2, rho, z, k)
        assert (1 + rho * rho) / b2 == pytest.approx(inv0, rel=1e-12)


def test_truncation_radius_mass_fixes_the_variance_reading():
    """Sec. "Wave-Optical Rendering": a radius 2.5 beta holds more than 99.8% of the ray.
    With |psi|^2 ~ exp(-r^2 / beta^2) (spatial variance beta^2/2 per axis) the 2-D mass is
    1 - exp(-6.25) = 0.998070; reading beta as the standard deviation gives 0.956 and fails."""
    beta = 1.0
    r = np.linspace(0, 10, 200001)
    dens = np.exp(-r * r / beta ** 2) * 2 * np.pi * r
    tot = np.trapezoid(dens, r)
    mass = np.trapezoid(dens[r <= 2.5 * beta], r[r <= 2.5 * beta]) / tot
    assert mass == pytest.approx(1 - math.exp(-6.25), abs=1e-6)
    assert mass > 0.998
    wrong = 1 - math.exp(-2.5 ** 2 / 2)
    assert wrong < 0.998


# --------------------------------------------------------------------------------------
# Windowed diffraction density p_w: brute-force quadrature of the defining integral
# --------------------------------------------------------------------------------------

def _window_grid(S, half, step):
    xs = np.arange(-half, half + step / 2, step)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Si = np.linalg.inv(np.array([[S[0], S[2]], [S[2], S[1]]]))
    q = Si[0, 0] * X * X + 2 * Si[0, 1] * X * Y + Si[1, 1] * Y * Y
    w = np.exp(-q / 4.0)
    return X, Y, w, step * step


def _brute_pw(X, Y, w, dA, kappa, phase):
    F = np.sum(w * np.exp(1j * (kappa[0] * X + kappa[1] * Y + phase))) * dA
    return abs(F) ** 2 / ((2 * np.pi) ** 2 * np.sum(w * w) * dA)


def test_pw_smooth_matches_defining_integral():
    S = (9.0, 4.0, 2.0)
    X, Y, w, dA = _window_grid(S, 40.0, 0.1)
    k = 2 * math.pi / 0.5
    kit = (3.0, -1.0)
    for dk in [(0.0, 0.0), (0.1, -0.05), (0.2, 0.3), (-0.25, 0.1)]:
        kot = (kit[0] + dk[0], kit[1] + dk[1])
        ref = _brute_pw(X, Y, w, dA, dk, 0.0)
        got = oracle.pw(0, 0.0, 1.0, k, kit, kot, S)
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-14 * oracle.pw(0, 0, 1, k, kit, kit, S))


def test_pw_grating_matches_defining_integral():
    """Sinusoidal phase screen h = A sin(K g.x) under the window, q_z from the query."""
    S = (16.0, 9.0, -3.0)
    X, Y, w, dA = _window_grid(S, 55.0, 0.08)
    lam, A, pitch = 0.55, 0.1, 2.0
    k = 2 * math.pi / lam
    K = 2 * math.pi / pitch
    ang = math.radians(30.0)
    g = (math.cos(ang), math.sin(ang))
    kit = (0.4 * k, 0.1 * k)
    peak = None
    for j, off in [(0, 0.0), (1, 0.0), (-1, 0.05), (2, -0.1), (1, 0.2), (0, 0.6)]:
        kappa = (-j * K * g[0] + off, -j * K * g[1] + 0.5 * off)
        kot = (kit[0] + kappa[0], kit[1] + kappa[1])
        ci = math.sqrt(1 - (kit[0] ** 2 + kit[1] ** 2) / k ** 2)
        co = math.sqrt(1 - (kot[0] ** 2 + kot[1] ** 2) / k ** 2)
        qz = k * (ci + co)
        ref = _brute_pw(X, Y, w, dA, kappa, qz * A * np.sin(K * (g[0] * X + g[1] * Y)))
        got = oracle.pw(2, A, pitch, k, kit, kot, S, g=g)
        if peak is None:
            peak = got
        assert got == pytest.approx(ref, rel=1e-8, abs=1e-12 * peak)


def test_pw_rough_matches_lag_space_integral():
    """Ensemble average of the Gaussian random phase screen in lag space:
    p = (1 / (2 pi)^2) int exp(-D^T S^-1 D / 8) exp(i kappa.D) exp(-g (1 - exp(-|D|^2 / l^2))) dD
    (the window autocorrelation is exp(-D^T S^-1 D / 8) times the window energy)."""
    S = (9.0, 6.0, 1.0)
    s_um, ell = 0.1, 1.0
    lam = 0.6
    k = 2 * math.pi / lam
    kit = (2.0, 0.5)
    Si = np.linalg.inv(np.array([[S[0], S[2]], [S[2], S[1]]]))
    step = 0.08
    xs = np.arange(-50, 50 + step / 2, step)
    DX, DY = np.meshgrid(xs, xs, indexing="ij")
    Rw = np.exp(-(Si[0, 0] * DX * DX + 2 * Si[0, 1] * DX * DY + Si[1, 1] * DY * DY) / 8.0)
    for dk in [(0.0, 0.0), (0.3, 0.0), (0.5, -0.7), (1.5, 1.0)]:
        kot = (kit[0] + dk[0], kit[1] + dk[1])
        ci = math.sqrt(1 - (kit[0] ** 2 + kit[1] ** 2) / k ** 2)
        co = math.sqrt(1 - (kot[0] ** 2 + kot[1] ** 2) / k ** 2)
        g = (k * (ci + co) * s_um) ** 2
        E = np.exp(-g * (1 - np.exp(-(DX * DX + DY * DY) / ell ** 2)))
        ref = np.sum(Rw * E * np.cos(dk[0] * DX + dk[1] * DY)) * step * step / (2 * np.pi) ** 2
        got = oracle.pw(1, s_um, ell, k, kit, kot, S)
        assert got == pytest.approx(ref, rel=1e-8)


def test_pw_rough_limits():
    k = 2 * math.pi / 0.5
    S = (30.0, 20.0, 0.0)
    kit = (1.0, 0.0)
    # g -> 0: the smooth kernel
    for dk in [(0, 0), (0.02, 0.01)]:
        kot = (kit[0] + dk[0], kit[1] + dk[1])
        assert oracle.pw(1, 0.0, 2.0, k, kit, kot, S) == pytest.approx(
            oracle.pw(0, 0.0, 2.0, k, kit, kot, S), rel=1e-14)
    # g >> 1: second moment of kappa is Sigma_k + 2 g / l^2 (ray-optics slope variance
    # 2 s^2 / l^2 scaled by q_z^2); checked at normal incidence where q_z ~ 2k near the peak
    s_um, ell = 0.3, 40.0
    kit = (0.0, 0.0)
    g0 = (2 * k * s_um) ** 2
    sd = math.sqrt(2 * g0) / ell
    ks = np.linspace(-6 * sd, 6 * sd, 241)
    KX, KY = np.meshgrid(ks, ks, indexing="ij")
    q = np.stack([np.full(KX.size, 1.0), np.full(KX.size, s_um), np.full(KX.size, ell),
                  np.ones(KX.size), np.full(KX.size, k), np.zeros(KX.size), np.zeros(KX.size),
                  KX.ravel(), KY.ravel(), np.full(KX.size, S[0]), np.full(KX.size, S[1]),
                  np.zeros(KX.size), np.ones(KX.size), np.zeros(KX.size)], 1)
    p = oracle.pw_batch(q).reshape(KX.shape)
    dk2 = (ks[1] - ks[0]) ** 2
    mass = p.sum() * dk2
    mxx = (p * KX * KX).sum() * dk2 / mass
    # q_z varies slightly across the lobe (q_z = k (cos i + cos o)); the slope limit holds
    # to the order of the lobe's angular width squared
    assert mass == pytest.approx(1.0, rel=2e-3)
    assert mxx == pytest.approx(0.25 / S[0] + 2 * g0 / ell ** 2, rel=2e-2)


def test_reciprocity():
    rng = np.random.default_rng(3)
    for _ in range(200):
        kind = int(rng.integers(0, 3))
        k = 2 * math.pi / rng.uniform(0.4, 0.7)
        kit = rng.uniform(-0.6, 0.6, 2) * k
        kot = kit + rng.normal(0, 0.3, 2)
        S = (rng.uniform(5, 50), rng.uniform(5, 50), rng.uniform(-2, 2))
        h = rng.uniform(0.05, 0.3)
        L = rng.uniform(0.8, 4.0)
        a = oracle.pw(kind, h, L, k, kit, kot, S)
        b = oracle.pw(kind, h, L, k, -kot, -kit, S)
        assert a == pytest.approx(b, rel=1e-12, abs=1e-300)


# --------------------------------------------------------------------------------------
# Bessel weights, grating orders, energy
# --------------------------------------------------------------------------------------

def test_bessel_against_scipy_and_jacobi_anger():
    for x in [0.0, 1e-3, 0.5, 1.97869, 3.3, 9.4, 17.0]:
        tot = 0.0
        for n in range(-60, 61):
            ref = special.jv(n, x)
            got = oracle.besselj(n, x)
            assert got == pytest.approx(ref, rel=1e-10, abs=1e-15)
            tot += got * got
        assert tot == pytest.approx(1.0, abs=1e-12)


def _golden_lobes():
    rows, total, centre = [], None, None
    with open(os.path.join(GOLD, "tiny_grating_lobes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "SUM":
                total = float(p[1])
            elif p[0] == "CENTRE":
                centre = float(p[1])
            else:
                rows.append((int(p[0]), float(p[1]), float(p[2])))
    return rows, total, centre


def test_tiny_grating_orders_and_weights():
    rows, total, _ = _golden_lobes()
    lam, A, pitch = 0.55, 0.1, 2.0
    k = 2 * math.pi / lam
    K = 2 * math.pi / pitch
    kit = (k * 0.5, 0.0)
    ci = math.cos(math.radians(30))
    res = oracle.sample_continuation(2, A, pitch, k, kit, ci, (0.3, 0.5, 0.5))
    assert res is not None
    assert res[2] == pytest.approx(total, abs=2e-6)
    # inverse-CDF order selection: the fraction of a fine uniform grid mapped to each order
    us = (np.arange(20000) + 0.5) / 20000
    counts = {}
    for u in us:
        kox, koy, _ = oracle.sample_continuation(2, A, pitch, k, kit, ci, (u, 0.5, 0.5))
        j = int(round((kit[0] - kox) / K))
        th = math.degrees(math.asin(kox / k))
        counts.setdefault(j, [0, th])[0] += 1
    for j, th, wgt in rows:
        assert counts.get(j, [0])[0] / len(us) == pytest.approx(wgt / total, abs=1e-4)
    # a uniform in the middle of each order's CDF interval selects that order, whose
    # direction obeys the grating equation
    c = 0.0
    for j, th, wgt in rows:
        u = (c + 0.5 * wgt) / total
        c += wgt
        kox, koy, _ = oracle.sample_continuation(2, A, pitch, k, kit, ci, (u, 0.5, 0.5))
        assert int(round((kit[0] - kox) / K)) == j
        assert math.degrees(math.asin(kox / k)) == pytest.approx(th, abs=1e-3)


def test_energy_bounds():
    k = 2 * math.pi / 0.55
    # smooth with a wide footprint: all energy in the propagating disk
    S = (400.0, 300.0, 50.0)
    ks = np.linspace(-0.2, 0.2, 301)
    KX, KY = np.meshgrid(ks, ks, indexing="ij")
    kit = np.array([2.0, 1.0])

    def integ(kind, h, L, S, extent=0.2, n=301, centre=None):
        c = kit if centre is None else centre
        ks = np.linspace(-extent, extent, n)
        KX, KY = np.meshgrid(ks, ks, indexing="ij")
        m = KX.size
        q = np.stack([np.full(m, float(kind)), np.full(m, h), np.full(m, L), np.ones(m),
                      np.full(m, k), np.full(m, kit[0]), np.full(m, kit[1]),
                      c[0] + KX.ravel(), c[1] + KY.ravel(), np.full(m, S[0]), np.full(m, S[1]),
                      np.full(m, S[2]), np.ones(m), np.zeros(m)], 1)
        return oracle.pw_batch(q).sum() * (ks[1] - ks[0]) ** 2

    assert integ(0, 0, 1, S) == pytest.approx(1.0, abs=1e-9)
    # grating: each lobe carries J_j(m_j)^2 (q_z varies across a narrow lobe only slightly)
    A, pitch = 0.1, 2.0
    K = 2 * math.pi / pitch
    ci = math.sqrt(1 - (kit ** 2).sum() / k ** 2)
    for j in [-1, 0, 1, 2]:
        c = kit - np.array([j * K, 0.0])
        co = math.sqrt(1 - (c ** 2).sum() / k ** 2)
        mj = k * A * (ci + co)
        assert integ(2, A, pitch, S, centre=c) == pytest.approx(special.jv(j, mj) ** 2, rel=2e-4)
    # rough: at most the incident energy
    assert integ(1, 0.2, 3.0, (30.0, 30.0, 0.0), extent=9.0, n=601) <= 1.0 + 1e-9


# --------------------------------------------------------------------------------------
# Tiny grating image: closed form per sample
# --------------------------------------------------------------------------------------

def _tiny_closed_form(wl):
    """Independent NumPy evaluation of the tiny workload: each sample's mean ray hits the
    quad after distance t; the generalized ray has sigma_r^2 = beta^2/2 + (t/k)^2/(2 beta^2);
    the view direction is exactly the +1 order, so its value is J_1(m_1)^2 times the peak
    of a Gaussian with covariance diag(1/(4 s_x^2), 1/(4 s_y^2)), s_x = sigma_r / cos(theta)."""
    sen = wl.sensor
    lam = wl.lambdas_um[0]
    k = 2 * math.pi / lam
    H, Wd = sen.height, sen.width
    ys, xs = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
    img = np.zeros((H, Wd))
    beta2 = 2 * (sen.sigma_m * 1e6) ** 2
    d = sen.dir
    cos_o = -d[2]
    sin_o = math.sqrt(1 - cos_o ** 2)
    m1 = k * 0.1 * (math.cos(math.radians(30)) + cos_o)
    J2 = special.jv(1, m1) ** 2
    for s in range(wl.spp):
        pid = ((s * H + ys) * Wd + xs).astype(np.uint64)
        ctr = np.stack([pid & 0xFFFFFFFF, pid >> 32, np.zeros_like(pid), np.zeros_like(pid)],
                       -1).reshape(-1, 4)
        r = oracle.philox(ctr, [wl.seed & 0xFFFFFFFF, wl.seed >> 32]).reshape(H, Wd, 4)
        u0 = (r[..., 0] >> 8) / 2.0 ** 24
        u1 = (r[..., 1] >> 8) / 2.0 ** 24
        o = (sen.origin[None, None, :] + ((xs + u0) * sen.pitch_m)[..., None] * sen.axis_u
             + ((ys + u1) * sen.pitch_m)[..., None] * sen.axis_v)
        t = -o[..., 2] / d[2]
        P = o + t[..., None] * d
        inside = (np.abs(P[..., 0]) <= 0.5e-3) & (np.abs(P[..., 1]) <= 0.5e-3)
        zb = t * 1e6 / k
        sr2 = 0.5 * (beta2 + zb * zb / beta2)
        sx2 = sr2 / cos_o ** 2
        sy2 = sr2
        val = J2 * 4.0 * np.sqrt(sx2 * sy2) / (2 * np.pi)
        img += np.where(inside, val, 0.0) / wl.spp
    return img, (k, sin_o, m1, J2)


def test_tiny_grating_image_closed_form():
    wl = W.tiny_grating()
    img, st = oracle.render(wl, use_bvh=False)
    ref, _ = _tiny_closed_form(wl)
    assert st["segments"] == 32 * 32 * 8
    np.testing.assert_allclose(img[0], ref, rtol=1e-9, atol=1e-9 * ref.max())


def test_tiny_grating_centre_value_golden():
    _, _, centre = _golden_lobes()
    wl = W.tiny_grating()
    k = 2 * math.pi / 0.55
    beta2 = 2 * 20.0 ** 2
    zb = 1e4 / k
    sr2 = 0.5 * (beta2 + zb * zb / beta2)
    cos_o = -wl.sensor.dir[2]
    kit = (0.5 * k, 0.0)
    kot = (-k * wl.sensor.dir[0], 0.0)
    S = (sr2 / cos_o ** 2, sr2, 0.0)
    assert math.sqrt(S[0]) == pytest.approx(30.426, abs=1e-3)
    assert math.sqrt(S[1]) == pytest.approx(29.646, abs=1e-3)
    assert oracle.pw(2, 0.1, 2.0, k, kit, kot, S) == pytest.approx(centre, abs=1e-3)


# --------------------------------------------------------------------------------------
# Measurement against a partially coherent source: expectation of the NEE estimator
# --------------------------------------------------------------------------------------

def _flat_quad_scene(kind=W.SMOOTH, h=0.0, L=1.0):
    half = 0.05
    verts = np.array([[-half, -half, 0], [half, -half, 0], [half, half, 0], [-half, half, 0]],
                     np.float64)
    return W.Scene(verts=verts, tris=np.array([[0, 1, 2], [0, 2, 3]], np.int32),
                   tri_mat=np.zeros(2, np.int32), materials=[W.Material(kind, h, L)])


def test_gsm_measurement_expectation():
    """Backward = forward for one bounce: the mean of the estimator with the source's angular
    density N(k_s,t, r_c^-2 I) sampled at NEE equals the overlap N(k_o,t; 0, Sigma_k +
    r_c^-2 I) (emitter axis along the normal, smooth surface, near-normal view so that the
    source spread and the window spectrum are of similar width)."""
    scene = _flat_quad_scene()
    lam = 0.5
    k = 2 * math.pi / lam
    rc = 60.0
    th = math.radians(0.1)
    sig = 20.0
    view = np.array([math.sin(th), 0.0, -math.cos(th)])
    sen = W._ortho_sensor(-0.01 * view, view, np.array([0, 1.0, 0]), 1, 1, 1e-6, sig * 1e-6)
    src = W.Source(W.GSM_AREA, dir=np.array([0, 0, -1.0]), pos=np.array([0, 0, 0.02]),
                   eu=np.array([0.5, 0, 0]), ev=np.array([0, 0.5, 0]),
                   coherence_radius_um=rc, power=1.0)
    spp = 20000
    wl = W.Workload("gsm-pin", scene, sen, [src], np.array([lam]), spp=spp, max_depth=1, seed=9)
    img, _, paths = oracle.render(wl, keep_paths=True)
    vals = paths[:, 0, 0] * spp
    beta2 = 2 * sig ** 2
    zb = 1e4 / k
    sr2 = 0.5 * (beta2 + zb * zb / beta2)
    cos_i = math.cos(th)
    Sk = np.diag([1 / (4 * sr2 / cos_i ** 2), 1 / (4 * sr2)]) + np.eye(2) / rc ** 2
    ko = np.array([-k * view[0], 0.0])   # outgoing tangential wavevector (toward the sensor)
    expect = math.exp(-0.5 * ko @ np.linalg.solve(Sk, ko)) / (2 * math.pi * math.sqrt(np.linalg.det(Sk)))
    se = vals.std() / math.sqrt(spp)
    assert abs(vals.mean() - expect) < 4 * se
    assert se < 0.02 * expect


def test_spp_ranges_sum_to_full_render():
    wl = W.mid_terrain(width=24, height=20, spp=6, n_lambda=2)
    osc = oracle.OracleScene(wl.scene)
    full, _ = oracle.render(wl, osc, spp_norm=6)
    a, _ = oracle.render(wl, osc, spp_begin=0, spp_count=2, spp_norm=6)
    b, _ = oracle.render(wl, osc, spp_begin=2, spp_count=4, spp_norm=6)
    np.testing.assert_allclose(a + b, full, rtol=1e-12, atol=1e-300)


def test_linear_in_source_multiplicity():
    """Two identical sources, one picked per vertex with probability 1/2 and weighted by 2:
    the image is exactly twice the single-source image (linearity in the source term)."""
    wl = W.mid_terrain(width=16, height=16, spp=2, n_lambda=2)
    osc = oracle.OracleScene(wl.scene)
    one, _ = oracle.render(wl, osc)
    wl2 = W.Workload(wl.name, wl.scene, wl.sensor, [wl.sources[0], wl.sources[0]], wl.lambdas_um,
                     wl.spp, wl.max_depth, wl.seed)
    two, _ = oracle.render(wl2, osc)
    np.testing.assert_array_equal(two, 2 * one)


# --------------------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------------------

def test_bvh_matches_brute_force():
    sc = W.terrain_scene(nx=32, ny=16, seed=4, tiles=4)
    osc = oracle.OracleScene(sc)
    rng = np.random.default_rng(5)
    n = 3000
    o = np.stack([rng.uniform(-0.02, 0.12, n), rng.uniform(-0.02, 0.12, n),
                  rng.uniform(0.01, 0.05, n)], 1)
    d = rng.normal(size=(n, 3))
    d[:, 2] = -np.abs(d[:, 2]) - 0.2
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # a few rays from below and grazing rays
    a = osc.intersect(o, d, use_bvh=True)
    b = osc.intersect(o, d, use_bvh=False)
    np.testing.assert_array_equal(a[:, 0], b[:, 0])
    np.testing.assert_array_equal(a[:, 1], b[:, 1])
    assert (a[:, 0] >= 0).mean() > 0.3


def test_watertight_shared_edge():
    """A ray through the shared diagonal of a quad hits one of its two triangles."""
    sc = _flat_quad_scene()
    osc = oracle.OracleScene(sc)
    t = np.linspace(-0.04, 0.04, 101)
    o = np.stack([t, t, np.full_like(t, 0.01)], 1)
    d = np.tile([0, 0, -1.0], (t.size, 1))
    h = osc.intersect(o, d)
    assert np.all(h[:, 0] >= 0)
    assert np.allclose(h[:, 1], 0.01)


# --------------------------------------------------------------------------------------
# Coherent measurement
# --------------------------------------------------------------------------------------

def test_hankel_against_scipy():
    for x in [10.0, 1e3, 2.5e5, 1.1e7, 1.6e8]:
        ref = special.hankel1(1, x)
        got = oracle.hankel1(x)
        # the phase of H1 at large x is limited by the representation of x itself
        assert abs(got - ref) <= max(1e-11, 8 * x * 2.0 ** -52) * abs(ref)


@pytest.mark.parametrize("sigma_mode", ["pitch", "quarter"])
def test_two_point_fringes_and_visibility(sigma_mode):
    """Two-point interference (eq. two_point_interference): fringe angular frequency
    k l_s / z; a Gaussian detection window of std sigma and the uniform pixel scale the
    fringe contrast by exp(-K^2 sigma^2 / 2) * sinc(K pitch / 2)."""
    case = W.coherent_case("points", z_m=1.0, lambda_um=0.55, sigma_mode=sigma_mode, width=1024,
                           height=1)
    xp = np.arange(480, 545)
    I = oracle.coherent_exact(case, xp)
    k = 2 * math.pi / case.lambda_um
    z = case.z_m * 1e6
    K = k * 50.0 / z
    X = (xp + 0.5 - case.width / 2) * case.pitch_um
    V = math.exp(-0.5 * (K * case.sigma_um) ** 2) * np.sinc(K * case.pitch_um / 2 / np.pi)
    model = (2.0 / z ** 2) * (1 + V * np.cos(K * X))
    np.testing.assert_allclose(I, model, rtol=2e-4)
    period = 2 * math.pi / K
    assert period == pytest.approx(case.lambda_um * z / 50.0, rel=1e-12)


def test_double_slit_far_field():
    """Slits b = 10 um, d = 50 um: Fraunhofer pattern sinc^2(pi b X / (lambda z)) *
    cos^2(pi d X / (lambda z)) of the 2-D Rayleigh-Sommerfeld integral (narrow window)."""
    case = W.coherent_case("slits", z_m=0.1, lambda_um=0.55, width=1024, height=1)
    case.sigma_um = 0.05 * case.pitch_um
    xp = np.arange(0, 1024, 16)
    I = oracle.coherent_exact(case, xp, n_gl=4)
    lam, z = case.lambda_um, case.z_m * 1e6
    X = (xp + 0.5 - case.width / 2) * case.pitch_um
    model = np.sinc(10.0 * X / (lam * z)) ** 2 * np.cos(np.pi * 50.0 * X / (lam * z)) ** 2
    model *= I[np.argmin(np.abs(X))] / model[np.argmin(np.abs(X))]
    np.testing.assert_allclose(I, model, atol=3e-3 * I.max())


def test_coherent_estimator_converges_to_expectation():
    case = W.coherent_case("slits", z_m=1.0, lambda_um=0.4, width=64, height=2, spp=512)
    mc = oracle.coherent_mc(case)
    ex = oracle.coherent_exact(case, np.arange(64))
    # rows are statistically identical (slits are y-invariant)
    est = mc.mean(0)
    assert np.abs(est - ex).max() < 0.08 * ex.max()


# --------------------------------------------------------------------------------------
# FP64 multilayer perceptron
# --------------------------------------------------------------------------------------

def test_mlp_backward_matches_finite_differences():
    from oracle import mlp
    Ws, bs = mlp.init_params(seed=2)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, 10))
    Y = rng.normal(size=7)
    dWs, dbs, _ = mlp.backward(Ws, bs, X, Y)
    h = 1e-6
    for l, (i, j) in [(0, (3, 5)), (2, (10, 60)), (4, (7, 0))]:
        Wp = [w.copy() for w in Ws]
        Wm = [w.copy() for w in Ws]
        Wp[l][i, j] += h
        Wm[l][i, j] -= h
        fd = (mlp.mse_loss(Wp, bs, X, Y) - mlp.mse_loss(Wm, bs, X, Y)) / (2 * h)
        assert dWs[l][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for l in [1, 4]:
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += h
        bm[l][0] -= h
        fd = (mlp.mse_loss(Ws, bp, X, Y) - mlp.mse_loss(Ws, bm, X, Y)) / (2 * h)
        assert dbs[l][0] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    # GELU (tanh form) against PyTorch's own implementation in double precision
    import torch
    x = np.linspace(-6, 6, 25)
    ref = torch.nn.functional.gelu(torch.tensor(x, dtype=torch.float64), approximate="tanh").numpy()
    np.testing.assert_allclose(mlp.gelu(x), ref, rtol=1e-13, atol=1e-15)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(xt, approximate="tanh").sum().backward()
    np.testing.assert_allclose(mlp.gelu_grad(x), xt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_rough_continuation_sampling_moments():
    """Unwindowed rough-surface kernel f_inf = sum_m Poisson(m; g) N(kappa; 0, 2m/l^2 I) with
    g = (2 k cos(i) s)^2: the sampler leaves the direction unchanged with probability e^-g and
    draws kappa with E|kappa|^2 = sum_m P(m) 4 m / l^2 = 4 g / l^2."""
    from scipy.stats import poisson
    k = 2 * math.pi / 0.6
    s_um, ell = 0.08, 2.0
    ci = 0.9
    g = (2 * k * ci * s_um) ** 2
    kit = (0.3, -0.2)
    rng = np.random.default_rng(8)
    n = 40000
    u = rng.uniform(0, 1, (n, 3))
    kap2, zero = [], 0
    for row in u:
        r = oracle.sample_continuation(1, s_um, ell, k, kit, ci, row)
        assert r is not None and r[2] == 1.0
        d2 = (r[0] - kit[0]) ** 2 + (r[1] - kit[1]) ** 2
        zero += d2 == 0.0
        kap2.append(d2)
    kap2 = np.array(kap2)
    assert zero / n == pytest.approx(math.exp(-g), abs=4 * math.sqrt(math.exp(-g) / n))
    se = kap2.std() / math.sqrt(n)
    assert abs(kap2.mean() - 4 * g / ell ** 2) < 4 * se
    # the term index follows the Poisson law exactly (inverse CDF of a fine uniform grid)
    us = (np.arange(2000) + 0.5) / 2000
    ms = []
    for uu in us:
        r = oracle.sample_continuation(1, s_um, ell, k, kit, ci, (uu, 0.1, 0.25))
        # with u1 = 0.1, u2 = 0.25 the Box-Muller pair is (0, r): |kappa| = sqrt(2m)/l * r
        rr = math.sqrt(-2 * math.log(1 - 0.1))
        d = math.hypot(r[0] - kit[0], r[1] - kit[1])
        ms.append(int(round((d * ell / rr) ** 2 / 2)))
    hist = np.bincount(ms, minlength=30)[:30] / len(us)
    np.testing.assert_allclose(hist, poisson.pmf(np.arange(30), g), atol=1.0 / len(us) + 1e-12)


def test_e4m3_rounding_against_format_definition():
    """OCP FP8 E4M3: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits, code 0x7F / 0xFF NaN.
    Every finite code (decoded from that definition) rounds to itself; every midpoint of two
    neighbours rounds to the one with an even mantissa; values beyond 448 clamp."""
    from oracle import mlp as omlp
    vals = []
    for c in range(256):
        if c & 0x7F == 0x7F:
            continue
        s = -1.0 if c & 0x80 else 1.0
        e, m = (c >> 3) & 15, c & 7
        v = s * (2.0 ** -6 * m / 8.0 if e == 0 else 2.0 ** (e - 7) * (1.0 + m / 8.0))
        vals.append((v, m))
    pos = sorted({(v, m) for v, m in vals if v >= 0})
    v = np.array([p[0] for p in pos])
    assert len(pos) == 127 and v[-1] == 448.0 and v[1] == 2.0 ** -9
    np.testing.assert_array_equal(omlp.e4m3_round(v), v)
    np.testing.assert_array_equal(omlp.e4m3_round(-v), -v)
    mids = 0.5 * (v[1:] + v[:-1])
    even = np.array([pos[i][0] if pos[i][1] % 2 == 0 else pos[i + 1][0] for i in range(len(pos) - 1)])
    np.testing.assert_array_equal(omlp.e4m3_round(mids), even)
    # just off the midpoints: the nearer neighbour
    np.testing.assert_array_equal(omlp.e4m3_round(mids * (1 - 1e-9)), v[:-1])
    np.testing.assert_array_equal(omlp.e4m3_round(mids * (1 + 1e-9)), v[1:])
    assert omlp.e4m3_round(1e6) == 448.0 and omlp.e4m3_round(-500.0) == -448.0


def test_bf16_rounding_against_format_definition():
    """bfloat16: float32 with the low 16 bits zero.  Random float32 values round to the nearer
    of the two neighbouring bfloat16 values, ties to the one with an even last bit."""
    from oracle import mlp as omlp
    rng = np.random.default_rng(8)
    bits = rng.integers(0, 2 ** 31 - 2 ** 23, size=20000, dtype=np.uint64).astype(np.uint32)
    bits[:64] = (bits[:64] & 0xFFFF0000) | 0x8000          # exact midpoints
    x = bits.view(np.float32).astype(np.float64)
    lo = (bits & 0xFFFF0000).view(np.float32).astype(np.float64)
    hi = ((bits & 0xFFFF0000) + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    dl, dh = x - lo, hi - x
    lo_even = ((bits >> 16) & 1) == 0
    want = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(lo_even, lo, hi)))
    np.testing.assert_array_equal(omlp.bf16_round(x.astype(np.float32)), want)
    np.testing.assert_array_equal(omlp.bf16_round(-x.astype(np.float32)), -want)


def test_e4m3_forward_reduces_to_exact_network():
    """The quantized passes are exact where the rounding is: a hidden layer whose weights and
    input rows are E4M3 values with max 448 in every neuron and every query (all scales 1), or
    whose activations sit one residual step off an E4M3 value, and an input layer on bfloat16
    values.  A full random network changes by no more than the formats' spacing allows."""
    from oracle import mlp as omlp
    rng = np.random.default_rng(3)
    grid = np.array([0.25, 0.5, 1.0, 2.0, -0.5, -1.0, 0.0, 0.75])
    W = rng.choice(grid, size=(64, 64))
    W[0, :] = 448.0                       # every neuron's scale is 1
    A = rng.choice(grid, size=(256, 64))
    A[:, 5] = -448.0                      # every query's scale is 1
    np.testing.assert_array_equal(omlp.e4m3_matmul(A, W), A @ W)
    # the residual term: an activation between two E4M3 values carries its rounding residual
    # at 16x, so a/s = 1.0625 (hi = 1, residual 1/16 -> lo = 1) is carried exactly
    A2 = A.copy()
    A2[:, 7] = 1.0625
    np.testing.assert_allclose(omlp.e4m3_matmul(A2, W), A2 @ W, rtol=0, atol=1e-12)
    assert omlp.e4m3_round(1.0625) == 1.0
    # input layer: bfloat16-exact inputs and weights pass unrounded
    W1 = rng.choice(grid, size=(10, 64)) * 3.0
    W2 = rng.normal(size=(64, 1))
    X = rng.choice(grid, size=(256, 10)) * 5.0
    bs = [rng.normal(size=64), np.zeros(1)]
    ref, _, _ = omlp.forward([W1, W2], bs, X)
    np.testing.assert_allclose(omlp.forward_e4m3([W1, W2], bs, X), ref[:, 0], rtol=1e-12, atol=1e-12)
    # full network, random weights: bounded quantization error, and not zero
    Ws = [rng.normal(0, np.sqrt(2.0 / a), size=(a, b)) for a, b in zip(omlp.SIZES[:-1], omlp.SIZES[1:])]
    bz = [rng.normal(0, 0.05, size=b) for b in omlp.SIZES[1:]]
    X = rng.uniform(-1, 1, size=(512, 10))
    ref, _, _ = omlp.forward(Ws, bz, X)
    got = omlp.forward_e4m3(Ws, bz, X)
    err = np.linalg.norm(got - ref[:, 0]) / np.linalg.norm(ref[:, 0])
    assert 1e-4 < err < 0.1
