"""Pins of the oracle's composite interaction (Sec. "Wave-Optical Rendering": a generalized ray
whose footprint covers two materials meets the composition of their interaction operators).

The operator is the Fourier integral of the Gaussian window times each side's reflection
function over its half-plane, averaged over the unknown position of each deterministic profile
(design notes, composite reading).  Everything here checks the oracle against something other
than itself: scipy's Faddeeva function, 2-D Gauss-Legendre quadrature of the defining
integrals, the single-material kernel in the limits, a brute-force boundary search in NumPy, and
the closed form of two mirrors meeting at a straight boundary, path by path.
"""

import math

import numpy as np
import pytest
from scipy import special

import oracle
from workloads import scenes as W

K550 = 2.0 * math.pi / 0.55


# --------------------------------------------------------------------------------------
# Faddeeva function
# --------------------------------------------------------------------------------------

def test_faddeeva_matches_library():
    """Library pin: scipy.special.wofz on the upper half-plane, from the real axis to Im z = 12,
    |Re z| from 0 to 1e4 (both branches of the oracle: series and continued fraction)."""
    xs = np.concatenate([-np.logspace(-3, 4, 90)[::-1], [0.0], np.logspace(-3, 4, 90)])
    ys = np.concatenate([[0.0], np.logspace(-4, math.log10(12.0), 30)])
    z = (xs[None, :] + 1j * ys[:, None]).ravel()
    got = oracle.faddeeva(z)
    ref = special.wofz(z)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-11


# --------------------------------------------------------------------------------------
# Half-plane window field against quadrature of its defining integral
# --------------------------------------------------------------------------------------

def _gl_panels(a, b, width, nodes=24):
    """Composite Gauss-Legendre nodes and weights on [a, b] with panels no wider than width."""
    npan = max(1, int(math.ceil((b - a) / width)))
    x0, w0 = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(a, b, npan + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x0 + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w0)
    return np.concatenate(xs), np.concatenate(ws)


def _edge_grid(S, n, c, side, vmax):
    """Quadrature over one half-plane in the boundary's frame x = a n + b e: side 1 is a > c,
    side 0 is a < c.  Returns points x [m][2] and weights."""
    smax = math.sqrt(max(np.linalg.eigvalsh(np.array([[S[0], S[2]], [S[2], S[1]]]))))
    L = 10.0 * smax            # the amplitude window is below 1.4e-11 beyond
    width = min(smax, 10.0 / max(vmax, 1e-9))
    if side == 1:
        a, wa = _gl_panels(c, c + L, width)
    else:
        a, wa = _gl_panels(-L, c, width)
    b, wb = _gl_panels(-L, L, width)
    e = np.array([-n[1], n[0]])
    A, B = np.meshgrid(a, b, indexing="ij")
    x = A[..., None] * np.asarray(n) + B[..., None] * e
    return x.reshape(-1, 2), (wa[:, None] * wb[None, :]).ravel()


def _window(S, x):
    Si = np.linalg.inv(np.array([[S[0], S[2]], [S[2], S[1]]]))
    return np.exp(-0.25 * np.einsum("mi,ij,mj->m", x, Si, x))


def _norm(S):
    """(2 pi)^2 times the window energy (the normalisation of p_w), by quadrature."""
    x0, w0 = _edge_grid(S, (1.0, 0.0), 0.0, 0, 1.0)
    x1, w1 = _edge_grid(S, (1.0, 0.0), 0.0, 1, 1.0)
    e = np.sum(w0 * _window(S, x0) ** 2) + np.sum(w1 * _window(S, x1) ** 2)
    return 4.0 * math.pi ** 2 * e


CASES = [
    ((9.0, 4.0, 1.5), (math.cos(0.4), math.sin(0.4)), 0.0),
    ((9.0, 4.0, 1.5), (math.cos(2.1), math.sin(2.1)), 2.5),
    ((2.0, 6.5, -1.2), (0.0, 1.0), 5.0),
    ((4.0, 4.0, 0.0), (1.0, 0.0), 1.0),
]


@pytest.mark.parametrize("S,n,c", CASES)
def test_halfplane_field_matches_quadrature(S, n, c):
    """2-D quadrature of int_{n.x > c} w(x) e^{i v.x} dx (and over the whole plane) at transfers
    from the lobe's centre out along the boundary's diffraction streak."""
    rng = np.random.default_rng(3)
    vs = np.concatenate([rng.normal(0.0, 0.3, (6, 2)), 2.5 * np.asarray(n)[None, :] * np.arange(1, 5)[:, None],
                         rng.normal(0.0, 1.5, (4, 2))])
    whole, far = oracle.halfplane_field(S, n, c, vs)
    nrm = math.sqrt(_norm(S))
    scale = whole.max()
    for v, g, f in zip(vs, whole, far):
        vmax = float(np.hypot(*v))
        x1, w1 = _edge_grid(S, n, c, 1, vmax)
        x0, w0 = _edge_grid(S, n, c, 0, vmax)
        F = np.sum(w1 * _window(S, x1) * np.exp(1j * x1 @ v)) / nrm
        G = F + np.sum(w0 * _window(S, x0) * np.exp(1j * x0 @ v)) / nrm
        assert abs(F - f) < 1e-9 * scale, (v, F, f)
        assert abs(G - g) < 1e-9 * scale, (v, G, g)


def test_window_field_is_the_window_spectrum():
    """|G(v)|^2 of the whole plane is the window spectrum density N(v; 0, S^-1 / 4), the
    single-material smooth kernel with reflectance 1."""
    S = (9.0, 4.0, 1.5)
    vs = np.random.default_rng(5).normal(0.0, 0.4, (20, 2))
    g, _ = oracle.halfplane_field(S, (1.0, 0.0), 0.0, vs)
    k = 20.0
    pw = [oracle.pw(0, 0.0, 1.0, k, (0.0, 0.0), tuple(v), S) for v in vs]
    assert np.allclose(g ** 2, pw, rtol=1e-12, atol=0.0)


# --------------------------------------------------------------------------------------
# Composite p_w against the phase-averaged defining integral
# --------------------------------------------------------------------------------------

def _side_field(S, n, c, side, kappa, qz, mat, g, phases):
    """int over the side's half-plane of w(x) t(x) e^{i kappa.x} for each profile phase.
    mat = (kind, h, Lambda, refl) with kind 0 smooth, 2 grating (h = amplitude)."""
    kind, h, lam, refl = mat
    vmax = float(np.hypot(*kappa)) + (2 * math.pi / lam if kind == 2 else 0.0) * (abs(qz * h) + 3)
    x, w = _edge_grid(S, n, c, side, vmax)
    base = w * _window(S, x) * np.exp(1j * x @ kappa) * math.sqrt(refl)
    if kind == 0:
        return np.array([np.sum(base)] * len(phases))
    K = 2 * math.pi / lam
    gx = x @ np.asarray(g)
    return np.array([np.sum(base * np.exp(1j * qz * h * np.sin(K * gx + ph))) for ph in phases])


def _brute_composite(S, n, c, kin, kout, k, near, far, gn, gf, P=24):
    kappa = np.asarray(kout) - np.asarray(kin)
    ci = math.sqrt(1 - (kin[0] ** 2 + kin[1] ** 2) / k ** 2)
    co = math.sqrt(1 - (kout[0] ** 2 + kout[1] ** 2) / k ** 2)
    qz = k * (ci + co)
    phases = 2 * math.pi * np.arange(P) / P
    un = _side_field(S, n, c, 0, kappa, qz, near, gn, phases)
    uf = _side_field(S, n, c, 1, kappa, qz, far, gf, phases)
    # independent uniform phases of the two profiles: E|U_n + U_f|^2
    val = np.mean(np.abs(un) ** 2) + np.mean(np.abs(uf) ** 2) + 2 * np.real(np.mean(un) * np.conj(np.mean(uf)))
    return val / _norm(S)


def _row(near, gn, far, gf, k, kin, kout, S, n, c):
    return [near[0], near[1], near[2], near[3], gn[0], gn[1], far[0], far[1], far[2], far[3], gf[0], gf[1],
            k, kin[0], kin[1], kout[0], kout[1], S[0], S[1], S[2], n[0], n[1], c]


SMOOTH1 = (0, 0.0, 1.0, 1.0)
SMOOTH03 = (0, 0.0, 1.0, 0.3)
GRAT_A = (2, 0.04, 2.0, 0.9)          # amplitude 0.04 um, pitch 2 um
GRAT_B = (2, 0.06, 1.3, 1.0)

COMPOSITE_CASES = [
    # near, gn, far, gf, S, n, c, kin, kout
    (SMOOTH1, (1, 0), SMOOTH03, (1, 0), (6.0, 4.0, 1.0), (math.cos(0.3), math.sin(0.3)), 1.0, (2.0, 0.5), (-2.2, -0.4)),
    (SMOOTH1, (1, 0), SMOOTH03, (1, 0), (6.0, 4.0, 1.0), (math.cos(0.3), math.sin(0.3)), 1.0, (2.0, 0.5), (-1.4, -0.1)),
    (SMOOTH1, (1, 0), GRAT_A, (math.cos(1.0), math.sin(1.0)), (2.0, 1.2, 0.3), (0.6, 0.8), 0.5, (1.0, 0.0), (-1.2, 0.3)),
    (GRAT_A, (1, 0), SMOOTH03, (1, 0), (2.0, 1.2, 0.3), (0.6, -0.8), 1.0, (1.0, 0.0), (-1.0 + 2 * math.pi / 2.0, 0.1)),
    (GRAT_A, (1, 0), GRAT_B, (0.0, 1.0), (1.5, 1.5, 0.0), (1.0, 0.0), 0.0, (0.5, 0.5), (-0.6, -0.3)),
]


@pytest.mark.parametrize("case", range(len(COMPOSITE_CASES)))
def test_composite_matches_phase_averaged_integral(case):
    """2-D quadrature of |int w t e^{i kappa.x}|^2 averaged over the two profiles' phases
    (24 equally spaced phases each: exact for these trigonometric polynomials, whose Bessel
    weights are below 1e-10 beyond order 10), normalised by (2 pi)^2 int |w|^2."""
    near, gn, far, gf, S, n, c, kin, kout = COMPOSITE_CASES[case]
    k = K550
    ref = _brute_composite(S, n, c, kin, kout, k, near, far, gn, gf)
    got = oracle.pw_composite_batch(np.array([_row(near, gn, far, gf, k, kin, kout, S, n, c)]))[0]
    assert ref > 0
    assert abs(got - ref) <= 1e-9 * ref, (got, ref)


def test_composite_rough_side():
    """A rough side's coherent part is its mean field exp(-g/2) (a smooth side of that
    amplitude, by quadrature); its diffuse Poisson terms n >= 1 are the single-material ones
    weighted by the window's intensity mass on its side."""
    S, n, c = (6.0, 4.0, 1.0), (math.cos(0.3), math.sin(0.3)), 1.5
    k = K550
    kin, kout = (2.0, 0.5), (-2.1, -0.6)
    h, ell, refl = 0.02, 1.5, 0.8
    ci = math.sqrt(1 - (kin[0] ** 2 + kin[1] ** 2) / k ** 2)
    co = math.sqrt(1 - (kout[0] ** 2 + kout[1] ** 2) / k ** 2)
    g = (k * (ci + co) * h) ** 2
    coh = _brute_composite(S, n, c, kin, kout, k, (0, 0.0, 1.0, refl * math.exp(-g)), SMOOTH03, (1, 0), (1, 0))
    snn = n[0] ** 2 * S[0] + 2 * n[0] * n[1] * S[2] + n[1] ** 2 * S[1]
    mass_near = 1.0 - 0.5 * math.erfc(c / math.sqrt(2 * snn))
    full = oracle.pw(1, h, ell, k, kin, kout, S, refl=refl)
    spec = refl * math.exp(-g) * oracle.pw(0, 0.0, 1.0, k, kin, kout, S)
    ref = coh + mass_near * (full - spec)
    got = oracle.pw_composite_batch(np.array([_row((1, h, ell, refl), (1, 0), SMOOTH03, (1, 0), k, kin, kout, S, n, c)]))[0]
    assert abs(got - ref) <= 1e-9 * ref


def test_composite_diffuse_reading_error_is_small():
    """The local reading of a rough side's diffuse part (the window's intensity mass on the
    side times the single-material terms) against the exact ensemble integral over the
    half-plane: for a lag D between two points of the side, the pair density of the window
    restricted to the side is Phi(-(c + |n.D|/2) / s_n) instead of Phi(-c / s_n), with s_n^2
    the window's intensity variance across the boundary.  Exact value by quadrature over the
    lag; at a correlation length of 1/20 of the footprint the reading is within 3 %."""
    S = (100.0, 64.0, 10.0)
    n, c = (1.0, 0.0), 6.0
    ell, g = 0.5, 4.0
    Sm = np.array([[S[0], S[2]], [S[2], S[1]]])
    A = 0.5 * np.linalg.inv(Sm)
    snn = Sm[0, 0]
    kappa = np.array([0.3, -0.2])
    # lag quadrature; the integrand is smooth on each side of n.D = 0
    xs, ws = _gl_panels(-6.0, 6.0, 0.5)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Wt = ws[:, None] * ws[None, :]
    D = np.stack([X, Y], -1)
    quadA = np.einsum("...i,ij,...j->...", D, A, D)
    ph = np.exp(1j * (D @ kappa))
    exact = local = 0.0
    Phi = lambda t: 0.5 * special.erfc(-t / math.sqrt(2.0))
    for m in range(1, 40):
        wgt = math.exp(-g + m * math.log(g) - math.lgamma(m + 1))
        base = Wt * ph * np.exp(-m * (X ** 2 + Y ** 2) / ell ** 2 - 0.25 * quadA)
        exact += wgt * np.real(np.sum(base * Phi(-(c + 0.5 * np.abs(X)) / math.sqrt(snn))))
        local += wgt * np.real(np.sum(base * Phi(-c / math.sqrt(snn))))
    assert local > 0 and exact > 0
    rel = abs(local - exact) / exact
    assert rel < 0.03, rel


def test_composite_limits_and_reciprocity():
    rng = np.random.default_rng(7)
    k = K550
    S = (20.0, 12.0, 3.0)
    n = (math.cos(0.9), math.sin(0.9))
    snn = n[0] ** 2 * S[0] + 2 * n[0] * n[1] * S[2] + n[1] ** 2 * S[1]
    rows, single = [], []
    for near in [SMOOTH1, GRAT_A, (1, 0.05, 2.0, 0.7)]:
        for _ in range(4):
            kin = rng.normal(0, 1.5, 2)
            kout = -kin + rng.normal(0, 0.3, 2)
            rows.append(_row(near, (1, 0), GRAT_B, (0, 1), k, kin, kout, S, n, 40.0 * math.sqrt(snn)))
            single.append(oracle.pw(near[0], near[1], near[2], k, tuple(kin), tuple(kout), S, refl=near[3]))
    got = oracle.pw_composite_batch(np.array(rows))
    # tolerance: relative, plus rounding of the lobe's peak density where the sides' fields
    # cancel (far out in the boundary's streak)
    peak = oracle.pw(0, 0.0, 1.0, k, (0.0, 0.0), (0.0, 0.0), S)
    # a boundary far outside the window leaves the near material's kernel
    assert np.allclose(got, single, rtol=1e-12, atol=1e-14 * peak)
    # the same smooth material on both sides: the single-material kernel at any distance
    same = [_row((0, 0, 1, 0.7), (1, 0), (0, 0, 1, 0.7), (1, 0), k, r[13:15], r[15:17], S, n, 0.4) for r in rows]
    ref = [oracle.pw(0, 0.0, 1.0, k, tuple(r[13:15]), tuple(r[15:17]), S, refl=0.7) for r in rows]
    assert np.allclose(oracle.pw_composite_batch(np.array(same)), ref, rtol=1e-12, atol=1e-14 * peak)
    # reciprocity: (k_i -> k_o) and (-k_o -> -k_i) with the same footprint and boundary
    mixed = np.array([_row(SMOOTH1, (1, 0), GRAT_A, (0.6, 0.8), k, r[13:15], r[15:17], S, n, 1.0) for r in rows])
    rev = mixed.copy()
    rev[:, 13:15], rev[:, 15:17] = -mixed[:, 15:17], -mixed[:, 13:15]
    a, b = oracle.pw_composite_batch(mixed), oracle.pw_composite_batch(rev)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * peak)


# --------------------------------------------------------------------------------------
# Boundary search
# --------------------------------------------------------------------------------------

def _np_boundaries(scene):
    tris = scene.tris.astype(np.int64)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    t = np.concatenate([np.arange(len(tris))] * 3)
    e.sort(1)
    key = e[:, 0] * (1 << 32) + e[:, 1]
    order = np.argsort(key, kind="stable")
    key, t, e = key[order], t[order], e[order]
    uniq, start, count = np.unique(key, return_index=True, return_counts=True)
    sel = start[count == 2]
    t0, t1 = t[sel], t[sel + 1]
    keep = scene.tri_mat[t0] != scene.tri_mat[t1]
    return e[sel][keep], scene.tri_mat[t0][keep], scene.tri_mat[t1][keep]


def _seg_dist(P, a, b):
    ab = b - a
    t = np.clip(np.einsum("...i,...i", P - a, ab) / np.einsum("...i,...i", ab, ab), 0.0, 1.0)
    return np.linalg.norm(P - (a + t[..., None] * ab), axis=-1)


def test_boundary_edges_and_nearest_match_brute_force():
    """The mid terrain's material boundaries (mesh edges shared by two triangles of different
    materials) and the nearest boundary of a hit's material, against NumPy brute force."""
    scene = W.terrain_scene()
    osc = oracle.OracleScene(scene)
    nb = osc.boundaries()
    edges, ma, mb = _np_boundaries(scene)
    assert nb == len(edges) > 1000
    got = osc.boundary_edges()
    key_got = {tuple(np.round(np.concatenate([np.sort(np.stack([r[0:3], r[3:6]]), 0).ravel()]), 12)) for r in got}
    v = scene.verts
    key_ref = {tuple(np.round(np.sort(np.stack([v[a], v[b]]), 0).ravel(), 12)) for a, b in edges}
    assert key_got == key_ref
    rng = np.random.default_rng(2)
    # within the grid's cell (2 mm, the default) the search goes through the grid, beyond it
    # over all of the material's edges
    for reach in [1.5e-3, 3e-3] * 3:
        mat = int(rng.integers(0, len(scene.materials)))
        tri_of = np.nonzero(scene.tri_mat == mat)[0]
        ts = rng.choice(tri_of, 40)
        bc = rng.dirichlet([1, 1, 1], 40)
        P = np.einsum("ti,tij->tj", bc, v[scene.tris[ts]])
        res = osc.nearest_boundary(mat, P, reach)
        mine = (got[:, 6] == mat) | (got[:, 7] == mat)
        idx = np.nonzero(mine)[0]
        d = _seg_dist(P[:, None, :], got[idx, 0:3][None], got[idx, 3:6][None])
        for i in range(len(P)):
            j = int(np.argmin(d[i]))
            if d[i, j] < reach:
                assert int(res[i, 0]) == idx[j] and abs(res[i, 1] - d[i, j]) < 1e-15
            else:
                assert int(res[i, 0]) == -1


# --------------------------------------------------------------------------------------
# Two mirrors meeting at a straight boundary: closed form per path
# --------------------------------------------------------------------------------------

def _propagated_sigma2(sigma_m, z_m, k):
    """Intensity variance of a generalized ray (beta^2 = 2 sigma^2, rho = 0) after z in free
    space (eq. K_free_space_propagation with rho = 0 at the start): beta^2 + zbar^2 / beta^2."""
    b2 = 2.0 * (sigma_m * 1e6) ** 2
    zb = z_m * 1e6 / k
    return 0.5 * (b2 + zb * zb / b2)


def test_split_mirror_composite_geometry_and_side_choice():
    wl = W.split_mirror()
    osc = oracle.OracleScene(wl.scene)
    k = K550
    beta2 = 2.0 * _propagated_sigma2(wl.sensor.sigma_m, 0.01, k)
    sr = math.sqrt(0.5 * beta2)
    for x_um, near_refl, far_refl in [(-20.0, 1.0, 0.25), (35.0, 0.25, 1.0), (-3.0, 1.0, 0.25)]:
        o = (x_um * 1e-6, 0.1e-3, 0.01)
        c_ref = abs(x_um)
        mf_ref = 0.5 * math.erfc(c_ref / (math.sqrt(2.0) * sr))
        lo = oracle.OracleScene.interaction_composite(osc, o, (0, 0, -1), k, beta2, (0.5, 0.5, 0.5, 1 - mf_ref - 1e-9))
        hi = oracle.OracleScene.interaction_composite(osc, o, (0, 0, -1), k, beta2, (0.5, 0.5, 0.5, 1 - mf_ref + 1e-9))
        assert lo["composite"] and abs(lo["c"] - c_ref) < 1e-9 and abs(abs(lo["n"][0]) + abs(lo["n"][1]) - 1) < 1e-12
        assert abs(lo["mass_far"] - mf_ref) < 1e-12
        assert not lo["far"] and lo["weight"] == pytest.approx(near_refl, abs=1e-15)
        assert hi["far"] and hi["weight"] == pytest.approx(far_refl, abs=1e-15)
    # beyond 2.5 beta of the boundary: no composite
    far_x = 2.5 * math.sqrt(beta2) * 1.01
    r = osc.interaction_composite((-far_x * 1e-6, 0.0, 0.01), (0, 0, -1), k, beta2, (0.5, 0.5, 0.5, 0.5))
    assert not r["composite"]
    r = osc.interaction_composite((-0.99 * 2.5 * math.sqrt(beta2) * 1e-6, 0.0, 0.01), (0, 0, -1), k, beta2,
                                  (0.5, 0.5, 0.5, 0.5))
    assert r["composite"]


@pytest.mark.parametrize("aniso", [False, True])
@pytest.mark.parametrize("reach_m", [2e-3, 60e-6])
def test_split_mirror_per_path_closed_form(reach_m, aniso):
    """Two smooth mirrors (reflectance a_l = 1, a_r = 0.25) meeting at x = 0, normal incidence,
    light at the mirror direction (kappa = 0).  At kappa = 0 the far half-plane's field is half
    the whole window's times erfc(c / (2 s)) (s: the window's intensity std), so a path that
    meets the surface at distance c from the boundary measures
        p_w = (2 s^2 / pi) [sqrt(a_near) (1 - E) + sqrt(a_far) E]^2,  E = erfc(c / (2 s)) / 2,
    inside min(2.5 beta, reach) of the boundary and a_near 2 s^2 / pi beyond it.  The hit point
    of each path is its pixel position plus the source draw's first two uniforms.  An
    anisotropic ray (its second moments carried as matrices) starts isotropic and stays so along
    the axis, so it meets the same closed form."""
    wl = W.split_mirror(width=64, height=2, spp=4)
    k = K550
    img, st, paths = oracle.render(wl, composite=True, reach_m=reach_m, keep_paths=True, aniso=aniso)
    s2 = _propagated_sigma2(wl.sensor.sigma_m, 0.01, k)
    s = math.sqrt(s2)
    rad = min(2.5 * math.sqrt(2.0 * s2) * 1e-6, reach_m)
    W_, H_ = wl.sensor.width, wl.sensor.height
    n_comp = 0
    for sl in range(wl.spp):
        for y in range(H_):
            for x in range(W_):
                pid = ((sl * H_ + y) * W_ + x) * 1 + 0
                r = oracle.philox(np.array([[pid & 0xFFFFFFFF, pid >> 32, 0, 0]], np.uint32),
                                  np.array([wl.seed & 0xFFFFFFFF, wl.seed >> 32], np.uint32))[0]
                u0 = (int(r[0]) >> 8) / 16777216.0
                xw = wl.sensor.origin[0] + (x + u0) * wl.sensor.pitch_m * wl.sensor.axis_u[0]
                a_n, a_f = (1.0, 0.25) if xw < 0 else (0.25, 1.0)
                c_m = abs(xw)
                if c_m < rad:
                    n_comp += 1
                    E = 0.5 * math.erfc(c_m * 1e6 / (2.0 * s))
                    ref = 2.0 * s2 / math.pi * (math.sqrt(a_n) * (1 - E) + math.sqrt(a_f) * E) ** 2
                else:
                    ref = a_n * 2.0 * s2 / math.pi
                got = paths[sl, y * W_ + x, 0] * wl.spp
                assert abs(got - ref) <= 1e-9 * ref, (x, y, sl, xw, got, ref)
    assert st["composite"] == n_comp > 0


# --------------------------------------------------------------------------------------
# Composite interactions on hero-wavelength paths (reading R31)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("reach_m", [2e-3, 60e-6])
def test_hero_split_mirror_per_path_closed_form(reach_m):
    """Hero-wavelength paths on the split mirror, four wavelengths per path: at the single
    vertex every member measures its own composite p_w (the closed form of
    test_split_mirror_per_path_closed_form with that member's window s_i), and the balance
    heuristic's weights are 1 there (T = R = 1, plane wave), so each member's record is its
    closed form.  The boundary is detected with the hero's window: min(2.5 beta_h, reach)."""
    wl = W.split_mirror(width=64, height=2, spp=4, n_lambda=4)
    img, st, paths = oracle.render(wl, composite=True, reach_m=reach_m, keep_paths=True, hero=True)
    W_, H_ = wl.sensor.width, wl.sensor.height
    ks = [2.0 * math.pi / lam for lam in wl.lambdas_um]
    s2 = [_propagated_sigma2(wl.sensor.sigma_m, 0.01, k) for k in ks]
    n_comp = 0
    for sl in range(wl.spp):
        for y in range(H_):
            for x in range(W_):
                pid = ((sl * H_ + y) * W_ + x) * 1 + 0          # one rotation group
                r = oracle.philox(np.array([[pid & 0xFFFFFFFF, pid >> 32, 0, 0]], np.uint32),
                                  np.array([wl.seed & 0xFFFFFFFF, wl.seed >> 32], np.uint32))[0]
                u0 = (int(r[0]) >> 8) / 16777216.0
                hs = int(r[3]) >> 30
                xw = wl.sensor.origin[0] + (x + u0) * wl.sensor.pitch_m * wl.sensor.axis_u[0]
                a_n, a_f = (1.0, 0.25) if xw < 0 else (0.25, 1.0)
                c_m = abs(xw)
                rad = min(2.5 * math.sqrt(2.0 * s2[hs]) * 1e-6, reach_m)
                comp = c_m < rad
                n_comp += comp
                for i in range(4):
                    if comp:
                        E = 0.5 * math.erfc(c_m * 1e6 / (2.0 * math.sqrt(s2[i])))
                        ref = 2.0 * s2[i] / math.pi * (math.sqrt(a_n) * (1 - E) + math.sqrt(a_f) * E) ** 2
                    else:
                        ref = a_n * 2.0 * s2[i] / math.pi
                    got = paths[sl, y * W_ + x, i] * wl.spp
                    assert abs(got - ref) <= 1e-9 * ref, (x, y, sl, i, hs, got, ref)
    assert st["composite"] == n_comp > 0


def test_hero_composite_unbiased_on_terrain():
    """Hero-wavelength paths with composite interactions against one-wavelength paths with
    them (pinned above) on the whole terrain at 41 x 29 pixels, where the ~1 mm footprints put
    most interactions within reach of a boundary: the per-wavelength totals agree within their
    Monte Carlo error (the companions' mixture densities, the members' far masses and the side
    choice all enter)."""
    wl = W.as_float32_inputs(W.mid_terrain(width=41, height=29, spp=64, n_lambda=8))
    sc = oracle.OracleScene(wl.scene)
    sc.boundaries(2e-3)
    _, sa, pa = oracle.render(wl, oscene=sc, composite=True, reach_m=2e-3, keep_paths=True)
    _, sb, pb = oracle.render(wl, oscene=sc, composite=True, reach_m=2e-3, keep_paths=True, hero=True)
    print("composite interactions: one-wavelength", sa["composite"], "hero", sb["composite"])
    assert sb["composite"] > 0.2 * sb["segments"]
    zs = []
    for w in range(len(wl.lambdas_um)):
        xa, xb = pa[:, :, w].sum(1), pb[:, :, w].sum(1)      # per-sample totals (independent)
        se = math.sqrt(wl.spp * (xa.var(ddof=1) + xb.var(ddof=1)))
        zs.append((xb.sum() - xa.sum()) / se)
    print("hero vs one-wavelength composite paths, z per wavelength:", np.round(zs, 2))
    assert np.all(np.abs(zs) < 4.5)


_SMOOTH = (0, 0.0, 1.0, 0.9, 1.0, 0.0)
_ROUGH_A = (1, 0.06, 2.0, 0.8, 1.0, 0.0)
_ROUGH_B = (1, 0.15, 4.0, 0.7, 1.0, 0.0)
_GRATING_A = (2, 0.08, 2.0, 0.85, 1.0, 0.0)
_GRATING_B = (2, 0.05, 1.2, 0.9, 0.6, 0.8)


@pytest.mark.parametrize("near,far", [(_SMOOTH, _ROUGH_A), (_ROUGH_A, _ROUGH_B), (_GRATING_A, _ROUGH_B),
                                      (_SMOOTH, _GRATING_B), (_GRATING_A, _GRATING_B), (_ROUGH_B, _SMOOTH)])
def test_hero_composite_step_importance_identity(near, far):
    """One continuation step at a composite interaction, hero and companion with different
    wavenumbers and far masses: the companion's ratios f_c / p_h and p_c / p_h, averaged over
    the hero's samples (side choice included), reproduce the averages over the companion's own
    mixture sampling, for Gaussian test functions of the outgoing direction centred on the
    specular direction, on a lobe, and off it.  The identity covers the classes the members
    share, the specular direction and the rough lobes: a grating's orders j != 0 move with the
    wavelength, so the hero never samples the companion's (those are covered when the
    companion is the hero), and the companion's own samples of them are left out."""
    rng = np.random.default_rng(sum(int(v * 100) for v in near + far))
    n = 200000
    kh, kc = 2 * math.pi / 0.45, 2 * math.pi / 0.65
    th = 0.45
    ui, ci = (math.sin(th), 0.0), math.cos(th)
    mh, mc = 0.3, 0.45
    a = oracle.hero_composite_step(near, far, mh, mc, kh, kc, ui, ci, rng.random((n, 4)))
    b = oracle.hero_composite_step(near, far, mc, mc, kc, kc, ui, ci, rng.random((n, 4)))
    ma, mb = np.isfinite(a[:, 0]), np.isfinite(b[:, 0])
    mb = mb & (np.nan_to_num(b[:, 5], nan=2.0) != 2.0)        # the companion's shared classes
    assert np.any(a[ma, 5] == 0.0)
    for cx, w in [(0.0, 0.02), (0.0, 0.1), (0.1, 0.1), (0.3, 0.2), (-0.2, 0.15)]:
        def phi(r, k, m):
            ux = np.where(m, r[:, 0], 0.0) / k - ui[0] - cx
            uy = np.where(m, r[:, 1], 0.0) / k
            return np.where(m, np.exp(-(ux ** 2 + uy ** 2) / (2 * w * w)), 0.0)
        pa, pb = phi(a, kh, ma), phi(b, kc, mb)
        for xa, xb in ((np.where(ma, a[:, 3], 0) * pa, np.where(mb, b[:, 2], 0) * pb),    # f
                       (np.where(ma, a[:, 4], 0) * pa, pb)):                               # p
            se = math.hypot(xa.std(), xb.std()) / math.sqrt(n)
            z = (xa.mean() - xb.mean()) / max(se, 1e-300)
            assert abs(z) < 5.0 or abs(xa.mean() - xb.mean()) <= 1e-12, (cx, w, xa.mean(), xb.mean(), z)
    # a companion identical to the hero (same wavenumber and far mass) has the hero's own
    # weight f_h / p_h and density ratio 1 in the shared classes
    c = oracle.hero_composite_step(near, far, mh, mh, kh, kh, ui, ci, rng.random((n, 4)))
    mcm = np.isfinite(c[:, 0]) & (np.nan_to_num(c[:, 5], nan=2.0) != 2.0)
    assert np.allclose(c[mcm, 2], c[mcm, 3], rtol=1e-12) and np.allclose(c[mcm, 4], 1.0, rtol=1e-12)
