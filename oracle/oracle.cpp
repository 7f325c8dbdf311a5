// FP64 reference implementation ("oracle") of the backward generalized-ray path tracer.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
// file; only the test-suite, the smoke check and the CPU baseline leg of the benchmark do.
// It shares no source with the HIP path: its own counter RNG, its own BVH, its own
// intersection routine, its own scattering kernels, all in double precision, written for
// clarity rather than speed.
//
// Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762).
// Each function names the section / equation it follows.  Readings of passages the paper
// leaves open are listed in the design notes and repeated next to the code that takes them.
//
// Parity status: every component below is pinned by the CPU test-suite except where a
// function header says "parity unpinned".

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

// Worker threads when the caller does not say: the hardware threads, at most 16 (a
// one-GPU share of a shared host).
static int default_threads() {
    const int hw = (int)std::thread::hardware_concurrency();
    return hw > 0 ? std::min(hw, 16) : 1;
}

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------------------------------
// Counter-based RNG: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11).  Round function: two 32x32->64 multiplies of counter
// words 0 and 2 by the published multipliers; the high halves are xored with the other counter
// words and the key; the key is bumped by the published Weyl constants between rounds.
// ------------------------------------------------------------------------------------------
struct U4 { uint32_t v[4]; };

U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = M0 * (uint64_t)x0;
        uint64_t p1 = M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += W0; k1 += W1;
    }
    return U4{{x0, x1, x2, x3}};
}

// 24-bit uniform in [0, 1): exactly representable in float and double.
inline double unif(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// Standard normal pair by the Box-Muller transform of two uniforms.
inline void box_muller(double u1, double u2, double& z1, double& z2) {
    double r = std::sqrt(-2.0 * std::log(1.0 - u1));
    double ph = 2.0 * kPi * u2;
    z1 = r * std::cos(ph);
    z2 = r * std::sin(ph);
}

// Random-stream layout.  Counter = (path id low, path id high, interaction index, stream).
enum { STREAM_SOURCE = 0, STREAM_NEE = 1, STREAM_SCATTER = 2 };

U4 draw(uint64_t pid, uint32_t depth, uint32_t stream, uint64_t seed) {
    return philox((uint32_t)pid, (uint32_t)(pid >> 32), depth, stream, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// ------------------------------------------------------------------------------------------
// Small vector helpers.
// ------------------------------------------------------------------------------------------
struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) { return (1.0 / norm(a)) * a; }
inline V3 ld3(const double* p) { return {p[0], p[1], p[2]}; }

// Self-intersection offset (metres): a fixed relative tolerance of the ray origin's size.
inline double t_eps(V3 o) {
    double m = std::max(std::fabs(o.x), std::max(std::fabs(o.y), std::fabs(o.z)));
    return 1e-7 * (1.0 + m);
}

}  // namespace

// ==========================================================================================
// C structures of the oracle's interface (its own; the product library defines its own).
// ==========================================================================================
extern "C" {

typedef struct {
    int32_t kind;               // 0 smooth, 1 gaussian random rough, 2 sinusoidal grating
    double height_um;           // rough: RMS height; grating: amplitude A
    double length_um;           // rough: 1/e correlation length; grating: pitch
    double gdir[3];             // grating vector direction (world)
    double reflectance;
} or_material;

typedef struct {
    double origin[3], axis_u[3], axis_v[3], dir[3];
    int32_t width, height;
    double pitch_m, sigma_m;
} or_sensor;

typedef struct {
    int32_t kind;               // 0 plane wave, 1 gaussian-schell area emitter
    double dir[3], pos[3], eu[3], ev[3];
    double rc_um, power;
} or_source;

typedef struct {
    int64_t spp_begin, spp_count;
    double spp_norm;            // contributions are divided by this (total samples per pixel)
    int32_t max_depth;
    int32_t rr_enable;
    uint32_t rr_threshold24;    // survive iff (draw >> 8) < threshold
    double rr_p;
    uint64_t seed;
    int32_t use_bvh;            // 0: brute-force closest hit
    int32_t n_threads;
    int32_t hero;               // 1: hero-wavelength paths over rotation groups (nl % 4 == 0)
    int32_t aniso;              // 1: anisotropic generalized rays (matrix beta, rho)
    int32_t composite;          // 1: composite interactions at material boundaries
    double reach_m;             // composite: largest boundary distance considered (metres)
} or_opts;

}  // extern "C"

namespace {

// ------------------------------------------------------------------------------------------
// Scattering of a curvature-free generalized ray by one surface patch (Sec. "Interaction
// Kernels": reflection, sinusoidal grating, rough surface).  The windowed diffraction
// density p_w over the outgoing tangential wavevector is the squared Fourier transform of
// the window times the surface phase screen, normalised by the window energy.  With the
// Gaussian window of the generalized ray it becomes a Gaussian mixture (see design notes).
// ------------------------------------------------------------------------------------------

// Bivariate normal density N(x; 0, S), S = [[a, c], [c, b]].
double gauss2(double x, double y, double a, double b, double c) {
    double det = a * b - c * c;
    double q = (b * x * x - 2.0 * c * x * y + a * y * y) / det;
    return std::exp(-0.5 * q) / (2.0 * kPi * std::sqrt(det));
}

// Bessel function of the first kind of integer order (library primitive; J_{-n} = (-1)^n J_n).
double besselj(int n, double x) {
    int an = std::abs(n);
    double v = (x < 0.0) ? ((an & 1) ? -std::cyl_bessel_j((double)an, -x)
                                     : std::cyl_bessel_j((double)an, -x))
                         : std::cyl_bessel_j((double)an, x);
    if (n < 0 && (an & 1)) v = -v;
    // Far beyond the turning point (order above the argument) J_n(x) underflows; the library
    // routine returns NaN there instead of 0 (e.g. order 1000 at x = 228).
    if (std::isnan(v) && (double)an > std::fabs(x)) v = 0.0;
    return v;
}

struct Mat {
    int kind; double h, L, refl; V3 gdir;
};

// p_w(k_i,t -> k_o,t), a density over the outgoing tangential wavevector (um^2).
// kit, kot: tangential wavevectors in the material frame (um^-1); k = 2 pi / lambda;
// (sxx, syy, sxy): intensity footprint covariance of the window on the surface (um^2);
// (gx, gy): grating direction in the frame.
double pw_eval(const Mat& m, double k, double kix, double kiy, double kox, double koy,
               double sxx, double syy, double sxy, double gx, double gy) {
    double ni = (kix * kix + kiy * kiy) / (k * k);
    double no = (kox * kox + koy * koy) / (k * k);
    if (ni >= 1.0 || no >= 1.0) return 0.0;
    double ci = std::sqrt(1.0 - ni), co = std::sqrt(1.0 - no);
    double qz = k * (ci + co);                       // normal wavevector transfer (reflection)
    double kx = kox - kix, ky = koy - kiy;            // tangential transfer kappa
    // Window spectrum covariance: the amplitude window exp(-x^T S^-1 x / 4) has a squared
    // Fourier transform with covariance S^-1 / 4.
    double det = sxx * syy - sxy * sxy;
    double a = 0.25 * syy / det, b = 0.25 * sxx / det, c = -0.25 * sxy / det;
    if (m.kind == 0) {
        return m.refl * gauss2(kx, ky, a, b, c);
    }
    if (m.kind == 2) {
        // Phase screen h(x) = A sin(K g.x): Jacobi-Anger expansion into orders j with
        // weights J_j(q_z A)^2 centred on kappa = -j K g (grating equation).
        double K = 2.0 * kPi / m.L;
        double mm = qz * m.h;
        int J = (int)std::ceil(std::fabs(mm)) + 40;
        double s = 0.0;
        for (int j = -J; j <= J; ++j) {
            double bj = besselj(j, mm);
            s += bj * bj * gauss2(kx + j * K * gx, ky + j * K * gy, a, b, c);
        }
        return m.refl * s;
    }
    // Gaussian random surface, RMS s, autocorrelation exp(-tau^2 / l^2), ensemble average:
    // exp(-g (1 - C)) expanded as a Poisson series in g = (q_z s)^2; term n carries the
    // window spectrum convolved with an isotropic Gaussian of variance 2 n / l^2.
    double g = qz * qz * m.h * m.h;
    double s = 0.0;
    if (g == 0.0) return m.refl * gauss2(kx, ky, a, b, c);
    int M = (int)std::ceil(g + 20.0 * std::sqrt(g) + 40.0);
    double lg = std::log(g);
    for (int n = 0; n <= M; ++n) {
        double lw = -g + n * lg - std::lgamma((double)n + 1.0);
        double w = std::exp(lw);
        if (w == 0.0) continue;
        double add = 2.0 * n / (m.L * m.L);
        s += w * gauss2(kx, ky, a + add, b + add, c);
    }
    return m.refl * s;
}

// Continuation sampling from the unwindowed kernel f_inf (the delta-lobe limit of p_w),
// Sec. "Interaction Kernels" (grating orders, rough-surface Monte Carlo) with the incident
// wave taken along the generalized ray's own travel direction (time reversal = wavevector
// reversal; the kernels used here are reciprocal).  Returns false when the path ends.
// comp (optional) receives the sampled component: the grating order j, the rough surface's
// Poisson term n (0 = the specular delta), 0 for a smooth surface.
bool sample_finf(const Mat& m, double k, double kix, double kiy, double ci, double u0, double u1,
                 double u2, double gx, double gy, double& kox, double& koy, double& weight,
                 int& evanescent, int* comp = nullptr) {
    evanescent = 0;
    if (comp) *comp = 0;
    if (m.kind == 0) {
        kox = kix; koy = kiy; weight = m.refl;
        return true;
    }
    if (m.kind == 2) {
        double K = 2.0 * kPi / m.L;
        int J = (int)std::ceil(2.0 * k / K) + 2;
        std::vector<double> w;
        std::vector<int> js;
        double W = 0.0;
        for (int j = -J; j <= J; ++j) {
            double ox = kix - j * K * gx, oy = kiy - j * K * gy;
            double no = (ox * ox + oy * oy) / (k * k);
            if (no >= 1.0) continue;                  // evanescent orders are dropped
            double mj = k * m.h * (ci + std::sqrt(1.0 - no));
            double bj = besselj(j, mj);
            w.push_back(bj * bj);
            js.push_back(j);
            W += bj * bj;
        }
        if (W <= 0.0) { evanescent = 1; return false; }
        double target = u0 * W, c = 0.0;
        int pick = js.back();
        for (size_t i = 0; i < w.size(); ++i) {
            c += w[i];
            if (target < c) { pick = js[i]; break; }
        }
        kox = kix - pick * K * gx;
        koy = kiy - pick * K * gy;
        weight = m.refl * W;
        if (comp) *comp = pick;
        return true;
    }
    // rough: term n ~ Poisson(g) at the specular normal transfer, then kappa ~ N(0, 2n/l^2 I)
    double g = 4.0 * k * k * ci * ci * m.h * m.h;
    int n = 0;
    if (g > 0.0) {
        int M = (int)std::ceil(g + 20.0 * std::sqrt(g) + 40.0);
        double lg = std::log(g), c = 0.0;
        n = M;
        for (int i = 0; i <= M; ++i) {
            c += std::exp(-g + i * lg - std::lgamma((double)i + 1.0));
            if (u0 < c) { n = i; break; }
        }
    }
    if (comp) *comp = n;
    double z1, z2;
    box_muller(u1, u2, z1, z2);
    double sd = std::sqrt(2.0 * n) / m.L;
    kox = kix + sd * z1;
    koy = kiy + sd * z2;
    if ((kox * kox + koy * koy) >= k * k) { evanescent = 1; return false; }
    weight = m.refl;
    return true;
}

// ------------------------------------------------------------------------------------------
// Composite interaction at a material boundary (Sec. "Wave-Optical Rendering", the second
// practical difficulty: a generalized ray whose footprint covers several materials meets the
// composition of their interaction operators, and the waves the materials scatter interfere;
// the paper leaves such composite operators to future work, so the operator below is this
// implementation's reading, listed in the design notes).
//
// The footprint meets one straight boundary: surface coordinates x about the hit, the near
// side (the hit's material) is n.x < c and the far side n.x > c, with n the unit normal of the
// boundary line (pointing to the far side) and c >= 0 its distance from the hit.  The field
// scattered towards the tangential transfer kappa is the Fourier integral of the amplitude
// window times each side's reflection function over its half-plane.  A deterministic surface
// (smooth, grating) has no stated position of its profile relative to the boundary, so its
// phase is averaged: cross terms survive between the two sides' undiffracted mean fields only.
// A rough side adds its ensemble mean field exp(-g/2) to that cross term and its diffuse
// (Poisson terms n >= 1) part weighted by the window's intensity mass on its side (the local
// reading: correlation length small against the footprint).  parity: pinned by 2-D quadrature
// of the defining integral (phase-averaged), the sides' limits, Parseval, the library Faddeeva
// function, and a closed-form mirror pair rendered per path.
// ------------------------------------------------------------------------------------------

// Faddeeva function w(z) = exp(-z^2) erfc(-i z), Im z >= 0.  |z| < 6 and Im z < 1: erf by
// its Maclaurin series (Abramowitz & Stegun 7.1.5) and w = exp(-z^2) (1 - erf(-i z));
// otherwise the Laplace continued fraction (A&S 7.1.4) evaluated backwards from depth 200
// (further from the real axis 1 - erf cancels, and the fraction converges well there).
std::complex<double> faddeeva(std::complex<double> z) {
    using cd = std::complex<double>;
    if (std::abs(z) < 6.0 && z.imag() < 1.0) {
        const cd zeta = cd(0.0, -1.0) * z;
        const cd z2 = zeta * zeta;
        cd term = zeta, sum = 0.0;
        for (int n = 0; n < 1000; ++n) {
            const cd add = term / (double)(2 * n + 1);
            sum += add;
            if (n > 5 && std::abs(add) <= 1e-17 * std::abs(sum)) break;
            term = -term * z2 / (double)(n + 1);
        }
        return std::exp(-z * z) * (1.0 - (2.0 / std::sqrt(kPi)) * sum);
    }
    cd t = z;
    for (int n = 200; n >= 1; --n) t = z - (0.5 * n) / t;
    return cd(0.0, 1.0 / std::sqrt(kPi)) / t;
}

// Window field over the whole plane, normalised so that its squared magnitude is the window
// spectrum density N(v; 0, S^-1 / 4): G(v) / sqrt((2 pi)^2 int |w|^2), with the amplitude
// window w(x) = exp(-x^T S^-1 x / 4) (S: intensity footprint covariance, um^2).
double window_field(double sxx, double syy, double sxy, double vx, double vy) {
    const double detS = sxx * syy - sxy * sxy;
    const double detA = 0.25 / detS;                       // A = S^-1 / 2
    const double G = 2.0 * kPi / std::sqrt(detA) * std::exp(-(sxx * vx * vx + 2.0 * sxy * vx * vy + syy * vy * vy));
    return G / std::sqrt(4.0 * kPi * kPi * kPi / std::sqrt(detA));
}

// The same integral over the far half-plane n.x > c only.  In the boundary's frame
// x = a n + b e (e = (-ny, nx)), with the window's precision A = S^-1 / 2 written Ann, Ane,
// Aee: the b integral is Gaussian, sqrt(2 pi / Aee) exp((i v_e - Ane a)^2 / (2 Aee)), and
// what remains is
//   int_c^inf exp(-p a^2 / 2 + i q a) da = sqrt(pi / (2 p)) exp(-p c^2 / 2 + i q c) w(z),
//   p = det A / Aee,  q = v_n - v_e Ane / Aee,  z = (q + i p c) / sqrt(2 p).
std::complex<double> halfplane_field(double sxx, double syy, double sxy, double nx, double ny, double c,
                                     double vx, double vy) {
    const double detS = sxx * syy - sxy * sxy;
    const double ixx = 0.5 * syy / detS, iyy = 0.5 * sxx / detS, ixy = -0.5 * sxy / detS;   // A
    const double ex = -ny, ey = nx;
    const double Ann = nx * nx * ixx + 2.0 * nx * ny * ixy + ny * ny * iyy;
    const double Aee = ex * ex * ixx + 2.0 * ex * ey * ixy + ey * ey * iyy;
    const double Ane = nx * ex * ixx + (nx * ey + ny * ex) * ixy + ny * ey * iyy;
    const double detA = Ann * Aee - Ane * Ane;
    const double vn = nx * vx + ny * vy, ve = ex * vx + ey * vy;
    const double p = detA / Aee, q = vn - ve * Ane / Aee;
    const std::complex<double> z(q / std::sqrt(2.0 * p), p * c / std::sqrt(2.0 * p));
    const std::complex<double> ph(-0.5 * p * c * c - 0.5 * ve * ve / Aee, q * c);
    const std::complex<double> F = std::sqrt(2.0 * kPi / Aee) * std::sqrt(kPi / (2.0 * p)) * std::exp(ph) * faddeeva(z);
    return F / std::sqrt(4.0 * kPi * kPi * kPi / std::sqrt(detA));
}

// One side of a composite interaction: its material and the grating direction in the frame.
struct Side { const Mat* m; double gx, gy; };

// p_w of the composite interaction (density over the outgoing tangential wavevector, um^2).
// near / far: the two sides; (nx, ny), c: the boundary in the frame; other arguments as
// pw_eval.
double pw_composite(const Side& nr, const Side& fr, double k, double kix, double kiy, double kox, double koy,
                    double sxx, double syy, double sxy, double nx, double ny, double c) {
    const double ni = (kix * kix + kiy * kiy) / (k * k);
    const double no = (kox * kox + koy * koy) / (k * k);
    if (ni >= 1.0 || no >= 1.0) return 0.0;
    const double ci = std::sqrt(1.0 - ni), co = std::sqrt(1.0 - no);
    const double qz = k * (ci + co);
    const double kx = kox - kix, ky = koy - kiy;
    const double snn = nx * nx * sxx + 2.0 * nx * ny * sxy + ny * ny * syy;
    const double mass_far = 0.5 * std::erfc(c / std::sqrt(2.0 * snn));
    const double mass[2] = {1.0 - mass_far, mass_far};
    // window spectrum covariance S^-1 / 4 (as pw_eval) for the diffuse terms
    const double det = sxx * syy - sxy * sxy;
    const double wa = 0.25 * syy / det, wb = 0.25 * sxx / det, wc = -0.25 * sxy / det;
    const Side* sd[2] = {&nr, &fr};
    std::complex<double> mean[2];
    double total = 0.0;
    for (int s = 0; s < 2; ++s) {
        const Mat& m = *sd[s]->m;
        // this side's half-plane field: far = F, near = G - F
        auto H = [&](double vx, double vy) {
            const std::complex<double> F = halfplane_field(sxx, syy, sxy, nx, ny, c, vx, vy);
            return s == 1 ? F : window_field(sxx, syy, sxy, vx, vy) - F;
        };
        if (m.kind == 0) {
            const std::complex<double> h = H(kx, ky);
            total += m.refl * std::norm(h);
            mean[s] = std::sqrt(m.refl) * h;
        } else if (m.kind == 2) {
            const double K = 2.0 * kPi / m.L;
            const double mm = qz * m.h;
            const int J = (int)std::ceil(std::fabs(mm)) + 40;
            mean[s] = 0.0;
            for (int j = -J; j <= J; ++j) {
                const double bj = besselj(j, mm);
                if (j != 0 && bj * bj < 1e-32) continue;   // orders weighing below 1e-32
                const std::complex<double> h = H(kx + j * K * sd[s]->gx, ky + j * K * sd[s]->gy);
                total += m.refl * bj * bj * std::norm(h);
                if (j == 0) mean[s] = std::sqrt(m.refl) * bj * h;
            }
        } else {
            const double g = qz * qz * m.h * m.h;
            const std::complex<double> h = H(kx, ky);
            total += m.refl * std::exp(-g) * std::norm(h);
            mean[s] = std::sqrt(m.refl) * std::exp(-0.5 * g) * h;
            if (g > 0.0) {
                const int M = (int)std::ceil(g + 20.0 * std::sqrt(g) + 40.0);
                const double lg = std::log(g);
                double dif = 0.0;
                for (int n = 1; n <= M; ++n) {
                    const double w = std::exp(-g + n * lg - std::lgamma((double)n + 1.0));
                    if (w == 0.0) continue;
                    const double add = 2.0 * n / (m.L * m.L);
                    dif += w * gauss2(kx, ky, wa + add, wb + add, wc);
                }
                total += m.refl * mass[s] * dif;
            }
        }
    }
    // non-negative in exact arithmetic (a phase average of squared magnitudes plus diffuse
    // terms); far out in the boundary's diffraction streak the sum cancels to rounding
    return std::max(0.0, total + 2.0 * std::real(mean[0] * std::conj(mean[1])));
}

// ------------------------------------------------------------------------------------------
// Hero-wavelength spectral sampling (Sec. "Interactive Rendering", implementation details: the
// hero wavelength drives the path, and paths without dispersive delta segments carry up to
// three more wavelengths).  The companions here are the other members of a rotation group of
// the wavelength grid, and the four estimates are combined by the one-sample balance heuristic
// over the four choices of hero (Wilkie, Nawaz, Droske, Weidlich, Hanika, "Hero wavelength
// spectral sampling", EGSR 2014): with f_i the path's contribution and p_i its sampling
// density at wavelength i, member i's estimate is 4 f_i / sum_k p_k.
//
// One continuation step, companion at wavenumber kc against the hero's kh.  Densities are over
// the outgoing tangential direction u_o = k_o,t / k for a continuous lobe; a delta component
// is compared by its probability.
//   smooth : one delta at the mirror direction for every wavelength: p = 1, f = refl.
//   grating: order j leaves at u_o = u_i - j K g / k, a delta that moves with the wavelength
//            (dispersive) unless j = 0, so a companion reaches the hero's direction only
//            through order 0, with probability J_0(m_0)^2 / W and value refl J_0(m_0)^2.
//   rough  : term 0 is the specular delta, probability e^-g; terms n >= 1 spread
//            kappa = k (u_o - u_i) as N(0, 2n/l^2 I), i.e. over u_o the density
//            k^2 sum_{n>=1} Poisson(n; g) N(k du; 0, 2n/l^2 I); f = refl p.
// ------------------------------------------------------------------------------------------

// Order weights of a grating at wavenumber k: W = sum of J_j(m_j)^2 over the propagating
// orders (the normalisation of order sampling) and w0 = J_0(m_0)^2.
void grating_weights(const Mat& m, double k, double kix, double kiy, double ci, double gx, double gy,
                     double& W, double& w0) {
    double K = 2.0 * kPi / m.L;
    int J = (int)std::ceil(2.0 * k / K) + 2;
    W = 0.0;
    w0 = 0.0;
    for (int j = -J; j <= J; ++j) {
        double ox = kix - j * K * gx, oy = kiy - j * K * gy;
        double no = (ox * ox + oy * oy) / (k * k);
        if (no >= 1.0) continue;
        double bj = besselj(j, k * m.h * (ci + std::sqrt(1.0 - no)));
        W += bj * bj;
        if (j == 0) w0 = bj * bj;
    }
}

// Continuous part (terms n >= 1) of the rough surface's sampling density over u_o, at squared
// direction change du2 = |u_o - u_i|^2.
double rough_lobe_density(const Mat& m, double k, double ci, double du2) {
    double g = 4.0 * k * k * ci * ci * m.h * m.h;
    if (g <= 0.0) return 0.0;
    int M = (int)std::ceil(g + 20.0 * std::sqrt(g) + 40.0);
    double lg = std::log(g), s = 0.0;
    for (int n = 1; n <= M; ++n) {
        double w = std::exp(-g + n * lg - std::lgamma((double)n + 1.0));
        double var = 2.0 * n / (m.L * m.L);
        s += w * std::exp(-0.5 * k * k * du2 / var) / (2.0 * kPi * var);
    }
    return k * k * s;
}

// f_c / p_h and p_c / p_h of a companion for the direction the hero sampled through component
// comp (as returned by sample_finf).  (ux, uy): incident tangential direction; (dux, duy):
// u_o - u_i.
void finf_companion(const Mat& m, double kh, double kc, double ux, double uy, double ci, double dux,
                    double duy, int comp, double gx, double gy, double& f_ph, double& p_ph) {
    if (m.kind == 0) {
        f_ph = m.refl;
        p_ph = 1.0;
        return;
    }
    if (m.kind == 2) {
        if (comp != 0) { f_ph = 0.0; p_ph = 0.0; return; }
        double Wh, w0h, Wc, w0c;
        grating_weights(m, kh, kh * ux, kh * uy, ci, gx, gy, Wh, w0h);
        grating_weights(m, kc, kc * ux, kc * uy, ci, gx, gy, Wc, w0c);
        double ph = w0h / Wh;                     // > 0: the hero drew order 0
        f_ph = m.refl * w0c / ph;
        p_ph = (Wc > 0.0 ? w0c / Wc : 0.0) / ph;
        return;
    }
    if (comp == 0) {
        double gh = 4.0 * kh * kh * ci * ci * m.h * m.h, gc = 4.0 * kc * kc * ci * ci * m.h * m.h;
        p_ph = std::exp(gh - gc);
        f_ph = m.refl * p_ph;
        return;
    }
    double du2 = dux * dux + duy * duy;
    p_ph = rough_lobe_density(m, kc, ci, du2) / rough_lobe_density(m, kh, ci, du2);
    f_ph = m.refl * p_ph;
}

// Companion ratios at a composite interaction of a hero-wavelength path (reading R31).  The
// continuation samples the near side's unwindowed kernel with probability 1 - m and the far
// side's with probability m (the window's intensity mass beyond the boundary), so over the
// outgoing direction member i meets the mixture (1 - m_i) f_near + m_i f_far, and the hero
// samples (1 - m_h) p_near + m_h p_far at its own wavenumber.  The sampled direction falls in
// one of three classes, and only components of that class have mass there:
//   specular : the mirror direction (smooth; a rough surface's term 0, probability e^-g; a
//              grating's order 0, probability J_0(m_0)^2 / W): shared by every wavelength;
//   lobe     : a rough surface's terms n >= 1 (a density over u_o, rough_lobe_density);
//   order    : a grating order j != 0 of the sampled side, whose direction moves with the
//              wavelength: the hero's alone.
// mass[i]: member i's far mass; far_chosen: the side the hero sampled; comp: the sampled
// component (sample_finf); (ux, uy): incident tangential direction and (dux, duy) = u_o - u_i,
// both in the near side's frame.  f_ph[i] = f_i / p_h, p_ph[i] = p_i / p_h (1 for the hero).
void composite_companions(const Side& near, const Side& far, bool far_chosen, const double mass[4],
                          const double k[4], int hi, double ux, double uy, double ci, double dux, double duy,
                          int comp, double f_ph[4], double p_ph[4]) {
    const Side& cs = far_chosen ? far : near;
    const Mat& cm = *cs.m;
    const int cls = (cm.kind == 0 || comp == 0) ? 0 : (cm.kind == 1 ? 1 : 2);   // specular, lobe, order
    const double du2 = dux * dux + duy * duy;
    const Side* sides[2] = {&near, &far};
    double f[4], p[4];
    for (int i = 0; i < 4; ++i) {
        const double a[2] = {1.0 - mass[i], mass[i]};
        f[i] = 0.0;
        p[i] = 0.0;
        if (cls == 2) {
            if (i != hi) continue;
            double W, w0;
            grating_weights(cm, k[i], k[i] * ux, k[i] * uy, ci, cs.gx, cs.gy, W, w0);
            const double K = 2.0 * kPi / cm.L;
            const double ox = k[i] * ux - comp * K * cs.gx, oy = k[i] * uy - comp * K * cs.gy;
            const double no = (ox * ox + oy * oy) / (k[i] * k[i]);
            const double bj = besselj(comp, k[i] * cm.h * (ci + std::sqrt(std::max(0.0, 1.0 - no))));
            const double as = a[far_chosen ? 1 : 0];
            p[i] = W > 0.0 ? as * bj * bj / W : 0.0;
            f[i] = as * cm.refl * bj * bj;
            continue;
        }
        for (int sd = 0; sd < 2; ++sd) {
            const Mat& M = *sides[sd]->m;
            double ps = 0.0, fs = 0.0;
            if (cls == 0) {
                if (M.kind == 0) {
                    ps = 1.0;
                    fs = M.refl;
                } else if (M.kind == 1) {
                    ps = std::exp(-4.0 * k[i] * k[i] * ci * ci * M.h * M.h);
                    fs = M.refl * ps;
                } else {
                    double W, w0;
                    grating_weights(M, k[i], k[i] * ux, k[i] * uy, ci, sides[sd]->gx, sides[sd]->gy, W, w0);
                    ps = W > 0.0 ? w0 / W : 0.0;
                    fs = M.refl * w0;
                }
            } else if (M.kind == 1) {
                ps = rough_lobe_density(M, k[i], ci, du2);
                fs = M.refl * ps;
            }
            p[i] += a[sd] * ps;
            f[i] += a[sd] * fs;
        }
    }
    const double ph = p[hi];
    for (int i = 0; i < 4; ++i) {
        f_ph[i] = ph > 0.0 ? f[i] / ph : 0.0;
        p_ph[i] = ph > 0.0 ? p[i] / ph : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// Geometry: FP64 Moller-Trumbore intersection, a median-split binary BVH, and brute force.
// Closest hit: smallest t > eps; equal t resolved to the lower triangle index.
// ------------------------------------------------------------------------------------------
struct Tri { V3 p0, p1, p2; };

bool isect_tri(const Tri& T, V3 o, V3 d, double tmin, double& t, double& u, double& v) {
    V3 e1 = T.p1 - T.p0, e2 = T.p2 - T.p0;
    V3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    V3 s = o - T.p0;
    u = dot(s, p) * inv;
    if (u < 0.0 || u > 1.0) return false;
    V3 q = cross(s, e1);
    v = dot(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return false;
    t = dot(e2, q) * inv;
    return t > tmin;
}

struct Node { V3 lo, hi; int left, right, first, count; };

struct SceneO {
    std::vector<Tri> tris;
    std::vector<V3> vn;            // per-vertex normals (3 per triangle); zero = use geometric
    std::vector<int> mat;
    std::vector<Mat> mats;
    std::vector<Node> nodes;
    std::vector<int> order;        // triangle indices referenced by leaves
    // Material boundaries (composite interactions): mesh edges shared by exactly two triangles
    // of different materials, and per material the boundary edges it lies on.
    struct BEdge { V3 p0, p1; int mat[2]; V3 opp[2]; };   // opp: each triangle's third vertex
    std::vector<BEdge> bedges;
    std::vector<std::vector<int>> mat_bedges;
    bool have_bedges = false;
    // Uniform grid over the boundary edges (cell size bcell, origin borg): each edge is listed,
    // in id order, in every cell that its box widened by bcell touches, so every edge within
    // bcell of a point is listed in the point's cell.
    double bcell = 0.0;
    V3 borg{0, 0, 0};
    std::unordered_map<uint64_t, std::vector<int>> bgrid;
};

void tri_bounds(const Tri& T, V3& lo, V3& hi) {
    lo = {std::min({T.p0.x, T.p1.x, T.p2.x}), std::min({T.p0.y, T.p1.y, T.p2.y}),
          std::min({T.p0.z, T.p1.z, T.p2.z})};
    hi = {std::max({T.p0.x, T.p1.x, T.p2.x}), std::max({T.p0.y, T.p1.y, T.p2.y}),
          std::max({T.p0.z, T.p1.z, T.p2.z})};
}

int build_rec(SceneO& S, int first, int count) {
    Node nd;
    V3 lo{1e300, 1e300, 1e300}, hi{-1e300, -1e300, -1e300};
    for (int i = first; i < first + count; ++i) {
        V3 a, b;
        tri_bounds(S.tris[S.order[i]], a, b);
        lo = {std::min(lo.x, a.x), std::min(lo.y, a.y), std::min(lo.z, a.z)};
        hi = {std::max(hi.x, b.x), std::max(hi.y, b.y), std::max(hi.z, b.z)};
    }
    nd.lo = lo; nd.hi = hi; nd.left = nd.right = -1; nd.first = first; nd.count = count;
    int id = (int)S.nodes.size();
    S.nodes.push_back(nd);
    if (count <= 4) return id;
    V3 ext = hi - lo;
    int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
    auto cen = [&](int t) {
        const Tri& T = S.tris[t];
        V3 c = (1.0 / 3.0) * (T.p0 + T.p1 + T.p2);
        return axis == 0 ? c.x : (axis == 1 ? c.y : c.z);
    };
    int mid = first + count / 2;
    std::nth_element(S.order.begin() + first, S.order.begin() + mid,
                     S.order.begin() + first + count,
                     [&](int a, int b) { return cen(a) < cen(b) || (cen(a) == cen(b) && a < b); });
    int l = build_rec(S, first, mid - first);
    int r = build_rec(S, mid, first + count - mid);
    S.nodes[id].left = l;
    S.nodes[id].right = r;
    S.nodes[id].count = 0;
    return id;
}

// Slab test; returns the entry distance in tnear.
bool box_hit(const Node& n, V3 o, V3 d, double tmax, double& tnear) {
    double t0 = 0.0, t1 = tmax;
    const double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    const double lo[3] = {n.lo.x, n.lo.y, n.lo.z}, hi[3] = {n.hi.x, n.hi.y, n.hi.z};
    for (int a = 0; a < 3; ++a) {
        if (dd[a] == 0.0) {
            if (oo[a] < lo[a] || oo[a] > hi[a]) return false;
            continue;
        }
        double inv = 1.0 / dd[a];
        double ta = (lo[a] - oo[a]) * inv, tb = (hi[a] - oo[a]) * inv;
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta);
        t1 = std::min(t1, tb);
        if (t0 > t1) return false;
    }
    tnear = t0;
    return true;
}

struct Hit { int tri; double t, u, v; };

// Closest hit along o + t d, t in (tmin, tmax).  any=true stops at the first hit found.
// skip: the triangle the ray leaves (a flat triangle cannot be hit again by a ray leaving
// it), or -1.
bool trace_ray(const SceneO& S, V3 o, V3 d, double tmin, double tmax, bool use_bvh, bool any,
               Hit& h, int skip = -1) {
    h.tri = -1;
    h.t = tmax;
    auto consider = [&](int ti) {
        if (ti == skip) return;
        double t, u, v;
        if (isect_tri(S.tris[ti], o, d, tmin, t, u, v) && t < tmax) {
            if (t < h.t || (t == h.t && ti < h.tri)) { h.t = t; h.u = u; h.v = v; h.tri = ti; }
        }
    };
    if (!use_bvh) {
        for (int i = 0; i < (int)S.tris.size(); ++i) {
            consider(i);
            if (any && h.tri >= 0) return true;
        }
        return h.tri >= 0;
    }
    std::vector<int> stack;
    stack.reserve(128);
    stack.push_back(0);
    while (!stack.empty()) {
        int ni = stack.back();
        stack.pop_back();
        const Node& n = S.nodes[ni];
        double tn;
        if (!box_hit(n, o, d, h.t, tn)) continue;
        if (n.left < 0) {
            for (int i = n.first; i < n.first + n.count; ++i) consider(S.order[i]);
            if (any && h.tri >= 0) return true;
        } else {
            stack.push_back(n.left);
            stack.push_back(n.right);
        }
    }
    return h.tri >= 0;
}

// ------------------------------------------------------------------------------------------
// One backward path (Algorithm 1 specialised to the interactive assumption of Sec.
// "Interactive Rendering": rays are traced as rays, the generalized-ray parameters are
// carried along; measurement by next-event estimation at every interaction).
// ------------------------------------------------------------------------------------------
// measured[kind]: vertices that evaluated a measurement (an emitter direction on the lit side
// of both normals), by the material kind of the hit (0 smooth, 1 rough, 2 grating)
struct Stats {
    uint64_t segments = 0, shadow = 0, evanescent = 0, backfacing = 0, composite = 0;
    uint64_t measured[3] = {0, 0, 0};
};

struct Ctx {
    const SceneO* S;
    const or_sensor* sen;
    const or_source* src;
    int nsrc;
    const double* lambdas;
    int nl;
    const or_opts* op;
};

// Build the tangent frame of the interaction: x axis = grating direction (gratings) or the
// projection of the travel direction (otherwise).
void make_frame(const Mat& m, V3 n, V3 d, V3& xa, V3& ya) {
    V3 t;
    if (m.kind == 2) {
        t = m.gdir - dot(m.gdir, n) * n;
        if (norm(t) > 1e-9) { xa = unit(t); ya = cross(n, xa); return; }
    }
    t = d - dot(d, n) * n;
    if (norm(t) > 1e-12) {
        xa = unit(t);
    } else {
        V3 a = std::fabs(n.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
        xa = unit(cross(n, a));
    }
    ya = cross(n, xa);
}

// Geometry of an interaction: hit point, geometric and shading normals (both facing the
// incoming ray), cosine of incidence, tangent frame and the travel direction in that frame.
struct Vertex {
    V3 P, ng, ns, xa, ya;
    double ci, dx, dy;
    const Mat* m;
};

// Incidence cosines at or below this end the path as back-facing: the footprint is stretched
// along the plane of incidence by 1 / cos, and beyond a millionfold it no longer is small
// against the geometry, which the ray-traced propagation of Sec. "Interactive Rendering"
// assumes.
constexpr double kGrazingCos = 1e-6;

// Returns false when the shading normal faces away from the incoming ray (or grazes it).
bool make_vertex(const SceneO& S, V3 o, V3 d, const Hit& h, Vertex& v) {
    v.P = o + h.t * d;
    const Tri& T = S.tris[h.tri];
    V3 ng = unit(cross(T.p1 - T.p0, T.p2 - T.p0));
    V3 ns = ng;
    {
        V3 n0 = S.vn[3 * h.tri], n1 = S.vn[3 * h.tri + 1], n2 = S.vn[3 * h.tri + 2];
        if (dot(n0, n0) > 0.0 && dot(n1, n1) > 0.0 && dot(n2, n2) > 0.0)
            ns = unit((1.0 - h.u - h.v) * n0 + h.u * n1 + h.v * n2);
    }
    if (dot(d, ng) > 0.0) ng = -1.0 * ng;
    if (dot(ns, ng) < 0.0) ns = -1.0 * ns;
    v.ng = ng;
    v.ns = ns;
    v.ci = -dot(d, ns);
    if (v.ci <= kGrazingCos) return false;
    v.m = &S.mats[S.mat[h.tri]];
    make_frame(*v.m, ns, d, v.xa, v.ya);
    v.dx = dot(d, v.xa);
    v.dy = dot(d, v.ya);
    return true;
}

// Footprint of the generalized ray on the surface: intensity variance beta^2/2 across the
// beam, stretched by 1/cos along the plane of incidence.
void footprint(const Vertex& v, double beta2, double& sxx, double& syy, double& sxy) {
    double sr2 = 0.5 * beta2;
    sxx = sr2 * (1.0 + v.dx * v.dx / (v.ci * v.ci));
    syy = sr2 * (1.0 + v.dy * v.dy / (v.ci * v.ci));
    sxy = sr2 * (v.dx * v.dy / (v.ci * v.ci));
}

// Material-boundary edges of a triangle mesh given by vertex indices tris [nt][3]: every edge
// (unordered vertex-index pair) used by exactly two triangles whose materials differ.
void find_boundaries(SceneO& S, const int32_t* tris, int64_t nt) {
    std::vector<std::pair<uint64_t, int>> keys;   // (edge key, 3 * triangle + local edge)
    keys.reserve(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int e = 0; e < 3; ++e) {
            uint64_t a = (uint32_t)tris[3 * t + e], b = (uint32_t)tris[3 * t + (e + 1) % 3];
            if (a > b) std::swap(a, b);
            keys.push_back({(a << 32) | b, (int)(3 * t + e)});
        }
    std::sort(keys.begin(), keys.end());
    S.bedges.clear();
    S.mat_bedges.assign(S.mats.size(), {});
    for (size_t i = 0; i < keys.size();) {
        size_t j = i;
        while (j < keys.size() && keys[j].first == keys[i].first) ++j;
        if (j - i == 2) {
            const int t0 = keys[i].second / 3, t1 = keys[i + 1].second / 3;
            const int e0 = keys[i].second % 3;
            if (S.mat[t0] != S.mat[t1]) {
                const Tri& T0 = S.tris[t0];
                const Tri& T1 = S.tris[t1];
                const V3 p[3] = {T0.p0, T0.p1, T0.p2};
                SceneO::BEdge E;
                E.p0 = p[e0];
                E.p1 = p[(e0 + 1) % 3];
                E.mat[0] = S.mat[t0];
                E.mat[1] = S.mat[t1];
                E.opp[0] = p[(e0 + 2) % 3];
                // the vertex of T1 that is on neither end of the edge
                const V3 q[3] = {T1.p0, T1.p1, T1.p2};
                const int e1 = keys[i + 1].second % 3;
                E.opp[1] = q[(e1 + 2) % 3];
                const int id = (int)S.bedges.size();
                S.bedges.push_back(E);
                S.mat_bedges[E.mat[0]].push_back(id);
                S.mat_bedges[E.mat[1]].push_back(id);
            }
        }
        i = j;
    }
    S.have_bedges = true;
}

// Distance from P to the segment [a, b].  Where the nearest point is an end, the distance is
// taken to that end itself, so that edges meeting at a vertex give equal distances there (the
// ties of the nearest-boundary rule then go to the lower edge id).
double point_segment_distance(V3 P, V3 a, V3 b) {
    const V3 ab = b - a;
    const double l2 = dot(ab, ab);
    const double t = l2 > 0.0 ? dot(P - a, ab) / l2 : 0.0;
    if (!(t > 0.0)) return norm(P - a);
    if (t >= 1.0) return norm(P - b);
    return norm(P - (a + t * ab));
}

// Nearest boundary edge of material mat within distance reach (metres) of P, -1 if none;
// equal distances go to the lower edge index.
uint64_t bcell_key(const SceneO& S, V3 P) {
    const int64_t x = (int64_t)std::floor((P.x - S.borg.x) / S.bcell);
    const int64_t y = (int64_t)std::floor((P.y - S.borg.y) / S.bcell);
    const int64_t z = (int64_t)std::floor((P.z - S.borg.z) / S.bcell);
    return ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) | (uint64_t)(z & 0x1FFFFF);
}

void build_bgrid(SceneO& S, double cell) {
    S.bgrid.clear();
    S.bcell = cell;
    S.borg = V3{1e300, 1e300, 1e300};
    for (const auto& E : S.bedges) {
        S.borg.x = std::min({S.borg.x, E.p0.x, E.p1.x});
        S.borg.y = std::min({S.borg.y, E.p0.y, E.p1.y});
        S.borg.z = std::min({S.borg.z, E.p0.z, E.p1.z});
    }
    S.borg = S.borg - V3{4 * cell, 4 * cell, 4 * cell};
    for (int id = 0; id < (int)S.bedges.size(); ++id) {
        const auto& E = S.bedges[id];
        const int64_t lo[3] = {(int64_t)std::floor((std::min(E.p0.x, E.p1.x) - cell - S.borg.x) / cell),
                               (int64_t)std::floor((std::min(E.p0.y, E.p1.y) - cell - S.borg.y) / cell),
                               (int64_t)std::floor((std::min(E.p0.z, E.p1.z) - cell - S.borg.z) / cell)};
        const int64_t hi[3] = {(int64_t)std::floor((std::max(E.p0.x, E.p1.x) + cell - S.borg.x) / cell),
                               (int64_t)std::floor((std::max(E.p0.y, E.p1.y) + cell - S.borg.y) / cell),
                               (int64_t)std::floor((std::max(E.p0.z, E.p1.z) + cell - S.borg.z) / cell)};
        for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
                for (int64_t z = lo[2]; z <= hi[2]; ++z) {
                    const uint64_t key = ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) |
                                         (uint64_t)(z & 0x1FFFFF);
                    S.bgrid[key].push_back(id);
                }
    }
}

int nearest_boundary(const SceneO& S, int mat, V3 P, double reach, double& dist) {
    int best = -1;
    dist = reach;
    if (S.bcell > 0.0 && reach <= S.bcell) {
        // every edge within reach of P is listed in P's cell (in id order)
        auto it = S.bgrid.find(bcell_key(S, P));
        if (it == S.bgrid.end()) return -1;
        for (int id : it->second) {
            const auto& E = S.bedges[id];
            if (E.mat[0] != mat && E.mat[1] != mat) continue;
            const double d = point_segment_distance(P, E.p0, E.p1);
            if (d < dist) { best = id; dist = d; }
        }
        return best;
    }
    for (int id : S.mat_bedges[mat]) {
        const double d = point_segment_distance(P, S.bedges[id].p0, S.bedges[id].p1);
        if (d < dist || (d == dist && best >= 0 && id < best)) {
            if (d < reach) { best = id; dist = d; }
        }
    }
    return best;
}

// Composite interaction at vertex v of triangle tri (material mat) with footprint S (um^2):
// the nearest boundary edge of mat within min(2.5 beta_max, reach_m) of the hit, with
// beta_max = sqrt(2) times the footprint's largest standard deviation (the ball that holds the
// generalized ray, Sec. "Wave-Optical Rendering"), carried onto the tangent plane of the frame:
// its unit normal (nx, ny) towards the far side (the side of the far triangle's third vertex),
// its distance c >= 0, the far side (material and grating direction in the frame) and the far
// side's share of the window's intensity mass.  False when there is none.
bool composite_at(const SceneO& S, const Vertex& v, int mat, double sxx, double syy, double sxy, double reach_m,
                  Side& far, double& nx, double& ny, double& c, double& mass_far) {
    if (!S.have_bedges || S.mat_bedges[mat].empty()) return false;
    const double lmax = 0.5 * (sxx + syy) + std::sqrt(0.25 * (sxx - syy) * (sxx - syy) + sxy * sxy);
    const double rad = std::min(2.5 * std::sqrt(2.0 * lmax) * 1e-6, reach_m);
    double dist;
    const int id = nearest_boundary(S, mat, v.P, rad, dist);
    if (id < 0) return false;
    const SceneO::BEdge& E = S.bedges[id];
    const int fs = E.mat[0] == mat ? 1 : 0;       // the far side: the other material
    const V3 a3 = E.p0 - v.P, b3 = E.p1 - v.P, q3 = E.opp[fs] - v.P;
    const double ax = dot(a3, v.xa) * 1e6, ay = dot(a3, v.ya) * 1e6;   // um
    const double bx = dot(b3, v.xa) * 1e6, by = dot(b3, v.ya) * 1e6;
    const double qx = dot(q3, v.xa) * 1e6, qy = dot(q3, v.ya) * 1e6;
    const double ex = bx - ax, ey = by - ay, el = std::sqrt(ex * ex + ey * ey);
    if (!(el > 1e-6 * norm(E.p1 - E.p0) * 1e6)) return false;   // edge seen end-on
    nx = -ey / el;
    ny = ex / el;
    if (nx * (qx - ax) + ny * (qy - ay) < 0.0) { nx = -nx; ny = -ny; }
    c = std::max(0.0, nx * ax + ny * ay);
    const Mat& fm = S.mats[E.mat[fs]];
    far.m = &fm;
    far.gx = 1.0;
    far.gy = 0.0;
    if (fm.kind == 2) {
        const double gx = dot(fm.gdir, v.xa), gy = dot(fm.gdir, v.ya), gl = std::sqrt(gx * gx + gy * gy);
        if (gl > 1e-9) { far.gx = gx / gl; far.gy = gy / gl; }
    }
    const double snn = nx * nx * sxx + 2.0 * nx * ny * sxy + ny * ny * syy;
    mass_far = 0.5 * std::erfc(c / std::sqrt(2.0 * snn));
    return true;
}

// Emitter sampling for next-event estimation from P at wavenumber k.  A plane wave arrives
// along its direction; a Gaussian-Schell emitter's arrival wavevector is drawn from its
// ensemble-averaged angular spectrum, a Gaussian of standard deviation 1/r_c per transverse
// axis, and must reach the emitter's rectangle.  om: travel direction of the arriving light;
// tmax: distance to the emitter; tt: squared transverse part of om (Gaussian-Schell).
bool nee_direction(const or_source& L, V3 P, double k, double u1, double u2, V3& om, double& tmax,
                   double& tt) {
    tmax = 1e300;
    tt = 0.0;
    if (L.kind == 0) {
        om = unit(ld3(L.dir));
        return true;
    }
    double z1, z2;
    box_muller(u1, u2, z1, z2);
    double du = z1 / L.rc_um, dv = z2 / L.rc_um;      // um^-1
    tt = (du * du + dv * dv) / (k * k);
    if (tt >= 1.0) return false;
    V3 ax = unit(ld3(L.dir));
    V3 eu = ld3(L.eu), ev = ld3(L.ev);
    double lu = norm(eu), lv = norm(ev);
    V3 bu = (1.0 / lu) * eu, bv = (1.0 / lv) * ev;
    om = (du / k) * bu + (dv / k) * bv + std::sqrt(1.0 - tt) * ax;
    double den = dot(om, ax);
    double te = dot(ld3(L.pos) - P, ax) / (-den);
    if (!(te > t_eps(P))) return false;
    V3 Q = P - te * om;
    double a = dot(Q - ld3(L.pos), bu) / lu, b = dot(Q - ld3(L.pos), bv) / lv;
    if (!(std::fabs(a) <= 1.0 && std::fabs(b) <= 1.0)) return false;
    tmax = te;
    return true;
}

// Free-space propagation of the generalized ray over z um (eq. K_free_space_propagation),
// with zbar = z / |k0| and the pre-update beta, rho.
void propagate(double z, double k, double& beta2, double& rho) {
    double zb = z / k;
    double rho_new = rho + zb * (1.0 + rho * rho) / beta2;
    double beta2_new = beta2 + zb * (2.0 * rho + zb * (1.0 + rho * rho) / beta2);
    rho = rho_new;
    beta2 = beta2_new;
}

// ------------------------------------------------------------------------------------------
// Anisotropic generalized rays (Sec. "Generalized rays" allows beta, rho to be positive-
// definite matrices; the formulas are in the paper's supplement, which is not available).
// Reading: the ray's phase-space Gaussian over the two axes transverse to its mean direction,
// kept as its 4x4 second-moment matrix [[Srr, Srk], [Srk^T, Skk]] in a transverse frame of
// the mean direction.  The scalar ray is Srr = beta^2 I, Srk = rho I, Skk = (1 + rho^2) /
// beta^2 I: its free-space law (eq. K_free_space_propagation) is the shear r -> r + zbar k of
// these moments, and the matrix form below is the same shear.  At an interaction the
// transverse plane of the incoming mean direction is carried onto the surface along that
// direction and the surface onto the transverse plane of the outgoing direction; positions
// map by that 2x2 G and wavevectors by G^-T (tangential wavevector deviations are conserved),
// a symplectic map, so a pure state stays pure.  A mirror reflection leaves an isotropic ray
// isotropic; a grating order or rough-surface lobe leaving at another angle stretches the ray
// along the plane of scattering by cos(o) / cos(i), the anamorphic beam magnification.
// ------------------------------------------------------------------------------------------
struct Aniso {
    double rr[2][2], rk[2][2], kk[2][2];
};

// Orthonormal basis (e1, e2) of the plane normal to the unit vector d (Duff et al., "Building
// an Orthonormal Basis, Revisited", JCGT 6(1), 2017).
void transverse_frame(V3 d, V3& e1, V3& e2) {
    double sg = d.z >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + d.z), b = d.x * d.y * a;
    e1 = V3{1.0 + sg * d.x * d.x * a, sg * b, -sg * d.x};
    e2 = V3{b, sg + d.y * d.y * a, -d.y};
}

Aniso aniso_isotropic(double beta2) {
    Aniso A{};
    for (int i = 0; i < 2; ++i) {
        A.rr[i][i] = beta2;
        A.kk[i][i] = 1.0 / beta2;
    }
    return A;
}

// Free space over z um: zbar = z / k, Srr += zbar (Srk + Srk^T) + zbar^2 Skk, Srk += zbar Skk.
void propagate_aniso(double z, double k, Aniso& A) {
    double zb = z / k;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) A.rr[i][j] += zb * (A.rk[i][j] + A.rk[j][i]) + zb * zb * A.kk[i][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) A.rk[i][j] += zb * A.kk[i][j];
}

// The surface point reached from transverse offset v along di: v - di (n . v) / (n . di).
V3 onto_surface(V3 v, V3 di, V3 n) { return v - (dot(n, v) / dot(n, di)) * di; }

// Interaction: incoming mean direction di, outgoing do_, surface normal n.
void interact_aniso(V3 di, V3 do_, V3 n, Aniso& A) {
    V3 ei[2], eo[2];
    transverse_frame(di, ei[0], ei[1]);
    transverse_frame(do_, eo[0], eo[1]);
    double G[2][2], Gi[2][2];
    for (int b = 0; b < 2; ++b) {
        V3 sp = onto_surface(ei[b], di, n);
        for (int a = 0; a < 2; ++a) G[a][b] = dot(eo[a], sp);
    }
    double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];   // +-cos(o) / cos(i)
    if (!(std::fabs(det) > 1e-6)) return;   // a continuation along the surface: the map is singular
    Gi[0][0] = G[1][1] / det;
    Gi[0][1] = -G[0][1] / det;
    Gi[1][0] = -G[1][0] / det;
    Gi[1][1] = G[0][0] / det;
    Aniso B{};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    B.rr[i][j] += G[i][a] * A.rr[a][b] * G[j][b];    // G Srr G^T
                    B.rk[i][j] += G[i][a] * A.rk[a][b] * Gi[b][j];   // G Srk G^-1
                    B.kk[i][j] += Gi[a][i] * A.kk[a][b] * Gi[b][j];  // G^-T Skk G^-1
                }
    A = B;
}

// Footprint covariance on the surface frame (xa, ya) of a ray arriving along d: the spatial
// variance Srr / 2 carried onto the surface along d (the scalar footprint() for Srr = beta^2 I).
void footprint_aniso(V3 d, V3 n, V3 xa, V3 ya, const Aniso& A, double& sxx, double& syy, double& sxy) {
    V3 e[2];
    transverse_frame(d, e[0], e[1]);
    double H[2][2];
    for (int b = 0; b < 2; ++b) {
        V3 sp = onto_surface(e[b], d, n);
        H[0][b] = dot(xa, sp);
        H[1][b] = dot(ya, sp);
    }
    double S[2][2] = {{0, 0}, {0, 0}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) S[i][j] += 0.5 * H[i][a] * A.rr[a][b] * H[j][b];
    sxx = S[0][0];
    syy = S[1][1];
    sxy = 0.5 * (S[0][1] + S[1][0]);
}

// vtx (optional, tests): per interaction, 12 values: depth, triangle, hit point (3), composite
// (1 or 0), boundary distance c (um), its normal (2), far-side mass, the measurement added,
// and the side the continuation took (0 near, 1 far, -1 none).
double trace_path(const Ctx& C, int px, int py, int64_t s, int w, Stats& st, std::vector<double>* vtx = nullptr) {
    const SceneO& S = *C.S;
    const or_sensor& sen = *C.sen;
    const or_opts& op = *C.op;
    const uint64_t W = (uint64_t)sen.width, H = (uint64_t)sen.height;
    const uint64_t pid = ((((uint64_t)s * H) + (uint64_t)py) * W + (uint64_t)px) * (uint64_t)C.nl +
                         (uint64_t)w;
    const double lam = C.lambdas[w];
    const double k = 2.0 * kPi / lam;                     // um^-1

    // Sourcing (Sec. "Interactive Rendering", implementation details): mean position uniform
    // on the pixel, mean direction the sensor axis, beta^2 / 2 = sigma^2, rho = 0, alpha = 1.
    U4 r0 = draw(pid, 0, STREAM_SOURCE, op.seed);
    V3 o = ld3(sen.origin) + ((px + unif(r0.v[0])) * sen.pitch_m) * ld3(sen.axis_u) +
           ((py + unif(r0.v[1])) * sen.pitch_m) * ld3(sen.axis_v);
    V3 d = ld3(sen.dir);
    double sig_um = sen.sigma_m * 1e6;
    double beta2 = 2.0 * sig_um * sig_um;
    double rho = 0.0;
    Aniso A = aniso_isotropic(beta2);   // the matrix form, when op.aniso
    double alpha = 1.0;
    double contrib = 0.0;
    int prev = -1;   // triangle the current segment leaves

    for (int depth = 0; depth < op.max_depth; ++depth) {
        st.segments++;
        Hit h;
        if (!trace_ray(S, o, d, t_eps(o), 1e300, op.use_bvh != 0, false, h, prev)) break;
        prev = h.tri;
        if (op.aniso) propagate_aniso(h.t * 1e6, k, A);
        else propagate(h.t * 1e6, k, beta2, rho);
        Vertex v;
        if (!make_vertex(S, o, d, h, v)) { st.backfacing++; break; }
        const Mat& m = *v.m;
        double sxx, syy, sxy;
        if (op.aniso) footprint_aniso(d, v.ns, v.xa, v.ya, A, sxx, syy, sxy);
        else footprint(v, beta2, sxx, syy, sxy);
        // The frame's x axis is the grating direction, so the grating vector is (1, 0).
        const double gx = 1.0, gy = 0.0;
        // Composite interaction when a material boundary lies within the footprint.
        Side near_side{&m, gx, gy}, far_side{&m, gx, gy};
        double bnx = 0.0, bny = 0.0, bc = 0.0, mass_far = 0.0;
        const bool comp = op.composite &&
                          composite_at(S, v, S.mat[h.tri], sxx, syy, sxy, op.reach_m, far_side, bnx, bny, bc, mass_far);
        if (comp) st.composite++;
        size_t vrow = 0;
        if (vtx) {
            vrow = vtx->size();
            const double row[12] = {(double)depth, (double)h.tri, v.P.x, v.P.y, v.P.z, comp ? 1.0 : 0.0, bc, bnx, bny,
                                    mass_far, 0.0, -1.0};
            vtx->insert(vtx->end(), row, row + 12);
        }

        // Measurement by next-event estimation (measurement operator, eq.
        // measurement_operator, with the ensemble-averaged source WDF).
        U4 rn = draw(pid, depth, STREAM_NEE, op.seed);
        if (C.nsrc > 0) {
            int si = std::min((int)(unif(rn.v[0]) * C.nsrc), C.nsrc - 1);
            const or_source& L = C.src[si];
            V3 om{0, 0, 0};
            double tmax, tt;
            bool ok = nee_direction(L, v.P, k, unif(rn.v[1]), unif(rn.v[2]), om, tmax, tt);
            if (ok && dot(om, v.ng) < 0.0 && dot(om, v.ns) < 0.0) {
                st.shadow++;
                st.measured[m.kind]++;
                Hit hs;
                bool occ = trace_ray(S, v.P, -1.0 * om, t_eps(v.P), tmax, op.use_bvh != 0, true, hs, h.tri);
                if (!occ) {
                    double kix = k * dot(om, v.xa), kiy = k * dot(om, v.ya);
                    double kox = -k * v.dx, koy = -k * v.dy;
                    double p = comp ? pw_composite(near_side, far_side, k, kix, kiy, kox, koy, sxx, syy, sxy, bnx, bny, bc)
                                    : pw_eval(m, k, kix, kiy, kox, koy, sxx, syy, sxy, gx, gy);
                    contrib += alpha * L.power * p * (double)C.nsrc;
                    if (vtx) (*vtx)[vrow + 10] = alpha * L.power * p * (double)C.nsrc;
                }
            }
        }
        if (depth + 1 >= op.max_depth) break;

        // Light-matter interaction: sample the continuation generalized ray.  At a composite
        // interaction the continuation samples the far side's unwindowed kernel with the
        // probability of the window's intensity mass there (word 3 of the NEE draw), else the
        // near side's: a one-sample estimate of the mass-weighted mixture of the two kernels.
        U4 rs = draw(pid, depth, STREAM_SCATTER, op.seed);
        const Side& cs = (comp && !(unif(rn.v[3]) < 1.0 - mass_far)) ? far_side : near_side;
        if (vtx) (*vtx)[vrow + 11] = (&cs == &far_side) ? 1.0 : 0.0;
        double kix = k * v.dx, kiy = k * v.dy, kox, koy, wgt;
        int ev;
        if (!sample_finf(*cs.m, k, kix, kiy, v.ci, unif(rs.v[0]), unif(rs.v[1]), unif(rs.v[2]), cs.gx, cs.gy,
                         kox, koy, wgt, ev)) {
            st.evanescent += ev;
            break;
        }
        alpha *= wgt;
        if (op.rr_enable && depth + 1 >= 2) {
            if (!((rs.v[3] >> 8) < op.rr_threshold24)) break;
            alpha /= op.rr_p;
        }
        double kn = std::sqrt(std::max(0.0, 1.0 - (kox * kox + koy * koy) / (k * k)));
        V3 din = d;
        d = (kox / k) * v.xa + (koy / k) * v.ya + kn * v.ns;
        d = unit(d);
        if (op.aniso) interact_aniso(din, d, v.ns, A);
        o = v.P;
    }
    return contrib;
}

// One hero-wavelength path: the path of trace_path, sampled at the hero wavelength, carrying
// the four wavelengths of rotation group grp of the grid (indices grp + i G, G = nl / 4; the
// hero is member r0.w >> 30 of the group).  Path id ((s H + y) W + x) G + grp.  Each member
// keeps its own beta, rho (the free-space law depends on |k|) and its own footprint; they share
// the geometric path.  Per member i: T_i = f_i / p_h and R_i = p_i / p_h along the path; next-
// event estimation at a vertex adds 4 T_i q_i M_i / sum_k R_k q_k, with M_i the member's
// measurement and q_i the ratio of its emitter-sampling density to the hero's.
// out[i]: contribution to wavelength grp + i G.
void trace_path_hero(const Ctx& C, int px, int py, int64_t s, int grp, Stats& st, double out[4]) {
    const SceneO& S = *C.S;
    const or_sensor& sen = *C.sen;
    const or_opts& op = *C.op;
    const uint64_t W = (uint64_t)sen.width, H = (uint64_t)sen.height;
    const int G = C.nl / 4;
    const uint64_t pid = ((((uint64_t)s * H) + (uint64_t)py) * W + (uint64_t)px) * (uint64_t)G +
                         (uint64_t)grp;
    double k[4];
    for (int i = 0; i < 4; ++i) k[i] = 2.0 * kPi / C.lambdas[grp + i * G];

    U4 r0 = draw(pid, 0, STREAM_SOURCE, op.seed);
    const int hi = (int)(r0.v[3] >> 30);
    const double kh = k[hi];
    V3 o = ld3(sen.origin) + ((px + unif(r0.v[0])) * sen.pitch_m) * ld3(sen.axis_u) +
           ((py + unif(r0.v[1])) * sen.pitch_m) * ld3(sen.axis_v);
    V3 d = ld3(sen.dir);
    double sig_um = sen.sigma_m * 1e6;
    double beta2[4], rho[4], T[4], R[4];
    for (int i = 0; i < 4; ++i) {
        beta2[i] = 2.0 * sig_um * sig_um;
        rho[i] = 0.0;
        T[i] = 1.0;
        R[i] = 1.0;
        out[i] = 0.0;
    }
    int prev = -1;

    for (int depth = 0; depth < op.max_depth; ++depth) {
        st.segments++;
        Hit h;
        if (!trace_ray(S, o, d, t_eps(o), 1e300, op.use_bvh != 0, false, h, prev)) break;
        prev = h.tri;
        for (int i = 0; i < 4; ++i) propagate(h.t * 1e6, k[i], beta2[i], rho[i]);
        Vertex v;
        if (!make_vertex(S, o, d, h, v)) { st.backfacing++; break; }
        const Mat& m = *v.m;
        const double gx = 1.0, gy = 0.0;
        // Composite interaction (reading R31): the boundary is found with the hero's footprint;
        // each member's window is the hero's scaled by its beta^2 (same frame and stretch), so
        // its far mass is erfc(c / sqrt(2 n^T S_i n)) / 2.
        Side near_side{&m, gx, gy}, far_side{&m, gx, gy};
        double bnx = 0.0, bny = 0.0, bc = 0.0, mass[4] = {0.0, 0.0, 0.0, 0.0};
        bool comp = false;
        if (op.composite) {
            double sxx, syy, sxy, mf;
            footprint(v, beta2[hi], sxx, syy, sxy);
            comp = composite_at(S, v, S.mat[h.tri], sxx, syy, sxy, op.reach_m, far_side, bnx, bny, bc, mf);
            if (comp) {
                st.composite++;
                for (int i = 0; i < 4; ++i) {
                    double ixx, iyy, ixy;
                    footprint(v, beta2[i], ixx, iyy, ixy);
                    const double snn = bnx * bnx * ixx + 2.0 * bnx * bny * ixy + bny * bny * iyy;
                    mass[i] = 0.5 * std::erfc(bc / std::sqrt(2.0 * snn));
                }
            }
        }

        U4 rn = draw(pid, depth, STREAM_NEE, op.seed);
        if (C.nsrc > 0) {
            int si = std::min((int)(unif(rn.v[0]) * C.nsrc), C.nsrc - 1);
            const or_source& L = C.src[si];
            V3 om{0, 0, 0};
            double tmax, tt;
            bool ok = nee_direction(L, v.P, kh, unif(rn.v[1]), unif(rn.v[2]), om, tmax, tt);
            if (ok && dot(om, v.ng) < 0.0 && dot(om, v.ns) < 0.0) {
                st.shadow++;
                st.measured[m.kind]++;
                Hit hs;
                bool occ = trace_ray(S, v.P, -1.0 * om, t_eps(v.P), tmax, op.use_bvh != 0, true, hs, h.tri);
                if (!occ) {
                    // emitter-sampling density of the arrival direction at each member,
                    // relative to the hero's: the angular spectrum N(k u_t; 0, rc^-2 I) k^2
                    double q[4], den = 0.0;
                    for (int i = 0; i < 4; ++i) {
                        q[i] = L.kind == 0 ? 1.0
                                           : (k[i] * k[i]) / (kh * kh) *
                                                 std::exp(-0.5 * (k[i] * k[i] - kh * kh) * tt * L.rc_um * L.rc_um);
                        den += R[i] * q[i];
                    }
                    for (int i = 0; i < 4; ++i) {
                        if (T[i] == 0.0) continue;
                        double sxx, syy, sxy;
                        footprint(v, beta2[i], sxx, syy, sxy);
                        const double kix = k[i] * dot(om, v.xa), kiy = k[i] * dot(om, v.ya);
                        const double kox = -k[i] * v.dx, koy = -k[i] * v.dy;
                        double p = comp ? pw_composite(near_side, far_side, k[i], kix, kiy, kox, koy, sxx, syy, sxy,
                                                       bnx, bny, bc)
                                        : pw_eval(m, k[i], kix, kiy, kox, koy, sxx, syy, sxy, gx, gy);
                        out[i] += 4.0 * T[i] * q[i] * L.power * p * (double)C.nsrc / den;
                    }
                }
            }
        }
        if (depth + 1 >= op.max_depth) break;

        U4 rs = draw(pid, depth, STREAM_SCATTER, op.seed);
        // at a composite interaction the hero's side as in trace_path (word 3 of the NEE draw,
        // the hero's far mass)
        const bool far_chosen = comp && !(unif(rn.v[3]) < 1.0 - mass[hi]);
        const Side& cs = far_chosen ? far_side : near_side;
        double kix = kh * v.dx, kiy = kh * v.dy, kox, koy, wgt;
        int ev, cj;
        if (!sample_finf(*cs.m, kh, kix, kiy, v.ci, unif(rs.v[0]), unif(rs.v[1]), unif(rs.v[2]), cs.gx, cs.gy,
                         kox, koy, wgt, ev, &cj)) {
            st.evanescent += ev;
            break;
        }
        if (comp) {
            double f_ph[4], p_ph[4];
            composite_companions(near_side, far_side, far_chosen, mass, k, hi, v.dx, v.dy, v.ci, (kox - kix) / kh,
                                 (koy - kiy) / kh, cj, f_ph, p_ph);
            for (int i = 0; i < 4; ++i) {
                T[i] *= f_ph[i];
                R[i] *= p_ph[i];
            }
        } else {
            for (int i = 0; i < 4; ++i) {
                if (i == hi) {
                    T[i] *= wgt;
                    continue;
                }
                double f_ph, p_ph;
                finf_companion(m, kh, k[i], v.dx, v.dy, v.ci, (kox - kix) / kh, (koy - kiy) / kh, cj, gx, gy,
                               f_ph, p_ph);
                T[i] *= f_ph;
                R[i] *= p_ph;
            }
        }
        if (op.rr_enable && depth + 1 >= 2) {
            if (!((rs.v[3] >> 8) < op.rr_threshold24)) break;
            for (int i = 0; i < 4; ++i) T[i] /= op.rr_p;
        }
        double kn = std::sqrt(std::max(0.0, 1.0 - (kox * kox + koy * koy) / (kh * kh)));
        d = (kox / kh) * v.xa + (koy / kh) * v.ya + kn * v.ns;
        d = unit(d);
        o = v.P;
    }
}

}  // namespace

// ==========================================================================================
// Exported entry points (ctypes).
// ==========================================================================================
extern "C" {

void or_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    U4 r = philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    std::memcpy(out, r.v, 16);
}

void or_philox_batch(const uint32_t* ctr, int64_t n, const uint32_t* key, uint32_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        U4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[0], key[1]);
        std::memcpy(out + 4 * i, r.v, 16);
    }
}

double or_besselj(int n, double x) { return besselj(n, x); }

// Free-space propagation of the generalized-ray parameters (eq. K_free_space_propagation):
// beta^2 -> beta^2 + zbar (2 rho + zbar (1 + rho^2) / beta^2), rho -> rho + zbar (1 + rho^2) /
// beta^2 with zbar = z / |k0|; z in um, k in um^-1, beta^2 in um^2.  out = (beta^2, rho).
void or_propagate(double beta2, double rho, double z_um, double k, double* out) {
    double zb = z_um / k;
    out[1] = rho + zb * (1.0 + rho * rho) / beta2;
    out[0] = beta2 + zb * (2.0 * rho + zb * (1.0 + rho * rho) / beta2);
}

// p_w for one query; material given by its fields.
double or_pw(int kind, double h, double L, double refl, double k, double kix, double kiy,
             double kox, double koy, double sxx, double syy, double sxy, double gx, double gy) {
    Mat m{kind, h, L, refl, {1, 0, 0}};
    return pw_eval(m, k, kix, kiy, kox, koy, sxx, syy, sxy, gx, gy);
}

void or_pw_batch(const double* q, int64_t n, double* out) {
    // q rows: kind, h, L, refl, k, kix, kiy, kox, koy, sxx, syy, sxy, gx, gy
    for (int64_t i = 0; i < n; ++i) {
        const double* r = q + 14 * i;
        Mat m{(int)r[0], r[1], r[2], r[3], {1, 0, 0}};
        out[i] = pw_eval(m, r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11], r[12], r[13]);
    }
}

// Continuation sample; returns 1 when a direction was produced.
int or_sample(int kind, double h, double L, double refl, double k, double kix, double kiy,
              double ci, double u0, double u1, double u2, double gx, double gy, double* out3) {
    Mat m{kind, h, L, refl, {1, 0, 0}};
    double kox = 0, koy = 0, w = 0;
    int ev = 0;
    bool ok = sample_finf(m, k, kix, kiy, ci, u0, u1, u2, gx, gy, kox, koy, w, ev);
    out3[0] = kox; out3[1] = koy; out3[2] = w;
    return ok ? 1 : 0;
}

// Hero-wavelength continuation step for a batch of uniforms u[n][3]: sample at kh from the
// incident tangential direction (ux, uy), then the companion ratios at kc.  out[n][5] =
// (kox, koy, hero weight, f_c / p_h, p_c / p_h), all NaN when the sample ends the path.
void or_hero_step_batch(int kind, double h, double L, double refl, double kh, double kc, double ux,
                        double uy, double ci, double gx, double gy, const double* u, int64_t n,
                        double* out) {
    Mat m{kind, h, L, refl, {1, 0, 0}};
    for (int64_t i = 0; i < n; ++i) {
        double* o = out + 5 * i;
        double kox, koy, w;
        int ev, comp;
        if (!sample_finf(m, kh, kh * ux, kh * uy, ci, u[3 * i], u[3 * i + 1], u[3 * i + 2], gx, gy, kox, koy, w,
                         ev, &comp)) {
            for (int j = 0; j < 5; ++j) o[j] = std::nan("");
            continue;
        }
        double f_ph, p_ph;
        finf_companion(m, kh, kc, ux, uy, ci, kox / kh - ux, koy / kh - uy, comp, gx, gy, f_ph, p_ph);
        o[0] = kox;
        o[1] = koy;
        o[2] = w;
        o[3] = f_ph;
        o[4] = p_ph;
    }
}

// One hero-wavelength continuation step at a composite interaction for uniforms u [n][4] (the
// sampler's three, then the side choice): sides near / far given by their fields (kind, h, L,
// refl, grating direction in the frame), far masses mass_h (hero) and mass_c (companion).
// out [n][6]: (kox, koy, f_h / p_h, f_c / p_h, p_c / p_h, class of the sampled direction: 0
// specular, 1 rough lobe, 2 dispersive grating order); NaN rows end the path.
void or_hero_composite_step_batch(const double* near_m, const double* far_m, double mass_h, double mass_c, double kh,
                                  double kc, double ux, double uy, double ci, const double* u, int64_t n,
                                  double* out) {
    const Mat mn{(int)near_m[0], near_m[1], near_m[2], near_m[3], {1, 0, 0}};
    const Mat mf{(int)far_m[0], far_m[1], far_m[2], far_m[3], {1, 0, 0}};
    const Side near{&mn, near_m[4], near_m[5]}, far{&mf, far_m[4], far_m[5]};
    const double k[4] = {kh, kc, kc, kc}, mass[4] = {mass_h, mass_c, mass_c, mass_c};
    for (int64_t i = 0; i < n; ++i) {
        const double* ui = u + 4 * i;
        double* o = out + 6 * i;
        const bool far_chosen = !(ui[3] < 1.0 - mass_h);
        const Side& cs = far_chosen ? far : near;
        double kox, koy, w;
        int ev, comp;
        if (!sample_finf(*cs.m, kh, kh * ux, kh * uy, ci, ui[0], ui[1], ui[2], cs.gx, cs.gy, kox, koy, w, ev,
                         &comp)) {
            for (int j = 0; j < 6; ++j) o[j] = std::nan("");
            continue;
        }
        double f_ph[4], p_ph[4];
        composite_companions(near, far, far_chosen, mass, k, 0, ux, uy, ci, kox / kh - ux, koy / kh - uy, comp, f_ph,
                             p_ph);
        o[0] = kox;
        o[1] = koy;
        o[2] = f_ph[0];
        o[3] = f_ph[1];
        o[4] = p_ph[1];
        o[5] = (cs.m->kind == 0 || comp == 0) ? 0.0 : (cs.m->kind == 1 ? 1.0 : 2.0);
    }
}

void* or_scene_create(const double* verts, int64_t nv, const double* normals,
                      const int32_t* tris, int64_t nt, const int32_t* tri_mat,
                      const or_material* mats, int32_t nm) {
    SceneO* S = new SceneO();
    S->tris.resize(nt);
    S->vn.assign(3 * nt, V3{0, 0, 0});
    S->mat.resize(nt);
    for (int64_t i = 0; i < nt; ++i) {
        int a = tris[3 * i], b = tris[3 * i + 1], c = tris[3 * i + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) { delete S; return nullptr; }
        S->tris[i] = Tri{ld3(verts + 3 * a), ld3(verts + 3 * b), ld3(verts + 3 * c)};
        if (normals) {
            S->vn[3 * i] = ld3(normals + 3 * a);
            S->vn[3 * i + 1] = ld3(normals + 3 * b);
            S->vn[3 * i + 2] = ld3(normals + 3 * c);
        }
        S->mat[i] = tri_mat[i];
        if (tri_mat[i] < 0 || tri_mat[i] >= nm) { delete S; return nullptr; }
    }
    for (int i = 0; i < nm; ++i) {
        const or_material& M = mats[i];
        V3 g = ld3(M.gdir);
        if (M.kind == 2) g = unit(g);
        S->mats.push_back(Mat{M.kind, M.height_um, M.length_um, M.reflectance, g});
    }
    S->order.resize(nt);
    for (int64_t i = 0; i < nt; ++i) S->order[i] = (int)i;
    if (nt > 0) build_rec(*S, 0, (int)nt);
    return S;
}

void or_scene_destroy(void* s) { delete (SceneO*)s; }

// Find the scene's material boundaries (needed by composite rendering) and grid them with
// cells of `cell` metres (the largest reach searched through the grid; farther searches scan
// the material's edges).  tris: the index array given to or_scene_create.  Returns the
// number of boundary edges.
int64_t or_scene_boundaries(void* s, const int32_t* tris, int64_t nt, double cell) {
    SceneO& S = *(SceneO*)s;
    if ((int64_t)S.tris.size() != nt || !(cell > 0.0)) return -1;
    if (!S.have_bedges) find_boundaries(S, tris, nt);
    if (S.bcell != cell) build_bgrid(S, cell);
    return (int64_t)S.bedges.size();
}

// Boundary edge i: out [14] = p0 (3), p1 (3), materials (2), third vertices (6).
void or_boundary_edge(void* s, int64_t i, double* out) {
    const SceneO::BEdge& E = ((SceneO*)s)->bedges[i];
    const V3 v[4] = {E.p0, E.p1, E.opp[0], E.opp[1]};
    for (int j = 0; j < 2; ++j) { out[3 * j] = v[j].x; out[3 * j + 1] = v[j].y; out[3 * j + 2] = v[j].z; }
    out[6] = E.mat[0];
    out[7] = E.mat[1];
    for (int j = 0; j < 2; ++j) { out[8 + 3 * j] = v[2 + j].x; out[9 + 3 * j] = v[2 + j].y; out[10 + 3 * j] = v[2 + j].z; }
}

// Nearest boundary edge of material mat within reach of points P [n][3]; out [n][2] = (edge
// index or -1, distance).
void or_nearest_boundary(void* s, int32_t mat, const double* P, int64_t n, double reach, double* out) {
    const SceneO& S = *(SceneO*)s;
    for (int64_t i = 0; i < n; ++i) {
        double d;
        const int id = nearest_boundary(S, mat, ld3(P + 3 * i), reach, d);
        out[2 * i] = id;
        out[2 * i + 1] = id >= 0 ? d : 0.0;
    }
}

// The interactions of one path (tests): pixel (px, py), sample s, wavelength w of a render
// with these options; out: up to max_rows rows of the 12 values trace_path records.  Returns
// the number of rows (the path's contribution in *value, already divided by spp_norm).
int32_t or_path_vertices(void* sc, const or_sensor* sen, const or_source* src, int32_t nsrc, const double* lambdas,
                         int32_t nl, const or_opts* op, int32_t px, int32_t py, int64_t s, int32_t w, double* out,
                         int32_t max_rows, double* value) {
    Ctx C{(const SceneO*)sc, sen, src, nsrc, lambdas, nl, op};
    Stats st;
    std::vector<double> v;
    *value = trace_path(C, px, py, s, w, st, &v) / op->spp_norm;
    const int32_t n = (int32_t)(v.size() / 12);
    std::memcpy(out, v.data(), sizeof(double) * 12 * (size_t)std::min(n, max_rows));
    return n;
}

// Faddeeva function (tests): z = (re, im), im >= 0; out [2].
void or_faddeeva(double re, double im, double* out) {
    const std::complex<double> w = faddeeva({re, im});
    out[0] = w.real();
    out[1] = w.imag();
}

// Normalised window fields (tests): S [3] = (sxx, syy, sxy), boundary (nx, ny, c), v [n][2];
// out [n][3] = (whole-plane field, far half-plane field re, im).
void or_halfplane_field(const double* S, double nx, double ny, double c, const double* v, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        const std::complex<double> F = halfplane_field(S[0], S[1], S[2], nx, ny, c, v[2 * i], v[2 * i + 1]);
        out[3 * i] = window_field(S[0], S[1], S[2], v[2 * i], v[2 * i + 1]);
        out[3 * i + 1] = F.real();
        out[3 * i + 2] = F.imag();
    }
}

// Composite p_w for a batch (tests).  q [n][23]: near material (kind, h, L, refl, gx, gy), far
// material (the same six), k, kix, kiy, kox, koy, sxx, syy, sxy, nx, ny, c.  out [n].
void or_pw_composite_batch(const double* q, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        const double* r = q + 23 * i;
        const Mat mn{(int)r[0], r[1], r[2], r[3], V3{1, 0, 0}};
        const Mat mf{(int)r[6], r[7], r[8], r[9], V3{1, 0, 0}};
        const Side sn{&mn, r[4], r[5]}, sf{&mf, r[10], r[11]};
        out[i] = pw_composite(sn, sf, r[12], r[13], r[14], r[15], r[16], r[17], r[18], r[19], r[20], r[21], r[22]);
    }
}

// One interaction with composite interactions enabled (tests): closest hit of (o, d), the
// footprint of a ray of beta^2 = beta2 (um^2) there, the boundary found and the continuation
// sampled with uniforms u[0..2] and side-choice uniform u[3].  out [11]: composite (1 or 0),
// c (um), nx, ny, far mass, side (0 near, 1 far), weight, direction (3), ended.
void or_interaction_composite(void* s, const double* ray, double k, double beta2, const double* u, double reach_m,
                              double* out) {
    const SceneO& S = *(SceneO*)s;
    for (int i = 0; i < 11; ++i) out[i] = 0.0;
    V3 o = ld3(ray), d = unit(ld3(ray + 3));
    Hit h;
    if (!trace_ray(S, o, d, t_eps(o), 1e300, true, false, h)) { out[10] = 1.0; return; }
    Vertex v;
    if (!make_vertex(S, o, d, h, v)) { out[10] = 1.0; return; }
    double sxx, syy, sxy;
    footprint(v, beta2, sxx, syy, sxy);
    Side near_side{v.m, 1.0, 0.0}, far_side{v.m, 1.0, 0.0};
    double nx = 0, ny = 0, c = 0, mf = 0;
    const bool comp = S.have_bedges && composite_at(S, v, S.mat[h.tri], sxx, syy, sxy, reach_m, far_side, nx, ny, c, mf);
    const bool far = comp && !(u[3] < 1.0 - mf);
    const Side& cs = far ? far_side : near_side;
    out[0] = comp; out[1] = c; out[2] = nx; out[3] = ny; out[4] = mf; out[5] = far;
    double kox, koy, wgt;
    int ev;
    if (!sample_finf(*cs.m, k, k * v.dx, k * v.dy, v.ci, u[0], u[1], u[2], cs.gx, cs.gy, kox, koy, wgt, ev)) {
        out[10] = 1.0;
        return;
    }
    double kn = std::sqrt(std::max(0.0, 1.0 - (kox * kox + koy * koy) / (k * k)));
    V3 dn = unit((kox / k) * v.xa + (koy / k) * v.ya + kn * v.ns);
    out[6] = wgt; out[7] = dn.x; out[8] = dn.y; out[9] = dn.z;
}

// Closest hit for a batch of rays (tests).  rays: [n][6] (origin, direction).  out: [n][4]
// (triangle, t, u, v); triangle = -1 on a miss.  tmin < 0 selects the default offset.
void or_intersect(void* s, const double* rays, int64_t n, double tmin, int use_bvh, double* out) {
    const SceneO& S = *(SceneO*)s;
    for (int64_t i = 0; i < n; ++i) {
        V3 o = ld3(rays + 6 * i), d = ld3(rays + 6 * i + 3);
        Hit h;
        double tm = tmin < 0 ? t_eps(o) : tmin;
        bool hit = trace_ray(S, o, d, tm, 1e300, use_bvh != 0, false, h);
        out[4 * i] = hit ? h.tri : -1;
        out[4 * i + 1] = hit ? h.t : 0;
        out[4 * i + 2] = hit ? h.u : 0;
        out[4 * i + 3] = hit ? h.v : 0;
    }
}

// One interaction of the path loop, exposed for checking: closest hit of the ray (o, d), the
// vertex (shading normal interpolated from the hit's barycentrics and oriented like the path
// loop orients it) and the continuation sampled from f_inf with uniforms u[3] at wavenumber k.
// out: [hit (1 or 0), ns (3), ng (3), cos i, continuation direction (3), weight, ended (1 when
// the path ends there: back-facing or evanescent)].
void or_interaction(void* s, const double* ray, double k, const double* u, double* out) {
    const SceneO& S = *(SceneO*)s;
    for (int i = 0; i < 13; ++i) out[i] = 0.0;
    V3 o = ld3(ray), d = unit(ld3(ray + 3));
    Hit h;
    if (!trace_ray(S, o, d, t_eps(o), 1e300, true, false, h)) return;
    out[0] = 1.0;
    Vertex v;
    const bool front = make_vertex(S, o, d, h, v);
    out[1] = v.ns.x; out[2] = v.ns.y; out[3] = v.ns.z;
    out[4] = v.ng.x; out[5] = v.ng.y; out[6] = v.ng.z;
    out[7] = v.ci;
    if (!front) { out[12] = 1.0; return; }
    double kox, koy, wgt;
    int ev;
    if (!sample_finf(*v.m, k, k * v.dx, k * v.dy, v.ci, u[0], u[1], u[2], 1.0, 0.0, kox, koy, wgt, ev)) {
        out[12] = 1.0;
        return;
    }
    double kn = std::sqrt(std::max(0.0, 1.0 - (kox * kox + koy * koy) / (k * k)));
    V3 dn = unit((kox / k) * v.xa + (koy / k) * v.ya + kn * v.ns);
    out[8] = dn.x; out[9] = dn.y; out[10] = dn.z;
    out[11] = wgt;
}

// Render.  pixels: optional list of (x, y) pairs (npix of them); when null, every pixel of
// the sensor in row-major order.  image: [nl][npix].  paths (optional):
// [spp_count][npix][nl] per-path contributions (already divided by spp_norm).
// stats: [segments, shadow rays, evanescent kills, backfacing kills, composite interactions,
// measurements at smooth, rough and grating surfaces].
int or_trace(void* s, const or_sensor* sen, const or_source* src, int32_t nsrc,
             const double* lambdas, int32_t nl, const or_opts* op, const int32_t* pixels,
             int64_t npix, double* image, double* paths, uint64_t* stats) {
    if (!s || !sen || !op || nl <= 0 || op->spp_count < 0 || op->max_depth < 0) return -1;
    if (op->hero && nl % 4 != 0) return -1;
    if (op->hero && op->aniso) return -1;   // hero paths carry scalar beta, rho
    if (op->composite && !((const SceneO*)s)->have_bedges) return -1;
    const SceneO* S = (const SceneO*)s;
    if (!pixels) npix = (int64_t)sen->width * sen->height;
    Ctx C{S, sen, src, nsrc, lambdas, nl, op};
    int nt = op->n_threads > 0 ? op->n_threads : default_threads();
    nt = std::max(1, nt);
    std::atomic<int64_t> next(0);
    std::vector<Stats> sts(nt);
    auto work = [&](int tid) {
        Stats& st = sts[tid];
        for (;;) {
            int64_t p = next.fetch_add(1);
            if (p >= npix) break;
            int px, py;
            if (pixels) { px = pixels[2 * p]; py = pixels[2 * p + 1]; }
            else { px = (int)(p % sen->width); py = (int)(p / sen->width); }
            if (op->hero) {
                const int G = nl / 4;
                for (int g = 0; g < G; ++g) {
                    double acc[4] = {0, 0, 0, 0};
                    for (int64_t sl = 0; sl < op->spp_count; ++sl) {
                        double c[4];
                        trace_path_hero(C, px, py, op->spp_begin + sl, g, st, c);
                        for (int i = 0; i < 4; ++i) {
                            c[i] /= op->spp_norm;
                            if (paths) paths[(sl * npix + p) * nl + g + i * G] = c[i];
                            acc[i] += c[i];
                        }
                    }
                    for (int i = 0; i < 4; ++i) image[(int64_t)(g + i * G) * npix + p] = acc[i];
                }
                continue;
            }
            for (int w = 0; w < nl; ++w) {
                double acc = 0.0;
                for (int64_t sl = 0; sl < op->spp_count; ++sl) {
                    double c = trace_path(C, px, py, op->spp_begin + sl, w, st) / op->spp_norm;
                    if (paths) paths[(sl * npix + p) * nl + w] = c;
                    acc += c;
                }
                image[(int64_t)w * npix + p] = acc;
            }
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(work, i);
    for (auto& t : th) t.join();
    uint64_t tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (auto& st : sts) {
        tot[0] += st.segments; tot[1] += st.shadow; tot[2] += st.evanescent; tot[3] += st.backfacing;
        tot[4] += st.composite;
        for (int i = 0; i < 3; ++i) tot[5 + i] += st.measured[i];
    }
    if (stats) std::memcpy(stats, tot, sizeof(tot));
    return 0;
}

// ------------------------------------------------------------------------------------------
// Coherent measurement of mutually coherent emitters (Sec. "Linearity of Generalized Rays",
// two-point interference, and "Numeric Validation", Rayleigh-Sommerfeld diffraction).
//
// Field at a sensor point X (um, x along the row, y across it), z = distance to the aperture
// plane:
//   points: U = sum_e exp(i k L_e) / L_e,   L_e = |X - s_e| (3-D spherical waves)
//   slits : U = sum_e c_e (i k z / 2) H1(k rho_e) / rho_e, the 2-D Rayleigh-Sommerfeld
//           first-kind kernel of a y-invariant aperture, integrated with Gauss-Legendre nodes
//           (positions xs, weights ws) over each slit under normal plane-wave illumination.
// A detection state centred at r0 with intensity standard deviation sigma, integrated over
// all mean wavevectors, measures |U|^2 averaged over the Gaussian N(r0, sigma^2) (the
// spatial marginal of the coherent state).
// ------------------------------------------------------------------------------------------
typedef struct {
    int32_t kind;          // 0 points, 1 slits
    int32_t n_nodes;       // points: number of emitters; slits: total quadrature nodes
    const double* xs;      // node x positions (um)
    const double* ws;      // node weights (slits) / ignored (points)
    double z_um, lambda_um;
    int32_t width, height;
    double pitch_um, sigma_um;
    int64_t spp;
    uint64_t seed;
} or_coherent;

static std::complex<double> field_at(const or_coherent& c, double X, double Y) {
    const double k = 2.0 * kPi / c.lambda_um;
    std::complex<double> U(0.0, 0.0);
    for (int e = 0; e < c.n_nodes; ++e) {
        double dx = X - c.xs[e];
        if (c.kind == 0) {
            double L = std::sqrt(c.z_um * c.z_um + dx * dx + Y * Y);
            U += std::polar(1.0 / L, k * L);
        } else {
            double rho = std::sqrt(c.z_um * c.z_um + dx * dx);
            double kr = k * rho;
            std::complex<double> H1(std::cyl_bessel_j(1.0, kr), std::cyl_neumann(1.0, kr));
            U += c.ws[e] * std::complex<double>(0.0, 0.5 * k * c.z_um) * H1 / rho;
        }
    }
    return U;
}

// Per-sample Monte Carlo estimator with the shared random streams: sample s of pixel (x, y)
// draws (u0, u1) on the pixel and a Gaussian offset (Box-Muller of u2, u3) of the detection
// state.  out: [height][width] mean of |U|^2 over the spp samples.
// rows: number of leading sensor rows to compute (<= height; path ids use the full height).
void or_coherent_mc(const or_coherent* c, double* out, int32_t n_threads, int32_t rows) {
    int nt = n_threads > 0 ? n_threads : default_threads();
    std::atomic<int64_t> next(0);
    if (rows <= 0 || rows > c->height) rows = c->height;
    int64_t np = (int64_t)c->width * rows;
    auto work = [&]() {
        for (;;) {
            int64_t p = next.fetch_add(1);
            if (p >= np) break;
            int x = (int)(p % c->width), y = (int)(p / c->width);
            double acc = 0.0;
            for (int64_t s = 0; s < c->spp; ++s) {
                uint64_t pid = ((uint64_t)s * c->height + y) * c->width + x;
                U4 r = draw(pid, 0, STREAM_SOURCE, c->seed);
                double z1, z2;
                box_muller(unif(r.v[2]), unif(r.v[3]), z1, z2);
                double X = (x + unif(r.v[0]) - 0.5 * c->width) * c->pitch_um + c->sigma_um * z1;
                double Y = (y + unif(r.v[1]) - 0.5 * c->height) * c->pitch_um + c->sigma_um * z2;
                acc += std::norm(field_at(*c, X, Y));
            }
            out[p] = acc / (double)c->spp;
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < std::max(1, nt); ++i) th.emplace_back(work);
    for (auto& t : th) t.join();
}

// The exact expectation of the estimator above for row y = 0 pixels, by Gauss-Hermite
// quadrature over the detection state's Gaussian and Gauss-Legendre quadrature over the pixel
// (x: pixel positions, n: count).  out[i] = E|U|^2 at pixel x[i]; rows are ignored (points:
// Y = 0 is used; the y dependence is a common factor near the axis).
void or_coherent_exact(const or_coherent* c, const int32_t* xpix, int64_t n, const double* gh_x,
                       const double* gh_w, int32_t ngh, const double* gl_x, const double* gl_w,
                       int32_t ngl, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int a = 0; a < ngl; ++a) {
            double u = 0.5 * (gl_x[a] + 1.0);
            double x0 = (xpix[i] + u - 0.5 * c->width) * c->pitch_um;
            for (int b = 0; b < ngh; ++b) {
                double X = x0 + std::sqrt(2.0) * c->sigma_um * gh_x[b];
                acc += 0.5 * gl_w[a] * gh_w[b] / std::sqrt(kPi) * std::norm(field_at(*c, X, 0.0));
            }
        }
        out[i] = acc;
    }
}

double or_hankel1_re(double x) { return std::cyl_bessel_j(1.0, x); }
double or_hankel1_im(double x) { return std::cyl_neumann(1.0, x); }

// Anisotropic generalized-ray steps, for the tests.  st: the 12 moments in row-major order,
// Srr[2][2], Srk[2][2], Skk[2][2], in the transverse frame of transverse_frame().
static Aniso aniso_from(const double* st) {
    Aniso A;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            A.rr[i][j] = st[2 * i + j];
            A.rk[i][j] = st[4 + 2 * i + j];
            A.kk[i][j] = st[8 + 2 * i + j];
        }
    return A;
}
static void aniso_to(const Aniso& A, double* st) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            st[2 * i + j] = A.rr[i][j];
            st[4 + 2 * i + j] = A.rk[i][j];
            st[8 + 2 * i + j] = A.kk[i][j];
        }
}
void or_transverse_frame(const double* d, double* e1, double* e2) {
    V3 a, b;
    transverse_frame(V3{d[0], d[1], d[2]}, a, b);
    e1[0] = a.x; e1[1] = a.y; e1[2] = a.z;
    e2[0] = b.x; e2[1] = b.y; e2[2] = b.z;
}
void or_aniso_free(double z_um, double k, double* st) {
    Aniso A = aniso_from(st);
    propagate_aniso(z_um, k, A);
    aniso_to(A, st);
}
void or_aniso_interact(const double* di, const double* dout, const double* n, double* st) {
    Aniso A = aniso_from(st);
    interact_aniso(V3{di[0], di[1], di[2]}, V3{dout[0], dout[1], dout[2]}, V3{n[0], n[1], n[2]}, A);
    aniso_to(A, st);
}
void or_aniso_footprint(const double* d, const double* n, const double* xa, const double* ya,
                        const double* st, double* out) {
    Aniso A = aniso_from(st);
    footprint_aniso(V3{d[0], d[1], d[2]}, V3{n[0], n[1], n[2]}, V3{xa[0], xa[1], xa[2]},
                    V3{ya[0], ya[1], ya[2]}, A, out[0], out[1], out[2]);
}

}  // extern "C"
