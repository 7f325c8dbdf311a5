// Device-side arithmetic of the generalized-ray tracer (gfx950, FP32 with FP64 where a
// discrete decision needs it).
//
// Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grw {

constexpr float kPiF = 3.14159265358979f;
constexpr float kTwoPiF = 6.28318530717959f;

// ------------------------------------------------------------------------------------------
// Small float3 helpers (registers only).
// ------------------------------------------------------------------------------------------
struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return f3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return f3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return f3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
    return f3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 normalize3(f3 a) { return rsqrtf(dot3(a, a)) * a; }
__device__ __forceinline__ float maxabs3(f3 a) {
    return fmaxf(fabsf(a.x), fmaxf(fabsf(a.y), fabsf(a.z)));
}

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 multiplies by the published
// multipliers, xor of the high halves with the other counter words and the key, Weyl-sequence
// key schedule.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32x32 -> 64-bit product as one multiply (both halves from one instruction)
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Streams of one path: counter = (path id lo, path id hi, interaction index, stream).
enum { STREAM_SOURCE = 0, STREAM_NEE = 1, STREAM_SCATTER = 2 };

__device__ __forceinline__ uint4 draw(uint64_t pid, uint32_t depth, uint32_t stream, uint64_t seed) {
    return philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), depth, stream, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// 24-bit uniform in [0, 1), exact in float.
__device__ __forceinline__ float unif(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// Box-Muller pair from two uniforms.
__device__ __forceinline__ void box_muller(float u1, float u2, float& z1, float& z2) {
    const float r = sqrtf(-2.0f * logf(1.0f - u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    z1 = r * c;
    z2 = r * s;
}

// ------------------------------------------------------------------------------------------
// Bivariate normal density N(x; 0, S), S = [[a, c], [c, b]].
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float gauss2(float x, float y, float a, float b, float c) {
    const float det = a * b - c * c;
    const float q = (b * x * x - 2.0f * c * x * y + a * y * y) * __builtin_amdgcn_rcpf(det);
    return __expf(-0.5f * q) * (1.0f / kTwoPiF) * rsqrtf(det);
}

// ------------------------------------------------------------------------------------------
// Bessel function of the first kind, integer order n >= 0.  Small arguments: the ascending
// series.  Larger ones: Miller's algorithm (backward recurrence for the minimal solution of a
// three-term recurrence, as analysed by W. Gautschi, "Computational aspects of three-term
// recurrence relations", SIAM Review 9, 1967), normalised by Neumann's identity
// J_0(x) + 2 sum_{k>=1} J_2k(x) = 1.
// ------------------------------------------------------------------------------------------
// Ascending series J_n(x) = (x/2)^n / n! * sum_k (-x^2/4)^k / (k! (n+1)(n+2)...(n+k)).  The
// terms stay below I_n(x) (x/2)^-n n!, so in FP32 the absolute error is ~2e-7 for x <= 4.5;
// about 14 terms there, far fewer for large n.
__device__ __forceinline__ float bessel_jn_series(int n, float x) {
    const float hx = 0.5f * x;
    // J_n(x) < (x/2)^n / n!: an order below 1e-10 weighs < 1e-20, far under one float ulp of
    // any sum of weights or lobe values it enters
    float p = 1.0f;
    if (n <= 4) {
        for (int i = 1; i <= n; ++i) p *= hx * __builtin_amdgcn_rcpf((float)i);
        if (p < 1e-10f) return 0.0f;
    } else {
        // (x/2)^n / n! = exp(n log(x/2) - log n!), log n! by Stirling's series (its first
        // omitted term, 1 / (1260 n^5), is below 3e-7 for n >= 5)
        const float nf = (float)n;
        const float rn = __builtin_amdgcn_rcpf(nf);
        const float lf = (nf + 0.5f) * __logf(nf) - nf + 0.91893853f + rn * (1.0f / 12.0f - rn * rn * (1.0f / 360.0f));
        const float e = nf * __logf(hx) - lf;
        if (!(e > -23.0258509f)) return 0.0f;   // log(1e-10); also x = 0
        p = __expf(e);
    }
    const float q = -hx * hx;
    float t = 1.0f, s = 1.0f, kf = 0.0f, nk = (float)n;
    for (int it = 0; it < 24; ++it) {
        kf += 1.0f;
        nk += 1.0f;
        t *= q * __builtin_amdgcn_rcpf(kf * nk);
        s += t;
        if (fabsf(t) < 1e-9f) break;
    }
    return p * s;
}

// x >= 0 (the phase-screen modulation depth q_z A is never negative here).
//
// Above the turning point k = x, J_k(x) decays like the Airy function of (k - x) / c with
// c = (x / 2)^(1/3).  Orders beyond x + 8 c + 12 are below 1.2e-10 (checked against scipy for
// x in [4.5, 2000]) and return 0.  The recurrence v_{k-1} = (2k / x) v_k - v_{k+1} runs down
// from v_{N+1} = 0, v_N = 1 with N = max(n, x) + 10 c + 16: the dominant solution's share,
// which the start sets, has decayed below FP32 rounding by order n (abs. error <= 2.3e-6 at
// x = 2000, 3e-7 for x <= 100; the callers keep x < 2000).  The v_k are J_k up to one common
// factor, fixed at the end by Neumann's identity; exact power-of-two rescaling keeps them in
// range.
__device__ inline float bessel_jn(int n, float x) {
    if (x <= 4.5f) return bessel_jn_series(n, x);
    const float c = cbrtf(0.5f * x);
    if ((float)n > x + 8.0f * c + 12.0f) return 0.0f;
    const int N = (int)(fmaxf((float)n, x) + 10.0f * c + 16.0f);
    const float two_over_x = 2.0f / x;
    float above = 0.0f, v = 1.0f;                  // v_{k+1}, v_k
    float neumann = (N & 1) ? 0.0f : 2.0f;         // v_0 + 2 (v_2 + v_4 + ...) so far
    float vn = (N == n) ? 1.0f : 0.0f;
    for (int k = N; k >= 1; --k) {
        const float below = (float)k * two_over_x * v - above;   // v_{k-1}
        above = v;
        v = below;
        const int idx = k - 1;
        if ((idx & 1) == 0) neumann += (idx == 0) ? v : 2.0f * v;
        if (idx == n) vn = v;
        if (fabsf(v) > 0x1p100f) {
            v *= 0x1p-100f;
            above *= 0x1p-100f;
            neumann *= 0x1p-100f;
            vn *= 0x1p-100f;
        }
    }
    return vn / neumann;
}

// ------------------------------------------------------------------------------------------
// log Poisson(m; g) without cancellation: Stirling's series for log m! in the form
// -m log1p((m - g) / g) + (m - g) - log(2 pi m) / 2 - 1 / (12 m) + 1 / (360 m^3).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float log_poisson(int m, float g, float logg) {
    if (m == 0) return -g;
    if (m < 10) {
        float lf = 0.0f;   // log m!
        for (int i = 2; i <= m; ++i) lf += logf((float)i);
        return -g + (float)m * logg - lf;
    }
    const float mf = (float)m;
    const float d = mf - g;
    return -mf * log1pf(d / g) + d - 0.5f * logf(kTwoPiF * mf) - 1.0f / (12.0f * mf) +
           1.0f / (360.0f * mf * mf * mf);
}

// Material record on the device.
struct DMat {
    int kind;
    float h, L, refl;
    float gx, gy, gz, pad;
};

enum { MAT_SMOOTH = 0, MAT_ROUGH = 1, MAT_GRATING = 2 };

// ------------------------------------------------------------------------------------------
// Windowed diffraction density p_w(k_i,t -> k_o,t) (um^2) of a curvature-free generalized ray
// on a surface patch (Sec. "Interaction Kernels"): the squared Fourier transform of the
// Gaussian window times the surface phase screen exp(i q_z h(x)), normalised by the window
// energy, as a Gaussian mixture in the tangential transfer kappa = k_o,t - k_i,t:
//   smooth : N(kappa; 0, Sk)
//   grating: sum_j J_j(q_z A)^2 N(kappa; -j K g, Sk)          (Jacobi-Anger, eq. K_grating)
//   rough  : sum_m Poisson(m; q_z^2 s^2) N(kappa; 0, Sk + 2m/l^2 I)   (ensemble average)
// with Sk = S_fp^-1 / 4, S_fp the footprint covariance, q_z = k (cos i + cos o).
// ------------------------------------------------------------------------------------------
// (Its reciprocals are the hardware's, 1 ulp: they scale the value, and no decision of the path
// depends on them.)
__device__ inline float pw_plain(int kind, float h, float L, float refl, float k, float kix,
                                 float kiy, float kox, float koy, float sxx, float syy, float sxy,
                                 float gx, float gy) {
    const float ik2 = __builtin_amdgcn_rcpf(k * k);
    const float ni = (kix * kix + kiy * kiy) * ik2;
    const float no = (kox * kox + koy * koy) * ik2;
    if (ni >= 1.0f || no >= 1.0f) return 0.0f;
    const float qz = k * (sqrtf(1.0f - ni) + sqrtf(1.0f - no));
    const float kx = kox - kix, ky = koy - kiy;
    const float det = sxx * syy - sxy * sxy;
    // a window thinner than float resolves (its determinant rounds to zero or below: extreme
    // anisotropic footprints after grazing interactions) measures nothing
    if (!(det > 0.0f)) return 0.0f;
    const float idet = 0.25f * __builtin_amdgcn_rcpf(det);
    const float a = syy * idet, b = sxx * idet, c = -sxy * idet;
    if (kind == MAT_SMOOTH) return refl * gauss2(kx, ky, a, b, c);
    if (kind == MAT_GRATING) {
        const float K = kTwoPiF / L;
        const float m = qz * h;
        const float proj = kx * gx + ky * gy;
        const float sg = sqrtf(fmaxf(a * gx * gx + 2.0f * c * gx * gy + b * gy * gy, 0.0f));
        int jlo = (int)ceilf((-proj - 8.0f * sg) / K);
        int jhi = (int)floorf((-proj + 8.0f * sg) / K);
        if (jhi < jlo) return 0.0f;
        jhi = min(jhi, jlo + 15);
        float s = 0.0f;
        for (int j = jlo; j <= jhi; ++j) {
            const float bj = bessel_jn(abs(j), m);
            s += bj * bj * gauss2(kx + (float)j * K * gx, ky + (float)j * K * gy, a, b, c);
        }
        return refl * s;
    }
    // rough
    const float g = qz * qz * h * h;
    if (g < 1e-12f) return refl * gauss2(kx, ky, a, b, c);
    const float sq = sqrtf(g);
    int mlo = max(0, (int)floorf(g - 6.0f * sq - 3.0f));
    int mhi = (int)ceilf(g + 6.0f * sq + 3.0f);
    if (mhi - mlo > 4095) {   // bound the work for out-of-range inputs
        mlo = max(0, (int)g - 2048);
        mhi = mlo + 4095;
    }
    const float add = 2.0f * __builtin_amdgcn_rcpf(L * L);
    const float logg = logf(g);
    const float c2 = c * c;
    // Poisson weights by the recurrence P(m + 1) = P(m) g / (m + 1) from the log-space first
    // term (relative drift ~1e-5 over the ~12 sqrt(g) terms, well inside FP32 tolerance of the
    // image); the exponent of the Gaussian is added to log P(mlo) once.
    const float lp0 = log_poisson(mlo, g, logg);
    float w = 1.0f;   // P(m) / P(mlo)
    float s = 0.0f;
    for (int m = mlo; m <= mhi; ++m) {
        const float aa = a + (float)m * add, bb = b + (float)m * add;
        const float dm = aa * bb - c2;
        const float q = (bb * kx * kx - 2.0f * c * kx * ky + aa * ky * ky) * __builtin_amdgcn_rcpf(dm);
        s += w * __expf(lp0 - 0.5f * q) * rsqrtf(dm);
        w *= g * __builtin_amdgcn_rcpf((float)(m + 1));
    }
    return refl * s * (1.0f / kTwoPiF);
}

// Smallest n with u < sum_{i <= n} Poisson(i; g), by inversion of the CDF in double precision
// (the decision must not depend on FP32 rounding of a long sum); terms below g - 7 sqrt(g)
// hold < 1e-11 mass and are skipped.  Kept out of line: its double-precision exp/log constants
// would otherwise be hoisted into registers for the whole path loop.
__device__ __noinline__ int poisson_inverse(double g, float u0) {
    int n = 0;
    if (g > 0.0) {
        const double sq = sqrt(g);
        const int mlo = g > 49.0 ? (int)floor(g - 7.0 * sq) : 0;
        const int mhi = min((int)ceil(g + 20.0 * sq + 40.0), mlo + 65536);
        // log of the first term: log Poisson(mlo; g) via Stirling (mlo >= 10 here) or exactly
        double lw;
        if (mlo == 0) {
            lw = -g;
        } else {
            const double mf = (double)mlo, d = mf - g;
            lw = -mf * log1p(d / g) + d - 0.5 * log(6.283185307179586 * mf) - 1.0 / (12.0 * mf) +
                 1.0 / (360.0 * mf * mf * mf);
        }
        double w = exp(lw), c = 0.0;
        const double uu = (double)u0;
        n = mhi;
        // w_{i+1} = w_i g / (i + 1); the reciprocal by the hardware estimate and one
        // Newton step (relative error ~1e-16, as a correctly rounded division)
        double t = (double)(mlo + 1);
        for (int i = mlo; i <= mhi; ++i) {
            c += w;
            if (uu < c) {
                n = i;
                break;
            }
            const double r0 = __builtin_amdgcn_rcp(t);
            const double r1 = fma(r0, fma(-t, r0, 1.0), r0);
            w *= g * r1;
            t += 1.0;
        }
    }
    return n;
}

// ------------------------------------------------------------------------------------------
// Continuation sampling from the unwindowed kernel f_inf (the delta-lobe limit of p_w),
// taking the generalized ray's own travel direction as the incident wave (time reversal is
// wavevector reversal, and these kernels are reciprocal).
//   smooth : mirror direction, weight = reflectance
//   grating: order j among the propagating ones with probability J_j(m_j)^2 / W,
//            m_j = k A (cos i + cos o_j); weight = reflectance * W (evanescent orders dropped)
//   rough  : term m ~ Poisson(g), g = (2 k cos i s)^2, then kappa ~ N(0, 2m/l^2 I);
//            weight = reflectance; an evanescent draw ends the path
// Returns 0 on success, 1 when the path ends evanescently.  comp (optional) receives the
// sampled component: the grating order, the rough surface's Poisson term (0 = the specular
// delta), 0 for a smooth surface; pick_p (optional) the probability of a grating's sampled
// order, w_j / W; off (optional, 2 floats) the rough surface's sampled transfer kappa (zero
// otherwise; a grating's is -j K along x); with off given, a rough surface's evanescent draw is
// left to the caller, which forms the direction in double.
// ------------------------------------------------------------------------------------------
__device__ inline int sample_finf(const DMat& m, float k, float kix, float kiy, float ci,
                                  float u0, float u1, float u2, float& kox, float& koy,
                                  float& weight, float* cache, int cache_n, int* comp = nullptr,
                                  float* pick_p = nullptr, float* off = nullptr, double g_rough = -1.0) {
    if (comp) *comp = 0;
    if (off) off[0] = off[1] = 0.0f;
    if (m.kind == MAT_SMOOTH) {
        kox = kix;
        koy = kiy;
        weight = m.refl;
        return 0;
    }
    const float k2 = k * k;
    const float ik2 = 1.0f / k2;
    if (m.kind == MAT_GRATING) {
        // grating vector = frame x axis; propagating orders: (kix - jK)^2 + kiy^2 < k^2.
        // cache: this lane's idle scratch (stride 64 floats) holding the order weights
        // between the summation and the inversion pass when the orders fit.
        const float K = kTwoPiF / m.L;
        const float rem = k2 - kiy * kiy;
        if (rem <= 0.0f) return 1;
        const float r = sqrtf(rem);
        const int jlo = (int)floorf((kix - r) / K) - 1;
        const int jhi = min((int)ceilf((kix + r) / K) + 1, jlo + 4096);
        const bool cached = jhi - jlo < cache_n;
        // pass 0 sums the weights W, pass 1 inverts the cumulative sum at u0 W (one Bessel
        // evaluation site for both)
        float W = 0.0f, c = 0.0f, target = 0.0f, wp = 0.0f;
        int pick = jhi, last = jlo;
#pragma nounroll
        for (int pass = 0; pass < 2; ++pass) {
            bool found = false;
            for (int j = jlo; j <= jhi; ++j) {
                const float ox = kix - (float)j * K;
                const float no = (ox * ox + kiy * kiy) * ik2;
                if (no >= 1.0f) continue;
                float w;
                if (pass == 1 && cached) {
                    w = cache[(j - jlo) * 64];
                } else {
                    const float bj = bessel_jn(abs(j), k * m.h * (ci + sqrtf(1.0f - no)));
                    w = bj * bj;
                }
                if (pass == 0) {
                    W += w;
                    if (cached) cache[(j - jlo) * 64] = w;
                } else {
                    c += w;
                    last = j;
                    wp = w;
                    if (target < c) {
                        pick = j;
                        found = true;
                        break;
                    }
                }
            }
            if (pass == 0) {
                if (!(W > 0.0f)) return 1;
                target = u0 * W;
            } else if (!found) {
                pick = last;
            }
        }
        kox = kix - (float)pick * K;
        koy = kiy;
        weight = m.refl * W;
        if (comp) *comp = pick;
        if (pick_p) *pick_p = wp / W;
        return 0;
    }
    // rough: Poisson term by inversion of the CDF in double precision (g_rough: the caller's
    // double-precision Poisson parameter, when it has one)
    const int n = poisson_inverse(g_rough >= 0.0 ? g_rough
                                                 : 4.0 * (double)k2 * (double)ci * (double)ci * (double)m.h * (double)m.h,
                                  u0);
    if (comp) *comp = n;
    float z1, z2;
    box_muller(u1, u2, z1, z2);
    const float sd = sqrtf(2.0f * (float)n) / m.L;
    kox = kix + sd * z1;
    koy = kiy + sd * z2;
    if (off) {
        // the caller forms the new direction in double and decides evanescence there
        off[0] = sd * z1;
        off[1] = sd * z2;
    } else if (kox * kox + koy * koy >= k2) {
        return 1;
    }
    weight = m.refl;
    return 0;
}

// ------------------------------------------------------------------------------------------
// Hero-wavelength companions.  A path sampled at its hero wavelength also carries the other
// members of the hero's rotation group of the wavelength grid; the members' estimates are
// combined by the one-sample balance heuristic over the choice of hero (Wilkie et al., "Hero
// wavelength spectral sampling", EGSR 2014).  For the direction the hero sampled, a member's
// value f_c and density p_c are compared with the hero's density p_h over the outgoing
// tangential direction u_o = k_o,t / k (continuous lobes) or by probability (deltas):
//   smooth : one non-dispersive delta: p_c / p_h = 1, f_c / p_h = refl
//   grating: order j != 0 is a delta whose direction moves with the wavelength (dispersive):
//            no member shares it; order 0 has probability J_0(m_0)^2 / W at every wavelength
//   rough  : the specular delta has probability exp(-g); the terms n >= 1 form the density
//            below; f_c / p_h = refl p_c / p_h
// ------------------------------------------------------------------------------------------

// Order weights of a grating at wavenumber k: W = sum of J_j(m_j)^2 over the propagating
// orders and w0 = J_0(m_0)^2, with m_j = k A (cos i + cos o_j) as in sample_finf.
__device__ inline void grating_weights(const DMat& m, float k, float kix, float kiy, float ci, float& W,
                                       float& w0) {
    W = 0.0f;
    w0 = 0.0f;
    const float k2 = k * k;
    const float ik2 = 1.0f / k2;
    const float K = kTwoPiF / m.L;
    const float rem = k2 - kiy * kiy;
    if (rem <= 0.0f) return;
    const float r = sqrtf(rem);
    const int jlo = (int)floorf((kix - r) / K) - 1;
    const int jhi = min((int)ceilf((kix + r) / K) + 1, jlo + 4096);
    for (int j = jlo; j <= jhi; ++j) {
        const float ox = kix - (float)j * K;
        const float no = (ox * ox + kiy * kiy) * ik2;
        if (no >= 1.0f) continue;
        const float bj = bessel_jn(abs(j), k * m.h * (ci + sqrtf(1.0f - no)));
        W += bj * bj;
        if (j == 0) w0 = bj * bj;
    }
}

// Continuous part (terms n >= 1) of a rough surface's continuation density over u_o at
// squared direction change du2 = |u_o - u_i|^2:
//   k^2 sum_{n>=1} Poisson(n; g) exp(-k^2 du2 l^2 / (4 n)) l^2 / (4 pi n),  g = (2 k cos i s)^2.
// Terms outside [g - 6 sqrt(g) - 3, g + 8 sqrt(g) + 8] are skipped (Poisson mass < 1e-9).
__device__ inline float rough_lobe_density(float k, float ci, float h, float L, float du2) {
    const float g = 4.0f * k * k * ci * ci * h * h;
    if (!(g > 1e-12f)) return 0.0f;
    const float sq = sqrtf(g);
    const int nlo = max(1, (int)floorf(g - 6.0f * sq - 3.0f));
    const int nhi = min((int)ceilf(g + 8.0f * sq + 8.0f), nlo + 8191);
    const float A = 0.25f * k * k * du2 * L * L;
    const float lp0 = log_poisson(nlo, g, logf(g));
    float w = 1.0f;   // Poisson(n; g) / Poisson(nlo; g)
    float s = 0.0f;
    float nf = (float)nlo;
    float rn = __builtin_amdgcn_rcpf(nf);   // 1 / n, carried to the next term
    for (int n = nlo; n <= nhi; ++n) {
        nf += 1.0f;
        const float rn1 = __builtin_amdgcn_rcpf(nf);
        s += w * __expf(lp0 - A * rn) * rn;
        w *= g * rn1;
        rn = rn1;
    }
    return s * k * k * L * L * (1.0f / (4.0f * kPiF));
}

}  // namespace grw
