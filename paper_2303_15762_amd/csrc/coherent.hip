// Coherent measurement of mutually coherent emitters (two points, or two slits under a normal
// plane wave), the precision-stress case of long optical paths.
//
// Paper (arXiv 2303.15762): Sec. "Linearity of Generalized Rays" (two-point interference and
// the sampling relation) and Sec. "Numeric Validation" (double slit, Rayleigh-Sommerfeld
// diffraction integrated over the detector).  A detection state integrated over all mean
// wavevectors measures the field's intensity averaged over the state's spatial density, so
// each sample draws a point on the pixel plus a Gaussian offset of std sigma and adds
// |sum_e c_e G_e exp(i k L_e)|^2 there.
//
// Phase modes: FP32 (naive), FP64, and compensated two-float (Dekker products by FMA, Knuth's
// TwoSum): the phase k L of a path of 0.1-10 m at sub-micron wavelengths needs ~50 bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/grwave.h"
#include "device_math.hpp"

namespace grw {

constexpr int kMaxNodes = 128;   // keeps the argument block under the 4 KB limit

struct CohArgs {
    int kind;          // 0 points, 1 slits
    int n;             // nodes
    double xs[kMaxNodes];
    double ws[kMaxNodes];
    double z, k, pitch, sigma;
    int W, H;
    int64_t spp;
    uint64_t seed;
};

// ---- two-float arithmetic --------------------------------------------------------------
// Error-free transformations need every rounding to happen where it is written, so FP
// contraction is switched off in them (a rounded product fused into a later add would count
// its rounding error twice).  Plain operators are used: the pragma governs only operations
// written in its scope, not those inside library intrinsics.
struct df {
    float hi, lo;
};
__device__ __forceinline__ df two_sum(float a, float b) {          // Knuth
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    return df{s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ df quick_two_sum(float a, float b) {    // |a| >= |b|
#pragma clang fp contract(off)
    const float s = a + b;
    return df{s, b - (s - a)};
}
__device__ __forceinline__ df two_prod(float a, float b) {         // exact by FMA
#pragma clang fp contract(off)
    const float p = a * b;
    return df{p, fmaf(a, b, -p)};
}
__device__ __forceinline__ df df_add(df x, df y) {
#pragma clang fp contract(off)
    df s = two_sum(x.hi, y.hi);
    s.lo = s.lo + (x.lo + y.lo);
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ df df_mul(df x, df y) {
#pragma clang fp contract(off)
    df p = two_prod(x.hi, y.hi);
    p.lo = p.lo + (x.hi * y.lo + x.lo * y.hi);
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ df df_sqrt(df x) {                       // one Newton correction
#pragma clang fp contract(off)
    const float s = sqrtf(x.hi);
    const df p = two_prod(s, s);
    const float diff = ((x.hi - p.hi) - p.lo) + x.lo;
    return quick_two_sum(s, diff / (2.0f * s));
}
__device__ __forceinline__ df df_from(double v) {
    const float hi = (float)v;
    return df{hi, (float)(v - (double)hi)};
}

template <int MODE>
__global__ __launch_bounds__(256) void coherent_kernel(const CohArgs A, float* __restrict__ img) {
    // block: 4 pixels x 64 sample lanes; samples of one pixel are spread over one wave
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t pix = (int64_t)blockIdx.x * 4 + wv;
    const int64_t npix = (int64_t)A.W * A.H;
    double acc = 0.0;
    // the slit kernel's constant factors (k z / 2) sqrt(2 / (pi k)) and 3 / (8 k), once per
    // thread (a thread draws few samples: the points case does not pay for them)
    double c_amp = 0.0, c_ci = 0.0;
    if (A.kind == 1) {
        c_amp = 0.5 * A.k * A.z * sqrt(2.0 / (M_PI * A.k));
        c_ci = 3.0 / (8.0 * A.k);
    }
    const float c_ampf = (float)c_amp, c_cif = (float)c_ci;
    if (pix < npix) {
        const int x = (int)(pix % A.W), y = (int)(pix / A.W);
        for (int64_t s = lane; s < A.spp; s += 64) {
            const uint64_t pid = ((uint64_t)s * A.H + y) * A.W + x;
            const uint4 r = draw(pid, 0, STREAM_SOURCE, A.seed);
            double re = 0.0, im = 0.0;
            if (MODE == GR_PHASE_FP64) {
                const double u0 = (double)(r.x >> 8) * (1.0 / 16777216.0);
                const double u1 = (double)(r.y >> 8) * (1.0 / 16777216.0);
                const double u2 = (double)(r.z >> 8) * (1.0 / 16777216.0);
                const double u3 = (double)(r.w >> 8) * (1.0 / 16777216.0);
                const double rr = sqrt(-2.0 * log(1.0 - u2));
                double sn, cs;
                sincospi(2.0 * u3, &sn, &cs);
                const double X = (x + u0 - 0.5 * A.W) * A.pitch + A.sigma * rr * cs;
                const double Y = (y + u1 - 0.5 * A.H) * A.pitch + A.sigma * rr * sn;
                // one double division per node: the distance's reciprocal
                const double z2y2 = A.z * A.z + Y * Y, z2 = A.z * A.z;
                for (int e = 0; e < A.n; ++e) {
                    const double dx = X - A.xs[e];
                    if (A.kind == 0) {
                        const double L = sqrt(z2y2 + dx * dx);
                        const double rL = 1.0 / L;
                        double ps, pc;
                        sincos(A.k * L, &ps, &pc);
                        re += pc * rL;
                        im += ps * rL;
                    } else {
                        // (i k z / 2) H1(k rho) / rho with the large-argument expansion of
                        // H1: sqrt(2 / (pi x)) exp(i (x - 3 pi / 4)) (1 + 3 i / (8 x)),
                        // x = k rho: amplitude (k z / 2) sqrt(2 / (pi k)) rho^-3/2
                        const double rho = sqrt(z2 + dx * dx);
                        const double rr = 1.0 / rho;
                        const double xk = A.k * rho;
                        const double amp = A.ws[e] * c_amp * rr * sqrt(rr);
                        double ps, pc;
                        sincos(xk - 0.75 * M_PI, &ps, &pc);
                        const double cr = 1.0, ci = c_ci * rr;
                        // i * (pc + i ps) * (cr + i ci)
                        const double ar = pc * cr - ps * ci, ai = pc * ci + ps * cr;
                        re += -amp * ai;
                        im += amp * ar;
                    }
                }
            } else {
                const float u0 = unif(r.x), u1 = unif(r.y);
                float z1, z2;
                box_muller(unif(r.z), unif(r.w), z1, z2);
                const float zf = (float)A.z, kf = (float)A.k;
                if (MODE == GR_PHASE_FP32) {
                    const float X = ((float)x + u0 - 0.5f * (float)A.W) * (float)A.pitch + (float)A.sigma * z1;
                    const float Y = ((float)y + u1 - 0.5f * (float)A.H) * (float)A.pitch + (float)A.sigma * z2;
                    float fre = 0.0f, fim = 0.0f;
                    for (int e = 0; e < A.n; ++e) {
                        const float dx = X - (float)A.xs[e];
                        if (A.kind == 0) {
                            const float L = sqrtf(zf * zf + dx * dx + Y * Y);
                            const float rL = 1.0f / L;
                            float ps, pc;
                            sincosf(kf * L, &ps, &pc);
                            fre += pc * rL;
                            fim += ps * rL;
                        } else {
                            const float rho = sqrtf(zf * zf + dx * dx);
                            const float rr = 1.0f / rho;
                            const float xk = kf * rho;
                            const float amp = (float)A.ws[e] * c_ampf * rr * sqrtf(rr);
                            float ps, pc;
                            sincosf(xk - 0.75f * kPiF, &ps, &pc);
                            const float ci = c_cif * rr;
                            fre += -amp * (pc * ci + ps);
                            fim += amp * (pc - ps * ci);
                        }
                    }
                    re = fre;
                    im = fim;
                } else {
                    // two-float: positions and the path length carried as (hi, lo) pairs, the
                    // phase reduced modulo 2 pi before the single-precision sincos
                    const df Xd = df_add(df_mul(two_sum((float)x - 0.5f * (float)A.W, u0), df_from(A.pitch)),
                                         two_prod((float)A.sigma, z1));
                    const df Yd = df_add(df_mul(two_sum((float)y - 0.5f * (float)A.H, u1), df_from(A.pitch)),
                                         two_prod((float)A.sigma, z2));
                    const df zz = df_from(A.z);
                    const df z2d = df_mul(zz, zz);
                    const df kd = df_from(A.k);
                    const df twopi = df_from(6.283185307179586);
                    float fre = 0.0f, fim = 0.0f;
                    for (int e = 0; e < A.n; ++e) {
                        const df dx = df_add(Xd, df_from(-A.xs[e]));
                        df r2 = df_add(z2d, df_mul(dx, dx));
                        if (A.kind == 0) r2 = df_add(r2, df_mul(Yd, Yd));
                        const df L = df_sqrt(r2);
                        const df ph = df_mul(kd, L);
                        const float nn = rintf(ph.hi * (1.0f / 6.283185307179586f));
                        const df red = df_add(ph, df_mul(df{-nn, 0.0f}, twopi));
                        const float phi = red.hi + red.lo;
                        const float Lf = L.hi;
                        const float rL = 1.0f / Lf;
                        if (A.kind == 0) {
                            float ps, pc;
                            sincosf(phi, &ps, &pc);
                            fre += pc * rL;
                            fim += ps * rL;
                        } else {
                            const float amp = (float)A.ws[e] * c_ampf * rL * sqrtf(rL);
                            float ps, pc;
                            sincosf(phi - 0.75f * kPiF, &ps, &pc);
                            const float ci = c_cif * rL;
                            fre += -amp * (pc * ci + ps);
                            fim += amp * (pc - ps * ci);
                        }
                    }
                    re = fre;
                    im = fim;
                }
            }
            acc += re * re + im * im;
        }
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (lane == 0 && pix < npix) {
        double t = 0.0;
        for (int i = 0; i < 64; ++i) t += part[wv][i];
        img[pix] = (float)(t / (double)A.spp);
    }
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = (n == 1) ? z : p1;
            const double pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace grw

extern "C" int grw_coherent_launch(const gr_coherent_desc* d, float* image, hipStream_t stream, float* ms,
                                   char* err, size_t errn) {
    using namespace grw;
    auto E = [&](const char* m) {
        std::snprintf(err, errn, "%s", m);
        return GR_E_INVALID;
    };
    if (!d || !image) return E("coherent: null argument");
    if (d->kind != 0 && d->kind != 1) return E("coherent: kind");
    if (d->n_slits < 1 || d->n_slits > 8) return E("coherent: 1..8 emitters");
    if (d->kind == 1 && (d->nodes_per_slit < 1 || d->n_slits * d->nodes_per_slit > kMaxNodes || !(d->width_um > 0)))
        return E("coherent: slit width / nodes (at most 128 nodes in total)");
    if (d->phase_mode < 0 || d->phase_mode > 2) return E("coherent: phase mode");
    if (!(d->z_um > 0) || !(d->lambda_um >= 0.1 && d->lambda_um <= 20.0)) return E("coherent: z / lambda");
    if (d->width < 1 || d->height < 1 || (int64_t)d->width * d->height > (1ll << 30)) return E("coherent: sensor size");
    if (!(d->pitch_um > 0) || !(d->sigma_um >= 0) || d->spp < 1) return E("coherent: pitch / sigma / spp");
    CohArgs a{};
    a.kind = d->kind;
    if (d->kind == 0) {
        a.n = d->n_slits;
        for (int i = 0; i < a.n; ++i) {
            a.xs[i] = d->centre_um[i];
            a.ws[i] = 1.0;
        }
    } else {
        std::vector<double> gx, gw;
        gauss_legendre(d->nodes_per_slit, gx, gw);
        a.n = d->n_slits * d->nodes_per_slit;
        for (int s = 0; s < d->n_slits; ++s)
            for (int j = 0; j < d->nodes_per_slit; ++j) {
                a.xs[s * d->nodes_per_slit + j] = d->centre_um[s] + 0.5 * d->width_um * gx[j];
                a.ws[s * d->nodes_per_slit + j] = 0.5 * d->width_um * gw[j];
            }
    }
    a.z = d->z_um;
    a.k = 2.0 * M_PI / d->lambda_um;
    a.pitch = d->pitch_um;
    a.sigma = d->sigma_um;
    a.W = d->width;
    a.H = d->height;
    a.spp = d->spp;
    a.seed = d->seed;
    const int64_t npix = (int64_t)a.W * a.H;
    const unsigned blocks = (unsigned)((npix + 3) / 4);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GR_E_DEVICE;
        (void)hipEventRecord(e0, stream);
    }
    if (d->phase_mode == GR_PHASE_FP32) hipLaunchKernelGGL(coherent_kernel<GR_PHASE_FP32>, dim3(blocks), dim3(256), 0, stream, a, image);
    else if (d->phase_mode == GR_PHASE_FP64) hipLaunchKernelGGL(coherent_kernel<GR_PHASE_FP64>, dim3(blocks), dim3(256), 0, stream, a, image);
    else hipLaunchKernelGGL(coherent_kernel<GR_PHASE_TWO_FLOAT>, dim3(blocks), dim3(256), 0, stream, a, image);
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
        std::snprintf(err, errn, "coherent launch: %s", hipGetErrorString(le));
        return GR_E_DEVICE;
    }
    if (ms) {
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) return GR_E_DEVICE;
        (void)hipEventElapsedTime(ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return GR_OK;
}
