// Composite interactions at material boundaries (Sec. "Wave-Optical Rendering", second
// practical difficulty: a generalized ray whose footprint covers several materials meets the
// composition of their interaction operators, and the waves the materials scatter interfere).
//
// The footprint meets one straight boundary, the nearest material-boundary edge of the hit's
// material within the ball that holds the ray, carried onto the tangent plane: surface
// coordinates x about the hit, near side (the hit's material) n.x < c, far side n.x > c
// (n the boundary's unit normal towards the far side, c >= 0).  p_w is the squared Fourier
// integral of the amplitude window w(x) = exp(-x^T S^-1 x / 4) times each side's reflection
// function over its half-plane, normalised like the single-material p_w, with the position
// of each deterministic profile (its phase at the boundary, which no input states) averaged:
// the orders of a side add in power and the sides interfere through their undiffracted mean
// fields.  A rough side's diffuse terms are the single-material ones weighted by the window's
// intensity mass on its side.
#pragma once

#include "trace_core.hpp"

namespace grw {

// Faddeeva function w(z) = exp(-z^2) erfc(-iz) for Im z >= 0 by Weideman's rational
// approximation (J. A. C. Weideman, "Computation of the complex error function", SIAM J.
// Numer. Anal. 31, 1994): with Z = (L + iz) / (L - iz),
//   w(z) = 2 sum_{n=1..N} a_n Z^(n-1) / (L - iz)^2 + pi^-1/2 / (L - iz),
// a_n the Fourier coefficients of exp(-t^2) (L^2 + t^2) in theta, t = L tan(theta / 2)
// (computed on the host).  N = 16: relative error below 6e-7 in float over the half-plane.
__device__ inline void faddeeva_w(float x, float y, const float (&a)[kWeidN], float L, float& wr, float& wi) {
    // D = L - iz = (L + y) - i x;  1 / D = ((L + y) + i x) / |D|^2
    const float dr = L + y;
    const float inv = 1.0f / (dr * dr + x * x);
    const float ir = dr * inv, ii = x * inv;
    // Z = (L + iz) / D with L + iz = (L - y) + i x
    const float nr = L - y, ni = x;
    const float zr = nr * ir - ni * ii, zi = nr * ii + ni * ir;
    float pr = a[kWeidN - 1], pi = 0.0f;
#pragma unroll
    for (int n = kWeidN - 2; n >= 0; --n) {
        const float tr = pr * zr - pi * zi + a[n];
        pi = pr * zi + pi * zr;
        pr = tr;
    }
    // (2 p / D + pi^-1/2) / D
    const float qr = 2.0f * (pr * ir - pi * ii) + 0.56418958354775628f;
    const float qi = 2.0f * (pr * ii + pi * ir);
    wr = qr * ir - qi * ii;
    wi = qr * ii + qi * ir;
}

// The window and one boundary in the surface frame, with what the half-plane fields reuse.
struct HalfPlane {
    float sxx, syy, sxy;     // intensity footprint covariance S (um^2)
    float nx, ny, c;         // boundary normal towards the far side and distance (um)
    float snn, sne;          // n^T S n, n^T S e  (e = (-ny, nx))
    float rsnn, rsq;         // 1 / snn, 1 / sqrt(snn)
    float along;             // det S / snn: the window's precision along the boundary
    float amp;               // sqrt(2 sqrt(det S) / pi): |whole-plane field|^2 at 0 is the peak density
    float e0;                // c^2 / (4 snn)
    float mass_far;          // the far side's share of the window's intensity
};

__device__ inline HalfPlane make_halfplane(float sxx, float syy, float sxy, float nx, float ny, float c) {
    HalfPlane H;
    H.sxx = sxx;
    H.syy = syy;
    H.sxy = sxy;
    H.nx = nx;
    H.ny = ny;
    H.c = c;
    const float ex = -ny, ey = nx;
    H.snn = nx * nx * sxx + 2.0f * nx * ny * sxy + ny * ny * syy;
    H.sne = nx * ex * sxx + (nx * ey + ny * ex) * sxy + ny * ey * syy;
    H.rsnn = 1.0f / H.snn;
    H.rsq = rsqrtf(H.snn);
    const float det = sxx * syy - sxy * sxy;
    H.along = det * H.rsnn;
    H.amp = sqrtf(2.0f * sqrtf(det) * (1.0f / kPiF));
    H.e0 = 0.25f * c * c * H.rsnn;
    H.mass_far = 0.5f * erfcf(c * H.rsq * 0.70710678118654752f);
    return H;
}

// Window fields at transfer v, normalised so that |.|^2 is a density: g over the whole plane
// (real), f over the far half-plane.  With a = n.v, b = e.v and m = a snn + b sne = n^T S v,
//   g = amp exp(-v^T S v)
//   f = amp / 2 exp(-b^2 det S / snn - c^2 / (4 snn)) exp(i c m / snn) w(m / sqrt(snn) + i c / (2 sqrt(snn)))
// (the Gaussian integral along the boundary, then the half-line integral across it).
__device__ inline void halfplane_fields(const HalfPlane& H, const BoundaryDev& B, float vx, float vy, float& g,
                                        float& fr, float& fi) {
    const float a = H.nx * vx + H.ny * vy, b = -H.ny * vx + H.nx * vy;
    const float m = a * H.snn + b * H.sne;
    const float vsv = H.sxx * vx * vx + 2.0f * H.sxy * vx * vy + H.syy * vy * vy;
    g = H.amp * __expf(-vsv);
    const float ex = -b * b * H.along - H.e0;
    fr = fi = 0.0f;
    if (ex < -80.0f) return;
    float wr, wi;
    faddeeva_w(m * H.rsq, 0.5f * H.c * H.rsq, B.weid, B.weid_L, wr, wi);
    float sn, cs;
    sincosf(H.c * m * H.rsnn, &sn, &cs);
    const float mag = 0.5f * H.amp * __expf(ex);
    fr = mag * (cs * wr - sn * wi);
    fi = mag * (sn * wr + cs * wi);
}

// p_w (um^2) of the composite interaction.  near, far: the two sides' materials with their
// grating directions (gnx, gny), (gfx, gfy) in the frame; other arguments as pw_plain.
__device__ inline float pw_composite(const DMat& near, float gnx, float gny, const DMat& far, float gfx,
                                           float gfy, float k, float kix, float kiy, float kox, float koy,
                                           const HalfPlane& H, const BoundaryDev& B) {
    const float ik2 = 1.0f / (k * k);
    const float ni = (kix * kix + kiy * kiy) * ik2;
    const float no = (kox * kox + koy * koy) * ik2;
    if (ni >= 1.0f || no >= 1.0f) return 0.0f;
    const float qz = k * (sqrtf(1.0f - ni) + sqrtf(1.0f - no));
    const float kx = kox - kix, ky = koy - kiy;
    float total = 0.0f;
    float mr0 = 0.0f, mi0 = 0.0f, mr1 = 0.0f, mi1 = 0.0f;   // the sides' mean fields
#pragma nounroll
    for (int s = 0; s < 2; ++s) {
        const DMat& M = s == 0 ? near : far;
        const float gx = s == 0 ? gnx : gfx, gy = s == 0 ? gny : gfy;
        const float sr = sqrtf(M.refl);
        if (M.kind == MAT_GRATING) {
            const float K = kTwoPiF / M.L;
            const float mm = qz * M.h;
            // orders beyond |m| + 10 carry J_j(m)^2 < 1e-13 of the total here
            const int J = min((int)ceilf(fabsf(mm)) + 10, 64);
#pragma nounroll
            for (int j = -J; j <= J; ++j) {
                const float vx = kx + (float)j * K * gx, vy = ky + (float)j * K * gy;
                // an order whose whole-plane field and half-plane field both vanish (its lobe
                // and its boundary streak both far from kappa) adds nothing
                const float bb = -H.ny * vx + H.nx * vy;
                if (H.sxx * vx * vx + 2.0f * H.sxy * vx * vy + H.syy * vy * vy > 80.0f &&
                    bb * bb * H.along + H.e0 > 80.0f && j != 0)
                    continue;
                const float bj = bessel_jn(abs(j), mm);
                float g, fr, fi;
                halfplane_fields(H, B, vx, vy, g, fr, fi);
                const float hr = s == 0 ? g - fr : fr, hi = s == 0 ? -fi : fi;
                total += M.refl * bj * bj * (hr * hr + hi * hi);
                if (j == 0) {
                    if (s == 0) {
                        mr0 = sr * bj * hr;
                        mi0 = sr * bj * hi;
                    } else {
                        mr1 = sr * bj * hr;
                        mi1 = sr * bj * hi;
                    }
                }
            }
        } else {
            float g, fr, fi;
            halfplane_fields(H, B, kx, ky, g, fr, fi);
            const float hr = s == 0 ? g - fr : fr, hi = s == 0 ? -fi : fi;
            const float gg = M.kind == MAT_ROUGH ? qz * qz * M.h * M.h : 0.0f;
            const float spec = __expf(-gg);
            total += M.refl * spec * (hr * hr + hi * hi);
            const float amp = sr * __expf(-0.5f * gg);
            if (s == 0) {
                mr0 = amp * hr;
                mi0 = amp * hi;
            } else {
                mr1 = amp * hr;
                mi1 = amp * hi;
            }
            if (M.kind == MAT_ROUGH && gg >= 1e-12f) {
                // diffuse terms n >= 1: the single-material series less its specular term,
                // weighted by this side's window mass
                const float det = H.sxx * H.syy - H.sxy * H.sxy;
                const float idet = 0.25f / det;
                const float full = pw_plain(MAT_ROUGH, M.h, M.L, M.refl, k, kix, kiy, kox, koy, H.sxx, H.syy,
                                            H.sxy, 1.0f, 0.0f);
                const float specn = M.refl * spec * gauss2(kx, ky, H.syy * idet, H.sxx * idet, -H.sxy * idet);
                total += (s == 0 ? 1.0f - H.mass_far : H.mass_far) * fmaxf(full - specn, 0.0f);
            }
        }
    }
    return fmaxf(0.0f, total + 2.0f * (mr0 * mr1 + mi0 * mi1));
}

// The boundary a hit meets, if any: the nearest boundary edge of the hit's material (listed
// for the hit's triangle, original index tri) within min(2.5 beta_max, reach) of the hit P,
// beta_max = sqrt(2) times the footprint's largest standard deviation (the ball that holds the
// generalized ray); equal distances go to the lower edge id.  Carried onto the tangent plane
// (xa, ya): the boundary's unit normal towards the far side (the side of the far triangle's
// third vertex) and its distance c >= 0 from the hit.  Fills the far side's material, its
// grating direction in the frame and the half-plane.  False when there is none, or when the
// edge is seen end-on.
__device__ inline bool find_boundary(const BoundaryDev& B, int tri, int mat, const d3& P, const f3& xa,
                                     const f3& ya, float sxx, float syy, float sxy, const DMat* mats, int& fmat,
                                     float& gfx, float& gfy, HalfPlane& H) {
    const uint4 L = B.tri_list[tri];
    if (L.y == 0u) return false;
    const float lmax = 0.5f * (sxx + syy) + sqrtf(0.25f * (sxx - syy) * (sxx - syy) + sxy * sxy);
    const float rad = fminf(2.5f * sqrtf(2.0f * lmax) * 1e-6f, B.reach_m);
    if (rad <= __uint_as_float(L.z)) return false;   // every listed edge is farther than rad
    float best_d = rad;
    int best = -1;
    for (uint32_t i = 0; i < L.y; ++i) {
        const uint32_t e = B.idx[L.x + i];
        const float4 p0 = B.edges[4 * e], p1 = B.edges[4 * e + 1];
        // the segment's ends relative to P (metres), each rounded once; where the nearest point
        // is an end, the distance is that end's own, so edges meeting at a vertex tie exactly
        // there and the lower id wins
        const f3 a = -1.0f * diff_f3(P, mk3(p0.x, p0.y, p0.z));
        const f3 b = -1.0f * diff_f3(P, mk3(p1.x, p1.y, p1.z));
        const f3 ab = b - a;
        const float l2 = dot3(ab, ab);
        const float t = l2 > 0.0f ? -dot3(a, ab) / l2 : 0.0f;
        const f3 q = !(t > 0.0f) ? a : (t >= 1.0f ? b : a + t * ab);
        const float dd = sqrtf(dot3(q, q));
        if (dd < best_d) {
            best_d = dd;
            best = (int)e;
        }
    }
    if (best < 0 || !(sxx * syy - sxy * sxy > 0.0f)) return false;
    const float4 p0 = B.edges[4 * best], p1 = B.edges[4 * best + 1];
    const int fs = __float_as_int(p0.w) == mat ? 1 : 0;   // the far side: the other material
    fmat = __float_as_int(fs ? p1.w : p0.w);
    const float4 qv = B.edges[4 * best + 2 + fs];
    const f3 a3 = -1.0f * diff_f3(P, mk3(p0.x, p0.y, p0.z));
    const f3 b3 = -1.0f * diff_f3(P, mk3(p1.x, p1.y, p1.z));
    const f3 q3 = -1.0f * diff_f3(P, mk3(qv.x, qv.y, qv.z));
    const float ax = dot3(a3, xa) * 1e6f, ay = dot3(a3, ya) * 1e6f;   // um
    const float ex = dot3(b3, xa) * 1e6f - ax, ey = dot3(b3, ya) * 1e6f - ay;
    const float qx = dot3(q3, xa) * 1e6f - ax, qy = dot3(q3, ya) * 1e6f - ay;
    const float el = sqrtf(ex * ex + ey * ey);
    const f3 seg = b3 - a3;
    if (!(el > 1e-6f * sqrtf(dot3(seg, seg)) * 1e6f)) return false;   // edge seen end-on
    float nx = -ey / el, ny = ex / el;
    if (nx * qx + ny * qy < 0.0f) {
        nx = -nx;
        ny = -ny;
    }
    const float c = fmaxf(0.0f, nx * ax + ny * ay);
    const DMat& fm = mats[fmat];
    gfx = 1.0f;
    gfy = 0.0f;
    if (fm.kind == MAT_GRATING) {
        const f3 gd = mk3(fm.gx, fm.gy, fm.gz);
        const float gx = dot3(gd, xa), gy = dot3(gd, ya), gl = sqrtf(gx * gx + gy * gy);
        if (gl > 1e-9f) {
            gfx = gx / gl;
            gfy = gy / gl;
        }
    }
    H = make_halfplane(sxx, syy, sxy, nx, ny, c);
    return true;
}

}  // namespace grw
