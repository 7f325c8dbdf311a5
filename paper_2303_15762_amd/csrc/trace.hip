// Backward generalized-ray path tracing on gfx950: one persistent kernel per trace.
//
// Each wave keeps 64 paths in registers.  Lanes whose path ended are refilled together: a
// ballot of the dead lanes, one atomic on the global path dispenser per wave, and the lane's
// rank among the dead lanes (mbcnt) as its offset.  Every iteration advances each live path by
// one segment: closest hit (4-wide BVH, per-lane stack in LDS), free-space update of the
// generalized ray, measurement by next-event estimation, continuation sampling.  Paths write
// one float each; a second kernel sums them per pixel in a fixed order, so the image does not
// depend on scheduling.
//
// Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762),
// Algorithm 1 under the interactive assumption of Sec. "Interactive Rendering".
#include <algorithm>

#include "composite.hpp"

namespace grw {

// Member i of a per-member register array.  Loops over the members that call a large function
// stay rolled, so that the kernel holds one copy of it; a chain of selects keeps the arrays in
// registers there (an indexed access would move them to scratch memory).
__device__ __forceinline__ float pick4(const float (&a)[4], int i) {
    return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

// Hero-wavelength continuation: the hero (member hs, wavenumber kh) sampled (kox, koy) with
// weight wgt through component comp (a grating order with probability ph) from the incident
// (kix, kiy); every member's value ratio f / p_h multiplies T and its density ratio p / p_h
// multiplies R.  A common factor of all T and R leaves the balance-heuristic estimates
// unchanged, so R is renormalised to max 1 (and the specular ratio exp(g_h - g_c) is formed
// relative to the largest member) to keep both in FP32 range.
__device__ inline void hero_continuation(const DMat& m, float kh, const float (&mk)[4], int hs, float kix,
                                         float kiy, float ci, float kox, float koy, float wgt, int comp,
                                         float ph, float (&T)[4], float (&R)[4]) {
    const float ux = kix / kh, uy = kiy / kh;
    float rf[4], rp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        rf[i] = 0.0f;
        rp[i] = 0.0f;
    }
    if (m.kind == MAT_SMOOTH) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            rf[i] = m.refl;
            rp[i] = 1.0f;
        }
    } else if (m.kind == MAT_GRATING) {
        if (comp == 0) {   // ph: the hero's probability of order 0
#pragma nounroll
            for (int i = 0; i < 4; ++i) {
                if (i == hs) continue;
                const float ki = pick4(mk, i);
                float Wc, w0c;
                grating_weights(m, ki, ki * ux, ki * uy, ci, Wc, w0c);
                const float f = m.refl * w0c / ph, p = (Wc > 0.0f ? w0c / Wc : 0.0f) / ph;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j == i) {
                        rf[j] = f;
                        rp[j] = p;
                    }
                }
            }
        }
    } else if (comp == 0) {
        const float c2h2 = 4.0f * ci * ci * m.h * m.h;
        const float gh = kh * kh * c2h2;
        float lr[4], mx = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            lr[i] = gh - mk[i] * mk[i] * c2h2;
            if (i != hs) mx = fmaxf(mx, lr[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            rp[i] = __expf((i == hs ? 0.0f : lr[i]) - mx);
            rf[i] = m.refl * rp[i];
        }
        wgt *= rp[hs];   // the hero's share of the common factor exp(-mx)
    } else {
        const float du2 = ((kox - kix) * (kox - kix) + (koy - kiy) * (koy - kiy)) / (kh * kh);
        float dn[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // lobe densities; mk[hs] is kh
#pragma nounroll
        for (int i = 0; i < 4; ++i) {
            const float di = rough_lobe_density(pick4(mk, i), ci, m.h, m.L, du2);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j == i) dn[j] = di;
            }
        }
        const float dh = pick4(dn, hs);
        if (dh > 0.0f) {
            const float idh = 1.0f / dh;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i == hs) continue;
                rp[i] = dn[i] * idh;
                rf[i] = m.refl * rp[i];
            }
        }
    }
    float rmax = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i == hs) {
            T[i] *= wgt;
            R[i] *= m.kind == MAT_ROUGH && comp == 0 ? rp[i] : 1.0f;
        } else {
            T[i] *= rf[i];
            R[i] *= rp[i];
        }
        rmax = fmaxf(rmax, R[i]);
    }
    const float inv = 1.0f / rmax;   // R of the hero > 0
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T[i] *= inv;
        R[i] *= inv;
    }
}

// The members' ratios at a composite interaction (reading R31): the hero sampled the side
// far_chosen (probability its far mass) and then that side's kernel, so member i meets the
// mixture (1 - m_i) f_near + m_i f_far and the hero's density is (1 - m_h) p_near + m_h p_far.
// The sampled direction is of one class, and only that class's components count: specular
// (smooth, a rough surface's term 0 with probability e^-g, a grating's order 0 with
// probability J_0(m_0)^2 / W: shared by every wavelength), a rough lobe (terms n >= 1, a density
// over u_o), or a grating order j != 0 of the sampled side (dispersive: the hero's alone, whose
// ratio is then its sampler's weight).  Member i's window is the hero's scaled by its beta^2,
// so its far mass is erfc(c / sqrt(2 snn_i)) / 2 with snn_i = snn_h beta_i^2 / beta_h^2.
// (kix, kiy): the hero's incident tangential wavevector and (kox, koy) the sampled one, both in
// the near side's frame; (gfx, gfy): a far grating's direction in that frame.
__device__ inline void hero_composite_continuation(const DMat& m, const DMat& fm, float gfx, float gfy,
                                                   bool far_chosen, float snn_h, float c, const float (&mb2)[4],
                                                   float kh, const float (&mk)[4], int hs, float kix, float kiy,
                                                   float ci, float kox, float koy, int comp, float wgt,
                                                   float (&T)[4], float (&R)[4]) {
    const DMat& cm = far_chosen ? fm : m;
    if (cm.kind == MAT_GRATING && comp != 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i == hs) {
                T[i] *= wgt;
            } else {
                T[i] = 0.0f;
                R[i] = 0.0f;
            }
        }
    } else {
        const bool spec = cm.kind == MAT_SMOOTH || comp == 0;
        const float ux = kix / kh, uy = kiy / kh;
        const float du2 = ((kox - kix) * (kox - kix) + (koy - kiy) * (koy - kiy)) / (kh * kh);
        const float b2h = pick4(mb2, hs);
        float f[4] = {0.0f, 0.0f, 0.0f, 0.0f}, p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma nounroll
        for (int i = 0; i < 4; ++i) {
            const float ki = pick4(mk, i);
            const float snn = snn_h * pick4(mb2, i) / b2h;
            const float af = 0.5f * erfcf(c * rsqrtf(snn) * 0.70710678118654752f);
            float fi = 0.0f, pi = 0.0f;
#pragma nounroll
            for (int sd = 0; sd < 2; ++sd) {
                const DMat& M = sd == 0 ? m : fm;
                const float a = sd == 0 ? 1.0f - af : af;
                float ps = 0.0f, fs = 0.0f;
                if (spec) {
                    if (M.kind == MAT_SMOOTH) {
                        ps = 1.0f;
                        fs = M.refl;
                    } else if (M.kind == MAT_ROUGH) {
                        ps = __expf(-4.0f * ki * ki * ci * ci * M.h * M.h);
                        fs = M.refl * ps;
                    } else {
                        // the grating's own frame (its direction along x): the far side's rotated
                        const float rx = sd == 0 ? 1.0f : gfx, ry = sd == 0 ? 0.0f : gfy;
                        float W, w0;
                        grating_weights(M, ki, ki * (rx * ux + ry * uy), ki * (-ry * ux + rx * uy), ci, W, w0);
                        ps = W > 0.0f ? w0 / W : 0.0f;
                        fs = M.refl * w0;
                    }
                } else if (M.kind == MAT_ROUGH) {
                    ps = rough_lobe_density(ki, ci, M.h, M.L, du2);
                    fs = M.refl * ps;
                }
                pi += a * ps;
                fi += a * fs;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j == i) {
                    f[j] = fi;
                    p[j] = pi;
                }
            }
        }
        const float ph = pick4(p, hs);
        if (ph > 0.0f) {
            const float iph = 1.0f / ph;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T[i] *= f[i] * iph;
                R[i] = i == hs ? R[i] : R[i] * p[i] * iph;
            }
        } else {
            // the hero's density underflows FP32 (a far lobe tail): the hero keeps its sampler's
            // weight and the companions are dropped, as in hero_continuation
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i == hs) {
                    T[i] *= wgt;
                } else {
                    T[i] = 0.0f;
                    R[i] = 0.0f;
                }
            }
        }
    }
    float rmax = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) rmax = fmaxf(rmax, R[i]);
    const float inv = rmax > 0.0f ? 1.0f / rmax : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T[i] *= inv;
        R[i] *= inv;
    }
}

// DEFER: rough-surface measurements inside the learned model's domain are not evaluated here;
// their encoded queries go to a queue that one batched matrix-core kernel evaluates after the
// trace (its results are added to the path records in a fixed order).
// HERO: each path carries the four wavelengths of a rotation group of the grid (indices
// g + i nl/4), sampled at the hero member drawn at sourcing; every member keeps its own beta,
// rho and footprint, and its estimate is 4 T_i q_i M_i / sum_k R_k q_k (one-sample balance
// heuristic over the hero choices), with q the members' emitter-sampling densities relative
// to the hero's and M the measurement.
// All instantiations ask for 4 waves per SIMD (128 VGPRs): a few path-state values spill to
// scratch, which costs less than the latency hidden by the fourth wave.
// ------------------------------------------------------------------------------------------
// Anisotropic generalized rays (Sec. "Generalized rays": beta, rho may be positive-definite
// matrices).  The ray's phase-space Gaussian over the two axes transverse to its mean direction
// is kept as its second moments Srr (symmetric), Srk, Skk (symmetric) in the transverse frame
// of the direction; the scalar ray is Srr = beta^2 I, Srk = rho I, Skk = (1 + rho^2) / beta^2 I,
// and free space (eq. K_free_space_propagation) is the shear r -> r + zbar k of these moments.
// An interaction carries the incoming transverse plane onto the surface along the incoming
// direction and the surface onto the outgoing transverse plane: positions map by that 2x2 G,
// wavevectors by G^-T (tangential wavevector deviations are conserved).
// ------------------------------------------------------------------------------------------
struct AnisoRay {
    float rr[3];   // Srr: xx, xy, yy
    float rk[4];   // Srk: xx, xy, yx, yy
    float kk[3];   // Skk: xx, xy, yy
};

// Orthonormal basis of the plane normal to the unit vector d (Duff et al., "Building an
// Orthonormal Basis, Revisited", JCGT 6(1), 2017).
__device__ __forceinline__ void transverse_frame(const f3& d, f3& e1, f3& e2) {
    const float sg = d.z >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (sg + d.z), b = d.x * d.y * a;
    e1 = mk3(1.0f + sg * d.x * d.x * a, sg * b, -sg * d.x);
    e2 = mk3(b, sg + d.y * d.y * a, -d.y);
}

__device__ __forceinline__ void aniso_iso(AnisoRay& R, float beta2) {
    R.rr[0] = R.rr[2] = beta2;
    R.rr[1] = 0.0f;
    R.rk[0] = R.rk[1] = R.rk[2] = R.rk[3] = 0.0f;
    R.kk[0] = R.kk[2] = 1.0f / beta2;
    R.kk[1] = 0.0f;
}

// Free space over zbar = z / k: Srr += zbar (Srk + Srk^T) + zbar^2 Skk, Srk += zbar Skk.
__device__ __forceinline__ void aniso_free(AnisoRay& R, float zb) {
    const float z2 = zb * zb;
    R.rr[0] += zb * (2.0f * R.rk[0]) + z2 * R.kk[0];
    R.rr[1] += zb * (R.rk[1] + R.rk[2]) + z2 * R.kk[1];
    R.rr[2] += zb * (2.0f * R.rk[3]) + z2 * R.kk[2];
    R.rk[0] += zb * R.kk[0];
    R.rk[1] += zb * R.kk[1];
    R.rk[2] += zb * R.kk[1];
    R.rk[3] += zb * R.kk[2];
}

// The 2x2 map from the transverse frame of di onto the surface (normal n) along di, expressed
// in the basis (t0, t1) (the outgoing transverse frame, or the surface's tangent frame).
__device__ __forceinline__ void onto_surface_map(const f3& di, const f3& n, const f3& t0, const f3& t1,
                                                 float (&G)[2][2]) {
    f3 e[2];
    transverse_frame(di, e[0], e[1]);
    const float ind = 1.0f / dot3(n, di);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const f3 sp = e[b] - (dot3(n, e[b]) * ind) * di;
        G[0][b] = dot3(t0, sp);
        G[1][b] = dot3(t1, sp);
    }
}

__device__ inline void aniso_interact(AnisoRay& R, const f3& di, const f3& dout, const f3& n) {
    f3 eo0, eo1;
    transverse_frame(dout, eo0, eo1);
    float G[2][2];
    onto_surface_map(di, n, eo0, eo1, G);
    const float det = G[0][0] * G[1][1] - G[0][1] * G[1][0];   // +-cos(o) / cos(i)
    if (!(fabsf(det) > 1e-6f)) return;   // a continuation along the surface: the map is singular
    const float idet = 1.0f / det;
    const float Gi[2][2] = {{G[1][1] * idet, -G[0][1] * idet}, {-G[1][0] * idet, G[0][0] * idet}};
    const float rr[2][2] = {{R.rr[0], R.rr[1]}, {R.rr[1], R.rr[2]}};
    const float rk[2][2] = {{R.rk[0], R.rk[1]}, {R.rk[2], R.rk[3]}};
    const float kk[2][2] = {{R.kk[0], R.kk[1]}, {R.kk[1], R.kk[2]}};
    float grr[2][2], grk[2][2], gkk[2][2];   // G Srr, G Srk, Gi^T Skk
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            grr[i][j] = G[i][0] * rr[0][j] + G[i][1] * rr[1][j];
            grk[i][j] = G[i][0] * rk[0][j] + G[i][1] * rk[1][j];
            gkk[i][j] = Gi[0][i] * kk[0][j] + Gi[1][i] * kk[1][j];
        }
    R.rr[0] = grr[0][0] * G[0][0] + grr[0][1] * G[0][1];
    R.rr[1] = grr[0][0] * G[1][0] + grr[0][1] * G[1][1];
    R.rr[2] = grr[1][0] * G[1][0] + grr[1][1] * G[1][1];
    R.rk[0] = grk[0][0] * Gi[0][0] + grk[0][1] * Gi[1][0];
    R.rk[1] = grk[0][0] * Gi[0][1] + grk[0][1] * Gi[1][1];
    R.rk[2] = grk[1][0] * Gi[0][0] + grk[1][1] * Gi[1][0];
    R.rk[3] = grk[1][0] * Gi[0][1] + grk[1][1] * Gi[1][1];
    R.kk[0] = gkk[0][0] * Gi[0][0] + gkk[0][1] * Gi[1][0];
    R.kk[1] = gkk[0][0] * Gi[0][1] + gkk[0][1] * Gi[1][1];
    R.kk[2] = gkk[1][0] * Gi[0][1] + gkk[1][1] * Gi[1][1];
}

// Footprint covariance in the surface frame (xa, ya): Srr / 2 carried onto the surface along d.
__device__ __forceinline__ void aniso_footprint(const AnisoRay& R, const f3& d, const f3& n, const f3& xa,
                                                const f3& ya, float& sxx, float& syy, float& sxy) {
    float H[2][2];
    onto_surface_map(d, n, xa, ya, H);
    const float h0[2] = {H[0][0] * R.rr[0] + H[0][1] * R.rr[1], H[0][0] * R.rr[1] + H[0][1] * R.rr[2]};
    const float h1[2] = {H[1][0] * R.rr[0] + H[1][1] * R.rr[1], H[1][0] * R.rr[1] + H[1][1] * R.rr[2]};
    sxx = 0.5f * (h0[0] * H[0][0] + h0[1] * H[0][1]);
    sxy = 0.5f * (h0[0] * H[1][0] + h0[1] * H[1][1]);
    syy = 0.5f * (h1[0] * H[1][0] + h1[1] * H[1][1]);
}

// COMPOSITE: where a material boundary of the hit's material lies within the ball holding the
// generalized ray, the measurement uses the composite p_w of the two sides and the
// continuation samples one side's kernel with the probability of its window mass.
template <int STACK, bool DEFER, bool HERO, bool ANISO = false, bool COMPOSITE = false>
__global__ __launch_bounds__(256, 4) void trace_kernel(const TraceArgs A) {
    __shared__ __attribute__((aligned(16))) int lds_stack[4][STACK][64];
    // the top levels of the BVH, read by every closest-hit query
    __shared__ float4 lds_nodes[kLdsNodes * 8];
    const int nln = stage_top_nodes(A.scene, lds_nodes);
    const lds_v4f* top = (const lds_v4f*)&lds_nodes[0];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    lds_int* stk = (lds_int*)&lds_stack[wv][0][lane];
    // the traversal's (child, key) pairs over the same wave-private region (the shading code
    // uses the lane's column of it as a cache between traversals)
    lds_v2i* stk2 = (lds_v2i*)&lds_stack[wv][0][0] + lane;
    // the child-code scratch: 16 contiguous bytes per lane in the last two entries' space
    lds_v4i* scr = (lds_v4i*)&lds_stack[wv][STACK - 4][0] + lane;
    // this wave's slice of the traversal-stack overflow (uniform; the lane adds its id)
    const size_t ostride = (size_t)gridDim.x * 256;
    v2i_t* ovf = A.ovf ? (v2i_t*)A.ovf + ((size_t)blockIdx.x * 256 + 64 * __builtin_amdgcn_readfirstlane(wv)) : nullptr;

    const SensorDev& sen = A.sensor;
    const uint32_t Wd = (uint32_t)sen.W, Hd = (uint32_t)sen.H, nl = (uint32_t)A.nl;
    // SHQ: shadow rays are queued for shadow_kernel (full waves of shadow rays instead of the
    // few lanes of a wave that measure at a vertex); a path's measurement values wait in its
    // (path, interaction) slots, and a merge writes the record once visibility is known.
    // DEFER (learned p_w) queues in-domain rough measurements for the batched network, whose
    // results land in the same slots before the shadow rays are traced.
    // Hero-wavelength paths store the four members' values per slot (four floats).
    constexpr bool SHQ = true;

    bool live = false, exhausted = false;
    uint64_t idx = 0, pid = 0;
    int depth = 0, prev = -1;
    d3 o = d3{0.0, 0.0, 0.0};
    // the path's direction, in double: it is renewed at every interaction from the double
    // shading normal, so that direction errors do not build up along chains of reflections
    d3 dd = d3{0.0, 0.0, 1.0};
    float beta2 = 1.0f, rho = 0.0f, alpha = 1.0f, k = 1.0f;
    AnisoRay ar;   // ANISO: the ray's second moments (beta2, rho unused)
    if constexpr (ANISO) aniso_iso(ar, 1.0f);
    // hero-wavelength members: wavenumber, beta^2, rho, T = f / p_h, R = p / p_h, estimate
    constexpr int NM = HERO ? 4 : 1;
    float mk[NM], mb2[NM], mrho[NM], mT[NM], mR[NM];
    int hs = 0;
#pragma unroll
    for (int i = 0; i < NM; ++i) mk[i] = mb2[i] = mrho[i] = mT[i] = mR[i] = 0.0f;
    // traversal work per lane; the per-path events are flagged per lane (one bit each) and
    // counted per wave with ballots, which keeps the counts in scalar registers
    uint32_t c_nodes = 0, c_tris = 0;
    // (32-bit: a launch holds at most 2^30 (path, interaction) slots, so no count of it reaches
    // 2^31; the narrower counters leave scalar registers to the rest of the kernel)
    uint32_t w_cnt[EV_COUNT] = {};

    while (true) {
        uint32_t ev = 0;
        if (!exhausted) {
            const unsigned long long need = __ballot(!live);
            if (need) {
                const int first = __ffsll((long long)need) - 1;
                const unsigned cnt = (unsigned)__popcll(need);
                unsigned long long base = 0;
                if (lane == first) base = atomicAdd(A.counter, (unsigned long long)cnt);
                base = __shfl(base, first);
                if (base + cnt >= A.n_paths) exhausted = true;   // n_paths: paths of this launch
                if (!live) {
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                    const uint64_t my = A.path_begin + base + rank;
                    if (base + rank < A.n_paths) {
                        // Sourcing (Sec. "Interactive Rendering"): mean position uniform on the
                        // pixel, mean direction the sensor axis, beta^2 = 2 sigma^2, rho = 0,
                        // alpha = 1.
                        idx = my;
                        const uint64_t sl = my / A.per_sample;
                        const uint32_t rem = (uint32_t)(my - sl * A.per_sample);
                        // hero paths: w is the rotation group, G = nl / 4 groups
                        const uint32_t nw = HERO ? (nl >> 2) : nl;
                        const uint32_t w = rem % nw;
                        const uint32_t pix = rem / nw;
                        const uint32_t x = pix % Wd, y = pix / Wd;
                        const uint64_t s_abs = (uint64_t)A.spp_begin + sl;
                        pid = ((s_abs * Hd + y) * Wd + x) * nw + w;
                        const uint4 r0 = draw(pid, 0, STREAM_SOURCE, A.seed);
                        if constexpr (HERO) {
                            hs = (int)(r0.w >> 30);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                mk[i] = kTwoPiF / A.lambda[w + i * nw];
                                if (i == hs) k = mk[i];
                            }
                        } else {
                            k = kTwoPiF / A.lambda[w];
                        }
                        const double fx = ((double)x + (double)unif(r0.x)) * (double)sen.pitch;
                        const double fy = ((double)y + (double)unif(r0.y)) * (double)sen.pitch;
                        o = d3{sen.o[0] + fx * sen.u[0] + fy * sen.v[0], sen.o[1] + fx * sen.u[1] + fy * sen.v[1],
                               sen.o[2] + fx * sen.u[2] + fy * sen.v[2]};
                        dd = d3{(double)sen.d[0], (double)sen.d[1], (double)sen.d[2]};
                        const f3 d = to_f3(dd);
                        beta2 = 2.0f * sen.sigma_um * sen.sigma_um;
                        rho = 0.0f;
                        // start where the ray enters the scene bounds, so that the float
                        // ray/triangle arithmetic works on in-scene rather than sensor
                        // distances; the free-space law composes, so the skipped stretch is
                        // propagated here
                        const float tadv = scene_entry(A.scene, o, d);
                        if constexpr (HERO) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                mb2[i] = beta2;
                                mrho[i] = 0.0f;
                                mT[i] = 1.0f;
                                mR[i] = 1.0f;
                                if (tadv > 0.0f) {
                                    const float zb = tadv * 1e6f / mk[i];
                                    mrho[i] = zb / beta2;
                                    mb2[i] = beta2 + zb * zb / beta2;
                                }
                            }
                        }
                        if constexpr (ANISO) aniso_iso(ar, beta2);
                        if (tadv > 0.0f) {
                            o = d3{o.x + (double)tadv * dd.x, o.y + (double)tadv * dd.y, o.z + (double)tadv * dd.z};
                            const float zb = tadv * 1e6f / k;
                            if constexpr (ANISO) {
                                aniso_free(ar, zb);
                            } else {
                                rho = zb / beta2;
                                beta2 = beta2 + zb * zb / beta2;
                            }
                        }
                        alpha = 1.0f;
                        depth = 0;
                        prev = -1;
                        live = true;
                        ev |= 1u << EV_PATH;
                    }
                }
            }
        }
        if (!__any(live)) break;

        // ---- one segment of every live path ------------------------------------------
        bool finish = false;
        bool wrote = false;   // SHQ: this vertex stored its measurement slot
        if (live) {
        ev |= 1u << EV_SEG;
        const f3 d = to_f3(dd);
        RayT ray;
        ray_setup(ray, o, d);
        const float tmin = 1e-7f * (1.0f + maxabs3(to_f3(o)));
        float thit = FLT_MAX, bu = 0.0f, bv = 0.0f;
        const int tri = traverse<STACK>(A.scene, ray, tmin, thit, false, prev, stk2, scr, A.lds_cap, ovf, ostride, c_nodes, c_tris, bu, bv,
                                        top, nln);
        if (tri < 0) {
            finish = true;
        } else {
            const float4* T = A.scene.tris + (size_t)tri * 3;
            const float4 v0 = T[0], v1 = T[1], v2 = T[2];
            double t64;
            double bu64 = (double)bu, bv64 = (double)bv;
            refine_hit(o, dd, v0, v1, v2, thit, bu64, bv64, t64);
            // Free-space propagation of the generalized ray (eq. K_free_space_propagation)
            // over the hit distance, zbar = z / |k0|, pre-update beta and rho on the right.
            if constexpr (HERO) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float zb = thit * 1e6f / mk[i];
                    const float orr = 1.0f + mrho[i] * mrho[i];
                    const float rho_n = mrho[i] + zb * orr / mb2[i];
                    mb2[i] = mb2[i] + zb * (2.0f * mrho[i] + zb * orr / mb2[i]);
                    mrho[i] = rho_n;
                }
            } else if constexpr (ANISO) {
                aniso_free(ar, thit * 1e6f / k);
            } else {
                // the free-space law with hardware reciprocals (1 ulp): beta and rho only scale
                // footprints and values
                const float zb = thit * 1e6f * __builtin_amdgcn_rcpf(k);
                const float orr = 1.0f + rho * rho;
                const float q = zb * orr * __builtin_amdgcn_rcpf(beta2);
                const float rho_n = rho + q;
                beta2 = beta2 + zb * (2.0f * rho + q);
                rho = rho_n;
            }
            const d3 P = d3{o.x + t64 * dd.x, o.y + t64 * dd.y, o.z + t64 * dd.z};
            prev = __float_as_int(v0.w);
            const DMat m = A.scene.mats[__float_as_int(v1.w)];
            f3 ng = normalize3(cross3(mk3(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z),
                                      mk3(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z)));
            // shading normal in double (barycentric interpolation of the vertex normals)
            d3 nsd = d3{(double)ng.x, (double)ng.y, (double)ng.z};
            {
                const float4* NN = A.scene.tnorm + (size_t)tri * 3;
                const float4 n0 = NN[0], n1 = NN[1], n2 = NN[2];
                if ((n0.x != 0.f || n0.y != 0.f || n0.z != 0.f) && (n1.x != 0.f || n1.y != 0.f || n1.z != 0.f) &&
                    (n2.x != 0.f || n2.y != 0.f || n2.z != 0.f)) {
                    const double w0 = 1.0 - bu64 - bv64;
                    const d3 sn = d3{w0 * n0.x + bu64 * n1.x + bv64 * n2.x, w0 * n0.y + bu64 * n1.y + bv64 * n2.y,
                                     w0 * n0.z + bu64 * n1.z + bv64 * n2.z};
                    const double r = 1.0 / sqrt(sn.x * sn.x + sn.y * sn.y + sn.z * sn.z);
                    nsd = d3{sn.x * r, sn.y * r, sn.z * r};
                }
            }
            if (dot3(d, ng) > 0.0f) ng = -1.0f * ng;
            if (nsd.x * ng.x + nsd.y * ng.y + nsd.z * ng.z < 0.0) nsd = d3{-nsd.x, -nsd.y, -nsd.z};
            const f3 ns = to_f3(nsd);
            const double cid = -(dd.x * nsd.x + dd.y * nsd.y + dd.z * nsd.z);
            // the float cosine for the float arithmetic below (footprint, p_w, sampling).  The
            // path ends at an incidence cosine of 1e-6 or less: the footprint, stretched by
            // 1 / cos along the plane of incidence, is then no longer small against the
            // geometry (and its float covariance would overflow)
            const float ci = -dot3(d, ns);
            if (!(cid > 1e-6) || !(ci > 1e-6f)) {
                ev |= 1u << EV_BACKFACING;
                finish = true;
            } else {
                // Tangent frame: x = grating direction (gratings), else the travel direction
                // projected onto the surface.
                f3 xa = mk3(0, 0, 0);
                bool have = false;
                if (m.kind == MAT_GRATING) {
                    const f3 g = mk3(m.gx, m.gy, m.gz);
                    const f3 t = g - dot3(g, ns) * ns;
                    if (dot3(t, t) > 1e-18f) {
                        xa = normalize3(t);
                        have = true;
                    }
                }
                if (!have) {
                    const f3 t = d - dot3(d, ns) * ns;
                    if (dot3(t, t) > 1e-24f) {
                        xa = normalize3(t);
                    } else {
                        const f3 a = fabsf(ns.x) < 0.9f ? mk3(1, 0, 0) : mk3(0, 1, 0);
                        xa = normalize3(cross3(ns, a));
                    }
                }
                const f3 ya = cross3(ns, xa);
                // Footprint on the surface: beam variance beta^2/2, stretched by 1/cos along
                // the plane of incidence.
                // (hero paths: the hero's own window, for the boundary search)
                float b2w = beta2;
                if constexpr (HERO) b2w = pick4(mb2, hs);
                const float sr2 = 0.5f * b2w;
                const float dx = dot3(d, xa), dy = dot3(d, ya);
                const float ic2 = __builtin_amdgcn_rcpf(ci * ci);   // scales the footprint only
                float sxx = 0.0f, syy = 0.0f, sxy = 0.0f;
                if constexpr (ANISO) {
                    aniso_footprint(ar, d, ns, xa, ya, sxx, syy, sxy);
                } else {
                    sxx = sr2 * (1.0f + dx * dx * ic2);
                    syy = sr2 * (1.0f + dy * dy * ic2);
                    sxy = sr2 * (dx * dy * ic2);
                }
                // composite interaction: the boundary within the footprint, if any
                bool comp = false;
                int fmat = 0;
                float gfx = 1.0f, gfy = 0.0f;
                HalfPlane hp{};
                if constexpr (COMPOSITE) {
                    comp = find_boundary(A.bnd, prev, __float_as_int(v1.w), P, xa, ya, sxx, syy, sxy, A.scene.mats,
                                         fmat, gfx, gfy, hp);
                    if (comp) ev |= 1u << EV_COMPOSITE;
                }

                // Measurement by next-event estimation (eq. measurement_operator).
                float sval = 0.0f;   // SHQ: the value for this vertex's slot
                float hv[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // HERO: the members' values
                if (A.nsrc > 0) {
                    const uint4 rn = draw(pid, (uint32_t)depth, STREAM_NEE, A.seed);
                    const int si = min((int)(unif(rn.x) * (float)A.nsrc), A.nsrc - 1);
                    const SourceDev& L = A.src[si];
                    f3 om = mk3(0, 0, 0);
                    bool ok = false;
                    float tmax_s = FLT_MAX, tt_s = 0.0f;
                    const float tminP = 1e-7f * (1.0f + maxabs3(to_f3(P)));
                    if (L.kind == 0) {
                        om = ld3(L.dir);
                        ok = true;
                    } else {
                        float z1, z2;
                        box_muller(unif(rn.y), unif(rn.z), z1, z2);
                        // one division: 1 / k (the emitter's reciprocal radius and extents
                        // come with it)
                        const float ik = 1.0f / k;
                        const float du = z1 * L.irc_um, dv = z2 * L.irc_um;
                        const float tt = (du * du + dv * dv) * (ik * ik);
                        tt_s = tt;
                        if (tt < 1.0f) {
                            const f3 ax = ld3(L.dir), eu = ld3(L.bu), ev = ld3(L.bv);
                            om = (du * ik) * eu + (dv * ik) * ev + sqrtf(1.0f - tt) * ax;
                            const f3 pp = diff_f3(P, ld3(L.pos));   // P - emitter centre
                            const float te = dot3(pp, ax) / dot3(om, ax);
                            if (te > tminP) {
                                const f3 qp = pp - te * om;           // Q - emitter centre
                                const float a = dot3(qp, eu) * L.ilu, b = dot3(qp, ev) * L.ilv;
                                if (fabsf(a) <= 1.0f && fabsf(b) <= 1.0f) {
                                    ok = true;
                                    tmax_s = te;
                                }
                            }
                        }
                    }
                    if constexpr (HERO) {
                      if (ok && dot3(om, ng) < 0.0f && dot3(om, ns) < 0.0f) {
                        // the four members' values now (their slot holds four floats), the
                        // visibility later (shadow_kernel clears all four)
                        ev |= 1u << EV_SHADOW;
                        ev |= 1u << (EV_MEAS_SMOOTH + m.kind);
                        const uint32_t slot = (uint32_t)((idx - A.path_begin) * (uint64_t)A.max_depth + depth);
                        // members: emitter-sampling density of om relative to the hero's
                        // (Gaussian angular spectrum N(k u_t; 0, rc^-2 I) k^2), then the
                        // balance-heuristic estimate of each
                        float q[4], den = 0.0f;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            q[i] = L.kind == 0 ? 1.0f
                                               : mk[i] * mk[i] / (k * k) *
                                                     __expf(-0.5f * (mk[i] * mk[i] - k * k) * tt_s * L.rc_um * L.rc_um);
                            den += mR[i] * q[i];
                        }
                        const float cx = dot3(om, xa), cy = dot3(om, ya);
                        const float scale = 4.0f * L.power * (float)A.nsrc / den;
                        // one p_w call site for the four members (a rolled loop; the member's
                        // registers are picked by selects)
#pragma nounroll
                        for (int i = 0; i < 4; ++i) {
                            const float Ti = pick4(mT, i);
                            if (Ti == 0.0f) continue;
                            const float ki = pick4(mk, i), sr = 0.5f * pick4(mb2, i);
                            const float fxx = sr * (1.0f + dx * dx * ic2), fyy = sr * (1.0f + dy * dy * ic2),
                                        fxy = sr * (dx * dy * ic2);
                            float p;
                            if (COMPOSITE && comp) {
                                // the member's own window against the boundary the hero found
                                const HalfPlane Hi = make_halfplane(fxx, fyy, fxy, hp.nx, hp.ny, hp.c);
                                p = pw_composite(m, 1.0f, 0.0f, A.scene.mats[fmat], gfx, gfy, ki, ki * cx, ki * cy,
                                                 -ki * dx, -ki * dy, Hi, A.bnd);
                            } else {
                                p = pw_plain(m.kind, m.h, m.L, m.refl, ki, ki * cx, ki * cy, -ki * dx, -ki * dy, fxx,
                                             fyy, fxy, 1.0f, 0.0f);
                            }
                            const float add = scale * Ti * pick4(q, i) * p;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                if (j == i) hv[j] = add;
                            }
                        }
                        const bool want = hv[0] != 0.0f || hv[1] != 0.0f || hv[2] != 0.0f || hv[3] != 0.0f;
                        const unsigned long long qm = __ballot(want);
                        if (want) {
                            const int leader = __ffsll((long long)qm) - 1;
                            unsigned long long qb = 0;
                            if (lane == leader) qb = atomicAdd(A.shq_count, (unsigned long long)__popcll(qm));
                            qb = __shfl(qb, leader);
                            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(qm >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)qm, 0u));
                            uint4* q4 = A.shq + 3 * (qb + r);
                            const unsigned long long px = __double_as_longlong(P.x), py = __double_as_longlong(P.y),
                                                     pz = __double_as_longlong(P.z);
                            q4[0] = make_uint4((uint32_t)px, (uint32_t)(px >> 32), (uint32_t)py, (uint32_t)(py >> 32));
                            q4[1] = make_uint4((uint32_t)pz, (uint32_t)(pz >> 32), __float_as_uint(om.x), __float_as_uint(om.y));
                            q4[2] = make_uint4(__float_as_uint(om.z), __float_as_uint(tmax_s), (uint32_t)prev, slot);
                        }
                      }
                    } else if constexpr (SHQ) {
                      if (ok && dot3(om, ng) < 0.0f && dot3(om, ns) < 0.0f) {
                        // the measurement value now, its visibility later (shadow_kernel)
                        ev |= 1u << EV_SHADOW;
                        ev |= 1u << (EV_MEAS_SMOOTH + m.kind);
                        const float kix = k * dot3(om, xa), kiy = k * dot3(om, ya);
                        const float kox = -k * dx, koy = -k * dy;
                        const float scale = alpha * L.power * (float)A.nsrc;
                        const uint32_t slot = (uint32_t)((idx - A.path_begin) * (uint64_t)A.max_depth + depth);
                        // e: 0 closed form, 1 queued for the network, 2 more than 8 lobe widths
                        // from the lobe (p_w taken as 0)
                        int e = 0;
                        // (a composite interaction keeps the closed form: the network knows one
                        // material's p_w only)
                        if (DEFER && m.kind == MAT_ROUGH && !(COMPOSITE && comp)) {
                            const SurDomain D{A.sur.gmin, A.sur.gmax, A.sur.smin, A.sur.smax};
                            float sx[MLP_IN] = {}, slp = 0.0f;
                            e = sur_encode(D, k, kix, kiy, kox, koy, sxx, syy, sxy, m.h, m.L, sx, slp);
                            if (e == 0) ev |= 1u << EV_FALLBACK;
                            // append the query (one atomic per wave); every (path, depth) appends
                            // at most once, so the queue is sized for the launch's slots
                            const bool wq = e == 1;
                            const unsigned long long nm = __ballot(wq);
                            if (wq) {
                                ev |= 1u << EV_SUR;
                                const int leader = __ffsll((long long)nm) - 1;
                                unsigned long long nb = 0;
                                if (lane == leader) nb = atomicAdd(A.sq_count, (unsigned long long)__popcll(nm));
                                nb = __shfl(nb, leader);
                                const uint32_t r = __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(nm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nm, 0u));
                                uint4* q = A.sq + 2 * (nb + r);
                                q[0] = make_uint4(bf16_pair(sx[0], sx[1]), bf16_pair(sx[2], sx[3]),
                                                  bf16_pair(sx[4], sx[5]), bf16_pair(sx[6], sx[7]));
                                q[1] = make_uint4(bf16_pair(sx[8], sx[9]), __float_as_uint(scale * m.refl),
                                                  __float_as_uint(slp), slot);
                            }
                        }
                        float v = 0.0f;
                        if (e == 0) {
                            if (COMPOSITE && comp)
                                v = scale * pw_composite(m, 1.0f, 0.0f, A.scene.mats[fmat], gfx, gfy, k, kix, kiy, kox,
                                                         koy, hp, A.bnd);
                            else
                                v = scale * pw_plain(m.kind, m.h, m.L, m.refl, k, kix, kiy, kox, koy, sxx, syy, sxy,
                                                     1.0f, 0.0f);
                        }
                        const bool want = v != 0.0f || e == 1;
                        const unsigned long long qm = __ballot(want);
                        if (want) {
                            const int leader = __ffsll((long long)qm) - 1;
                            unsigned long long qb = 0;
                            if (lane == leader) qb = atomicAdd(A.shq_count, (unsigned long long)__popcll(qm));
                            qb = __shfl(qb, leader);
                            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(qm >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)qm, 0u));
                            sval = v;
                            uint4* q = A.shq + 3 * (qb + r);
                            const unsigned long long px = __double_as_longlong(P.x), py = __double_as_longlong(P.y),
                                                     pz = __double_as_longlong(P.z);
                            q[0] = make_uint4((uint32_t)px, (uint32_t)(px >> 32), (uint32_t)py, (uint32_t)(py >> 32));
                            q[1] = make_uint4((uint32_t)pz, (uint32_t)(pz >> 32), __float_as_uint(om.x), __float_as_uint(om.y));
                            q[2] = make_uint4(__float_as_uint(om.z), __float_as_uint(tmax_s), (uint32_t)prev, slot);
                        }
                      }
                    }
                }
                // every vertex that reaches the measurement stores its slot (zero without a
                // measurement; a queued network query overwrites it, an occluded shadow ray
                // clears it), so the merge reads the path's first slots only
                if constexpr (HERO) {
                    float4* h4 = reinterpret_cast<float4*>(A.sdense) + ((idx - A.path_begin) * (uint64_t)A.max_depth + depth);
                    *h4 = make_float4(hv[0], hv[1], hv[2], hv[3]);
                } else {
                    A.sdense[(idx - A.path_begin) * (uint64_t)A.max_depth + depth] = sval;
                }
                wrote = true;
                if (depth + 1 >= A.max_depth) {
                    finish = true;
                } else {
                    // Light-matter interaction: sample the continuation generalized ray.  At a
                    // composite interaction, the far side's kernel with the probability of its
                    // window mass (word 3 of the interaction's NEE draw), else the near side's:
                    // a one-sample estimate of the mass-weighted mixture of the two kernels.  A
                    // far grating is sampled in its own frame (grating vector along x).
                    const uint4 rs = draw(pid, (uint32_t)depth, STREAM_SCATTER, A.seed);
                    float kox = 0.0f, koy = 0.0f, wgt = 0.0f;
                    int comp_j = 0;
                    float ph = 0.0f;
                    float off[2];
                    DMat cm = m;
                    float rcx = 1.0f, rcy = 0.0f;   // the sampled side's grating direction
                    bool far_chosen = false;
                    if constexpr (COMPOSITE) {
                        if (comp && !(unif(draw(pid, (uint32_t)depth, STREAM_NEE, A.seed).w) < 1.0f - hp.mass_far)) {
                            far_chosen = true;
                            cm = A.scene.mats[fmat];
                            if (cm.kind == MAT_GRATING) {
                                rcx = gfx;
                                rcy = gfy;
                            }
                        }
                    }
                    const float kix_s = rcx * k * dx + rcy * k * dy, kiy_s = -rcy * k * dx + rcx * k * dy;
                    // a rough surface's Poisson parameter (2 k cos i s)^2 in double, from the path's
                    // wavelength and double cosine (its decision must not depend on float rounding)
                    double g_rough = -1.0;
                    if (cm.kind == MAT_ROUGH) {
                        const uint32_t nw = HERO ? (nl >> 2) : nl;
                        const uint32_t wi = (uint32_t)(pid % nw) + (HERO ? (uint32_t)hs * nw : 0u);
                        const double kd = 6.283185307179586 / (double)A.lambda[wi];
                        g_rough = 4.0 * kd * kd * cid * cid * (double)cm.h * (double)cm.h;
                    }
                    if (sample_finf(cm, k, kix_s, kiy_s, ci, unif(rs.x), unif(rs.y), unif(rs.z), kox, koy, wgt,
                                    (float*)(int*)stk, STACK, &comp_j, HERO ? &ph : nullptr, off, g_rough)) {
                        ev |= 1u << EV_EVANESCENT;
                        finish = true;
                    } else {
                        if constexpr (COMPOSITE) {
                            const float ox = rcx * kox - rcy * koy, oy = rcy * kox + rcx * koy;
                            kox = ox;
                            koy = oy;
                        }
                        if constexpr (HERO) {
                            if (COMPOSITE && comp)
                                hero_composite_continuation(m, A.scene.mats[fmat], gfx, gfy, far_chosen, hp.snn, hp.c,
                                                            mb2, k, mk, hs, k * dx, k * dy, ci, kox, koy, comp_j, wgt,
                                                            mT, mR);
                            else
                                hero_continuation(m, k, mk, hs, k * dx, k * dy, ci, kox, koy, wgt, comp_j, ph, mT, mR);
                        } else {
                            alpha *= wgt;
                        }
                        if (A.rr_enable && depth + 1 >= 2) {
                            if ((rs.w >> 8) < A.rr_thr) {
                                alpha *= A.inv_rr_p;
                                if constexpr (HERO) {
#pragma unroll
                                    for (int i = 0; i < NM; ++i) mT[i] *= A.inv_rr_p;
                                }
                            } else {
                                finish = true;
                            }
                        }
                        if (!finish) {
                            // the new direction in double: the tangential part of the old one
                            // plus the sampled transfer (a grating order's -j K in its own
                            // frame, rotated into the hit's), normal part from |d| = 1; the
                            // frame rebuilt in double by the float frame's rule
                            double ox = (double)off[0], oy = (double)off[1];
                            if (cm.kind == MAT_GRATING) {
                                ox = -(double)comp_j * (6.283185307179586 / (double)cm.L);
                                oy = 0.0;
                            }
                            const double fx = (double)rcx * ox - (double)rcy * oy, fy = (double)rcy * ox + (double)rcx * oy;
                            const d3 td = d3{dd.x + cid * nsd.x, dd.y + cid * nsd.y, dd.z + cid * nsd.z};
                            // (one candidate and one normalisation, selected without branches:
                            // a value assigned only on some divergent paths would be carried
                            // around the path loop)
                            d3 t = td;
                            double t2 = td.x * td.x + td.y * td.y + td.z * td.z;
                            bool hx = t2 > 1e-24;
                            if (m.kind == MAT_GRATING) {
                                const double gn = (double)m.gx * nsd.x + (double)m.gy * nsd.y + (double)m.gz * nsd.z;
                                const d3 tg = d3{m.gx - gn * nsd.x, m.gy - gn * nsd.y, m.gz - gn * nsd.z};
                                const double tg2 = tg.x * tg.x + tg.y * tg.y + tg.z * tg.z;
                                if (tg2 > 1e-18) {
                                    t = tg;
                                    t2 = tg2;
                                    hx = true;
                                }
                            }
                            const double rx = hx ? 1.0 / sqrt(t2) : 0.0;
                            const d3 xd = hx ? d3{t.x * rx, t.y * rx, t.z * rx} : d3{(double)xa.x, (double)xa.y, (double)xa.z};
                            const d3 yd = d3{nsd.y * xd.z - nsd.z * xd.y, nsd.z * xd.x - nsd.x * xd.z,
                                             nsd.x * xd.y - nsd.y * xd.x};
                            const double ik = 1.0 / (double)k;
                            const d3 tn = d3{td.x + (fx * xd.x + fy * yd.x) * ik, td.y + (fx * xd.y + fy * yd.y) * ik,
                                             td.z + (fx * xd.z + fy * yd.z) * ik};
                            const double kn2 = 1.0 - (tn.x * tn.x + tn.y * tn.y + tn.z * tn.z);
                            if (!(kn2 > 0.0)) {
                                // evanescent in double although the float sampler kept it
                                ev |= 1u << EV_EVANESCENT;
                                finish = true;
                            }
                            const double kn = sqrt(fmax(0.0, kn2));
                            const d3 nd = d3{tn.x + kn * nsd.x, tn.y + kn * nsd.y, tn.z + kn * nsd.z};
                            const double r = 1.0 / sqrt(nd.x * nd.x + nd.y * nd.y + nd.z * nd.z);
                            dd = d3{nd.x * r, nd.y * r, nd.z * r};
                            if constexpr (ANISO) aniso_interact(ar, d, to_f3(dd), ns);
                            o = P;
                            if (!finish) ++depth;
                        }
                    }
                }
            }
        }
        }   // live
        if (finish) {
            // slots the path stored: one per vertex that reached the measurement
            A.snd[idx - A.path_begin] = (uint8_t)(depth + (wrote ? 1 : 0));
            live = false;
        }
#pragma unroll
        for (int b = 0; b < EV_COUNT; ++b) w_cnt[b] += (uint32_t)__popcll(__ballot((ev >> b) & 1u));
    }

    const unsigned long long s8 = wave_sum(c_nodes), s9 = wave_sum(c_tris);
    if (lane == 0) {
        atomicAdd(A.stats + ST_PATHS, (unsigned long long)w_cnt[EV_PATH]);
        atomicAdd(A.stats + ST_SEGMENTS, (unsigned long long)w_cnt[EV_SEG]);
        atomicAdd(A.stats + ST_SHADOW, (unsigned long long)w_cnt[EV_SHADOW]);
        atomicAdd(A.stats + ST_EVANESCENT, (unsigned long long)w_cnt[EV_EVANESCENT]);
        atomicAdd(A.stats + ST_BACKFACING, (unsigned long long)w_cnt[EV_BACKFACING]);
        atomicAdd(A.stats + ST_NONFINITE, (unsigned long long)w_cnt[EV_NONFINITE]);
        atomicAdd(A.stats + ST_NODES, s8);
        atomicAdd(A.stats + ST_TRIS, s9);
        atomicAdd(A.stats + ST_SUR, (unsigned long long)w_cnt[EV_SUR]);
        atomicAdd(A.stats + ST_FALLBACK, (unsigned long long)w_cnt[EV_FALLBACK]);
        atomicAdd(A.stats + ST_COMPOSITE, (unsigned long long)w_cnt[EV_COMPOSITE]);
        atomicAdd(A.stats + ST_MEAS_SMOOTH, (unsigned long long)w_cnt[EV_MEAS_SMOOTH]);
        atomicAdd(A.stats + ST_MEAS_ROUGH, (unsigned long long)w_cnt[EV_MEAS_ROUGH]);
        atomicAdd(A.stats + ST_MEAS_GRATING, (unsigned long long)w_cnt[EV_MEAS_GRATING]);
    }
}

// Shadow rays queued by the trace kernel (48 B each: mean position in double, the direction
// the light travels, the emitter distance, the triangle the ray leaves, the slot), one per
// lane in full waves.  An occluded ray clears the measurement value in its slot.  The grid is
// the trace kernel's, so the traversal-stack overflow region fits.
template <int STACK>
__global__ __launch_bounds__(256, 4) void shadow_kernel(const TraceArgs A) {
    __shared__ __attribute__((aligned(16))) int lds_stack[4][STACK][64];
    __shared__ float4 lds_nodes[kLdsNodes * 8];
    const int nln = stage_top_nodes(A.scene, lds_nodes);
    const lds_v4f* top = (const lds_v4f*)&lds_nodes[0];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // the traversal's (child, key) pairs over the wave-private region
    lds_v2i* stk2 = (lds_v2i*)&lds_stack[wv][0][0] + lane;
    // the child-code scratch: 16 contiguous bytes per lane in the last two entries' space
    lds_v4i* scr = (lds_v4i*)&lds_stack[wv][STACK - 4][0] + lane;
    const size_t ostride = (size_t)gridDim.x * 256;
    v2i_t* ovf = A.ovf ? (v2i_t*)A.ovf + ((size_t)blockIdx.x * 256 + 64 * __builtin_amdgcn_readfirstlane(wv)) : nullptr;
    const uint64_t n = *A.shq_count;
    uint32_t c_nodes = 0, c_tris = 0;
    for (uint64_t base = ((uint64_t)blockIdx.x * 4 + wv) * 64; base < n; base += (uint64_t)gridDim.x * 256) {
        const uint64_t i = base + lane;
        if (i < n) {
            const uint4* q = A.shq + 3 * i;
            const uint4 a = q[0], b = q[1], c = q[2];
            const d3 P = d3{__longlong_as_double((long long)(((uint64_t)a.y << 32) | a.x)),
                            __longlong_as_double((long long)(((uint64_t)a.w << 32) | a.z)),
                            __longlong_as_double((long long)(((uint64_t)b.y << 32) | b.x))};
            const f3 om = mk3(__uint_as_float(b.z), __uint_as_float(b.w), __uint_as_float(c.x));
            const float tminP = 1e-7f * (1.0f + maxabs3(to_f3(P)));
            RayT sray;
            ray_setup(sray, P, -1.0f * om);
            float tm = __uint_as_float(c.y), su, sv;
            const int occ = traverse<STACK>(A.scene, sray, tminP, tm, true, (int)c.z, stk2, scr, A.lds_cap, ovf, ostride,
                                            c_nodes, c_tris, su, sv, top, nln);
            if (occ >= 0) {
                if (A.hero) reinterpret_cast<float4*>(A.sdense)[c.w] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                else A.sdense[c.w] = 0.0f;
            }
        }
    }
    const unsigned long long s8 = wave_sum(c_nodes), s9 = wave_sum(c_tris);
    if (lane == 0) {
        atomicAdd(A.stats + ST_NODES, s8);
        atomicAdd(A.stats + ST_TRIS, s9);
    }
}

// Records of a launch's paths: the measurement values of each path's interactions summed in
// depth order (the order in which the path would have added them itself); path i stored its
// first nd[i] slots.
__global__ __launch_bounds__(256) void shadow_merge_kernel(const float* __restrict__ val,
                                                           const uint8_t* __restrict__ nd, int depth,
                                                           float* __restrict__ records, uint64_t p0, uint64_t n,
                                                           float inv_spp_norm, unsigned long long* stats) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const int m = nd[i];
        const float* vp = val + i * depth;
        float s = 0.0f;
        if (depth <= 8) {
            // the stored slots' loads issue together; the sum keeps depth order
            float v8[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) v8[d] = d < m ? vp[d] : 0.0f;
#pragma unroll
            for (int d = 0; d < 8; ++d)
                if (d < m) s += v8[d];
        } else {
            for (int d = 0; d < m; ++d) s += vp[d];
        }
        float v = s * inv_spp_norm;
        if (!isfinite(v)) {
            bad = true;
            v = 0.0f;
        }
        records[p0 + i] = v;
    }
    const unsigned long long nb = __popcll(__ballot(bad));
    if ((threadIdx.x & 63) == 0 && nb) atomicAdd(stats + ST_NONFINITE, nb);
}

// Records of a launch's hero-wavelength paths: member i's values summed over the path's
// stored slots in depth order (four floats per slot) into the record of wavelength g + i G of
// its (sample, pixel): path index p -> record (p / G) nl + p % G + i G.
__global__ __launch_bounds__(256) void hero_merge_kernel(const float4* __restrict__ val,
                                                         const uint8_t* __restrict__ nd, int depth,
                                                         float* __restrict__ records, uint64_t p0, uint64_t n,
                                                         uint32_t G, uint32_t nl, float inv_spp_norm,
                                                         unsigned long long* stats) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned nbad = 0;
    if (i < n) {
        const int m = nd[i];
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
        for (int d = 0; d < m; ++d) {
            const float4 v = val[i * depth + d];
            s0 += v.x;
            s1 += v.y;
            s2 += v.z;
            s3 += v.w;
        }
        const uint64_t p = p0 + i;
        const uint64_t rb = (p / G) * nl + p % G;
        const float sv[4] = {s0 * inv_spp_norm, s1 * inv_spp_norm, s2 * inv_spp_norm, s3 * inv_spp_norm};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = sv[j];
            if (!isfinite(v)) {
                ++nbad;
                v = 0.0f;
            }
            records[rb + (uint64_t)j * G] = v;
        }
    }
    unsigned long long nb = 0;
    for (int b = 0; b < 4; ++b) nb += __popcll(__ballot(nbad > (unsigned)b));
    if ((threadIdx.x & 63) == 0 && nb) atomicAdd(stats + ST_NONFINITE, nb);
}

// Per-pixel sum of the path records in sample order (deterministic).
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ rec, float* __restrict__ img,
                                                     int64_t S, uint32_t H, uint32_t W, uint32_t nl) {
    const uint32_t per = H * W * nl;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per) return;
    float acc = 0.0f;
    // eight samples' loads in flight at a time; the sum keeps sample order
#pragma unroll 8
    for (int64_t s = 0; s < S; ++s) acc += rec[(size_t)s * per + t];
    const uint32_t w = t % nl;
    const uint32_t pix = t / nl;
    img[(size_t)w * H * W + pix] += acc;
}

__global__ __launch_bounds__(256) void bsdf_eval_kernel(const float* __restrict__ q, int64_t n,
                                                        float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* r = q + i * 14;
    out[i] = pw_plain((int)r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11],
                      r[12], r[13]);
}

template <bool DEFER, bool HERO, bool ANISO = false, bool COMPOSITE = false>
static int grid_for(int device) {
    int ncu = 0, nb = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, trace_kernel<kLdsStack, DEFER, HERO, ANISO, COMPOSITE>, 256,
                                                     0) != hipSuccess)
        return 0;
    return ncu * (nb > 0 ? nb : 1);
}

int trace_grid_size(int device, bool sur, bool hero, bool aniso, bool composite) {
    if (composite && aniso) return grid_for<false, false, true, true>(device);
    if (composite && hero) return grid_for<false, true, false, true>(device);
    if (composite) return sur ? grid_for<true, false, false, true>(device) : grid_for<false, false, false, true>(device);
    if (aniso) return grid_for<false, false, true>(device);
    if (hero) return grid_for<false, true>(device);
    return sur ? grid_for<true, false>(device) : grid_for<false, false>(device);
}

hipError_t launch_trace(const TraceArgs& a, int grid, hipStream_t s) {
    if (a.composite && a.aniso)
        hipLaunchKernelGGL((trace_kernel<kLdsStack, false, false, true, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.composite && a.hero)
        hipLaunchKernelGGL((trace_kernel<kLdsStack, false, true, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.composite && a.bsdf_mode != 0)
        hipLaunchKernelGGL((trace_kernel<kLdsStack, true, false, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.composite)
        hipLaunchKernelGGL((trace_kernel<kLdsStack, false, false, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.aniso) hipLaunchKernelGGL((trace_kernel<kLdsStack, false, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.hero) hipLaunchKernelGGL((trace_kernel<kLdsStack, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (a.bsdf_mode != 0) hipLaunchKernelGGL((trace_kernel<kLdsStack, true, false>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((trace_kernel<kLdsStack, false, false>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void chunk_reset_kernel(unsigned long long* counter, unsigned long long* sq_count,
                                                          unsigned long long* shq_count, float* dense, uint64_t n) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *counter = 0ull;
        *sq_count = 0ull;
        if (shq_count) *shq_count = 0ull;
    }
    for (uint64_t i = t; i < n; i += (uint64_t)gridDim.x * blockDim.x) dense[i] = 0.0f;
}

// Zero n 32-bit words (a kernel rather than a memset node, so a captured graph replays it
// like any other launch).
__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_shadow(const TraceArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((shadow_kernel<kLdsStack>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_shadow_merge(const float* val, const uint8_t* nd, int depth, float* records, uint64_t p0,
                               uint64_t n, float inv_spp_norm, unsigned long long* stats, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(shadow_merge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, val, nd, depth,
                       records, p0, n, inv_spp_norm, stats);
    return hipGetLastError();
}

hipError_t launch_hero_merge(const float* val, const uint8_t* nd, int depth, float* records, uint64_t p0,
                             uint64_t n, uint32_t G, uint32_t nl, float inv_spp_norm, unsigned long long* stats,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(hero_merge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(val), nd, depth, records, p0, n, G, nl, inv_spp_norm, stats);
    return hipGetLastError();
}

hipError_t launch_chunk_reset(unsigned long long* counter, unsigned long long* sq_count,
                              unsigned long long* shq_count, float* dense, uint64_t n, hipStream_t s) {
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(chunk_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, counter, sq_count, shq_count,
                       dense, n);
    return hipGetLastError();
}

hipError_t launch_reduce(const float* records, float* image, int64_t spp_count, uint32_t H, uint32_t W,
                         uint32_t nl, hipStream_t s) {
    const uint32_t per = H * W * nl;
    hipLaunchKernelGGL(reduce_kernel, dim3((per + 255) / 256), dim3(256), 0, s, records, image, spp_count,
                       H, W, nl);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void composite_eval_kernel(const float* __restrict__ q, int64_t n,
                                                             float* __restrict__ out, const BoundaryDev B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* r = q + i * 23;
    DMat mn, mf;
    mn.kind = (int)r[0];
    mn.h = r[1];
    mn.L = r[2];
    mn.refl = r[3];
    mf.kind = (int)r[6];
    mf.h = r[7];
    mf.L = r[8];
    mf.refl = r[9];
    mn.gx = mn.gy = mn.gz = mn.pad = mf.gx = mf.gy = mf.gz = mf.pad = 0.0f;
    const HalfPlane H = make_halfplane(r[17], r[18], r[19], r[20], r[21], r[22]);
    out[i] = pw_composite(mn, r[4], r[5], mf, r[10], r[11], r[12], r[13], r[14], r[15], r[16], H, B);
}

hipError_t launch_composite_eval(const float* q, int64_t n, float* out, const BoundaryDev& b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(composite_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, n, out, b);
    return hipGetLastError();
}

hipError_t launch_bsdf_eval(const float* q, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(bsdf_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, n, out);
    return hipGetLastError();
}

}  // namespace grw
