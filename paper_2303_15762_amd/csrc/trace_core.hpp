// Device building blocks of the path tracer shared by its kernels: double-precision path
// positions, the float ray set-up and watertight triangle test, hit refinement, BVH4
// traversal, and small wave helpers.
//
// Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762).
#pragma once

#include <float.h>

#include "kernels.hpp"
#include "mlp_core.hpp"

namespace grw {

// A pointer into LDS typed as such, so that LDS accesses stay LDS instructions (a generic
// pointer lets the compiler merge an LDS and a global access into one flat access).
typedef __attribute__((address_space(3))) int lds_int;
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4f_t lds_v4f;
typedef int v2i_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) v2i_t lds_v2i;
typedef __attribute__((address_space(3))) v4i_t lds_v4i;

// Copy BVH nodes 0 .. min(kLdsNodes, node count) - 1 into the block's LDS (8 float4 each) and
// return how many; all threads of the block call it.
__device__ __forceinline__ int stage_top_nodes(const SceneDev& S, float4* lds) {
    const int n = min(kLdsNodes, (int)(S.node_bytes >> 7));
    for (int i = threadIdx.x; i < n * 8; i += blockDim.x) lds[i] = S.nodes[i];
    __syncthreads();
    return n;
}

// Path positions are kept in double precision: at metre-scale coordinates one float ulp is
// 0.06 um, and steep shading-normal gradients turn such offsets into direction errors that
// grow along the path.  A ray carries its origin as the nearest float o plus the float
// residual lo, so that vertex - origin keeps float precision relative to the segment.
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 add_scaled(d3 a, float t, f3 v) {
    return d3{a.x + (double)t * (double)v.x, a.y + (double)t * (double)v.y, a.z + (double)t * (double)v.z};
}
__device__ __forceinline__ f3 to_f3(d3 a) { return mk3((float)a.x, (float)a.y, (float)a.z); }
// (a - b) rounded once to float
__device__ __forceinline__ f3 diff_f3(d3 a, f3 b) {
    return mk3((float)(a.x - (double)b.x), (float)(a.y - (double)b.y), (float)(a.z - (double)b.z));
}

// Distance along (o, d) at which the ray enters the scene bounds (widened by 1 mm on the
// host), or 0 when it starts inside or misses them.  The float slab test errs by far less
// than the margin.
__device__ __forceinline__ float scene_entry(const SceneDev& S, d3 o, f3 d) {
    const f3 of = to_f3(o);
    const float t0x = (S.lo[0] - of.x) / d.x, t1x = (S.hi[0] - of.x) / d.x;
    const float t0y = (S.lo[1] - of.y) / d.y, t1y = (S.hi[1] - of.y) / d.y;
    const float t0z = (S.lo[2] - of.z) / d.z, t1z = (S.hi[2] - of.z) / d.z;
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
    return (tn > 0.0f && tn <= tf) ? tn : 0.0f;
}

// Hit distance and barycentric weights of the triangle the float test found, recomputed in
// double precision (Moller-Trumbore on the float vertices, along the path's double direction):
// the position the path continues from, and the shading normal interpolated there, then carry
// no error of the float ray-space arithmetic.  Keeps the float test's values (bu, bv on entry)
// when the double test degenerates.
__device__ __forceinline__ void refine_hit(d3 o, d3 d, float4 a, float4 b, float4 c, float& t,
                                           double& bu, double& bv, double& t64) {
    t64 = (double)t;
    const double e1x = (double)b.x - a.x, e1y = (double)b.y - a.y, e1z = (double)b.z - a.z;
    const double e2x = (double)c.x - a.x, e2y = (double)c.y - a.y, e2z = (double)c.z - a.z;
    const double dx = d.x, dy = d.y, dz = d.z;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0) return;
    const double inv = 1.0 / det;
    const double sx = o.x - a.x, sy = o.y - a.y, sz = o.z - a.z;
    const double u = (sx * px + sy * py + sz * pz) * inv;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const double v = (dx * qx + dy * qy + dz * qz) * inv;
    const double tt = (e2x * qx + e2y * qy + e2z * qz) * inv;
    if (!(tt > 0.0)) return;
    t64 = tt;
    t = (float)tt;
    bu = fmin(fmax(u, 0.0), 1.0);
    bv = fmin(fmax(v, 0.0), 1.0);
}

struct RayT {
    f3 o, lo, d, inv;
    int kx, ky, kz;
    float Sx, Sy, Sz;
};

__device__ __forceinline__ float comp(f3 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }

__device__ __forceinline__ void ray_setup(RayT& r, d3 o, f3 d) {
    r.o = to_f3(o);
    r.lo = diff_f3(o, r.o);
    r.d = d;
    const float tiny = 1e-30f;
    r.inv = mk3(1.0f / (fabsf(d.x) > tiny ? d.x : copysignf(tiny, d.x)),
                1.0f / (fabsf(d.y) > tiny ? d.y : copysignf(tiny, d.y)),
                1.0f / (fabsf(d.z) > tiny ? d.z : copysignf(tiny, d.z)));
    // Watertight ray/triangle test set-up (Woop, Benthin, Wald, JCGT 2013): permute so that
    // the dominant direction axis is z, keep the winding, shear onto the ray.
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    const int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    const float dz = comp(d, kz);
    if (dz < 0.0f) {
        const int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.Sx = comp(d, kx) / dz;
    r.Sy = comp(d, ky) / dz;
    r.Sz = 1.0f / dz;
}

// Returns true with t and the barycentric weights (bu of v1, bv of v2) when the ray's line
// crosses the triangle (edges inclusive, shared edges decided consistently).
__device__ __forceinline__ bool tri_isect(const RayT& r, float4 a4, float4 b4, float4 c4, float& t,
                                          float& bu, float& bv) {
    // no FP contraction here: an edge shared by two triangles must get exactly opposite edge
    // function values (a fused multiply-add would round the two orientations differently)
#pragma clang fp contract(off)
    const f3 A = mk3((a4.x - r.o.x) - r.lo.x, (a4.y - r.o.y) - r.lo.y, (a4.z - r.o.z) - r.lo.z);
    const f3 B = mk3((b4.x - r.o.x) - r.lo.x, (b4.y - r.o.y) - r.lo.y, (b4.z - r.o.z) - r.lo.z);
    const f3 C = mk3((c4.x - r.o.x) - r.lo.x, (c4.y - r.o.y) - r.lo.y, (c4.z - r.o.z) - r.lo.z);
    const float Az0 = comp(A, r.kz), Bz0 = comp(B, r.kz), Cz0 = comp(C, r.kz);
    const float Ax = comp(A, r.kx) - r.Sx * Az0, Ay = comp(A, r.ky) - r.Sy * Az0;
    const float Bx = comp(B, r.kx) - r.Sx * Bz0, By = comp(B, r.ky) - r.Sy * Bz0;
    const float Cx = comp(C, r.kx) - r.Sx * Cz0, Cy = comp(C, r.ky) - r.Sy * Cz0;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float T = U * (r.Sz * Az0) + V * (r.Sz * Bz0) + W * (r.Sz * Cz0);
    // hardware reciprocal (1 ulp): the hit found is recomputed in double (refine_hit), and t
    // only orders this ray's candidates
    const float rcp = __builtin_amdgcn_rcpf(det);
    t = T * rcp;
    bu = V * rcp;
    bv = W * rcp;
    return true;
}


// BVH4 traversal.  closest: smallest t in (tmin, tmax), equal t resolved to the lower original
// triangle index; any: stop at the first t in (tmin, tmax).  skip: original index of the
// triangle the ray leaves (never hit again), or -1.  stk: this lane's LDS stack (stride 64),
// of which the first cap (<= STACK / 2 - 2) entries are used, each a (child code, entry key)
// pair; entry cap + i goes to ovf[i * ostride + lane], ovf being the wave's slice of the
// overflow region, which the caller sizes for the tree: at most 3 entries per inner node on the
// current root path.  scr: 16 bytes of LDS of this lane (the space of the stack's last two
// entries) that hold a node's child codes while its children are ordered.
// Returns the triangle (leaf order) or -1.
// Traversal loop structure (Aila and Laine, "Understanding the efficiency of ray traversal on
// GPUs", HPG 2009: while-while with postponed leaves): each lane descends inner nodes until it
// has found a leaf, which it parks while it keeps descending; the wave leaves the node loop once
// every lane still in it holds a leaf, and then the lanes test their leaves together.  Node
// and triangle code thus run on fuller waves than when every iteration does either one.
// Nodes below nln are read from top (their LDS copy), the others from the node array.
template <int STACK>
__device__ __forceinline__ int traverse(const SceneDev& S, const RayT& r, float tmin, float& tmax,
                                        bool any, int skip, lds_v2i* stk, lds_v4i* scr, int cap, v2i_t* ovf, size_t ostride,
                                        uint32_t& n_nodes, uint32_t& n_tris, float& hu, float& hv,
                                        const lds_v4f* top, int nln) {
    constexpr int kDone = 0x7FFFFFFF;   // nothing left to visit (never a node index)
    int best = -1;
    int best_orig = 0x7FFFFFFF;
    float best_t = tmax;
    int sp = 0;
    int cur = 0;    // next inner node (>= 0) or leaf (< 0) to visit, or kDone
    int leaf = 0;   // a parked leaf (< 0), or 0
    // The LDS entry is always read (in range) and replaced by the overflow entry when the
    // stack is that deep, so the common pop stays an LDS read.  A closest-hit query skips an
    // inner node whose entry distance lies beyond the closest hit found since it was pushed:
    // its children's boxes lie inside its (widened) box and the slab distances are monotonic
    // in the planes, so each child's entry distance is at least the node's and the node test
    // would reject all four.  The stored key is the entry distance's bit pattern with its four
    // low bits replaced by 4 x slot, hence "beyond" is key > bits(t_best) + 15.  Leaves are
    // always tested (a triangle's own distance can round below its box's).
    auto read_top = [&]() -> v2i_t {
        --sp;
        v2i_t e = stk[min(sp, cap - 1) * 64];
        if (sp >= cap) e = ovf[(size_t)(sp - cap) * ostride + __lane_id()];
        return e;
    };
    auto pop = [&]() -> int {
        if (sp == 0) return kDone;
        v2i_t e = read_top();
        if (!any) {
            const int ib = __float_as_int(best_t) + 15;
            while (e.x >= 0 && e.y > ib) {   // a stale inner node: take the next entry
                if (sp == 0) return kDone;
                e = read_top();
            }
        }
        return e.x;
    };
    // slab distances as (lo - o) / d = lo * inv - o * inv: one FMA per plane (the node boxes
    // are widened by more than the extra rounding of o * inv)
    const float ix = r.inv.x, iy = r.inv.y, iz = r.inv.z;
    const float oix = r.o.x * ix, oiy = r.o.y * iy, oiz = r.o.z * iz;
    // The ray's direction signs fix which plane of each slab it meets first: the near planes
    // are the low ones along positive directions.  Each lane fetches its near and far planes by
    // byte offset within the 128-byte node (lo x at 0, hi x at 16, lo y 32, hi y 48, lo z 64,
    // hi z 80, children 96), so the slab test needs no min/max per plane.  Buffer loads take
    // the per-lane offsets (reads past the node array return zero instead of faulting).
    const __amdgpu_buffer_rsrc_t nb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float4*>(S.nodes), (short)0, (int)S.node_bytes, 0x00020000);
    const int sx = ix < 0.0f ? 16 : 0, sy = iy < 0.0f ? 48 : 32, sz = iz < 0.0f ? 80 : 64;
    while (cur != kDone) {
        while (cur >= 0 && cur != kDone) {
            ++n_nodes;
            const int base = cur << 7;
            const int onx = base + sx, ony = base + sy, onz = base + sz;
            v4f_t nx, fx, ny, fy, nz, fz;
            v4i_t chv;
            if (cur < nln) {
                // the same 16-byte rows of the node's LDS copy, at the same byte offsets (the
                // copy's base folds into the LDS reads' immediate offset)
                const __attribute__((address_space(3))) char* L = (const __attribute__((address_space(3))) char*)top;
                nx = *(const lds_v4f*)(L + onx);
                fx = *(const lds_v4f*)(L + (onx ^ 16));
                ny = *(const lds_v4f*)(L + ony);
                fy = *(const lds_v4f*)(L + (ony ^ 16));
                nz = *(const lds_v4f*)(L + onz);
                fz = *(const lds_v4f*)(L + (onz ^ 16));
                chv = __builtin_bit_cast(v4i_t, *(const lds_v4f*)(L + base + 96));
            } else {
                nx = __builtin_amdgcn_raw_buffer_load_b128(nb, onx, 0, 0);
                fx = __builtin_amdgcn_raw_buffer_load_b128(nb, onx ^ 16, 0, 0);
                ny = __builtin_amdgcn_raw_buffer_load_b128(nb, ony, 0, 0);
                fy = __builtin_amdgcn_raw_buffer_load_b128(nb, ony ^ 16, 0, 0);
                nz = __builtin_amdgcn_raw_buffer_load_b128(nb, onz, 0, 0);
                fz = __builtin_amdgcn_raw_buffer_load_b128(nb, onz ^ 16, 0, 0);
                chv = __builtin_bit_cast(v4i_t, __builtin_amdgcn_raw_buffer_load_b128(nb, base + 96, 0, 0));
            }
            const int4 ch = make_int4(chv.x, chv.y, chv.z, chv.w);
            const float lxa[4] = {nx.x, nx.y, nx.z, nx.w}, hxa[4] = {fx.x, fx.y, fx.z, fx.w};
            const float lya[4] = {ny.x, ny.y, ny.z, ny.w}, hya[4] = {fy.x, fy.y, fy.z, fy.w};
            const float lza[4] = {nz.x, nz.y, nz.z, nz.w}, hza[4] = {fz.x, fz.y, fz.z, fz.w};
            // key = entry distance with 4 x slot in its four low bits (distances are positive, so
            // their bit patterns order like the values; distances within 16 ulps order by slot);
            // a miss keys as 0xFFFFFFFF.  Empty slots
            // hold boxes at +inf and always miss.  The interval ends are taken as signed integers:
            // the entry is at least tmin > 0, and positive floats order like their bit patterns
            // while any negative float is a negative integer, so the hit decision and the entry
            // distance equal the float ones (no NaN arises: the inverse direction is finite).
            uint32_t key[4];
            int chd[4] = {ch.x, ch.y, ch.z, ch.w};
            const int itmin = __float_as_int(tmin), ibest = __float_as_int(best_t);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // lxa..: near planes, hxa..: far planes (see above)
                const float t0x = fmaf(lxa[i], ix, -oix), t1x = fmaf(hxa[i], ix, -oix);
                const float t0y = fmaf(lya[i], iy, -oiy), t1y = fmaf(hya[i], iy, -oiy);
                const float t0z = fmaf(lza[i], iz, -oiz), t1z = fmaf(hza[i], iz, -oiz);
                const int tn = max(max(__float_as_int(t0x), __float_as_int(t0y)), max(__float_as_int(t0z), itmin));
                const int tf = min(min(__float_as_int(t1x), __float_as_int(t1y)), min(__float_as_int(t1z), ibest));
                key[i] = tn <= tf ? (((uint32_t)tn & ~15u) | (uint32_t)(4 * i)) : 0xFFFFFFFFu;
            }
            auto push = [&](int v, uint32_t k) {
                if (sp < cap) stk[sp * 64] = v2i_t{v, (int)k};
                else ovf[(size_t)(sp - cap) * ostride + __lane_id()] = v2i_t{v, (int)k};
                ++sp;
            };
            if (any) {
                // any hit ends the query, so the order of the visits only changes the work:
                // descend into the lowest hit slot and push the other hits, unsorted
                bool have = false;
                int nxt = 0;
#pragma unroll
                for (int i = 3; i >= 0; --i) {
                    if (key[i] != 0xFFFFFFFFu) {
                        if (have) push(nxt, 0u);
                        nxt = chd[i];
                        have = true;
                    }
                }
                cur = have ? nxt : pop();
            } else {
                // ascending sorting network on the keys alone; the child codes wait in the
                // lane's scratch and each is read back at the byte offset its key's slot bits
                // give (4 x slot)
                *scr = chv;
#define GRW_KSWAP(i, j)                                 \
        {                                                   \
            const uint32_t lo_ = min(key[i], key[j]);       \
            key[j] = max(key[i], key[j]);                   \
            key[i] = lo_;                                   \
        }
                GRW_KSWAP(0, 1)
                GRW_KSWAP(2, 3)
                GRW_KSWAP(0, 2)
                GRW_KSWAP(1, 3)
                GRW_KSWAP(1, 2)
#undef GRW_KSWAP
                const uint32_t sbase = (uint32_t)(uintptr_t)scr;
                auto child = [&](uint32_t k) -> int {
                    return *(const __attribute__((address_space(3))) int*)(uintptr_t)((k & 12u) | sbase);
                };
                // descend into the nearest hit and push the farther ones (farthest first); the
                // nearest child's code is read first, since the next node fetch waits on it
                // (with no hit there is nothing to push: the keys are sorted)
                if (key[0] != 0xFFFFFFFFu) {
                    cur = child(key[0]);
#pragma unroll
                    for (int i = 3; i >= 1; --i) {
                        if (key[i] != 0xFFFFFFFFu) push(child(key[i]), key[i]);
                    }
                } else {
                    cur = pop();
                }
            }
            if (cur < 0 && leaf == 0) {   // park the leaf and keep descending
                leaf = cur;
                cur = pop();
            }
            if (!__any(leaf == 0)) break;
        }
        while (leaf < 0) {
            const int first = leaf & 0x0FFFFFFF;
            const int cnt = ((leaf >> 28) & 7) + 1;
            for (int i = 0; i < cnt; ++i) {
                const float4* T = S.tris + (size_t)(first + i) * 3;
                const float4 a = T[0], b = T[1], cc = T[2];
                ++n_tris;
                const int orig = __float_as_int(a.w);
                float t, u, v;
                if (orig != skip && tri_isect(r, a, b, cc, t, u, v) && t > tmin) {
                    if (t < best_t || (t == best_t && orig < best_orig)) {
                        best_t = t;
                        best = first + i;
                        best_orig = orig;
                        hu = u;
                        hv = v;
                        if (any) {
                            tmax = best_t;
                            return best;
                        }
                    }
                }
            }
            leaf = 0;
            if (cur < 0) {   // the next node is a leaf too: test it in this loop
                leaf = cur;
                cur = pop();
            }
        }
    }
    tmax = best_t;
    return best;
}

__device__ __forceinline__ f3 ld3(const float* p) { return mk3(p[0], p[1], p[2]); }

__device__ __forceinline__ unsigned long long wave_sum(uint32_t v) {
    unsigned long long x = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// EV_MEAS_SMOOTH + kind: a vertex that evaluated a measurement at a surface of that kind
enum {
    EV_PATH = 0, EV_SEG, EV_SHADOW, EV_SUR, EV_FALLBACK, EV_EVANESCENT, EV_BACKFACING, EV_NONFINITE, EV_COMPOSITE,
    EV_MEAS_SMOOTH, EV_MEAS_ROUGH, EV_MEAS_GRATING, EV_COUNT
};

// bfloat16 pair (a in the low half), rounded to nearest even as the network's input stage does.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
    uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b);
    ua += 0x7FFFu + ((ua >> 16) & 1u);
    ub += 0x7FFFu + ((ub >> 16) & 1u);
    return (ua >> 16) | (ub & 0xFFFF0000u);
}

}  // namespace grw
