// Wavefront form of the backward generalized-ray path tracer (gfx950).
//
// The paths of one launch advance one interaction per bounce through five kernels that work
// on queues in HBM (structure-of-arrays state, one entry per path):
//   extend  : closest hit of every path in the bounce's list (a persistent kernel; each wave
//             takes the next 64 rays of the list with one atomic).
//   shade   : the hits: free-space update, frame and footprint, next-event sample (a shadow
//             record), continuation sample (the path enters the next list).
//   shadow  : any-hit rays of the shadow records, the same way as extend.
//   measure : p_w of the visible records added to the path's contribution (or, with the
//             learned p_w, a queued query).
//   finish  : one float per path into the records the per-pixel reduction sums.
// Every path draws the same counter-based random numbers as in the persistent kernel, and its
// contribution is summed in interaction order, so the image does not depend on scheduling.
//
// Measured on the mid terrain this form is 2.3x slower than the persistent kernel: after the
// first bounce the lists are in completion order, so each stage reads and writes the per-path
// state at scattered addresses of a 1.5 GB launch, which HBM serves one 64-byte line per
// access, while the persistent kernel keeps the state in registers.  Refilling lanes in the
// middle of a traversal (so that waves do not wait for their slowest ray) and sorting hits by
// material were tried and were slower still, for the same reason plus the atomics they add.
//
// Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762),
// Algorithm 1 under the interactive assumption of Sec. "Interactive Rendering".
#include <algorithm>

#include "trace_core.hpp"

namespace grw {

namespace {

constexpr int kDoneNode = 0x7FFFFFFF;   // nothing left to visit (never a node index)

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Append one entry per lane in `want` to a list; returns this lane's position.
__device__ __forceinline__ uint32_t wave_append(unsigned int* count, bool want) {
    const unsigned long long m = __ballot(want);
    const int lane = threadIdx.x & 63;
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    unsigned int base = 0;
    if (m && lane == leader) base = atomicAdd(count, (unsigned int)__popcll(m));
    base = __shfl(base, leader);
    return base + lane_rank(m);
}

__device__ __forceinline__ uint64_t wave_append64(unsigned long long* count, bool want) {
    const unsigned long long m = __ballot(want);
    const int lane = threadIdx.x & 63;
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    unsigned long long base = 0;
    if (m && lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    return base + lane_rank(m);
}

// Path id (the random streams' key), wavelength index of path p (global index).
__device__ __forceinline__ void path_ids(const TraceArgs& A, uint64_t p, uint64_t& pid, uint32_t& w,
                                         uint32_t& x, uint32_t& y) {
    const uint32_t Wd = (uint32_t)A.sensor.W, Hd = (uint32_t)A.sensor.H, nl = (uint32_t)A.nl;
    const uint64_t sl = p / A.per_sample;
    const uint32_t rem = (uint32_t)(p - sl * A.per_sample);
    w = rem % nl;
    const uint32_t pix = rem / nl;
    x = pix % Wd;
    y = pix / Wd;
    const uint64_t s_abs = (uint64_t)A.spp_begin + sl;
    pid = ((s_abs * Hd + y) * Wd + x) * nl + w;
}

// BVH4 traversal of one ray (the stack and the traversal state are the caller's).  Closest hit:
// smallest t in (tmin, best_t), equal t to the lower original index; ANY: stop at the first
// hit.  Same node test and child ordering as traverse().
template <bool ANY>
__device__ __forceinline__ void trav_steps(const SceneDev& S, const RayT& r, float tmin, int skip, int* stk,
                                           int cap, int* ovf, size_t ostride, int& cur, int& sp, float& best_t,
                                           int& best, int& best_orig, float& hu, float& hv, uint32_t& n_nodes,
                                           uint32_t& n_tris) {
    const float ix = r.inv.x, iy = r.inv.y, iz = r.inv.z;
    const float oix = r.o.x * ix, oiy = r.o.y * iy, oiz = r.o.z * iz;
    while (true) {
        if (cur >= 0) {
            ++n_nodes;
            const float4* N = S.nodes + (size_t)cur * 8;
            const float4 lx = N[0], hx = N[1], ly = N[2], hy = N[3], lz = N[4], hz = N[5];
            const int4 ch = *reinterpret_cast<const int4*>(N + 6);
            const float lxa[4] = {lx.x, lx.y, lx.z, lx.w}, hxa[4] = {hx.x, hx.y, hx.z, hx.w};
            const float lya[4] = {ly.x, ly.y, ly.z, ly.w}, hya[4] = {hy.x, hy.y, hy.z, hy.w};
            const float lza[4] = {lz.x, lz.y, lz.z, lz.w}, hza[4] = {hz.x, hz.y, hz.z, hz.w};
            uint32_t key[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float t0x = fmaf(lxa[i], ix, -oix), t1x = fmaf(hxa[i], ix, -oix);
                const float t0y = fmaf(lya[i], iy, -oiy), t1y = fmaf(hya[i], iy, -oiy);
                const float t0z = fmaf(lza[i], iz, -oiz), t1z = fmaf(hza[i], iz, -oiz);
                const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
                const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), best_t));
                key[i] = tn <= tf ? ((__float_as_uint(tn) & ~3u) | (uint32_t)i) : 0xFFFFFFFFu;
            }
#define GRW_CSWAP(i, j)                               \
    {                                                 \
        const uint32_t lo_ = min(key[i], key[j]);     \
        key[j] = max(key[i], key[j]);                 \
        key[i] = lo_;                                 \
    }
            GRW_CSWAP(0, 1)
            GRW_CSWAP(2, 3)
            GRW_CSWAP(0, 2)
            GRW_CSWAP(1, 3)
            GRW_CSWAP(1, 2)
#undef GRW_CSWAP
#pragma unroll
            for (int i = 3; i >= 1; --i) {
                if (key[i] != 0xFFFFFFFFu) {
                    const int v = child_of(ch, key[i]);
                    if (sp < cap) stk[sp * 64] = v;
                    else ovf[(size_t)(sp - cap) * ostride + __lane_id()] = v;
                    ++sp;
                }
            }
            if (key[0] != 0xFFFFFFFFu) {
                cur = child_of(ch, key[0]);
            } else if (sp == 0) {
                cur = kDoneNode;
            } else {
                --sp;
                cur = sp < cap ? stk[sp * 64] : ovf[(size_t)(sp - cap) * ostride + __lane_id()];
            }
        } else {
            const int first = cur & 0x0FFFFFFF;
            const int cnt = ((cur >> 28) & 7) + 1;
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
                        if (ANY) return;
                    }
                }
            }
            if (sp == 0) {
                cur = kDoneNode;
            } else {
                --sp;
                cur = sp < cap ? stk[sp * 64] : ovf[(size_t)(sp - cap) * ostride + __lane_id()];
            }
        }
        if (cur == kDoneNode) return;
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Sourcing (Sec. "Interactive Rendering"): every path of the launch, in index order.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wf_generate_kernel(const TraceArgs A, const WfArgs W) {
    const SensorDev& sen = A.sensor;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W.n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t pid;
        uint32_t w, x, y;
        path_ids(A, A.path_begin + i, pid, w, x, y);
        const float k = kTwoPiF / A.lambda[w];
        const uint4 r0 = draw(pid, 0, STREAM_SOURCE, A.seed);
        const double fx = ((double)x + (double)unif(r0.x)) * (double)sen.pitch;
        const double fy = ((double)y + (double)unif(r0.y)) * (double)sen.pitch;
        d3 o = d3{sen.o[0] + fx * sen.u[0] + fy * sen.v[0], sen.o[1] + fx * sen.u[1] + fy * sen.v[1],
                  sen.o[2] + fx * sen.u[2] + fy * sen.v[2]};
        const f3 d = mk3(sen.d[0], sen.d[1], sen.d[2]);
        float beta2 = 2.0f * sen.sigma_um * sen.sigma_um, rho = 0.0f;
        // start at the scene bounds; the skipped free-space stretch is propagated here
        const float tadv = scene_entry(A.scene, o, d);
        if (tadv > 0.0f) {
            o = add_scaled(o, tadv, d);
            const float zb = tadv * 1e6f / k;
            rho = zb / beta2;
            beta2 = beta2 + zb * zb / beta2;
        }
        W.ox[i] = o.x;
        W.oy[i] = o.y;
        W.oz[i] = o.z;
        W.dx[i] = d.x;
        W.dy[i] = d.y;
        W.dz[i] = d.z;
        W.beta2[i] = beta2;
        W.rho[i] = rho;
        W.alpha[i] = 1.0f;
        W.contrib[i] = 0.0f;
        W.prev[i] = -1;
        W.list[0][i] = (uint32_t)i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        W.cnt[WC_LIST0] = (unsigned int)W.n;
        atomicAdd(A.stats + ST_PATHS, (unsigned long long)W.n);
    }
}

// Counters of bounce b: the next list, the shadow list, the fetches.
__global__ void wf_reset_kernel(const WfArgs W, int b) {
    const int t = threadIdx.x;
    if (t == 0) W.cnt[WC_LIST0 + ((b + 1) & 1)] = 0u;
    if (t == 1) W.cnt[WC_SHADOW] = 0u;
    if (t == 2) W.cnt[WC_FETCH_E] = 0u;
    if (t == 3) W.cnt[WC_FETCH_S] = 0u;
}

// ------------------------------------------------------------------------------------------
// Closest hit (ANY = false) of the bounce's paths, or visibility (ANY = true) of its shadow
// records; waves take rays from the list as they finish.
// ------------------------------------------------------------------------------------------
template <bool ANY>
__global__ __launch_bounds__(256) void wf_trace_kernel(const TraceArgs A, const WfArgs W, int b) {
    __shared__ int lds_stack[4][kLdsStack][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    int* stk = &lds_stack[wv][0][lane];
    const size_t ostride = (size_t)gridDim.x * 256;
    int* ovf = A.ovf ? A.ovf + ((size_t)blockIdx.x * 256 + 64 * __builtin_amdgcn_readfirstlane(wv)) : nullptr;
    const uint32_t n = ANY ? W.cnt[WC_SHADOW] : W.cnt[WC_LIST0 + (b & 1)];
    unsigned int* fetch = W.cnt + (ANY ? WC_FETCH_S : WC_FETCH_E);
    const uint32_t* list = W.list[b & 1];

    bool has = false, exhausted = n == 0;
    uint32_t pi = 0;
    RayT r;
    float tmin = 0.0f, best_t = 0.0f, hu = 0.0f, hv = 0.0f;
    int cur = kDoneNode, sp = 0, best = -1, best_orig = 0, skip = -1;
    uint32_t c_nodes = 0, c_tris = 0, c_rays = 0;
    while (true) {
        if (!exhausted) {
            const unsigned long long idle = __ballot(!has);
            if (idle) {
                const int first = __ffsll((long long)idle) - 1;
                const unsigned cnt = (unsigned)__popcll(idle);
                unsigned int base = 0;
                if (lane == first) base = atomicAdd(fetch, cnt);
                base = __shfl(base, first);
                if (base + cnt >= n) exhausted = true;
                if (!has) {
                    const uint32_t my = base + lane_rank(idle);
                    if (my < n) {
                        d3 o;
                        f3 d;
                        if (ANY) {
                            pi = my;
                            o = d3{W.s_px[my], W.s_py[my], W.s_pz[my]};
                            d = mk3(W.s_dx[my], W.s_dy[my], W.s_dz[my]);
                            best_t = W.s_tmax[my];
                            skip = W.s_skip[my];
                        } else {
                            pi = list[my];
                            o = d3{W.ox[pi], W.oy[pi], W.oz[pi]};
                            d = mk3(W.dx[pi], W.dy[pi], W.dz[pi]);
                            best_t = FLT_MAX;
                            skip = W.prev[pi];
                        }
                        ray_setup(r, o, d);
                        tmin = 1e-7f * (1.0f + maxabs3(to_f3(o)));
                        cur = 0;
                        sp = 0;
                        best = -1;
                        best_orig = 0x7FFFFFFF;
                        has = true;
                        ++c_rays;
                    }
                }
            }
        }
        if (!__any(has)) break;
        if (has) {
            trav_steps<ANY>(A.scene, r, tmin, skip, stk, A.lds_cap, ovf, ostride, cur, sp, best_t, best, best_orig,
                            hu, hv, c_nodes, c_tris);
            has = false;
            if (ANY) {
                W.s_vis[pi] = best < 0 ? 1 : 0;
            } else {
                W.hit[pi] = best;
                if (best >= 0) {
                    W.ht[pi] = best_t;
                    W.hu[pi] = hu;
                    W.hv[pi] = hv;
                }
            }
        }
    }
    const unsigned long long sn = wave_sum(c_nodes), st = wave_sum(c_tris), sr = wave_sum(c_rays);
    if (lane == 0) {
        atomicAdd(A.stats + ST_NODES, sn);
        atomicAdd(A.stats + ST_TRIS, st);
        if (!ANY) atomicAdd(A.stats + ST_SEGMENTS, sr);
    }
}

// ------------------------------------------------------------------------------------------
// Shading of the bounce's hits: free-space update, frame, footprint, next-event sample,
// continuation.  Same arithmetic as the persistent kernel's segment body.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wf_shade_kernel(const TraceArgs A, const WfArgs W, int b) {
    __shared__ float gcache[4][kLdsStack][64];   // grating order weights of sample_finf
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    float* cache = &gcache[wv][0][lane];
    const uint64_t total = W.cnt[WC_LIST0 + (b & 1)];
    const uint32_t* lin = W.list[b & 1];
    uint32_t* out = W.list[(b + 1) & 1];
    unsigned int* out_cnt = W.cnt + WC_LIST0 + ((b + 1) & 1);
    uint32_t c_sh = 0, c_ev = 0, c_bf = 0;
    // block-uniform trip count: every lane of a wave reaches the list appends together
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < total; base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = base + threadIdx.x;
        bool cont = false, shadow = false;
        uint32_t pi = 0;
        d3 P = d3{0.0, 0.0, 0.0};
        f3 dn = mk3(0, 0, 1), om = mk3(0, 0, 1);
        float beta2 = 0.0f, rho = 0.0f, alpha = 0.0f, tmax_s = FLT_MAX, k = 1.0f;
        float kix = 0.0f, kiy = 0.0f, kox_m = 0.0f, koy_m = 0.0f, sxx = 0.0f, syy = 0.0f, sxy = 0.0f, scale = 0.0f;
        int prev = -1, matidx = 0;
        bool act = j < total;
        if (act) {
            pi = lin[j];
            act = W.hit[pi] >= 0;   // a miss ends the path
        }
        if (act) {
            uint64_t pid;
            uint32_t w, x, y;
            path_ids(A, A.path_begin + pi, pid, w, x, y);
            k = kTwoPiF / A.lambda[w];
            const d3 o = d3{W.ox[pi], W.oy[pi], W.oz[pi]};
            const f3 d = mk3(W.dx[pi], W.dy[pi], W.dz[pi]);
            beta2 = W.beta2[pi];
            rho = W.rho[pi];
            alpha = W.alpha[pi];
            const int tri = W.hit[pi];
            float thit = W.ht[pi], bu = W.hu[pi], bv = W.hv[pi];
            const float4* T = A.scene.tris + (size_t)tri * 3;
            const float4 v0 = T[0], v1 = T[1], v2 = T[2];
            double t64;
            refine_hit(o, d, v0, v1, v2, thit, bu, bv, t64);
            // Free-space propagation of the generalized ray (eq. K_free_space_propagation)
            // over the hit distance, zbar = z / |k0|, pre-update beta and rho on the right.
            const float zb = thit * 1e6f / k;
            const float orr = 1.0f + rho * rho;
            const float rho_n = rho + zb * orr / beta2;
            beta2 = beta2 + zb * (2.0f * rho + zb * orr / beta2);
            rho = rho_n;
            P = d3{o.x + t64 * d.x, o.y + t64 * d.y, o.z + t64 * d.z};
            prev = __float_as_int(v0.w);
            matidx = __float_as_int(v1.w);
            const DMat m = A.scene.mats[matidx];
            f3 ng = normalize3(cross3(mk3(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z),
                                      mk3(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z)));
            f3 ns = ng;
            {
                const float4* NN = A.scene.tnorm + (size_t)tri * 3;
                const float4 q0 = NN[0], q1 = NN[1], q2 = NN[2];
                if ((q0.x != 0.f || q0.y != 0.f || q0.z != 0.f) && (q1.x != 0.f || q1.y != 0.f || q1.z != 0.f) &&
                    (q2.x != 0.f || q2.y != 0.f || q2.z != 0.f)) {
                    const float w0 = 1.0f - bu - bv;
                    ns = normalize3(mk3(w0 * q0.x + bu * q1.x + bv * q2.x, w0 * q0.y + bu * q1.y + bv * q2.y,
                                        w0 * q0.z + bu * q1.z + bv * q2.z));
                }
            }
            if (dot3(d, ng) > 0.0f) ng = -1.0f * ng;
            if (dot3(ns, ng) < 0.0f) ns = -1.0f * ns;
            const float ci = -dot3(d, ns);
            if (ci <= 0.0f) {
                ++c_bf;
            } else {
                // Tangent frame: x = grating direction (gratings), else the travel direction
                // projected onto the surface.
                f3 xa;
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
                const float sr2 = 0.5f * beta2;
                const float dx = dot3(d, xa), dy = dot3(d, ya);
                const float ic2 = 1.0f / (ci * ci);
                sxx = sr2 * (1.0f + dx * dx * ic2);
                syy = sr2 * (1.0f + dy * dy * ic2);
                sxy = sr2 * (dx * dy * ic2);
                // Measurement by next-event estimation (eq. measurement_operator): the shadow
                // ray is traced by the next kernel.
                if (A.nsrc > 0) {
                    const uint4 rn = draw(pid, (uint32_t)b, STREAM_NEE, A.seed);
                    const int si = min((int)(unif(rn.x) * (float)A.nsrc), A.nsrc - 1);
                    const SourceDev& L = A.src[si];
                    bool ok = false;
                    const float tminP = 1e-7f * (1.0f + maxabs3(to_f3(P)));
                    if (L.kind == 0) {
                        om = ld3(L.dir);
                        ok = true;
                    } else {
                        float z1, z2;
                        box_muller(unif(rn.y), unif(rn.z), z1, z2);
                        const float du = z1 / L.rc_um, dv = z2 / L.rc_um;
                        const float tt = (du * du + dv * dv) / (k * k);
                        if (tt < 1.0f) {
                            const f3 ax = ld3(L.dir), eu = ld3(L.bu), ev = ld3(L.bv);
                            om = (du / k) * eu + (dv / k) * ev + sqrtf(1.0f - tt) * ax;
                            const f3 pp = diff_f3(P, ld3(L.pos));   // P - emitter centre
                            const float te = dot3(pp, ax) / dot3(om, ax);
                            if (te > tminP) {
                                const f3 qp = pp - te * om;           // Q - emitter centre
                                const float a = dot3(qp, eu) / L.lu, bb = dot3(qp, ev) / L.lv;
                                if (fabsf(a) <= 1.0f && fabsf(bb) <= 1.0f) {
                                    ok = true;
                                    tmax_s = te;
                                }
                            }
                        }
                    }
                    if (ok && dot3(om, ng) < 0.0f && dot3(om, ns) < 0.0f) {
                        shadow = true;
                        ++c_sh;
                        kix = k * dot3(om, xa);
                        kiy = k * dot3(om, ya);
                        kox_m = -k * dx;
                        koy_m = -k * dy;
                        scale = alpha * L.power * (float)A.nsrc;
                    }
                }
                if (b + 1 < A.max_depth) {
                    // Light-matter interaction: sample the continuation generalized ray.
                    const uint4 rs = draw(pid, (uint32_t)b, STREAM_SCATTER, A.seed);
                    float kox, koy, wgt;
                    if (sample_finf(m, k, k * dx, k * dy, ci, unif(rs.x), unif(rs.y), unif(rs.z), kox, koy, wgt,
                                    cache, kLdsStack)) {
                        ++c_ev;
                    } else {
                        alpha *= wgt;
                        cont = true;
                        if (A.rr_enable && b + 1 >= 2) {
                            if ((rs.w >> 8) < A.rr_thr) alpha *= A.inv_rr_p;
                            else cont = false;
                        }
                        if (cont) {
                            const float kn = sqrtf(fmaxf(0.0f, 1.0f - (kox * kox + koy * koy) / (k * k)));
                            dn = normalize3((kox / k) * xa + (koy / k) * ya + kn * ns);
                        }
                    }
                }
            }
        }
        const uint32_t spos = wave_append(W.cnt + WC_SHADOW, shadow);
        if (shadow) {
            W.s_path[spos] = pi;
            W.s_px[spos] = P.x;
            W.s_py[spos] = P.y;
            W.s_pz[spos] = P.z;
            W.s_dx[spos] = -om.x;
            W.s_dy[spos] = -om.y;
            W.s_dz[spos] = -om.z;
            W.s_tmax[spos] = tmax_s;
            W.s_skip[spos] = prev;
            W.s_mat[spos] = matidx;
            const size_t n = W.n;
            W.s_q[spos] = kix;
            W.s_q[n + spos] = kiy;
            W.s_q[2 * n + spos] = kox_m;
            W.s_q[3 * n + spos] = koy_m;
            W.s_q[4 * n + spos] = sxx;
            W.s_q[5 * n + spos] = syy;
            W.s_q[6 * n + spos] = sxy;
            W.s_q[7 * n + spos] = scale;
            W.s_q[8 * n + spos] = k;
        }
        const uint32_t cpos = wave_append(out_cnt, cont);
        if (cont) {
            W.ox[pi] = P.x;
            W.oy[pi] = P.y;
            W.oz[pi] = P.z;
            W.dx[pi] = dn.x;
            W.dy[pi] = dn.y;
            W.dz[pi] = dn.z;
            W.beta2[pi] = beta2;
            W.rho[pi] = rho;
            W.alpha[pi] = alpha;
            W.prev[pi] = prev;
            out[cpos] = pi;
        }
    }
    const unsigned long long s0 = wave_sum(c_sh), s1 = wave_sum(c_ev), s2 = wave_sum(c_bf);
    if (lane == 0) {
        atomicAdd(A.stats + ST_SHADOW, s0);
        atomicAdd(A.stats + ST_EVANESCENT, s1);
        atomicAdd(A.stats + ST_BACKFACING, s2);
    }
}

// ------------------------------------------------------------------------------------------
// Measurement of the visible shadow records: p_w added to the path's contribution (each path
// has at most one record per bounce, so no two lanes write the same path); with the learned
// p_w, in-domain rough queries are queued instead.
// ------------------------------------------------------------------------------------------
template <bool DEFER>
__global__ __launch_bounds__(256) void wf_measure_kernel(const TraceArgs A, const WfArgs W, int b) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = W.cnt[WC_SHADOW];
    uint32_t c_sur = 0, c_fb = 0;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = base + threadIdx.x;
        const bool vis = j < n && W.s_vis[j] != 0;
        bool want = false;
        float sx[MLP_IN], slp = 0.0f, scale = 0.0f, refl = 0.0f;
        uint32_t pi = 0;
        if (vis) {
            pi = W.s_path[j];
            const size_t nn = W.n;
            const float kix = W.s_q[j], kiy = W.s_q[nn + j], kox = W.s_q[2 * nn + j], koy = W.s_q[3 * nn + j];
            const float sxx = W.s_q[4 * nn + j], syy = W.s_q[5 * nn + j], sxy = W.s_q[6 * nn + j];
            scale = W.s_q[7 * nn + j];
            const float k = W.s_q[8 * nn + j];
            const DMat m = A.scene.mats[W.s_mat[j]];
            refl = m.refl;
            int e = 0;
            if (DEFER && m.kind == MAT_ROUGH) {
                const SurDomain D{A.sur.gmin, A.sur.gmax, A.sur.smin, A.sur.smax};
                e = sur_encode(D, k, kix, kiy, kox, koy, sxx, syy, sxy, m.h, m.L, sx, slp);
                if (e == 0) ++c_fb;
                want = e == 1;
            }
            if (e == 0)
                W.contrib[pi] += scale * pw_plain(m.kind, m.h, m.L, m.refl, k, kix, kiy, kox, koy, sxx, syy, sxy,
                                                  1.0f, 0.0f);
            // e == 2: more than 8 lobe widths from the lobe, p_w taken as 0
        }
        if (DEFER) {
            const uint64_t r = wave_append64(A.sq_count, want);
            if (want) {
                ++c_sur;
                uint4* q = A.sq + 2 * r;
                const uint32_t slot = (uint32_t)((uint64_t)pi * (uint64_t)A.max_depth + (uint64_t)b);
                q[0] = make_uint4(bf16_pair(sx[0], sx[1]), bf16_pair(sx[2], sx[3]), bf16_pair(sx[4], sx[5]),
                                  bf16_pair(sx[6], sx[7]));
                q[1] = make_uint4(bf16_pair(sx[8], sx[9]), __float_as_uint(scale * refl * A.inv_spp_norm),
                                  __float_as_uint(slp), slot);
            }
        }
    }
    const unsigned long long s0 = wave_sum(c_sur), s1 = wave_sum(c_fb);
    if (lane == 0) {
        atomicAdd(A.stats + ST_SUR, s0);
        atomicAdd(A.stats + ST_FALLBACK, s1);
    }
}

__global__ __launch_bounds__(256) void wf_finish_kernel(const TraceArgs A, const WfArgs W) {
    uint32_t c_nf = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W.n; i += (uint64_t)gridDim.x * blockDim.x) {
        float val = W.contrib[i] * A.inv_spp_norm;
        if (!isfinite(val)) {
            ++c_nf;
            val = 0.0f;
        }
        A.records[A.path_begin + i] = val;
    }
    const unsigned long long s = wave_sum(c_nf);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(A.stats + ST_NONFINITE, s);
}

int wavefront_trav_grid(int device) {
    int ncu = 0, nb = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wf_trace_kernel<false>, 256, 0) != hipSuccess) return 0;
    int nb2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, wf_trace_kernel<true>, 256, 0) != hipSuccess) return 0;
    return ncu * std::max(1, std::min(nb, nb2));
}

// One launch of paths [a.path_begin, a.path_begin + w.n): sourcing, max_depth bounces, records.
hipError_t launch_wavefront(const TraceArgs& a, const WfArgs& w, int grid_trav, int grid_work, hipStream_t s) {
    if (w.n == 0) return hipSuccess;
    const unsigned gw = (unsigned)grid_work;
    hipLaunchKernelGGL(wf_generate_kernel, dim3(gw), dim3(256), 0, s, a, w);
    const bool defer = a.bsdf_mode != 0;
    for (int b = 0; b < a.max_depth; ++b) {
        hipLaunchKernelGGL(wf_reset_kernel, dim3(1), dim3(64), 0, s, w, b);
        hipLaunchKernelGGL((wf_trace_kernel<false>), dim3(grid_trav), dim3(256), 0, s, a, w, b);
        hipLaunchKernelGGL(wf_shade_kernel, dim3(gw), dim3(256), 0, s, a, w, b);
        hipLaunchKernelGGL((wf_trace_kernel<true>), dim3(grid_trav), dim3(256), 0, s, a, w, b);
        if (defer) hipLaunchKernelGGL((wf_measure_kernel<true>), dim3(gw), dim3(256), 0, s, a, w, b);
        else hipLaunchKernelGGL((wf_measure_kernel<false>), dim3(gw), dim3(256), 0, s, a, w, b);
    }
    hipLaunchKernelGGL(wf_finish_kernel, dim3(gw), dim3(256), 0, s, a, w);
    return hipGetLastError();
}

}  // namespace grw
