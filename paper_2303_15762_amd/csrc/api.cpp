// C ABI of libgrwave.so: argument validation, scene upload, launch orchestration.
// Validation runs before any HIP call, so every error path is reachable without a GPU.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/grwave.h"
#include "bvh_build.hpp"
#include "kernels.hpp"

static_assert(grw::kLdsNodes <= grw::kTopNodes, "the LDS copy must hold top-level nodes only");
#include "surrogate.hpp"

extern "C" int grw_coherent_launch(const gr_coherent_desc* d, float* image, hipStream_t stream, float* ms,
                                   char* err, size_t errn);

struct gr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // scene (device)
    void* d_nodes = nullptr;
    void* d_tris = nullptr;
    void* d_tnorm = nullptr;
    void* d_mats = nullptr;
    int64_t n_tris = 0;
    int64_t n_nodes = 0;
    int bvh_depth = 0;
    int max_leaf = 0;
    int64_t scene_bytes = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // vertex bounds
    float build_ms = 0.0f;
    bool has_scene = false;
    // sensor and sources (host copies)
    bool has_sensor = false;
    gr_sensor sensor{};
    std::vector<gr_source> sources;
    int grid_plain = 0;              // persistent grids (blocks), set at scene upload
    int grid_sur = 0;
    int grid_hero = 0;
    int grid_aniso = 0;
    int grid_comp = 0;
    int grid_sur_comp = 0;
    int grid_aniso_comp = 0;
    int grid_hero_comp = 0;
    int grid_batch = 0;              // blocks of the batched network pass
    // host copies of the mesh (material boundaries are found on request)
    std::vector<float> h_verts;
    std::vector<int32_t> h_tris, h_tri_mat;
    // material boundaries (gr_scene_boundaries)
    void* d_bedges = nullptr;
    void* d_btri = nullptr;
    void* d_bidx = nullptr;
    int64_t n_bedges = 0;
    float reach_m = 0.0f;
    bool has_boundaries = false;
    float weid[grw::kWeidN] = {};
    float weid_L = 0.0f;
    grw::SurrogateState sur;
};

namespace {

int fail(gr_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(gr_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define GR_HIP(c, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail(c, GR_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }
bool unit3(const float* v) {
    if (!finite3(v)) return false;
    const double n = std::sqrt((double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2]);
    return std::fabs(n - 1.0) < 1e-3;
}

void free_boundaries(gr_ctx* c) {
    if (c->d_bedges) (void)hipFree(c->d_bedges);
    if (c->d_btri) (void)hipFree(c->d_btri);
    if (c->d_bidx) (void)hipFree(c->d_bidx);
    c->d_bedges = c->d_btri = c->d_bidx = nullptr;
    c->n_bedges = 0;
    c->has_boundaries = false;
}

void free_scene(gr_ctx* c) {
    free_boundaries(c);
    if (c->d_nodes) (void)hipFree(c->d_nodes);
    if (c->d_tris) (void)hipFree(c->d_tris);
    if (c->d_tnorm) (void)hipFree(c->d_tnorm);
    if (c->d_mats) (void)hipFree(c->d_mats);
    c->d_nodes = c->d_tris = c->d_tnorm = c->d_mats = nullptr;
    c->has_scene = false;
}

constexpr size_t kWsHeader = 4096;   // dispenser counter + statistics

// Traversal stack bound: at most 3 pending siblings per inner node on the root path.
int stack_for_depth(int depth) { return 3 * (depth + 1) + 1; }
constexpr int kMaxStack = 256;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// (child, key) entries per lane kept in LDS: the lane's LDS words hold kLdsStack / 2 entries,
// of which the last two are the traversal's child-code scratch
int lds_cap_for(const gr_trace_opts* o) { return (o->flags & GR_TRACE_SHORT_LDS_STACK) ? 4 : grw::kLdsStack / 2 - 2; }

// The learned-p_w path renders in launches of at most this many paths: each launch queues at
// most one query per path and interaction (32 B) and owns one result float per slot.  Each
// launch ends in a tail where waves wait for their slowest path, so launches are made as
// large as the memory allows.
constexpr uint64_t kSurChunk = 1ull << 28;
// ... and at most this many (path, interaction) slots per launch, which bounds deep paths
// (slot numbers stay below 2^30) ...
constexpr uint64_t kSurSlots = 1ull << 30;
// ... within this many bytes of queued network queries, queued shadow rays and results (2^30
// slots of a shadow ray and a result; the learned p_w adds a query per slot).
constexpr uint64_t kQueueBytes = (1ull << 30) * 52;
struct WsLayout {
    size_t records = 0, ovf = 0, queue = 0, shadow = 0, dense = 0, nd = 0, total = 0;
    uint64_t chunk = 0;
};

bool hero_of(const gr_trace_opts* o) { return (o->flags & GR_TRACE_HERO) != 0; }
bool composite_of(const gr_trace_opts* o) { return (o->flags & GR_TRACE_COMPOSITE) != 0; }
bool aniso_of(const gr_trace_opts* o) { return (o->flags & GR_TRACE_ANISO) != 0; }
// shadow rays go through a queue of their own (hero-wavelength paths store four member values
// per slot)
bool shadow_queue_of(const gr_trace_opts*) { return true; }
uint64_t slot_values(const gr_trace_opts* o) { return hero_of(o) ? 4 : 1; }

// Traversal-stack entries per lane that do not fit the LDS part.
uint32_t overflow_entries(const gr_ctx* c, const gr_trace_opts* o) {
    return c->has_scene ? (uint32_t)std::max(0, stack_for_depth(c->bvh_depth) - lds_cap_for(o)) : 0u;
}

}  // namespace

extern "C" {

int gr_create(gr_ctx** out, int device, void* hip_stream) {
    if (!out) return GR_E_INVALID;
    *out = nullptr;
    if (device < 0) return GR_E_INVALID;
    // No HIP call here: the device is selected (and checked) by the first entry point that
    // touches it, so argument validation is usable without a GPU.
    gr_ctx* c = new gr_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return GR_OK;
}

void gr_destroy(gr_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    free_scene(c);
    grw::surrogate_free(c->sur);
    delete c;
}

const char* gr_last_error(const gr_ctx* c) { return c ? c->err.c_str() : "null context"; }

int gr_scene_upload(gr_ctx* c, const float* verts, int64_t nv, const float* normals, const int32_t* tris,
                    int64_t nt, const int32_t* tri_mat, const gr_material* mats, int32_t nm) {
    if (!c) return GR_E_INVALID;
    if (!verts || !tris || !tri_mat || !mats) return fail(c, GR_E_INVALID, "scene: null pointer");
    if (nv < 3 || nt < 1 || nm < 1) return fail(c, GR_E_INVALID, "scene: nv=%lld nt=%lld nm=%d", (long long)nv, (long long)nt, nm);
    if (nt >= (1ll << 28)) return fail(c, GR_E_UNSUPPORTED, "scene: at most 2^28 triangles");
    for (int64_t i = 0; i < nv; ++i)
        if (!finite3(verts + 3 * i)) return fail(c, GR_E_INVALID, "scene: vertex %lld not finite", (long long)i);
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (tris[i] < 0 || tris[i] >= nv) return fail(c, GR_E_INVALID, "scene: triangle index out of range at %lld", (long long)i);
    for (int64_t i = 0; i < nt; ++i)
        if (tri_mat[i] < 0 || tri_mat[i] >= nm) return fail(c, GR_E_INVALID, "scene: material index out of range at %lld", (long long)i);
    for (int i = 0; i < nm; ++i) {
        const gr_material& m = mats[i];
        if (m.kind < 0 || m.kind > 2) return fail(c, GR_E_INVALID, "material %d: kind %d", i, m.kind);
        if (!(m.reflectance >= 0.0f && m.reflectance <= 1.0f)) return fail(c, GR_E_INVALID, "material %d: reflectance", i);
        if (m.kind != GR_MAT_SMOOTH) {
            // the scattering kernels are meant for optical surface detail: heights up to 10 um,
            // lengths (correlation length, pitch) from 0.01 um to 1 mm
            if (!(m.height_um >= 0.0f && m.height_um <= 10.0f)) return fail(c, GR_E_INVALID, "material %d: height_um outside [0, 10]", i);
            if (!(m.length_um >= 0.01f && m.length_um <= 1000.0f)) return fail(c, GR_E_INVALID, "material %d: length_um outside [0.01, 1000]", i);
        }
        if (m.kind == GR_MAT_GRATING && !unit3(m.gdir)) return fail(c, GR_E_INVALID, "material %d: grating direction not unit", i);
    }
    if (normals)
        for (int64_t i = 0; i < nv; ++i)
            if (!finite3(normals + 3 * i)) return fail(c, GR_E_INVALID, "scene: normal %lld not finite", (long long)i);

    const auto t0 = std::chrono::steady_clock::now();
    grw::BuiltBVH bvh = grw::build_bvh4(verts, tris, nt);
    const auto t1 = std::chrono::steady_clock::now();
    if (stack_for_depth(bvh.depth) > kMaxStack)
        return fail(c, GR_E_UNSUPPORTED, "scene: BVH depth %d too deep", bvh.depth);

    std::vector<float> tri_data(12 * (size_t)nt), tri_norm(12 * (size_t)nt, 0.0f);
    for (int64_t j = 0; j < nt; ++j) {
        const int32_t t = bvh.tri_order[j];
        for (int cidx = 0; cidx < 3; ++cidx) {
            const float* p = verts + 3 * (int64_t)tris[3 * t + cidx];
            float* q = &tri_data[12 * j + 4 * cidx];
            q[0] = p[0];
            q[1] = p[1];
            q[2] = p[2];
            q[3] = 0.0f;
            if (normals) {
                const float* n = normals + 3 * (int64_t)tris[3 * t + cidx];
                float* r = &tri_norm[12 * j + 4 * cidx];
                r[0] = n[0];
                r[1] = n[1];
                r[2] = n[2];
            }
        }
        int32_t orig = t, mat = tri_mat[t];
        std::memcpy(&tri_data[12 * j + 3], &orig, 4);
        std::memcpy(&tri_data[12 * j + 7], &mat, 4);
    }
    std::vector<grw::DMat> dm(nm);
    for (int i = 0; i < nm; ++i) {
        dm[i].kind = mats[i].kind;
        dm[i].h = mats[i].height_um;
        dm[i].L = mats[i].length_um;
        dm[i].refl = mats[i].reflectance;
        dm[i].gx = mats[i].gdir[0];
        dm[i].gy = mats[i].gdir[1];
        dm[i].gz = mats[i].gdir[2];
        dm[i].pad = 0.0f;
    }
    GR_HIP(c, hipSetDevice(c->device));
    free_scene(c);
    const size_t nb = bvh.nodes.size() * sizeof(grw::BVH4Node);
    const size_t tb = tri_data.size() * 4, mb = dm.size() * sizeof(grw::DMat);
    if (hipMalloc(&c->d_nodes, nb) != hipSuccess || hipMalloc(&c->d_tris, tb) != hipSuccess ||
        hipMalloc(&c->d_tnorm, tb) != hipSuccess || hipMalloc(&c->d_mats, mb) != hipSuccess) {
        free_scene(c);
        (void)hipGetLastError();
        return fail(c, GR_E_OOM, "scene: device allocation of %zu bytes failed", nb + 2 * tb + mb);
    }
    GR_HIP(c, hipMemcpy(c->d_nodes, bvh.nodes.data(), nb, hipMemcpyHostToDevice));
    GR_HIP(c, hipMemcpy(c->d_tris, tri_data.data(), tb, hipMemcpyHostToDevice));
    GR_HIP(c, hipMemcpy(c->d_tnorm, tri_norm.data(), tb, hipMemcpyHostToDevice));
    GR_HIP(c, hipMemcpy(c->d_mats, dm.data(), mb, hipMemcpyHostToDevice));
    c->n_tris = nt;
    for (int a = 0; a < 3; ++a) {
        c->lo[a] = std::numeric_limits<float>::infinity();
        c->hi[a] = -std::numeric_limits<float>::infinity();
    }
    for (int64_t i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) {
            c->lo[a] = std::min(c->lo[a], verts[3 * i + a]);
            c->hi[a] = std::max(c->hi[a], verts[3 * i + a]);
        }
    c->n_nodes = (int64_t)bvh.nodes.size();
    c->bvh_depth = bvh.depth;
    c->max_leaf = bvh.max_leaf;
    c->scene_bytes = (int64_t)(nb + 2 * tb + mb);
    c->build_ms = std::chrono::duration<float, std::milli>(t1 - t0).count();
    c->grid_plain = grw::trace_grid_size(c->device, false);
    c->grid_sur = grw::trace_grid_size(c->device, true);
    c->grid_hero = grw::trace_grid_size(c->device, false, true);
    c->grid_aniso = grw::trace_grid_size(c->device, false, false, true);
    c->grid_comp = grw::trace_grid_size(c->device, false, false, false, true);
    c->grid_sur_comp = grw::trace_grid_size(c->device, true, false, false, true);
    c->grid_aniso_comp = grw::trace_grid_size(c->device, false, false, true, true);
    c->grid_hero_comp = grw::trace_grid_size(c->device, false, true, false, true);
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) ncu = 0;
        c->grid_batch = 4 * std::max(ncu, 1);
    }
    if (c->grid_plain <= 0 || c->grid_sur <= 0 || c->grid_hero <= 0 || c->grid_aniso <= 0 || c->grid_comp <= 0 ||
        c->grid_sur_comp <= 0 || c->grid_aniso_comp <= 0 || c->grid_hero_comp <= 0) {
        free_scene(c);
        return fail(c, GR_E_DEVICE, "scene: occupancy query failed");
    }
    c->h_verts.assign(verts, verts + 3 * nv);
    c->h_tris.assign(tris, tris + 3 * nt);
    c->h_tri_mat.assign(tri_mat, tri_mat + nt);
    c->has_scene = true;
    return GR_OK;
}

int gr_scene_boundaries(gr_ctx* c, float reach_m, int64_t* n_edges) {
    if (!c) return GR_E_INVALID;
    if (!(reach_m >= 1e-6f && reach_m <= 1.0f)) return fail(c, GR_E_INVALID, "boundaries: reach_m outside [1e-6, 1] m");
    if (!c->has_scene) return fail(c, GR_E_NO_SCENE, "boundaries: no scene");
    grw::BuiltBoundaries B;
    const int64_t nt = (int64_t)c->h_tri_mat.size();
    if (!grw::build_boundaries(c->h_verts.data(), c->h_tris.data(), c->h_tri_mat.data(), nt, reach_m, B))
        return fail(c, GR_E_UNSUPPORTED, "boundaries: more than 2^32 candidate entries");
    std::vector<uint32_t> tl(4 * (size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        tl[4 * t] = B.first[t];
        tl[4 * t + 1] = B.count[t];
        std::memcpy(&tl[4 * t + 2], &B.gap[t], 4);
        tl[4 * t + 3] = 0u;
    }
    GR_HIP(c, hipSetDevice(c->device));
    free_boundaries(c);
    const size_t eb = std::max<size_t>(B.edges.size(), 16) * 4, tb = tl.size() * 4,
                 ib = std::max<size_t>(B.idx.size(), 1) * 4;
    if (hipMalloc(&c->d_bedges, eb) != hipSuccess || hipMalloc(&c->d_btri, tb) != hipSuccess ||
        hipMalloc(&c->d_bidx, ib) != hipSuccess) {
        free_boundaries(c);
        (void)hipGetLastError();
        return fail(c, GR_E_OOM, "boundaries: device allocation of %zu bytes failed", eb + tb + ib);
    }
    if (!B.edges.empty()) GR_HIP(c, hipMemcpy(c->d_bedges, B.edges.data(), B.edges.size() * 4, hipMemcpyHostToDevice));
    GR_HIP(c, hipMemcpy(c->d_btri, tl.data(), tb, hipMemcpyHostToDevice));
    if (!B.idx.empty()) GR_HIP(c, hipMemcpy(c->d_bidx, B.idx.data(), B.idx.size() * 4, hipMemcpyHostToDevice));
    grw::weideman_coefficients(grw::kWeidN, c->weid, &c->weid_L);
    c->n_bedges = B.n_edges;
    c->reach_m = reach_m;
    c->has_boundaries = true;
    if (n_edges) *n_edges = B.n_edges;
    return GR_OK;
}

int gr_scene_info_get(const gr_ctx* c, gr_scene_info* info) {
    if (!c || !info) return GR_E_INVALID;
    if (!c->has_scene) return GR_E_NO_SCENE;
    info->n_tris = c->n_tris;
    info->n_nodes = c->n_nodes;
    info->depth = c->bvh_depth;
    info->max_leaf = c->max_leaf;
    info->device_bytes = c->scene_bytes;
    info->build_ms = c->build_ms;
    info->reserved = 0.0f;
    return GR_OK;
}

int gr_set_sensor(gr_ctx* c, const gr_sensor* s) {
    if (!c) return GR_E_INVALID;
    if (!s) return fail(c, GR_E_INVALID, "sensor: null");
    if (!finite3(s->origin) || !unit3(s->axis_u) || !unit3(s->axis_v) || !unit3(s->dir))
        return fail(c, GR_E_INVALID, "sensor: origin must be finite and axes / direction unit vectors");
    if (s->width < 1 || s->height < 1 || s->width > (1 << 16) || s->height > (1 << 16))
        return fail(c, GR_E_INVALID, "sensor: %d x %d pixels", s->width, s->height);
    if (!(s->pitch_m > 0.0f) || !(s->sigma_m > 0.0f) || !std::isfinite(s->pitch_m) || !std::isfinite(s->sigma_m))
        return fail(c, GR_E_INVALID, "sensor: pitch and sigma must be positive");
    c->sensor = *s;
    c->has_sensor = true;
    return GR_OK;
}

int gr_set_sources(gr_ctx* c, const gr_source* s, int32_t n) {
    if (!c) return GR_E_INVALID;
    if (n < 0 || n > grw::kMaxSources) return fail(c, GR_E_INVALID, "sources: count %d (max %d)", n, grw::kMaxSources);
    if (n > 0 && !s) return fail(c, GR_E_INVALID, "sources: null");
    for (int i = 0; i < n; ++i) {
        const gr_source& q = s[i];
        if (q.kind != GR_SRC_PLANE_WAVE && q.kind != GR_SRC_GSM_AREA) return fail(c, GR_E_INVALID, "source %d: kind %d", i, q.kind);
        if (!unit3(q.dir)) return fail(c, GR_E_INVALID, "source %d: direction not unit", i);
        if (!(q.power >= 0.0f) || !std::isfinite(q.power)) return fail(c, GR_E_INVALID, "source %d: power", i);
        if (q.kind == GR_SRC_GSM_AREA) {
            if (!(q.coherence_radius_um > 0.0f) || !finite3(q.pos) || !finite3(q.eu) || !finite3(q.ev))
                return fail(c, GR_E_INVALID, "source %d: emitter geometry / coherence radius", i);
            const double lu = std::sqrt((double)q.eu[0] * q.eu[0] + (double)q.eu[1] * q.eu[1] + (double)q.eu[2] * q.eu[2]);
            const double lv = std::sqrt((double)q.ev[0] * q.ev[0] + (double)q.ev[1] * q.ev[1] + (double)q.ev[2] * q.ev[2]);
            if (!(lu > 0.0) || !(lv > 0.0)) return fail(c, GR_E_INVALID, "source %d: empty emitter", i);
            const double du = (q.eu[0] * q.dir[0] + q.eu[1] * q.dir[1] + q.eu[2] * q.dir[2]) / lu;
            const double dv = (q.ev[0] * q.dir[0] + q.ev[1] * q.dir[1] + q.ev[2] * q.dir[2]) / lv;
            const double uv = (q.eu[0] * q.ev[0] + q.eu[1] * q.ev[1] + q.eu[2] * q.ev[2]) / (lu * lv);
            if (std::fabs(du) > 1e-4 || std::fabs(dv) > 1e-4 || std::fabs(uv) > 1e-4)
                return fail(c, GR_E_INVALID, "source %d: emitter edges must be orthogonal to each other and the axis", i);
        }
    }
    c->sources.assign(s, s + n);
    return GR_OK;
}

}  // extern "C"

namespace {
// header | path records | traversal-stack overflow of the scene's BVH (per persistent lane) |
// learned-p_w queue and per-(path, interaction) results of one launch
WsLayout ws_layout(const gr_ctx* c, const gr_trace_opts* o, int32_t nl) {
    WsLayout L;
    const uint64_t per = (uint64_t)c->sensor.width * (uint64_t)c->sensor.height * (uint64_t)nl;
    const uint64_t n = per * (uint64_t)std::max<int64_t>(o->spp_count, 0);
    const uint64_t n_paths = hero_of(o) ? n / 4 : n;   // records per path: 4 for hero paths
    const size_t lanes =
        (size_t)std::max({c->grid_plain, c->grid_sur, c->grid_hero, c->grid_aniso, c->grid_comp, c->grid_sur_comp,
                                   c->grid_aniso_comp, c->grid_hero_comp}) * 256;
    L.records = kWsHeader;
    L.ovf = L.records + align256((size_t)n * sizeof(float));
    L.queue = L.ovf + align256(lanes * overflow_entries(c, o) * 2 * sizeof(int));
    const bool defer = o->bsdf_mode != GR_BSDF_PLAIN, shq = shadow_queue_of(o);
    // bytes per (path, interaction) slot: a network query, a shadow ray, the result float (and
    // one byte per path: its stored slot count)
    const uint64_t slot_bytes =
        (defer ? grw::kSurQueryBytes : 0) + (shq ? grw::kShadowQueryBytes : 0) + 4 * slot_values(o);
    const uint64_t slots_max = std::min<uint64_t>(kSurSlots, kQueueBytes / slot_bytes);
    const uint64_t sur_chunk = std::min<uint64_t>(kSurChunk, slots_max / (uint64_t)std::max(o->max_depth, 1));
    L.chunk = std::min<uint64_t>(n_paths, sur_chunk);
    const uint64_t slots = L.chunk * (uint64_t)std::max(o->max_depth, 1);
    L.shadow = L.queue + (defer ? align256((size_t)slots * grw::kSurQueryBytes) : 0);
    L.dense = L.shadow + (shq ? align256((size_t)slots * grw::kShadowQueryBytes) : 0);
    L.nd = L.dense + (defer || shq ? align256((size_t)slots * sizeof(float) * slot_values(o)) : 0);
    L.total = L.nd + (shq ? align256((size_t)L.chunk) : 0);
    return L;
}
}  // namespace

extern "C" {

int gr_workspace_size(const gr_ctx* c, const gr_trace_opts* o, int32_t nl, size_t* bytes) {
    if (!c || !o || !bytes) return GR_E_INVALID;
    if (!c->has_sensor) return GR_E_NO_SCENE;
    if (o->spp_count < 0 || nl < 1 || nl > grw::kMaxLambda) return GR_E_INVALID;
    *bytes = ws_layout(c, o, nl).total;
    return GR_OK;
}

int gr_workspace_paths(const gr_ctx* c, void* ws, float** paths) {
    if (!c || !ws || !paths) return GR_E_INVALID;
    *paths = reinterpret_cast<float*>(static_cast<char*>(ws) + kWsHeader);
    return GR_OK;
}

}  // extern "C"

namespace {

// Allocation-free traces run in this file-scope device array instead of a caller workspace.
// Host code never passes `scratch` itself to a kernel (on the host the name is a stand-in, not
// a device address): each device's copy is looked up once with hipGetSymbolAddress, with that
// device current, and only that address is used.
constexpr size_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up on the first call).
hipError_t scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

// gr_trace and gr_trace_noalloc: ws == nullptr with use_scratch selects the static array.
int trace_impl(gr_ctx* c, const float* lambda, int32_t nl, const gr_trace_opts* o, void* ws, size_t ws_bytes,
               float* image, gr_stats* st, bool use_scratch) {
    if (!c) return GR_E_INVALID;
    if (!lambda || !o || !image) return fail(c, GR_E_INVALID, "trace: null argument");
    if (nl < 1 || nl > grw::kMaxLambda) return fail(c, GR_E_INVALID, "trace: n_lambda %d", nl);
    for (int i = 0; i < nl; ++i)
        if (!(lambda[i] >= 0.1f && lambda[i] <= 20.0f)) return fail(c, GR_E_INVALID, "trace: wavelength %d outside [0.1, 20] um", i);
    if (o->spp_begin < 0 || o->spp_count < 0 || o->spp_norm < 1) return fail(c, GR_E_INVALID, "trace: spp range");
    if (o->max_depth < 1 || o->max_depth > 64) return fail(c, GR_E_INVALID, "trace: max_depth %d", o->max_depth);
    if (o->bsdf_mode < 0 || o->bsdf_mode > 2) return fail(c, GR_E_INVALID, "trace: bsdf_mode %d", o->bsdf_mode);
    if (o->rr_enable && !(o->rr_p > 0.0f && o->rr_p <= 1.0f)) return fail(c, GR_E_INVALID, "trace: rr_p");
    if (o->flags &
        ~(GR_TRACE_KEEP_PATHS | GR_TRACE_SHORT_LDS_STACK | GR_TRACE_HERO | GR_TRACE_ANISO | GR_TRACE_COMPOSITE))
        return fail(c, GR_E_INVALID, "trace: flags");
    if (aniso_of(o) && (hero_of(o) || o->bsdf_mode != GR_BSDF_PLAIN))
        return fail(c, GR_E_UNSUPPORTED,
                    "trace: anisotropic rays with the closed-form p_w and one wavelength per path only");
    if (hero_of(o)) {
        if (nl % 4 != 0) return fail(c, GR_E_INVALID, "trace: hero wavelengths need n_lambda %% 4 == 0 (got %d)", nl);
        if (o->bsdf_mode != GR_BSDF_PLAIN)
            return fail(c, GR_E_UNSUPPORTED, "trace: hero wavelengths with the closed-form p_w only");
    }
    if (!c->has_scene || !c->has_sensor) return fail(c, GR_E_NO_SCENE, "trace: scene and sensor must be set");
    if (composite_of(o) && !c->has_boundaries)
        return fail(c, GR_E_NO_SCENE, "trace: composite interactions need gr_scene_boundaries");
    if (o->bsdf_mode != GR_BSDF_PLAIN && !c->sur.ready)
        return fail(c, GR_E_INVALID, "trace: surrogate mode without gr_set_surrogate");
    if (o->bsdf_mode != GR_BSDF_PLAIN && (c->sensor.width * (int64_t)c->sensor.height < 1))
        return fail(c, GR_E_INVALID, "trace: sensor");
    size_t need = 0;
    gr_workspace_size(c, o, nl, &need);
    if (use_scratch) {
        if (need > kScratchBytes)
            return fail(c, GR_E_WORKSPACE,
                        "trace_noalloc: this trace needs %zu bytes of workspace, more than the %zu-byte static "
                        "scratch array; use gr_trace with a caller workspace",
                        need, kScratchBytes);
        GR_HIP(c, hipSetDevice(c->device));
        GR_HIP(c, scratch_address(c->device, &ws));
        ws_bytes = kScratchBytes;
    }
    if (!ws || ws_bytes < need) return fail(c, GR_E_WORKSPACE, "trace: workspace %zu < %zu bytes", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(ws) & 15) != 0) return fail(c, GR_E_INVALID, "trace: workspace alignment");
    const uint64_t per = (uint64_t)c->sensor.width * (uint64_t)c->sensor.height * (uint64_t)nl;
    if (per >= (1ull << 32)) return fail(c, GR_E_UNSUPPORTED, "trace: width * height * n_lambda >= 2^32");

    grw::TraceArgs a{};
    a.scene.nodes = static_cast<const float4*>(c->d_nodes);
    a.scene.tris = static_cast<const float4*>(c->d_tris);
    a.scene.tnorm = static_cast<const float4*>(c->d_tnorm);
    a.scene.mats = static_cast<const grw::DMat*>(c->d_mats);
    a.scene.n_tris = c->n_tris;
    a.scene.node_bytes = (uint32_t)(c->n_nodes * 128);
    for (int i = 0; i < 3; ++i) {
        a.scene.lo[i] = c->lo[i] - 1e-3f;
        a.scene.hi[i] = c->hi[i] + 1e-3f;
    }
    const gr_sensor& s = c->sensor;
    for (int i = 0; i < 3; ++i) {
        a.sensor.o[i] = s.origin[i];
        a.sensor.u[i] = s.axis_u[i];
        a.sensor.v[i] = s.axis_v[i];
        a.sensor.d[i] = s.dir[i];
    }
    a.sensor.W = s.width;
    a.sensor.H = s.height;
    a.sensor.pitch = s.pitch_m;
    a.sensor.sigma_um = s.sigma_m * 1e6f;
    a.nsrc = (int)c->sources.size();
    for (int i = 0; i < a.nsrc; ++i) {
        const gr_source& q = c->sources[i];
        grw::SourceDev& d = a.src[i];
        d.kind = q.kind;
        for (int j = 0; j < 3; ++j) {
            d.dir[j] = q.dir[j];
            d.pos[j] = q.pos[j];
        }
        if (q.kind == GR_SRC_GSM_AREA) {
            const float lu = std::sqrt(q.eu[0] * q.eu[0] + q.eu[1] * q.eu[1] + q.eu[2] * q.eu[2]);
            const float lv = std::sqrt(q.ev[0] * q.ev[0] + q.ev[1] * q.ev[1] + q.ev[2] * q.ev[2]);
            for (int j = 0; j < 3; ++j) {
                d.bu[j] = q.eu[j] / lu;
                d.bv[j] = q.ev[j] / lv;
            }
            d.ilu = 1.0f / lu;
            d.ilv = 1.0f / lv;
        } else {
            d.ilu = d.ilv = 0.0f;
        }
        d.rc_um = q.coherence_radius_um;
        d.irc_um = q.kind == GR_SRC_GSM_AREA ? 1.0f / q.coherence_radius_um : 0.0f;
        d.power = q.power;
    }
    a.nl = nl;
    for (int i = 0; i < nl; ++i) a.lambda[i] = lambda[i];
    a.spp_begin = o->spp_begin;
    a.hero = hero_of(o) ? 1 : 0;
    a.aniso = aniso_of(o) ? 1 : 0;
    a.composite = composite_of(o) ? 1 : 0;
    if (a.composite) {
        a.bnd.edges = static_cast<const float4*>(c->d_bedges);
        a.bnd.tri_list = static_cast<const uint4*>(c->d_btri);
        a.bnd.idx = static_cast<const uint32_t*>(c->d_bidx);
        a.bnd.reach_m = c->reach_m;
        a.bnd.weid_L = c->weid_L;
        for (int i = 0; i < grw::kWeidN; ++i) a.bnd.weid[i] = c->weid[i];
    }
    a.per_sample = (uint32_t)(a.hero ? per / 4 : per);   // hero: one path per group of 4 wavelengths
    a.n_paths = (uint64_t)a.per_sample * (uint64_t)o->spp_count;
    a.inv_spp_norm = (float)(1.0 / (double)o->spp_norm);
    a.max_depth = o->max_depth;
    a.rr_enable = o->rr_enable;
    a.rr_thr = (uint32_t)std::lround((double)o->rr_p * 16777216.0);
    a.inv_rr_p = o->rr_enable ? 1.0f / o->rr_p : 1.0f;
    a.seed = o->seed;
    a.bsdf_mode = o->bsdf_mode;
    if (o->bsdf_mode != GR_BSDF_PLAIN) grw::surrogate_fill(c->sur, a.sur);
    char* base = static_cast<char*>(ws);
    const WsLayout WL = ws_layout(c, o, nl);
    const uint64_t total = a.n_paths;
    a.counter = reinterpret_cast<unsigned long long*>(base);
    a.sq_count = reinterpret_cast<unsigned long long*>(base + 128);
    a.shq_count = reinterpret_cast<unsigned long long*>(base + 2048);
    a.stats = reinterpret_cast<unsigned long long*>(base + 256);
    a.records = reinterpret_cast<float*>(base + WL.records);
    a.lds_cap = lds_cap_for(o);
    a.ovf_n = overflow_entries(c, o);
    a.ovf = a.ovf_n ? reinterpret_cast<int*>(base + WL.ovf) : nullptr;
    const bool defer = o->bsdf_mode != GR_BSDF_PLAIN;
    const bool shq = shadow_queue_of(o);
    const bool fp8 = o->bsdf_mode == GR_BSDF_SURROGATE_FP8;
    a.sq = defer ? reinterpret_cast<uint4*>(base + WL.queue) : nullptr;
    a.shq = shq ? reinterpret_cast<uint4*>(base + WL.shadow) : nullptr;
    float* dense = defer || shq ? reinterpret_cast<float*>(base + WL.dense) : nullptr;
    a.sdense = dense;
    a.snd = shq ? reinterpret_cast<uint8_t*>(base + WL.nd) : nullptr;

    GR_HIP(c, hipSetDevice(c->device));
    const int grid = defer ? (a.composite ? c->grid_sur_comp : c->grid_sur)
                           : (a.hero ? (a.composite ? c->grid_hero_comp : c->grid_hero)
                                     : (a.aniso ? (a.composite ? c->grid_aniso_comp : c->grid_aniso)
                                                : (a.composite ? c->grid_comp : c->grid_plain)));
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (st)
        for (auto& e : ev) GR_HIP(c, hipEventCreate(&e));
    GR_HIP(c, grw::launch_zero_words(reinterpret_cast<uint32_t*>(ws), kWsHeader / 4, c->stream));
    if (st) GR_HIP(c, hipEventRecord(ev[0], c->stream));
    if (shq) {
        // launches of at most WL.chunk paths: trace (measurement values to the path's slots,
        // learned-p_w queries and shadow rays queued; each path clears its own slots), one
        // batched network pass over the query queue (its results to their slots), the queued
        // shadow rays in full waves (an occluded one clears its slot), records from the slots
        const int D = o->max_depth;
        for (uint64_t p0 = 0; p0 < total; p0 += WL.chunk) {
            const uint64_t pn = std::min<uint64_t>(WL.chunk, total - p0);
            a.path_begin = p0;
            a.n_paths = pn;
            GR_HIP(c, grw::launch_chunk_reset(a.counter, a.sq_count, a.shq_count, dense, 0, c->stream));
            GR_HIP(c, grw::launch_trace(a, grid, c->stream));
            if (defer)
                GR_HIP(c, grw::launch_sur_batch(c->sur, fp8, a.sq, a.sq_count, dense, a.stats, c->grid_batch, c->stream));
            GR_HIP(c, grw::launch_shadow(a, grid, c->stream));
            if (a.hero)
                GR_HIP(c, grw::launch_hero_merge(dense, a.snd, D, a.records, p0, pn, (uint32_t)(nl / 4), (uint32_t)nl,
                                                 a.inv_spp_norm, a.stats, c->stream));
            else
                GR_HIP(c, grw::launch_shadow_merge(dense, a.snd, D, a.records, p0, pn, a.inv_spp_norm, a.stats,
                                                   c->stream));
        }
        a.n_paths = total;
    }
    if (st) GR_HIP(c, hipEventRecord(ev[1], c->stream));
    if (total > 0)
        GR_HIP(c, grw::launch_reduce(a.records, image, o->spp_count, (uint32_t)s.height, (uint32_t)s.width,
                                     (uint32_t)nl, c->stream));
    if (st) {
        GR_HIP(c, hipEventRecord(ev[2], c->stream));
        GR_HIP(c, hipStreamSynchronize(c->stream));
        unsigned long long h[grw::ST_COUNT];
        GR_HIP(c, hipMemcpy(h, a.stats, sizeof(h), hipMemcpyDeviceToHost));
        float ms = 0.0f, ms_r = 0.0f;
        GR_HIP(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
        GR_HIP(c, hipEventElapsedTime(&ms_r, ev[1], ev[2]));
        for (auto& e : ev) (void)hipEventDestroy(e);
        st->paths = h[grw::ST_PATHS];
        st->segments = h[grw::ST_SEGMENTS];
        st->shadow_rays = h[grw::ST_SHADOW];
        st->surrogate_evals = h[grw::ST_SUR];
        st->fallbacks = h[grw::ST_FALLBACK];
        st->evanescent = h[grw::ST_EVANESCENT];
        st->backfacing = h[grw::ST_BACKFACING];
        st->nonfinite = h[grw::ST_NONFINITE];
        st->node_visits = h[grw::ST_NODES];
        st->tri_tests = h[grw::ST_TRIS];
        st->composite = h[grw::ST_COMPOSITE];
        st->measured_smooth = h[grw::ST_MEAS_SMOOTH];
        st->measured_rough = h[grw::ST_MEAS_ROUGH];
        st->measured_grating = h[grw::ST_MEAS_GRATING];
        st->ms = ms;
        st->ms_reduce = ms_r;
    }
    return GR_OK;
}

}  // namespace

extern "C" {

int gr_trace(gr_ctx* c, const float* lambda, int32_t nl, const gr_trace_opts* o, void* ws, size_t ws_bytes,
             float* image, gr_stats* st) {
    return trace_impl(c, lambda, nl, o, ws, ws_bytes, image, st, false);
}

int gr_trace_noalloc(gr_ctx* c, const float* lambda, int32_t nl, const gr_trace_opts* o, float* image) {
    return trace_impl(c, lambda, nl, o, nullptr, 0, image, nullptr, true);
}

int gr_bsdf_eval(gr_ctx* c, const float* q, int64_t n, int32_t mode, float* out) {
    if (!c) return GR_E_INVALID;
    if (n < 0 || (n > 0 && (!q || !out))) return fail(c, GR_E_INVALID, "bsdf_eval: arguments");
    if (mode != GR_BSDF_PLAIN) {
        if (!c->sur.ready) return fail(c, GR_E_INVALID, "bsdf_eval: surrogate mode without gr_set_surrogate");
        if (mode != GR_BSDF_SURROGATE_BF16 && mode != GR_BSDF_SURROGATE_FP8)
            return fail(c, GR_E_INVALID, "bsdf_eval: mode %d", mode);
    }
    GR_HIP(c, hipSetDevice(c->device));
    if (mode == GR_BSDF_PLAIN) {
        GR_HIP(c, grw::launch_bsdf_eval(q, n, out, c->stream));
    } else {
        GR_HIP(c, grw::launch_bsdf_eval_surrogate(c->sur, mode == GR_BSDF_SURROGATE_FP8, q, n, out, c->stream));
    }
    return GR_OK;
}

int gr_pw_composite_eval(gr_ctx* c, const float* q, int64_t n, float* out) {
    if (!c) return GR_E_INVALID;
    if (n < 0 || (n > 0 && (!q || !out))) return fail(c, GR_E_INVALID, "pw_composite_eval: arguments");
    grw::BoundaryDev b{};
    grw::weideman_coefficients(grw::kWeidN, b.weid, &b.weid_L);
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::launch_composite_eval(q, n, out, b, c->stream));
    return GR_OK;
}

int gr_coherent_measure(gr_ctx* c, const gr_coherent_desc* d, float* image, float* ms) {
    if (!c) return GR_E_INVALID;
    GR_HIP(c, hipSetDevice(c->device));
    char buf[256] = {0};
    const int rc = grw_coherent_launch(d, image, c->stream, ms, buf, sizeof(buf));
    if (rc != GR_OK) return fail(c, rc, "%s", buf);
    return GR_OK;
}

static bool domain_ok(const float* d) {
    return d && d[0] > 0.0f && d[1] >= d[0] && d[2] > 0.0f && d[3] >= d[2] && std::isfinite(d[1]) &&
           std::isfinite(d[3]);
}

int gr_surrogate_samples(gr_ctx* c, int64_t n, uint64_t seed, const float* domain, float* x, float* y, float* q) {
    if (!c) return GR_E_INVALID;
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, GR_E_INVALID, "surrogate_samples: arguments");
    if (!domain_ok(domain)) return fail(c, GR_E_INVALID, "surrogate_samples: domain");
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::surrogate_samples(n, seed, domain, x, y, q, c->stream));
    return GR_OK;
}

int gr_mlp_workspace_size(int64_t n, size_t* bytes) {
    if (n < 0 || !bytes) return GR_E_INVALID;
    *bytes = grw::mlp_workspace_bytes(n);
    return GR_OK;
}

int gr_mlp_forward(gr_ctx* c, const float* params, const float* x, int64_t n, int32_t dtype, void* ws, float* y) {
    if (!c) return GR_E_INVALID;
    if (!params || !ws || n < 0 || (n > 0 && (!x || !y))) return fail(c, GR_E_INVALID, "mlp_forward: arguments");
    if (dtype != GR_BSDF_SURROGATE_BF16 && dtype != GR_BSDF_SURROGATE_FP8)
        return fail(c, GR_E_INVALID, "mlp_forward: dtype %d", dtype);
    if ((reinterpret_cast<uintptr_t>(ws) & 15) != 0) return fail(c, GR_E_INVALID, "mlp_forward: workspace alignment");
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::mlp_forward(params, x, n, dtype == GR_BSDF_SURROGATE_FP8, ws, y, c->stream));
    return GR_OK;
}

int gr_mlp_backward(gr_ctx* c, const float* params, const float* x, const float* t, int64_t n, void* ws, float* grad,
                    float* loss) {
    if (!c) return GR_E_INVALID;
    if (!params || !x || !t || !ws || !grad || !loss || n < 1) return fail(c, GR_E_INVALID, "mlp_backward: arguments");
    if ((reinterpret_cast<uintptr_t>(ws) & 15) != 0) return fail(c, GR_E_INVALID, "mlp_backward: workspace alignment");
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::mlp_backward(params, x, t, n, ws, grad, loss, c->stream));
    return GR_OK;
}

int gr_mlp_activation(gr_ctx* c, const float* x, int64_t n, float* y, float* dy) {
    if (!c) return GR_E_INVALID;
    if (n < 0 || n > ((int64_t)1 << 40) || (n > 0 && (!x || !y || !dy)))
        return fail(c, GR_E_INVALID, "mlp_activation: arguments");
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::activation(x, n, y, dy, c->stream));
    return GR_OK;
}

int gr_adam_step(gr_ctx* c, float* p, const float* g, float* m, float* v, int32_t t, float lr, float b1, float b2,
                 float eps) {
    if (!c) return GR_E_INVALID;
    if (!p || !g || !m || !v || t < 1 || !(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(c, GR_E_INVALID, "adam_step: arguments");
    GR_HIP(c, hipSetDevice(c->device));
    GR_HIP(c, grw::adam(p, g, m, v, t, lr, b1, b2, eps, c->stream));
    return GR_OK;
}

int gr_set_surrogate(gr_ctx* c, const float* params, const float* domain) {
    if (!c) return GR_E_INVALID;
    if (!params || !domain_ok(domain)) return fail(c, GR_E_INVALID, "set_surrogate: arguments");
    GR_HIP(c, hipSetDevice(c->device));
    const hipError_t e = grw::surrogate_set(c->sur, params, domain, c->stream);
    if (e == hipErrorOutOfMemory) return fail(c, GR_E_OOM, "set_surrogate: allocation failed");
    if (e != hipSuccess) return fail(c, GR_E_DEVICE, "set_surrogate: %s", hipGetErrorString(e));
    return GR_OK;
}

}  // extern "C"
