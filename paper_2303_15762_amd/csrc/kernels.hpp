// Device-side argument blocks shared by the kernels and the host ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.hpp"

namespace grw {

constexpr int kMaxSources = 16;
constexpr int kMaxLambda = 64;
// LDS words per lane of the traversal stack: kLdsStack / 2 - 2 entries of (child code, entry
// key) and 16 bytes of child-code scratch; deeper entries go to the overflow region.
constexpr int kLdsStack = 32;
// BVH nodes 0 .. kLdsNodes - 1 (the builder puts the top levels there, breadth-first) are
// copied into each block's LDS by the traversal kernels: 8 KB beside the 32 KB of stacks,
// so that four blocks still fill the 160 KB of a compute unit.
constexpr int kLdsNodes = 64;

struct SceneDev {
    const float4* nodes;     // BVH4Node as 8 float4 each
    const float4* tris;      // 3 float4 per triangle in leaf order: v0 (w = original id), v1 (w = material), v2
    const float4* tnorm;     // 3 float4 per triangle: per-vertex shading normals (zero = geometric)
    const DMat* mats;
    int64_t n_tris;
    float lo[3], hi[3];      // bounds of all vertices widened by 1 mm
    uint32_t node_bytes;     // size of the node array (bounds of its buffer loads)
};

struct SensorDev {
    double o[3], u[3], v[3];  // origin and pixel axes (the float inputs, exactly)
    float d[3];
    int W, H;
    float pitch;      // metres
    float sigma_um;
};

struct SourceDev {
    int kind;         // 0 plane wave, 1 gaussian-schell area
    float dir[3];     // travel direction / emission axis (unit)
    float pos[3];
    float bu[3], bv[3];   // unit in-plane axes of the emitter
    float ilu, ilv;       // reciprocal half extents (1/m)
    float rc_um, irc_um;  // coherence radius (um) and its reciprocal
    float power;
};

// Trained domain of the learned p_w (the trace kernel encodes queries; a batched
// matrix-core kernel evaluates them after the trace).
struct SurrogateDev {
    float gmin, gmax, smin, smax;
    int enabled;
};

// One deferred learned-p_w query, 32 bytes: the 10 network inputs as bfloat16 pairs (the
// network rounds its inputs to bfloat16 anyway), the contribution scale (the merge divides it
// by the sample count), log of the lobe peak, and the (path, depth) slot of the result.
constexpr int kSurQueryBytes = 32;

// Terms of the rational approximation of the Faddeeva function (composite interactions).
constexpr int kWeidN = 16;

// Material boundaries of the scene (gr_scene_boundaries) for composite interactions, and the
// constants of the device's Faddeeva approximation.
struct BoundaryDev {
    const float4* edges;     // 4 float4 per boundary edge: p0 (w: material of triangle a, as int
                             // bits), p1 (w: material of triangle b), the third vertex of a, of b
    const uint4* tri_list;   // per original triangle: first and count into idx, a lower bound
                             // of its distance to those edges (float bits, metres), 0
    const uint32_t* idx;     // boundary edges of the triangle's material near it, ascending
    float reach_m;           // largest boundary distance considered
    float weid_L;
    float weid[kWeidN];      // a_1 .. a_N
};

struct TraceArgs {
    SceneDev scene;
    SensorDev sensor;
    SourceDev src[kMaxSources];
    int nsrc;
    int nl;
    float lambda[kMaxLambda];
    int64_t spp_begin;
    uint64_t path_begin;       // first path index of this launch
    uint64_t n_paths;          // paths of this launch: [path_begin, path_begin + n_paths)
    uint32_t per_sample;       // paths per sample: H * W * nl, or H * W * nl / 4 with hero
    int hero;                  // 1: hero-wavelength paths over rotation groups of 4 wavelengths
    int aniso;                 // 1: anisotropic generalized rays (matrix beta, rho)
    int composite;             // 1: composite interactions at material boundaries
    BoundaryDev bnd;
    float inv_spp_norm;
    int max_depth;
    int rr_enable;
    uint32_t rr_thr;           // survive iff (draw >> 8) < rr_thr
    float inv_rr_p;
    uint64_t seed;
    int bsdf_mode;
    SurrogateDev sur;
    uint4* sq;                       // deferred learned-p_w queries (2 uint4 each), or null
    unsigned long long* sq_count;
    uint4* shq;                      // queued shadow rays (3 uint4 each), or null
    unsigned long long* shq_count;
    float* sdense;                   // measurement values by (path, interaction) slot
                                     // [paths of the launch][max_depth] (four floats per slot
                                     // for hero-wavelength paths); a path stores the slots of
                                     // its first snd[path] interactions
    uint8_t* snd;                    // [paths of the launch]
    float* records;                  // [n_paths]
    int* ovf;                        // traversal stack overflow [ovf_n][grid * 256][2] (child, key), or null
    uint32_t ovf_n;                  // overflow entries per lane
    int lds_cap;                     // stack entries kept in LDS (<= kLdsStack / 2 - 2: two ints each)
    unsigned long long* counter;     // path dispenser
    unsigned long long* stats;       // [16]
};

enum {
    ST_PATHS = 0, ST_SEGMENTS, ST_SHADOW, ST_SUR, ST_FALLBACK, ST_EVANESCENT, ST_BACKFACING,
    ST_NONFINITE, ST_NODES, ST_TRIS, ST_COMPOSITE, ST_MEAS_SMOOTH, ST_MEAS_ROUGH, ST_MEAS_GRATING, ST_COUNT
};
static_assert(ST_COUNT <= 16, "the statistics array holds 16 counters");

// Launchers (trace.hip).
hipError_t launch_trace(const TraceArgs& a, int grid, hipStream_t s);
hipError_t launch_reduce(const float* records, float* image, int64_t spp_count, uint32_t H, uint32_t W,
                         uint32_t nl, hipStream_t s);
// Zero the path dispenser, the query and shadow-ray counts (shq_count may be null) and n
// floats of per-(path, depth) results.
hipError_t launch_chunk_reset(unsigned long long* counter, unsigned long long* sq_count,
                              unsigned long long* shq_count, float* dense, uint64_t n, hipStream_t s);
hipError_t launch_shadow(const TraceArgs& a, int grid, hipStream_t s);
// p[0 .. n) = 0 (32-bit words)
hipError_t launch_zero_words(uint32_t* p, uint64_t n, hipStream_t s);
// records[p0 + i] = inv_spp_norm * sum over d < nd[i] of val[i * depth + d], i < n (fixed order)
hipError_t launch_shadow_merge(const float* val, const uint8_t* nd, int depth, float* records, uint64_t p0,
                               uint64_t n, float inv_spp_norm, unsigned long long* stats, hipStream_t s);
// hero-wavelength records: member j of path p0 + i gets the sum over d < nd[i] of
// val[(i * depth + d) * 4 + j], at record ((p0 + i) / G) nl + (p0 + i) % G + j G
hipError_t launch_hero_merge(const float* val, const uint8_t* nd, int depth, float* records, uint64_t p0,
                             uint64_t n, uint32_t G, uint32_t nl, float inv_spp_norm, unsigned long long* stats,
                             hipStream_t s);
// a queued shadow ray: mean position (3 doubles), travel direction of the light, emitter
// distance, triangle left, slot
constexpr int kShadowQueryBytes = 48;
int trace_grid_size(int device, bool sur, bool hero = false, bool aniso = false, bool composite = false);

// Batch p_w evaluation (trace.hip).
hipError_t launch_bsdf_eval(const float* q, int64_t n, float* out, hipStream_t s);
// Batch composite p_w evaluation: rows of 23 floats (see gr_pw_composite_eval).
hipError_t launch_composite_eval(const float* q, int64_t n, float* out, const BoundaryDev& b, hipStream_t s);

}  // namespace grw
