/* grwave: backward generalized-ray wave-optical path tracing on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libgrwave.so.  Plain pointers and sizes only.
 *
 * Paper: "A Generalized Ray Formulation for Wave-Optics Rendering" (arXiv 2303.15762).
 *
 * Conventions (all entry points):
 *  - Every function returns GR_OK (0) or a negative GR_E_* status; gr_last_error() then holds a
 *    message.  No C++ exception and no abort crosses the ABI.
 *  - "host" pointers are read (and copied) before the call returns.  "device" pointers must
 *    point to memory on the context's device, be suitably aligned (4 bytes for float data,
 *    16 bytes for workspaces) and stay alive until the work enqueued on the context's stream has
 *    completed; they are owned by the caller.
 *  - Work is enqueued on the stream given to gr_create and is asynchronous unless stated.
 *  - Geometry is in metres, surface heights, lengths, coherence radii and wavelengths in
 *    micrometres.
 *  - A context is not thread-safe; use one per thread (and per device / stream).
 */
#ifndef GRWAVE_H
#define GRWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gr_ctx gr_ctx;

enum {
    GR_OK = 0,
    GR_E_INVALID = -1,      /* bad argument: null pointer, size, enum or range */
    GR_E_NO_SCENE = -2,     /* trace before scene / sensor upload */
    GR_E_DEVICE = -3,       /* HIP runtime error */
    GR_E_OOM = -4,          /* device allocation failed (scene upload, surrogate upload) */
    GR_E_UNSUPPORTED = -5,  /* valid request this build does not implement */
    GR_E_WORKSPACE = -6     /* workspace missing or smaller than gr_workspace_size */
};

enum { GR_MAT_SMOOTH = 0, GR_MAT_ROUGH = 1, GR_MAT_GRATING = 2 };
enum { GR_SRC_PLANE_WAVE = 0, GR_SRC_GSM_AREA = 1 };
enum { GR_BSDF_PLAIN = 0, GR_BSDF_SURROGATE_BF16 = 1, GR_BSDF_SURROGATE_FP8 = 2 };

/* Surface material.  Sec. "Interaction Kernels":
 *   SMOOTH  : reflection by a flat interface (eq. K_reflection_refraction), Fresnel factor
 *             = reflectance.
 *   GRATING : 1-D sinusoidal height h(x) = height_um * sin(2 pi g.x / length_um) (eq. K_grating):
 *             height_um = amplitude A (half the peak-to-valley depth), length_um = pitch,
 *             gdir = grating vector direction in world space (projected onto the surface).
 *   ROUGH   : Gaussian random surface (eq. K_surface_HS, ensemble-averaged scatter):
 *             height_um = RMS height, length_um = 1/e correlation length of the Gaussian
 *             autocorrelation. */
typedef struct {
    int32_t kind;
    float height_um;
    float length_um;
    float gdir[3];
    float reflectance;
} gr_material;

/* Orthographic sensor: pixel (x, y) covers origin + [x, x+1) pitch axis_u + [y, y+1) pitch axis_v.
 * Each detection state (Sec. "Measurement of the WDF", coherent states) is sourced with its mean
 * position uniform on the pixel, mean direction dir, intensity standard deviation sigma_m
 * (beta^2 / 2 = sigma^2) and rho = 0 (Sec. "Interactive Rendering", implementation details).
 * axis_u, axis_v, dir must be unit vectors; width, height >= 1; pitch_m, sigma_m > 0. */
typedef struct {
    float origin[3];
    float axis_u[3];
    float axis_v[3];
    float dir[3];
    int32_t width;
    int32_t height;
    float pitch_m;
    float sigma_m;
} gr_sensor;

/* Light source (Sec. "Interactive Rendering": distant sources and emitting areas).
 *   PLANE_WAVE: spatially coherent plane wave travelling along dir (unit); power = irradiance
 *               scale.  Visible where a ray along -dir escapes the scene.
 *   GSM_AREA  : Gaussian-Schell emitter: parallelogram pos +- eu +- ev (eu, ev orthogonal to
 *               the unit emission axis dir and to each other) emitting around dir with the
 *               tangential wavevector density N(0, coherence_radius_um^-2 I) (Sec.
 *               "Sample-Solve": source coherence fixes the angular spread). */
typedef struct {
    int32_t kind;
    float dir[3];
    float pos[3];
    float eu[3];
    float ev[3];
    float coherence_radius_um;
    float power;
} gr_source;

enum {
    GR_TRACE_KEEP_PATHS = 1,
    GR_TRACE_SHORT_LDS_STACK = 2,
    /* 4 is not used */
    GR_TRACE_HERO = 8,
    GR_TRACE_ANISO = 16,
    GR_TRACE_COMPOSITE = 32
};

/* Trace options.
 *   spp_begin, spp_count : sample indices [spp_begin, spp_begin + spp_count) of every pixel and
 *                          wavelength.  The random streams are keyed by the absolute index, so
 *                          disjoint ranges add up to the full render.
 *   spp_norm             : every path contribution is divided by this (normally the total
 *                          number of samples per pixel).
 *   max_depth            : number of surface interactions per path (>= 1, <= 64).
 *   bsdf_mode            : GR_BSDF_* (surrogate modes need gr_set_surrogate).
 *   rr_enable, rr_p      : Russian roulette from the third path segment on, survival
 *                          probability rr_p in (0, 1].
 *   seed                 : Philox key.
 *   flags                : GR_TRACE_KEEP_PATHS keeps the per-path contributions in the
 *                          workspace (see gr_workspace_paths).  GR_TRACE_SHORT_LDS_STACK keeps
 *                          only 4 BVH traversal-stack entries per lane in LDS and the rest in
 *                          the workspace (normally 14 stay in LDS, and the workspace holds the
 *                          deeper entries of BVHs of more than 3 levels); the image is
 *                          identical, the render slower.  It
 *                          exists to exercise the overflow path.  GR_TRACE_HERO traces
 *                          hero-wavelength paths (Sec. "Interactive Rendering", implementation
 *                          details: the hero wavelength drives the path and up to three more
 *                          wavelengths ride along): the n_lambda wavelengths (a multiple of 4)
 *                          form G = n_lambda / 4 rotation groups {g, g + G, g + 2G, g + 3G}; one
 *                          path per (pixel, sample, group) is sampled at a member drawn
 *                          uniformly (the hero), every member keeps its own beta, rho and
 *                          footprint, and the members' estimates are combined by the one-sample
 *                          balance heuristic over the choice of hero (grating orders other than
 *                          0 are dispersive and carry the hero alone).  A quarter of the paths
 *                          of the default render, a different estimator of the same image; the
 *                          records keep their layout.  Closed-form p_w only (else
 *                          GR_E_UNSUPPORTED).  GR_TRACE_ANISO carries
 *                          anisotropic generalized rays (Sec. "Generalized rays": beta, rho as
 *                          positive-definite matrices): the ray's phase-space second moments
 *                          over its two transverse axes go through the free-space law in matrix
 *                          form, and every interaction maps them from the incoming to the
 *                          outgoing transverse plane through the surface (positions by the
 *                          projection map G, wavevectors by G^-T), so a grating order or rough
 *                          lobe leaving at another angle than it arrived stretches the ray
 *                          along the plane of scattering; the footprint at each hit is the
 *                          ray's spatial moments on the surface.  Without the flag beta, rho
 *                          stay scalar and interactions leave them unchanged.  Closed-form p_w
 *                          and one wavelength per path only (else GR_E_UNSUPPORTED).
 *                          GR_TRACE_COMPOSITE applies composite interactions (Sec. "Wave-Optical
 *                          Rendering": a generalized ray whose footprint covers two materials
 *                          meets the composition of their interaction operators, whose scattered
 *                          waves interfere) where a material boundary found by
 *                          gr_scene_boundaries lies within the ball that holds the ray: the
 *                          measurement takes the composite p_w of the two sides (see
 *                          gr_pw_composite_eval) and the continuation samples the far side's
 *                          unwindowed kernel with the probability of the window's intensity mass
 *                          beyond the boundary, else the near side's.  Needs gr_scene_boundaries
 *                          (else GR_E_NO_SCENE).  With GR_TRACE_ANISO the footprint is the
 *                          anisotropic ray's; with GR_TRACE_HERO the boundary is found with the
 *                          hero's window, each member measures with its own window and the
 *                          companions' ratios follow the sides' mixture (reading R31).  With
 *                          a surrogate bsdf_mode the composite
 *                          measurements keep the closed form (the network holds one material's
 *                          p_w) and the other rough ones in the trained domain go to the
 *                          network.  Other bits are invalid. */
typedef struct {
    int64_t spp_begin;
    int64_t spp_count;
    int64_t spp_norm;
    int32_t max_depth;
    int32_t bsdf_mode;
    int32_t rr_enable;
    float rr_p;
    uint64_t seed;
    int32_t flags;
    int32_t reserved;
} gr_trace_opts;

/* Counters of one trace (filled only when a gr_stats pointer is passed; that call then
 * synchronises the stream). */
typedef struct {
    uint64_t paths;
    uint64_t segments;          /* closest-hit queries, escaping ones included */
    uint64_t shadow_rays;       /* any-hit queries of next-event estimation */
    uint64_t surrogate_evals;   /* learned-p_w queries evaluated by the network (the persistent
                                   kernel queues them before their shadow rays are traced, so
                                   occluded ones count too) */
    uint64_t fallbacks;         /* surrogate mode queries outside the trained domain */
    uint64_t evanescent;        /* paths ended by an evanescent continuation */
    uint64_t backfacing;        /* paths ended at a back-facing shading normal */
    uint64_t nonfinite;         /* non-finite contributions dropped */
    uint64_t node_visits;       /* BVH nodes fetched (closest-hit and any-hit) */
    uint64_t tri_tests;         /* triangle tests (closest-hit and any-hit) */
    uint64_t composite;         /* interactions that met a material boundary (GR_TRACE_COMPOSITE) */
    uint64_t measured_smooth;   /* vertices that evaluated a measurement (an emitter direction on
                                   the lit side of the geometric and shading normals), at smooth, */
    uint64_t measured_rough;    /* rough */
    uint64_t measured_grating;  /* and grating surfaces; their sum is shadow_rays */
    float ms;                   /* device time of the path-tracing kernels (trace, network
                                   pass, shadow rays, record merge) */
    float ms_reduce;            /* device time of the per-pixel reduction */
} gr_stats;

typedef struct {
    int64_t n_tris;
    int64_t n_nodes;            /* 4-wide BVH nodes (128 bytes each) */
    int32_t depth;              /* deepest node level (root = 0) */
    int32_t max_leaf;           /* largest leaf size */
    int64_t device_bytes;       /* scene bytes resident on the device */
    float build_ms;             /* host BVH build time */
    float reserved;
} gr_scene_info;

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t, or
 * NULL for the default stream).  The library allocates device memory only in
 * gr_scene_upload and gr_set_surrogate; the trace path uses the caller's workspace. */
int gr_create(gr_ctx** out, int device, void* hip_stream);
void gr_destroy(gr_ctx* ctx);
const char* gr_last_error(const gr_ctx* ctx);

/* Upload a triangle scene (host arrays, copied).  verts_m: [nv][3]; normals: [nv][3] unit
 * per-vertex shading normals or NULL (a zero normal selects the geometric normal of the
 * triangles using that vertex); tris: [nt][3] vertex indices; tri_mat: [nt] material
 * indices into mats[nm].  Builds a 4-wide SAH BVH on the host.  Replaces any previous scene.
 * Ray tracing of the generalized ray's mean is valid under the paper's interactive assumption
 * (footprint small against geometric detail, Sec. "Interactive Rendering"). */
int gr_scene_upload(gr_ctx* ctx, const float* verts_m, int64_t nv, const float* normals,
                    const int32_t* tris, int64_t nt, const int32_t* tri_mat,
                    const gr_material* mats, int32_t nm);
int gr_scene_info_get(const gr_ctx* ctx, gr_scene_info* info);

/* Material boundaries of the uploaded scene, for GR_TRACE_COMPOSITE (Sec. "Wave-Optical
 * Rendering", composite interactions): every mesh edge used by exactly two triangles (same
 * vertex indices) whose materials differ.  For each triangle, the boundary edges of its own
 * material within reach_m metres of it are listed on the device; a hit then takes the nearest
 * of them within min(2.5 beta_max, reach_m), beta_max = sqrt(2) times the footprint's largest
 * standard deviation, as one straight boundary carried onto the hit's tangent plane.
 * reach_m in [1e-6, 1]; n_edges (optional, host) receives the number of boundary edges.
 * Allocates device memory (64 B per edge, 8 B per triangle, 4 B per list entry); replaced by
 * the next call and freed with the scene.  Errors: GR_E_NO_SCENE before gr_scene_upload,
 * GR_E_INVALID for reach_m, GR_E_OOM, GR_E_UNSUPPORTED beyond 2^32 list entries. */
int gr_scene_boundaries(gr_ctx* ctx, float reach_m, int64_t* n_edges);

int gr_set_sensor(gr_ctx* ctx, const gr_sensor* sensor);
/* Up to 16 sources; next-event estimation picks one uniformly per interaction. */
int gr_set_sources(gr_ctx* ctx, const gr_source* sources, int32_t n);

/* Workspace (device memory) needed by gr_trace for these options and n_lambda wavelengths:
 * a header, one float per (sample, pixel, wavelength) record, the traversal-stack overflow of
 * the uploaded scene's BVH (one region per persistent lane, 3 entries per BVH level beyond the
 * LDS part), and for one launch of the persistent kernel its queued shadow rays (48 B),
 * measurement slots (4 B, or 16 B with hero wavelengths: one float per member) and, with a
 * learned p_w, network queries (32 B) per (path, interaction), plus one byte per path (at most
 * 52 GiB of these per launch).  Call it after gr_scene_upload: the size depends on the scene
 * and the device. */
int gr_workspace_size(const gr_ctx* ctx, const gr_trace_opts* opts, int32_t n_lambda,
                      size_t* bytes);
/* Device pointer (inside `workspace`) of the per-path contributions kept by
 * GR_TRACE_KEEP_PATHS: float [spp_count][height][width][n_lambda], already divided by
 * spp_norm. */
int gr_workspace_paths(const gr_ctx* ctx, void* workspace, float** paths_dev);

/* Render: Algorithm 1 under the interactive assumption (ray-traced propagation, next-event
 * estimation as the measurement, continuation sampled from the interaction kernel).
 *   lambda_um : host [n_lambda] wavelengths (um), 1 <= n_lambda <= 64.
 *   workspace : device, >= gr_workspace_size bytes.
 *   image     : device float [n_lambda][height][width]; contributions are ADDED to it.
 *   stats     : optional; when given the call synchronises the stream and fills it.
 * The path kernel stores each measurement value in its (path, interaction) slot (the four
 * members' values for hero-wavelength paths) and queues the measurement's shadow ray (48 B);
 * a shadow-ray kernel traces the queue in full waves and clears the slots of occluded ones,
 * and a merge sums each path's slots in depth order into its record(s).  Surrogate modes also queue
 * in-domain rough-surface measurements (32 B each) for one batched matrix-core pass, which
 * writes their slots before the shadow rays are traced.  Launches hold at most 256M paths and
 * 2^30 slots within 52 GiB of queues and slots (the workspace holds one launch's).
 * Same options and seed give a bitwise identical image. */
int gr_trace(gr_ctx* ctx, const float* lambda_um, int32_t n_lambda, const gr_trace_opts* opts,
             void* workspace, size_t workspace_bytes, float* image, gr_stats* stats);

/* gr_trace without a workspace argument and without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same kernels, launches and image as gr_trace (bit for bit); the workspace
 * is a 64 MiB array in the library's device memory (one per GPU, held until the process
 * ends; its address is looked up on the first call on each device).  The call allocates
 * nothing (no hipMalloc, hipFree, events or library allocations), clears what must start at
 * zero with kernels (no memset nodes), enqueues on the context's stream and returns without
 * synchronising; no statistics.
 *   image : device float [n_lambda][height][width], caller-owned; contributions are ADDED.
 * Errors: as gr_trace; GR_E_WORKSPACE when gr_workspace_size for these options exceeds
 * 64 MiB (e.g. a 41 x 29 sensor with 8 wavelengths, 16 samples and depth 4 over a
 * 65,536-triangle terrain needs about 62 MB, half of it the traversal stack's overflow region
 * for every persistent lane; full-size frames need gr_trace).  Every call on one GPU shares that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU (two streams, two
 * contexts, two threads) race and must be serialised by the caller.  The per-path records
 * of GR_TRACE_KEEP_PATHS stay in the array and are not accessible. */
int gr_trace_noalloc(gr_ctx* ctx, const float* lambda_um, int32_t n_lambda, const gr_trace_opts* opts,
                     float* image);

/* Windowed diffraction density p_w(k_i,t -> k_o,t) (um^2) for a batch of queries (device).
 * Row layout (14 floats): kind, height_um, length_um, reflectance, k (um^-1), kix, kiy, kox,
 * koy (tangential wavevectors in the material frame, um^-1), sxx, syy, sxy (footprint
 * covariance of the window on the surface, um^2), gx, gy (grating direction in the frame).
 * mode GR_BSDF_PLAIN evaluates the closed form; surrogate modes evaluate the uploaded network
 * where the query is inside its domain and the closed form elsewhere.  out: device [n]. */
int gr_bsdf_eval(gr_ctx* ctx, const float* queries, int64_t n, int32_t mode, float* out);

/* Composite p_w (um^2) at a straight material boundary for a batch of queries (device), the
 * operator GR_TRACE_COMPOSITE applies (Sec. "Wave-Optical Rendering": composition of two
 * materials' interaction operators).  In surface coordinates x about the hit, the near
 * material fills n.x < c and the far one n.x > c; p_w is the squared Fourier integral of the
 * amplitude window exp(-x^T S^-1 x / 4) times each side's reflection function over its
 * half-plane, normalised like gr_bsdf_eval's p_w, averaged over the (unstated) position of
 * each side's deterministic profile, so that the orders of a side add in power and the sides
 * interfere through their undiffracted mean fields; a rough side's diffuse terms are its
 * single-material ones weighted by the window's intensity mass on its side.
 * Row layout (23 floats): near material kind, height_um, length_um, reflectance, grating
 * direction (gx, gy) in the frame; far material (the same six); k (um^-1); kix, kiy, kox, koy
 * (um^-1); sxx, syy, sxy (footprint covariance, um^2); nx, ny (unit normal of the boundary,
 * towards the far side); c >= 0 (um).  out: device [n]. */
int gr_pw_composite_eval(gr_ctx* ctx, const float* queries, int64_t n, float* out);

/* Learned scattering model (the surrogate of p_w for Gaussian rough surfaces): a
 * 10 -> 64 -> 64 -> 64 -> 64 -> 1 perceptron with GELU (tanh form).
 * params: device float [13249] laid out W1[10][64], b1[64], W2[64][64], b2, W3, b3, W4, b4,
 * W5[64][1], b5[1] (row-major [fan_in][fan_out]; a layer computes x W + b).  The matrix-core
 * passes accumulate in FP32.  GR_BSDF_SURROGATE_BF16 rounds weights and activations to
 * bfloat16.  GR_BSDF_SURROGATE_FP8 runs the input layer on bfloat16 operands and the three
 * 64 x 64 hidden layers on OCP E4M3 operands: weights per output neuron with scale
 * max|W| / 448 over its 64 inputs (and a second E4M3 copy of the quantized weights divided by
 * 16), activations per query and layer with scale max|a| / 448 as two E4M3 terms (the value
 * and 16 times its rounding residual), accumulated in FP32; the output layer runs on the
 * vector ALUs in FP32 in both modes.
 *
 * Input encoding of a query (sur_encode in the sources; rough surfaces only): the tangential
 * transfer in lobe widths sqrt(2 g) / l (g = (q_z s)^2), the incident tangential direction,
 * log wavelength, log footprint std devs (diagonal footprint), log s, log l, log g, each
 * affinely scaled to about [-1, 1]; the output is log p_w minus log(l^2 / (4 pi g)).
 * domain (host [4]): {g_min, g_max, sigma_min_um, sigma_max_um} of the queries the network
 * covers; elsewhere the closed form is used. */
enum { GR_MLP_PARAMS = 13249 };

/* Draw n training samples on the device: x_out [n][10] encoded inputs, y_out [n] targets
 * (closed-form log p_w relative to the lobe peak, floored at -20), q_out [n][14] the raw
 * queries in the gr_bsdf_eval row layout (may be NULL).  Deterministic in seed. */
int gr_surrogate_samples(gr_ctx* ctx, int64_t n, uint64_t seed, const float* domain, float* x_out,
                         float* y_out, float* q_out);
/* Device workspace for gr_mlp_forward / gr_mlp_backward on n rows. */
int gr_mlp_workspace_size(int64_t n, size_t* bytes);
/* y [n] = network(x [n][10]); dtype GR_BSDF_SURROGATE_BF16 or GR_BSDF_SURROGATE_FP8. */
int gr_mlp_forward(gr_ctx* ctx, const float* params, const float* x, int64_t n, int32_t dtype,
                   void* workspace, float* y);
/* Gradient of the mean squared error (1/n) sum (network(x_i) - target_i)^2 into grad (device
 * float [13249], overwritten; deterministic) and the loss into loss_dev (device float [1]). */
int gr_mlp_backward(gr_ctx* ctx, const float* params, const float* x, const float* target,
                    int64_t n, void* workspace, float* grad, float* loss_dev);
/* The network's activation, GELU in its tanh form x / (1 + 2^(x (a + b x^2))) with
 * a = -2 sqrt(2/pi) log2(e), b = 0.044715 a, and its derivative, elementwise in float as the
 * forward and backward kernels compute them (for checking them on their own): y[i] = GELU(x[i]),
 * dy[i] = GELU'(x[i]), i < n.  x, y, dy: device float [n] (n = 0 does nothing).  Asynchronous
 * on the context's stream. */
int gr_mlp_activation(gr_ctx* ctx, const float* x, int64_t n, float* y, float* dy);
/* Adam (Kingma & Ba, bias-corrected) update of params in place; m, v device float [13249]
 * moments (start at zero); step t >= 1. */
int gr_adam_step(gr_ctx* ctx, float* params, const float* grad, float* m, float* v, int32_t t,
                 float lr, float beta1, float beta2, float eps);
/* Install a trained network for both surrogate modes (copied and packed on the device in
 * bfloat16 and in E4M3; allocates on first use). */
int gr_set_surrogate(gr_ctx* ctx, const float* params, const float* domain);

/* Coherent measurement of mutually coherent emitters (Sec. "Linearity of Generalized Rays",
 * two-point interference; Sec. "Numeric Validation", double slit).  For each pixel and sample,
 * a point is drawn from the detection state's spatial density (uniform on the pixel plus a
 * Gaussian of std sigma_um) and |sum_e c_e G_e exp(i k L_e)|^2 is accumulated, L_e the exact
 * distance from emitter node e to the point.  phase_mode: 0 FP32, 1 FP64, 2 compensated
 * two-float.  image: device float [height][width], overwritten with the per-pixel mean. */
enum { GR_PHASE_FP32 = 0, GR_PHASE_FP64 = 1, GR_PHASE_TWO_FLOAT = 2 };
typedef struct {
    int32_t kind;          /* 0 points (3-D spherical waves), 1 slits (2-D, y-invariant) */
    int32_t n_slits;       /* points: number of points; slits: number of slits (<= 8) */
    double centre_um[8];   /* x centres */
    double width_um;       /* slit width */
    int32_t nodes_per_slit;/* Gauss-Legendre nodes per slit (<= 64) */
    int32_t phase_mode;
    double z_um;           /* aperture plane to sensor distance */
    double lambda_um;
    int32_t width, height;
    double pitch_um, sigma_um;
    int64_t spp;
    uint64_t seed;
} gr_coherent_desc;
int gr_coherent_measure(gr_ctx* ctx, const gr_coherent_desc* desc, float* image, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* GRWAVE_H */
