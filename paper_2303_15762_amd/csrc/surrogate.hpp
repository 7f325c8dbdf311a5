// Learned scattering model (perceptron surrogate of p_w): host-side state and entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace grw {

struct SurrogateState {
    bool ready = false;
    void* d_pack = nullptr;      // weights in matrix-core operand order + hidden biases
    void* d_pack8 = nullptr;     // E4M3 forward weights + per-layer scales
    float* d_params = nullptr;   // FP32 copy of the installed parameters
    float domain[4] = {0, 0, 0, 0};
};

void surrogate_free(SurrogateState& s);
void surrogate_fill(const SurrogateState& s, SurrogateDev& d);
hipError_t launch_bsdf_eval_surrogate(const SurrogateState& s, bool fp8, const float* q, int64_t n, float* out,
                                      hipStream_t stream);
// Evaluate the *count deferred queries of a trace (kSurQueryBytes each) with the installed
// network and write each result to dense[slot]; non-finite results count into stats.
hipError_t launch_sur_batch(const SurrogateState& s, bool fp8, const uint4* queries, const unsigned long long* count,
                            float* dense, unsigned long long* stats, int grid, hipStream_t stream);
size_t mlp_workspace_bytes(int64_t n);
hipError_t mlp_forward(const float* params, const float* x, int64_t n, bool fp8, void* ws, float* y, hipStream_t s);
hipError_t mlp_backward(const float* params, const float* x, const float* t, int64_t n, void* ws, float* grad,
                        float* loss, hipStream_t s);
// y[i] = GELU(x[i]), dy[i] = GELU'(x[i]) for i < n (the kernels' float forms)
hipError_t activation(const float* x, int64_t n, float* y, float* dy, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, int t, float lr, float b1, float b2, float eps,
                hipStream_t s);
hipError_t surrogate_samples(int64_t n, uint64_t seed, const float* domain, float* x, float* y, float* q,
                             hipStream_t s);
hipError_t surrogate_set(SurrogateState& st, const float* params, const float* domain, hipStream_t s);

}  // namespace grw
