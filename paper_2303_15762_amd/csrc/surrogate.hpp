// Learned scattering model (perceptron surrogate of p_w): device state and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace grw {

struct SurrogateState {
    bool ready = false;
    uint16_t* d_wpack = nullptr;   // BF16 weights in matrix-core operand order
    float* d_bias = nullptr;       // hidden biases [4][64] then the output bias
    float* d_wout = nullptr;       // output layer weights [64]
    float domain[4] = {0, 0, 0, 0};
};

void surrogate_free(SurrogateState& s);
void surrogate_fill(const SurrogateState& s, SurrogateDev& d);
hipError_t launch_bsdf_eval_surrogate(const SurrogateState& s, const float* q, int64_t n, float* out,
                                      hipStream_t stream);

}  // namespace grw
