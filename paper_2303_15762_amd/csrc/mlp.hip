// Learned scattering model kernels (placeholder until the matrix-core implementation lands).
#include "../../include/grwave.h"
#include "surrogate.hpp"

namespace grw {

void surrogate_free(SurrogateState& s) {
    if (s.d_wpack) (void)hipFree(s.d_wpack);
    if (s.d_bias) (void)hipFree(s.d_bias);
    if (s.d_wout) (void)hipFree(s.d_wout);
    s = SurrogateState();
}

void surrogate_fill(const SurrogateState& s, SurrogateDev& d) {
    d.w_bf16 = s.d_wpack;
    d.bias = s.d_bias;
    d.w_out = s.d_wout;
    d.gmin = s.domain[0];
    d.gmax = s.domain[1];
    d.smin = s.domain[2];
    d.smax = s.domain[3];
    d.enabled = s.ready ? 1 : 0;
}

hipError_t launch_bsdf_eval_surrogate(const SurrogateState&, const float*, int64_t, float*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace grw

extern "C" {
int gr_surrogate_samples(gr_ctx*, int64_t, uint64_t, float*, float*, float*) { return GR_E_UNSUPPORTED; }
int gr_mlp_forward(gr_ctx*, const float*, const float*, int64_t, int32_t, float*) { return GR_E_UNSUPPORTED; }
int gr_mlp_workspace_size(int64_t, size_t*) { return GR_E_UNSUPPORTED; }
int gr_mlp_backward(gr_ctx*, const float*, const float*, const float*, int64_t, void*, float*, float*) {
    return GR_E_UNSUPPORTED;
}
int gr_adam_step(gr_ctx*, float*, const float*, float*, float*, int32_t, float, float, float, float) {
    return GR_E_UNSUPPORTED;
}
int gr_set_surrogate(gr_ctx*, const float*, const float*) { return GR_E_UNSUPPORTED; }
}
