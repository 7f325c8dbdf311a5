// Learned scattering model on gfx950: training-set generation from the closed-form p_w,
// forward / backward passes on the matrix cores (BF16 operands, FP32 accumulation), a
// deterministic gradient reduction, Adam, and the surrogate p_w evaluator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "../../include/grwave.h"
#include "device_math.hpp"
#include "mlp_core.hpp"
#include "surrogate.hpp"

namespace grw {

// ------------------------------------------------------------------------------------------
// Weight packing into matrix-core operand order (see mlp_core.hpp).
// wf: [FWD_FRAGS][64] bf16x8, A[row = out 16mt + c][slot 8g + j] = W[in = 32kb + kperm(slot)][out]
// wb: [BWD_FRAGS][64] bf16x8, A[row = in 16mt + c][slot 8g + j] = W[in][out = 32kb + kperm(slot)]
// bias: [4][64] hidden biases.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void pack_kernel(const float* __restrict__ P, bf16x8* __restrict__ wf,
                                                  bf16x8* __restrict__ wb, float* __restrict__ bias) {
    const int f = blockIdx.x;   // fragment index over FWD_FRAGS + BWD_FRAGS, then 4 bias blocks
    const int lane = threadIdx.x;
    const int g = lane >> 4, c = lane & 15;
    if (f < FWD_FRAGS) {
        int layer, mt, kb;
        if (f < 4) { layer = 0; mt = f; kb = 0; }
        else { const int q = f - 4; layer = 1 + q / 8; mt = (q % 8) / 2; kb = q % 2; }
        const int fan_in = layer == 0 ? MLP_IN : MLP_H;
        const int out = 16 * mt + c;
        bf16x8 v;
        for (int j = 0; j < 8; ++j) {
            const int in = 32 * kb + kperm(8 * g + j);
            v[j] = to_bf16(in < fan_in ? P[w_off(layer) + in * MLP_H + out] : 0.0f);
        }
        wf[f * 64 + lane] = v;
    } else if (f < FWD_FRAGS + BWD_FRAGS) {
        const int q = f - FWD_FRAGS;
        const int layer = 1 + q / 8, mt = (q % 8) / 2, kb = q % 2;
        const int in = 16 * mt + c;
        bf16x8 v;
        for (int j = 0; j < 8; ++j) {
            const int out = 32 * kb + kperm(8 * g + j);
            v[j] = to_bf16(P[w_off(layer) + in * MLP_H + out]);
        }
        wb[q * 64 + lane] = v;
    } else {
        const int layer = f - FWD_FRAGS - BWD_FRAGS;   // 0..3
        bias[layer * 64 + lane] = P[b_off(layer) + lane];
    }
}

// Packed-weight workspace layout (bytes).
constexpr size_t kPackWf = (size_t)FWD_FRAGS * 64 * 16;
constexpr size_t kPackWb = (size_t)BWD_FRAGS * 64 * 16;
constexpr size_t kPackBias = 4 * 64 * 4;
constexpr size_t kPackBytes = kPackWf + kPackWb + kPackBias;
// E4M3 forward fragments of Wq and Wq16, then the per-neuron weight scales [4][64].
constexpr size_t kPack8Wf = (size_t)FWD_FRAGS * 64 * 8;
constexpr size_t kPack8Bytes = 2 * kPack8Wf + 4 * 64 * 4;

// One wave per hidden layer: lane t finds output neuron t's weight scale (max |W| over its 64
// inputs / 448), then the forward fragments of Wq = E4M3(W / scale) and Wq16 = E4M3(Wq / 16)
// in the bfloat16 fragments' order and operand layout.  The input layer stays bfloat16.
__global__ __launch_bounds__(64) void pack8_kernel(const float* __restrict__ P, long* __restrict__ wf8,
                                                   long* __restrict__ wf16, float* __restrict__ wscale) {
    __shared__ float inv_s[64];
    const int layer = 1 + blockIdx.x, lane = threadIdx.x;
    float am = 0.0f;
    for (int in = 0; in < MLP_H; ++in) am = fmaxf(am, fabsf(P[w_off(layer) + in * MLP_H + lane]));
    float sw, inv;
    e4m3_scale(am, sw, inv);
    wscale[layer * 64 + lane] = sw;
    if (layer == 1) wscale[lane] = 1.0f;   // input layer: not quantized
    inv_s[lane] = inv;
    __syncthreads();
    const int g = lane >> 4, c = lane & 15;
    for (int mt = 0; mt < 4; ++mt)
        for (int kb = 0; kb < 2; ++kb) {
            const int out = 16 * mt + c;
            const float io = inv_s[out];
            float v[8];
            for (int j = 0; j < 8; ++j) {
                const int in = 32 * kb + kperm(8 * g + j);
                v[j] = clamp448(P[w_off(layer) + in * MLP_H + out] * io);
            }
            const long hi = e4m3x8(v);
            float q[8];
            e4m3x8_to_f32(hi, q);
            for (int j = 0; j < 8; ++j) q[j] *= 0.0625f;
            wf8[fwd_frag(layer, mt, kb) * 64 + lane] = hi;
            wf16[fwd_frag(layer, mt, kb) * 64 + lane] = e4m3x8(q);
        }
}

static hipError_t pack8(const float* params, void* buf, hipStream_t s) {
    char* b = static_cast<char*>(buf);
    hipLaunchKernelGGL(pack8_kernel, dim3(3), dim3(64), 0, s, params, reinterpret_cast<long*>(b),
                       reinterpret_cast<long*>(b + kPack8Wf), reinterpret_cast<float*>(b + 2 * kPack8Wf));
    return hipGetLastError();
}

// pack: the bfloat16 pack (for the hidden biases); pack8: the E4M3 pack
static MlpDev8 mlp_dev8(const float* params, const void* pack, const void* pack8buf) {
    const char* b = static_cast<const char*>(pack);
    const char* b8 = static_cast<const char*>(pack8buf);
    MlpDev8 M;
    M.wf1 = reinterpret_cast<const bf16x8*>(b);
    M.wf = reinterpret_cast<const long*>(b8);
    M.wf16 = reinterpret_cast<const long*>(b8 + kPack8Wf);
    M.wscale = reinterpret_cast<const float*>(b8 + 2 * kPack8Wf);
    M.bias = reinterpret_cast<const float*>(b + kPackWf + kPackWb);
    M.w5 = params + OFF_W5;
    M.b5 = params + OFF_B5;
    return M;
}

static hipError_t pack(const float* params, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    hipLaunchKernelGGL(pack_kernel, dim3(FWD_FRAGS + BWD_FRAGS + 4), dim3(64), 0, s, params,
                       reinterpret_cast<bf16x8*>(b), reinterpret_cast<bf16x8*>(b + kPackWf),
                       reinterpret_cast<float*>(b + kPackWf + kPackWb));
    return hipGetLastError();
}

static MlpDev mlp_dev(const float* params, const void* ws) {
    const char* b = static_cast<const char*>(ws);
    MlpDev M;
    M.wf = reinterpret_cast<const bf16x8*>(b);
    M.bias = reinterpret_cast<const float*>(b + kPackWf + kPackWb);
    M.w5 = params + OFF_W5;
    M.b5 = params + OFF_B5;
    return M;
}

// ------------------------------------------------------------------------------------------
// Forward: one wave per 64 rows.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256, 4) void mlp_forward_kernel(const MlpDev M, const float* __restrict__ x, int64_t n,
                                                          float* __restrict__ y) {
    __shared__ float stage[4][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row = ((int64_t)blockIdx.x * 4 + wv) * 64 + lane;
    float xi[MLP_IN];
    for (int f = 0; f < MLP_IN; ++f) xi[f] = row < n ? x[row * MLP_IN + f] : 0.0f;
    const float o = mlp_forward_wave(M, xi, stage[wv], nullptr);
    if (row < n) y[row] = o;
}

__global__ __launch_bounds__(256, 4) void mlp_forward8_kernel(const MlpDev8 M, const float* __restrict__ x, int64_t n,
                                                           float* __restrict__ y) {
    __shared__ float stage[4][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row = ((int64_t)blockIdx.x * 4 + wv) * 64 + lane;
    float xi[MLP_IN];
    for (int f = 0; f < MLP_IN; ++f) xi[f] = row < n ? x[row * MLP_IN + f] : 0.0f;
    const float o = mlp_forward_wave_fp8(M, xi, stage[wv]);
    if (row < n) y[row] = o;
}

// ------------------------------------------------------------------------------------------
// Backward: forward with saved pre-activations, then the gradient of the mean squared error,
// per wave of 64 rows, into a per-wave partial gradient (summed in a fixed order afterwards).
// ------------------------------------------------------------------------------------------
struct TrainArgs {
    MlpDev M;
    const bf16x8* wb;
    const float* params;
    const float* x;
    const float* t;
    int64_t n;
    float two_over_n;
    float* zs;        // [n_waves][16384]
    float* part;      // [n_waves][MLP_NPARAM]
    float* loss;      // [n_waves]
};

__device__ __forceinline__ float zload(const float* zw, int layer, int mt, int nb, int i, int lane) {
    return zw[((((layer * 4 + mt) * 4 + nb) * 4 + i) << 6) + lane];
}

__device__ __forceinline__ float reduce16(float v) {   // sum over the 16 lanes sharing l / 16
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

constexpr int kTS = 72;   // LDS tile row stride (bf16 elements, 144 bytes)

__global__ __launch_bounds__(64) void mlp_backward_kernel(const TrainArgs T) {
    __shared__ float stage[64 * 16];
    __shared__ __attribute__((aligned(16))) uint16_t HT[64 * kTS];
    __shared__ __attribute__((aligned(16))) uint16_t DT[64 * kTS];
    const int lane = threadIdx.x;
    const int g = lane >> 4, c = lane & 15;
    const int64_t wave = blockIdx.x;
    const int64_t row = wave * 64 + lane;
    const bool valid = row < T.n;
    float xi[MLP_IN];
    for (int f = 0; f < MLP_IN; ++f) xi[f] = valid ? T.x[row * MLP_IN + f] : 0.0f;
    float* zw = T.zs + wave * 16384;
    const float out = mlp_forward_wave(T.M, xi, stage, zw);
    const float r = valid ? out - T.t[row] : 0.0f;
    float* P = T.part + wave * MLP_NPARAM;
    {
        float l2 = r * r;
        for (int off = 32; off > 0; off >>= 1) l2 += __shfl_xor(l2, off);
        if (lane == 0) T.loss[wave] = l2;
    }
    const float d5 = T.two_over_n * r;
    float d5c[4];
    for (int nb = 0; nb < 4; ++nb) d5c[nb] = __shfl(d5, 16 * nb + c);
    {
        float s = d5;
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) P[OFF_B5] = s;
    }
    // output layer: dW5 and the gradient at the last hidden pre-activation
    f32x4 dl[4][4];
    for (int mt = 0; mt < 4; ++mt)
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * mt + 4 * g + i;
            float acc = 0.0f;
            for (int nb = 0; nb < 4; ++nb) {
                const float z = zload(zw, 3, mt, nb, i, lane);
                acc += gelu_f(z) * d5c[nb];
                dl[mt][nb][i] = T.params[OFF_W5 + f] * d5c[nb] * gelu_grad_f(z);
            }
            acc = reduce16(acc);
            if (c == 0) P[OFF_W5 + f] = acc;
        }
    for (int layer = 3; layer >= 0; --layer) {
        // bias gradient
        for (int mt = 0; mt < 4; ++mt)
            for (int i = 0; i < 4; ++i) {
                float s = dl[mt][0][i] + dl[mt][1][i] + dl[mt][2][i] + dl[mt][3][i];
                s = reduce16(s);
                if (c == 0) P[b_off(layer) + 16 * mt + 4 * g + i] = s;
            }
        // transpose the layer input (rows = features) and the gradient into LDS
        if (layer > 0) {
            for (int mt = 0; mt < 4; ++mt)
                for (int nb = 0; nb < 4; ++nb)
                    for (int i = 0; i < 4; ++i)
                        HT[(16 * mt + 4 * g + i) * kTS + 16 * nb + c] =
                            __builtin_bit_cast(uint16_t, to_bf16(gelu_f(zload(zw, layer - 1, mt, nb, i, lane))));
        } else {
            for (int f = 0; f < 16; ++f)
                HT[f * kTS + lane] = __builtin_bit_cast(uint16_t, to_bf16(f < MLP_IN ? xi[f] : 0.0f));
        }
        for (int mt = 0; mt < 4; ++mt)
            for (int nb = 0; nb < 4; ++nb)
                for (int i = 0; i < 4; ++i)
                    DT[(16 * mt + 4 * g + i) * kTS + 16 * nb + c] = __builtin_bit_cast(uint16_t, to_bf16(dl[mt][nb][i]));
        wave_sync_lds();
        // dW[in][out] = sum over the 64 rows of input[in] * grad[out]
        const int nmi = layer == 0 ? 1 : 4;
        const int fan_in = layer == 0 ? MLP_IN : MLP_H;
        for (int mi = 0; mi < nmi; ++mi)
            for (int no = 0; no < 4; ++no) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int kb = 0; kb < 2; ++kb) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&HT[(16 * mi + c) * kTS + 32 * kb + 8 * g]);
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(&DT[(16 * no + c) * kTS + 32 * kb + 8 * g]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
                }
                for (int i = 0; i < 4; ++i) {
                    const int in = 16 * mi + 4 * g + i;
                    if (in < fan_in) P[w_off(layer) + in * MLP_H + 16 * no + c] = acc[i];
                }
            }
        wave_sync_lds();
        if (layer > 0) {
            // gradient at the previous pre-activation: (W dl) * gelu'(z)
            bf16x8 b[2][4];
            for (int kb = 0; kb < 2; ++kb)
                for (int nb = 0; nb < 4; ++nb) b[kb][nb] = act_frag(dl, kb, nb);
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 a0 = T.wb[bwd_frag(layer, mt, 0) * 64 + lane];
                const bf16x8 a1 = T.wb[bwd_frag(layer, mt, 1) * 64 + lane];
                for (int nb = 0; nb < 4; ++nb) {
                    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
                    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[0][nb], zero, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[1][nb], acc, 0, 0, 0);
                    for (int i = 0; i < 4; ++i) acc[i] *= gelu_grad_f(zload(zw, layer - 1, mt, nb, i, lane));
                    dl[mt][nb] = acc;
                }
            }
        }
    }
}

// Per-wave partial gradients summed in a fixed order: a block takes 64 parameters (one per
// lane) and its four waves take every fourth partial each (wave g: partials g, g + 4, ...);
// the four sums are then added in wave order.  The last block sums the loss partials the same
// way.  Deterministic for a given n_waves.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float* __restrict__ part, const float* __restrict__ lpart,
                                                          int64_t n_waves, float inv_n, float* __restrict__ grad,
                                                          float* __restrict__ loss) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const bool is_loss = blockIdx.x == gridDim.x - 1;
    const int p = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (is_loss) {
        // lane l of wave g sums loss partials g + 4 (l + 64 j)
        for (int64_t w = g + 4 * lane; w < n_waves; w += 256) s += lpart[w];
    } else if (p < MLP_NPARAM) {
#pragma unroll 8
        for (int64_t w = g; w < n_waves; w += 4) s += part[w * MLP_NPARAM + p];
    }
    red[g][lane] = s;
    __syncthreads();
    if (g != 0) return;
    float t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    if (is_loss) {
        // fixed-order sum over the 64 lanes
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off);
        if (lane == 0) loss[0] = t * inv_n;
    } else if (p < MLP_NPARAM) {
        grad[p] = t;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------------------------------
// Training set: rough-surface queries in the canonical frame of the tracer's next-event
// estimation (outgoing direction in the x-z plane, diagonal footprint), outgoing transfers
// 70 % from a Gaussian around the lobe and 30 % uniform within 8 lobe widths; target log p_w
// (closed form) relative to the lobe's Gaussian peak, floored at -20 (e^-20 of the peak).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void samples_kernel(int64_t n, uint64_t seed, SurDomain D, float* __restrict__ xo,
                                                      float* __restrict__ yo, float* __restrict__ qo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[MLP_IN];
    float logpeak = 0.0f;
    float q[14];
    bool ok = false;
    for (uint32_t attempt = 0; attempt < 64 && !ok; ++attempt) {
        const uint4 r0 = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), attempt, 0x5A11u, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint4 r1 = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), attempt, 0x5A12u, (uint32_t)seed, (uint32_t)(seed >> 32));
        const float lam = 0.4f + 0.3f * unif(r0.x);
        const float k = kTwoPiF / lam;
        float s = 0.05f + 0.45f * unif(r0.y);
        const float ell = 0.5f + 4.5f * unif(r0.z);
        const float co = 0.2f + 0.8f * unif(r0.w);
        const float so = sqrtf(1.0f - co * co);
        const float sr = expf(logf(D.smin) + (logf(D.smax / 4.0f) - logf(D.smin)) * unif(r1.x));
        const float sxx = sr * sr / (co * co), syy = sr * sr;
        // smallest RMS height that reaches the domain's phase variance at this geometry
        const float smin_g = sqrtf(D.gmin) / (2.0f * k * co) * 1.02f;
        if (s < smin_g) s = smin_g + (0.5f - smin_g) * unif(r1.y);
        if (s > 0.5f) continue;
        const float g0 = 4.0f * k * k * co * co * s * s;
        const float sc = sqrtf(2.0f * g0) / ell;
        float vx, vy;
        if ((r1.z >> 24) < 180u) {   // 70 %: around the lobe
            float z1, z2;
            box_muller(unif(r1.z), unif(r1.w), z1, z2);
            vx = 1.2f * z1;
            vy = 1.2f * z2;
        } else {
            const float rr = 8.0f * sqrtf(unif(r1.z << 1));
            float sn, cs;
            sincospif(2.0f * unif(r1.w), &sn, &cs);
            vx = rr * cs;
            vy = rr * sn;
        }
        const float kox = -k * so, koy = 0.0f;
        const float kix = kox - vx * sc, kiy = koy - vy * sc;
        if ((kix * kix + kiy * kiy) >= 0.995f * k * k) continue;
        const int e = sur_encode(D, k, kix, kiy, kox, koy, sxx, syy, 0.0f, s, ell, x, logpeak);
        if (e != 1) continue;
        const float p = pw_plain(MAT_ROUGH, s, ell, 1.0f, k, kix, kiy, kox, koy, sxx, syy, 0.0f, 1.0f, 0.0f);
        const float y = logf(fmaxf(p, 1e-37f)) - logpeak;
        q[0] = 1.0f; q[1] = s; q[2] = ell; q[3] = 1.0f; q[4] = k; q[5] = kix; q[6] = kiy; q[7] = kox;
        q[8] = koy; q[9] = sxx; q[10] = syy; q[11] = 0.0f; q[12] = 1.0f; q[13] = 0.0f;
        yo[i] = fmaxf(y, -20.0f);
        ok = true;
    }
    if (!ok) {   // practically unreachable: a specular query at the domain's centre
        const float k = kTwoPiF / 0.55f, co = 0.8f, s = 0.3f, ell = 2.0f, sr = 100.0f;
        const float kox = -k * 0.6f;
        const float sxx = sr * sr / (co * co), syy = sr * sr;
        sur_encode(D, k, kox, 0.0f, kox, 0.0f, sxx, syy, 0.0f, s, ell, x, logpeak);
        const float p = pw_plain(MAT_ROUGH, s, ell, 1.0f, k, kox, 0.0f, kox, 0.0f, sxx, syy, 0.0f, 1.0f, 0.0f);
        yo[i] = fmaxf(logf(fmaxf(p, 1e-37f)) - logpeak, -20.0f);
        q[0] = 1.0f; q[1] = s; q[2] = ell; q[3] = 1.0f; q[4] = k; q[5] = kox; q[6] = 0.0f; q[7] = kox;
        q[8] = 0.0f; q[9] = sxx; q[10] = syy; q[11] = 0.0f; q[12] = 1.0f; q[13] = 0.0f;
    }
    for (int f = 0; f < MLP_IN; ++f) xo[i * MLP_IN + f] = x[f];
    if (qo)
        for (int f = 0; f < 14; ++f) qo[i * 14 + f] = q[f];
}

// ------------------------------------------------------------------------------------------
// Surrogate p_w for a batch of queries (gr_bsdf_eval rows); out-of-domain rows use the closed
// form.  One wave per 64 queries: every lane takes part in the matrix-core pass.
// ------------------------------------------------------------------------------------------
template <bool FP8>
__global__ __launch_bounds__(256, FP8 ? 3 : 4) void sur_eval_kernel(const MlpDev M, const MlpDev8 M8, SurDomain D,
                                                       const float* __restrict__ q, int64_t n, float* __restrict__ out) {
    __shared__ float stage[4][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = ((int64_t)blockIdx.x * 4 + wv) * 64 + lane;
    float x[MLP_IN] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    float logpeak = 0.0f;
    int e = 0;
    const float* r = q + (i < n ? i : 0) * 14;
    if (i < n && (int)r[0] == MAT_ROUGH)
        e = sur_encode(D, r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11], r[1], r[2], x, logpeak);
    const float y = FP8 ? mlp_forward_wave_fp8(M8, x, stage[wv]) : mlp_forward_wave(M, x, stage[wv], nullptr);
    if (i >= n) return;
    float v;
    if (e == 1) v = r[3] * __expf(y + logpeak);
    else if (e == 2) v = 0.0f;
    else v = pw_plain((int)r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11], r[12], r[13]);
    out[i] = v;
}

// ------------------------------------------------------------------------------------------
// Deferred queries of a trace: one wave per 64 queries, grid-stride over the count the trace
// kernel left in device memory (every lane of a wave takes part in the matrix-core pass).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void bf16_unpair(uint32_t u, float& a, float& b) {
    a = __uint_as_float(u << 16);
    b = __uint_as_float(u & 0xFFFF0000u);
}

template <bool FP8>
__global__ __launch_bounds__(256, FP8 ? 3 : 4) void sur_batch_kernel(const MlpDev M, const MlpDev8 M8, const uint4* __restrict__ q,
                                                        const unsigned long long* __restrict__ count,
                                                        float* __restrict__ dense, unsigned long long* stats) {
    __shared__ float stage[4][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t n = *count;
    for (uint64_t base = ((uint64_t)blockIdx.x * 4 + wv) * 64; base < n; base += (uint64_t)gridDim.x * 256) {
        const uint64_t i = base + lane;
        float x[MLP_IN] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        float scale = 0.0f, logpeak = 0.0f;
        uint32_t slot = 0;
        if (i < n) {
            const uint4 a = q[2 * i], b = q[2 * i + 1];
            bf16_unpair(a.x, x[0], x[1]);
            bf16_unpair(a.y, x[2], x[3]);
            bf16_unpair(a.z, x[4], x[5]);
            bf16_unpair(a.w, x[6], x[7]);
            bf16_unpair(b.x, x[8], x[9]);
            scale = __uint_as_float(b.y);
            logpeak = __uint_as_float(b.z);
            slot = b.w;
        }
        // the weight fragments are read again in every iteration (the compiler would otherwise
        // hoist them into ~100 registers for the whole loop and hold the kernel at one wave
        // per SIMD)
        MlpDev Mi = M;
        MlpDev8 M8i = M8;
        asm volatile("" : "+s"(Mi.wf));
        asm volatile("" : "+s"(M8i.wf), "+s"(M8i.wf16), "+s"(M8i.wf1));
        const float y = FP8 ? mlp_forward_wave_fp8(M8i, x, stage[wv]) : mlp_forward_wave(Mi, x, stage[wv], nullptr);
        if (i < n) {
            float v = scale * __expf(y + logpeak);
            if (!isfinite(v)) {
                atomicAdd(stats + ST_NONFINITE, 1ull);
                v = 0.0f;
            }
            dense[slot] = v;
        }
    }
}

hipError_t launch_sur_batch(const SurrogateState& s, bool fp8, const uint4* queries, const unsigned long long* count,
                            float* dense, unsigned long long* stats, int grid, hipStream_t stream) {
    const MlpDev M = mlp_dev(s.d_params, s.d_pack);
    const MlpDev8 M8 = mlp_dev8(s.d_params, s.d_pack, s.d_pack8);
    if (fp8)
        hipLaunchKernelGGL(sur_batch_kernel<true>, dim3(grid), dim3(256), 0, stream, M, M8, queries, count, dense, stats);
    else
        hipLaunchKernelGGL(sur_batch_kernel<false>, dim3(grid), dim3(256), 0, stream, M, M8, queries, count, dense, stats);
    return hipGetLastError();
}

void surrogate_free(SurrogateState& s) {
    if (s.d_pack8) (void)hipFree(s.d_pack8);
    if (s.d_pack) (void)hipFree(s.d_pack);
    if (s.d_params) (void)hipFree(s.d_params);
    s = SurrogateState();
}

void surrogate_fill(const SurrogateState& s, SurrogateDev& d) {
    d.gmin = s.domain[0];
    d.gmax = s.domain[1];
    d.smin = s.domain[2];
    d.smax = s.domain[3];
    d.enabled = s.ready ? 1 : 0;
}

hipError_t launch_bsdf_eval_surrogate(const SurrogateState& s, bool fp8, const float* q, int64_t n, float* out,
                                      hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const MlpDev M = mlp_dev(s.d_params, s.d_pack);
    const MlpDev8 M8 = mlp_dev8(s.d_params, s.d_pack, s.d_pack8);
    const SurDomain D{s.domain[0], s.domain[1], s.domain[2], s.domain[3]};
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (fp8) hipLaunchKernelGGL(sur_eval_kernel<true>, dim3(blocks), dim3(256), 0, stream, M, M8, D, q, n, out);
    else hipLaunchKernelGGL(sur_eval_kernel<false>, dim3(blocks), dim3(256), 0, stream, M, M8, D, q, n, out);
    return hipGetLastError();
}

// Host entry points used by the C ABI (api.cpp).
size_t mlp_workspace_bytes(int64_t n) {
    const int64_t waves = (n + 63) / 64;
    return kPackBytes + std::max(kPack8Bytes, (size_t)waves * (16384 + MLP_NPARAM + 1) * sizeof(float)) + 256;
}

hipError_t mlp_forward(const float* params, const float* x, int64_t n, bool fp8, void* ws, float* y, hipStream_t s) {
    hipError_t e = pack(params, ws, s);
    if (e != hipSuccess || n <= 0) return e;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (fp8) {
        void* p8 = static_cast<char*>(ws) + kPackBytes;
        e = pack8(params, p8, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(mlp_forward8_kernel, dim3(blocks), dim3(256), 0, s, mlp_dev8(params, ws, p8), x, n, y);
    } else {
        hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, s, mlp_dev(params, ws), x, n, y);
    }
    return hipGetLastError();
}

hipError_t mlp_backward(const float* params, const float* x, const float* t, int64_t n, void* ws, float* grad,
                        float* loss, hipStream_t s) {
    hipError_t e = pack(params, ws, s);
    if (e != hipSuccess) return e;
    const int64_t waves = (n + 63) / 64;
    char* b = static_cast<char*>(ws);
    TrainArgs T;
    T.M = mlp_dev(params, ws);
    T.wb = reinterpret_cast<const bf16x8*>(b + kPackWf);
    T.params = params;
    T.x = x;
    T.t = t;
    T.n = n;
    T.two_over_n = 2.0f / (float)n;
    float* f = reinterpret_cast<float*>(b + kPackBytes);
    T.zs = f;
    T.part = f + waves * 16384;
    T.loss = T.part + waves * MLP_NPARAM;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3((unsigned)waves), dim3(64), 0, s, T);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one block per 64 parameters, plus one for the loss
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((MLP_NPARAM + 63) / 64 + 1), dim3(256), 0, s, T.part, T.loss, waves,
                       1.0f / (float)n, grad, loss);
    return hipGetLastError();
}

// The network's activation and its derivative, elementwise, as the forward and backward
// kernels compute them.
__global__ __launch_bounds__(256) void activation_kernel(const float* __restrict__ x, int64_t n,
                                                         float* __restrict__ y, float* __restrict__ dy) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float v = x[i];
    y[i] = gelu_f(v);
    dy[i] = gelu_grad_f(v);
}

hipError_t activation(const float* x, int64_t n, float* y, float* dy, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(activation_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, y, dy);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int t, float lr, float b1, float b2, float eps,
                hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t surrogate_samples(int64_t n, uint64_t seed, const float* domain, float* x, float* y, float* q,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const SurDomain D{domain[0], domain[1], domain[2], domain[3]};
    hipLaunchKernelGGL(samples_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, seed, D, x, y, q);
    return hipGetLastError();
}

hipError_t surrogate_set(SurrogateState& st, const float* params, const float* domain, hipStream_t s) {
    if (!st.d_pack) {
        if (hipMalloc(&st.d_pack, kPackBytes) != hipSuccess) return hipErrorOutOfMemory;
        if (hipMalloc(&st.d_pack8, kPack8Bytes) != hipSuccess) return hipErrorOutOfMemory;
        if (hipMalloc(&st.d_params, MLP_NPARAM * sizeof(float)) != hipSuccess) return hipErrorOutOfMemory;
    }
    hipError_t e = hipMemcpyAsync(st.d_params, params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = pack(st.d_params, st.d_pack, s);
    if (e != hipSuccess) return e;
    e = pack8(st.d_params, st.d_pack8, s);
    if (e != hipSuccess) return e;
    for (int i = 0; i < 4; ++i) st.domain[i] = domain[i];
    st.ready = true;
    return hipStreamSynchronize(s);
}

}  // namespace grw
