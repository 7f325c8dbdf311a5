// Learned scattering model: 10 -> 64 -> 64 -> 64 -> 64 -> 1 perceptron with GELU, evaluated by
// one wave for 64 queries on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// The layers are computed transposed, out^T = W^T h^T: queries are the N dimension, so every
// lane keeps one query's column of activations in registers.  The matrix-core result layout
// (lane l holds rows 4(l/16)+i, i < 4, of column l%16) is reused directly as the next layer's
// B operand (lane l holds eight K values 8(l/16)+j of column l%16) by permuting the K order of
// each 32-wide block: slot 8g+j carries feature 4g+j (j < 4) or 16+4g+(j-4) (j >= 4).  The
// weights are stored pre-permuted in operand order, so no activation ever goes through LDS
// between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_IN = 10;
constexpr int MLP_H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 640, OFF_W2 = 704, OFF_B2 = 4800, OFF_W3 = 4864, OFF_B3 = 8960,
              OFF_W4 = 9024, OFF_B4 = 13120, OFF_W5 = 13184, OFF_B5 = 13248, MLP_NPARAM = 13249;
constexpr int FWD_FRAGS = 4 + 3 * 8;   // A fragments of W1^T (1 K-block) and W2..W4^T (2 K-blocks)
constexpr int BWD_FRAGS = 3 * 8;       // A fragments of W2..W4 (input-gradient products)

__host__ __device__ inline int w_off(int layer) {   // layer 0..3 -> W1..W4
    return layer == 0 ? OFF_W1 : (layer == 1 ? OFF_W2 : (layer == 2 ? OFF_W3 : OFF_W4));
}
__host__ __device__ inline int b_off(int layer) {
    return layer == 0 ? OFF_B1 : (layer == 1 ? OFF_B2 : (layer == 2 ? OFF_B3 : OFF_B4));
}
// K slot -> feature inside a 32-wide block
__host__ __device__ inline int kperm(int slot) {
    const int g = slot >> 3, j = slot & 7;
    return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
}
__host__ __device__ inline int fwd_frag(int layer, int mt, int kb) {
    return layer == 0 ? mt : 4 + (layer - 1) * 8 + mt * 2 + kb;
}
__host__ __device__ inline int bwd_frag(int layer, int mt, int kb) {   // layer 1..3 (W2..W4)
    return (layer - 1) * 8 + mt * 2 + kb;
}

// GELU, tanh form: 0.5 x (1 + tanh(y)), y = sqrt(2/pi) (x + 0.044715 x^3), and its
// derivative.  Since 0.5 (1 + tanh(y)) = 1 / (1 + exp(-2 y)), the activation is x s with
// s = 1 / (1 + 2^(x (a + b x^2))), a = -2 sqrt(2/pi) log2(e), b = 0.044715 a: one hardware
// base-2 exponential and one reciprocal (1 ulp each).  Large |x| saturates to x or -0.
constexpr float kGeluA = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
constexpr float kGeluB = 0.044715f * kGeluA;
__device__ __forceinline__ float gelu_gate(float x) {
    const float a = x * fmaf(kGeluB, x * x, kGeluA);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a));
}
__device__ __forceinline__ float gelu_f(float x) { return x * gelu_gate(x); }
// d/dx [x s] = s + x s (1 - s) 2 y', y' = sqrt(2/pi) (1 + 3 * 0.044715 x^2).  x^2 is capped so
// that y' stays finite where s (1 - s) is 0 (|x| beyond 1e15; uncapped, 0 * inf would give NaN).
__device__ __forceinline__ float gelu_grad_f(float x) {
    const float sg = gelu_gate(x);
    return sg + x * sg * (1.0f - sg) * (2.0f * 0.7978845608028654f) * fmaf(0.134145f, fminf(x * x, 1e30f), 1.0f);
}

// Round-to-nearest-even float -> bfloat16 (v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

struct MlpDev {
    const bf16x8* wf;    // [FWD_FRAGS][64] forward A fragments
    const float* bias;   // [4][64]
    const float* w5;     // [64]
    const float* b5;     // [1]
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// B fragment (one 32-wide K block) of the first layer from the staged inputs of the wave:
// stage[row * 16 + f] holds input feature f of query (lane) row.
__device__ __forceinline__ bf16x8 input_frag(const float* stage, int nb, int lane) {
    const int g = lane >> 4, c = lane & 15;
    const float* row = stage + (16 * nb + c) * 16;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int f = kperm(8 * g + j);
        v[j] = to_bf16(f < MLP_IN ? row[f] : 0.0f);
    }
    return v;
}

// Pack C-layout activations of M tiles (2kb, 2kb+1) of column block nb into a B fragment.
__device__ __forceinline__ bf16x8 act_frag(const f32x4 (&h)[4][4], int kb, int nb) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = to_bf16(h[2 * kb][nb][j]);
        v[4 + j] = to_bf16(h[2 * kb + 1][nb][j]);
    }
    return v;
}

// Forward pass of the 64 queries of this wave.  x: this lane's 10 inputs; stage: 64 x 16 floats
// of LDS private to the wave.  Optional zsave (global, per wave): pre-activations, layout
// [layer][mt][nb][i][lane].  Returns this lane's output.
__device__ inline float mlp_forward_wave(const MlpDev& M, const float* x, float* stage, float* zsave) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
#pragma unroll
    for (int f = 0; f < 16; ++f) stage[lane * 16 + f] = f < MLP_IN ? x[f] : 0.0f;
    wave_sync_lds();
    // every accumulation starts from the layer's bias: this lane's output rows 16 mt + 4 g + i
    // of the result tile are the bias's entries, whatever the column
    f32x4 h[4][4];
    {
        bf16x8 bin[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) bin[nb] = input_frag(stage, nb, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = M.wf[fwd_frag(0, mt, 0) * 64 + lane];
            const f32x4 bias = *reinterpret_cast<const f32x4*>(M.bias + 16 * mt + 4 * g);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) h[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bin[nb], bias, 0, 0, 0);
        }
    }
    wave_sync_lds();   // stage is free again for the caller
#pragma unroll
    for (int layer = 0; layer < 4; ++layer) {
        if (layer > 0) {
            bf16x8 b[2][4];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) b[kb][nb] = act_frag(h, kb, nb);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 a0 = M.wf[fwd_frag(layer, mt, 0) * 64 + lane];
                const bf16x8 a1 = M.wf[fwd_frag(layer, mt, 1) * 64 + lane];
                const f32x4 bias = *reinterpret_cast<const f32x4*>(M.bias + layer * 64 + 16 * mt + 4 * g);
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[0][nb], bias, 0, 0, 0);
                    h[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[1][nb], acc, 0, 0, 0);
                }
            }
        }
        // activation; the layer's output features of this lane are 16 mt + 4 g + i
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = h[mt][nb][i];
                    if (zsave) zsave[((((layer * 4 + mt) * 4 + nb) * 4 + i) << 6) + lane] = z;
                    h[mt][nb][i] = gelu_f(z);
                }
    }
    // output layer on the vector ALUs: partial dot products, then a reduction over the four
    // lane groups that hold the same query column
    float part[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        float s = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) s += M.w5[16 * mt + 4 * g + i] * h[mt][nb][i];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        part[nb] = s;
    }
    // lane 16 g + c owns query column 16 nb + c with nb = g
    const float o = g == 0 ? part[0] : (g == 1 ? part[1] : (g == 2 ? part[2] : part[3]));
    return o + M.b5[0];
}

// ------------------------------------------------------------------------------------------
// FP8 (OCP E4M3) forward pass.  The input layer (10 -> 64, 2.5 % of the multiply-adds) keeps
// bfloat16 operands: its ten encoded inputs (the transfer in lobe widths among them) would
// lose their position along the lobe to E4M3's three mantissa bits.  The three 64 x 64 hidden
// layers run on E4M3 operands:
//  - weights per output neuron (a row of the transposed product) with scale max|W| / 448 over
//    that neuron's 64 inputs: Wq = E4M3(W / scale), and a second copy Wq16 = E4M3(Wq / 16);
//  - activations per query with scale s = max|a| / 448 over its 64 values, as two E4M3 terms:
//    hi = E4M3(a / s) and lo = E4M3(16 (a / s - hi)), the rounding residual magnified 16x;
//  - one FP32 accumulation of Wq hi + Wq16 lo (four 16x16x32 products per 32 x 32 block),
//    multiplied by the two scales.
// Per-layer weight scales and a single activation term left 6.5 % and 5.6 % RMS error in the
// network's log p_w; this form leaves 3 %.  The E4M3 16x16x32 matrix-core product has the
// bfloat16 one's operand layout (8 values per lane, value j in byte j).
// ------------------------------------------------------------------------------------------
struct MlpDev8 {
    const bf16x8* wf1;     // [4][64] input-layer A fragments, bfloat16 (the BF16 pack's first 4)
    const long* wf;        // [FWD_FRAGS][64] forward A fragments Wq, E4M3 (hidden layers used)
    const long* wf16;      // [FWD_FRAGS][64] the same fragments of Wq16
    const float* wscale;   // [4][64] per-neuron weight scales (hidden layers used)
    const float* bias;     // [4][64]
    const float* w5;       // [64]
    const float* b5;       // [1]
};

constexpr float kE4M3Max = 448.0f;

// Four floats (already scaled into [-448, 448]) to E4M3, round to nearest even.
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

__device__ __forceinline__ long e4m3x8(const float (&v)[8]) {
    const uint32_t lo = e4m3x4(v[0], v[1], v[2], v[3]), hi = e4m3x4(v[4], v[5], v[6], v[7]);
    return (long)(((uint64_t)hi << 32) | lo);
}

// Eight E4M3 values (byte j = value j) to float.
__device__ __forceinline__ void e4m3x8_to_f32(long w, float (&q)[8]) {
    const int w0 = (int)(uint32_t)w, w1 = (int)(uint32_t)((uint64_t)w >> 32);
    const auto a = __builtin_amdgcn_cvt_pk_f32_fp8(w0, false), b = __builtin_amdgcn_cvt_pk_f32_fp8(w0, true);
    const auto c = __builtin_amdgcn_cvt_pk_f32_fp8(w1, false), d = __builtin_amdgcn_cvt_pk_f32_fp8(w1, true);
    q[0] = a[0];
    q[1] = a[1];
    q[2] = b[0];
    q[3] = b[1];
    q[4] = c[0];
    q[5] = c[1];
    q[6] = d[0];
    q[7] = d[1];
}

__device__ __forceinline__ float wave_absmax(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// scale (amax / 448) and its reciprocal; an all-zero tile quantizes to zeros
__device__ __forceinline__ void e4m3_scale(float amax, float& s, float& inv) {
    if (amax > 1e-30f) {
        s = amax * (1.0f / kE4M3Max);
        inv = kE4M3Max / amax;
    } else {
        s = 0.0f;
        inv = 0.0f;
    }
}

__device__ __forceinline__ float clamp448(float v) { return fminf(fmaxf(v, -kE4M3Max), kE4M3Max); }

// B fragments of the two activation terms of M tiles (2kb, 2kb+1), column block nb: hi =
// E4M3(a / s), lo = E4M3(16 (a / s - hi)) (|16 residual| <= 256, no clamp needed).
__device__ __forceinline__ void act_frag8x2(const f32x4 (&h)[4][4], int kb, int nb, float inv, long& hi, long& lo) {
    float v[8], r[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = clamp448(h[2 * kb][nb][j] * inv);
        v[4 + j] = clamp448(h[2 * kb + 1][nb][j] * inv);
    }
    hi = e4m3x8(v);
    float q[8];
    e4m3x8_to_f32(hi, q);
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = 16.0f * (v[j] - q[j]);
    lo = e4m3x8(r);
}

__device__ inline float mlp_forward_wave_fp8(const MlpDev8& M, const float* x, float* stage) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
#pragma unroll
    for (int f = 0; f < 16; ++f) stage[lane * 16 + f] = f < MLP_IN ? x[f] : 0.0f;
    wave_sync_lds();
    f32x4 h[4][4];
    float s_act[4] = {1.0f, 1.0f, 1.0f, 1.0f};   // scale of query 16 nb + (lane & 15) (hidden layers)
    {
        bf16x8 bin[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) bin[nb] = input_frag(stage, nb, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = M.wf1[mt * 64 + lane];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
                h[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bin[nb], zero, 0, 0, 0);
            }
        }
    }
    wave_sync_lds();   // stage is free again for the caller
#pragma unroll
    for (int layer = 0; layer < 4; ++layer) {
        if (layer > 0) {
            // per query: the 16 of its features in this lane, then the lanes c, c + 16, c + 32,
            // c + 48 that hold the rest
            float inv_act[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                float m = 0.0f;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) m = fmaxf(m, fabsf(h[mt][nb][i]));
                m = fmaxf(m, __shfl_xor(m, 16));
                m = fmaxf(m, __shfl_xor(m, 32));
                e4m3_scale(m, s_act[nb], inv_act[nb]);
            }
            long bh[2][4], bl[2][4];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) act_frag8x2(h, kb, nb, inv_act[nb], bh[kb][nb], bl[kb][nb]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const long a0 = M.wf[fwd_frag(layer, mt, 0) * 64 + lane];
                const long a1 = M.wf[fwd_frag(layer, mt, 1) * 64 + lane];
                const long c0 = M.wf16[fwd_frag(layer, mt, 0) * 64 + lane];
                const long c1 = M.wf16[fwd_frag(layer, mt, 1) * 64 + lane];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
                    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, bh[0][nb], zero, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, bh[1][nb], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(c0, bl[0][nb], acc, 0, 0, 0);
                    h[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(c1, bl[1][nb], acc, 0, 0, 0);
                }
            }
        }
        // dequantize, bias, activation; the layer's output features of this lane are 16 mt + 4 g + i
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            float bb[4], ws[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bb[i] = M.bias[layer * 64 + 16 * mt + 4 * g + i];
                ws[i] = layer == 0 ? 1.0f : M.wscale[layer * 64 + 16 * mt + 4 * g + i];
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) h[mt][nb][i] = gelu_f(h[mt][nb][i] * (ws[i] * s_act[nb]) + bb[i]);
        }
    }
    float part[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        float s = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) s += M.w5[16 * mt + 4 * g + i] * h[mt][nb][i];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        part[nb] = s;
    }
    const float o = g == 0 ? part[0] : (g == 1 ? part[1] : (g == 2 ? part[2] : part[3]));
    return o + M.b5[0];
}

// ------------------------------------------------------------------------------------------
// Input encoding of a rough-surface query for the learned model.
//
// The network sees the outgoing tangential wavevector relative to the incident one in units of
// the lobe width sqrt(2 g) / l (g = (q_z s)^2, the phase variance of the surface), the incident
// tangential direction, log wavelength, log footprint standard deviations (diagonal footprint
// frame), log RMS height, log correlation length and log g, each shifted and scaled to about
// [-1, 1].  It predicts log p_w relative to the peak l^2 / (4 pi g) of the single Gaussian
// with the mean Poisson term's variance.  Returns 0 outside the trained domain (g, footprint
// range, or an unscattered spike above 1e-4 of the lobe peak), 1 inside, 2 inside but beyond
// 8 lobe widths (where p_w is below 1e-9 of its peak and is taken as 0).
// ------------------------------------------------------------------------------------------
struct SurDomain {
    float gmin, gmax, smin, smax;
};

__device__ __forceinline__ int sur_encode(const SurDomain& D, float k, float kix, float kiy, float kox,
                                          float koy, float sxx, float syy, float sxy, float s_um,
                                          float ell_um, float* x, float& logpeak) {
    const float ik2 = 1.0f / (k * k);
    const float ni = (kix * kix + kiy * kiy) * ik2, no = (kox * kox + koy * koy) * ik2;
    if (ni >= 1.0f || no >= 1.0f) return 0;
    const float qz = k * (sqrtf(1.0f - ni) + sqrtf(1.0f - no));
    const float g = qz * qz * s_um * s_um;
    if (!(g >= D.gmin && g <= D.gmax)) return 0;
    if (fabsf(sxy) > 1e-6f * sqrtf(sxx * syy)) return 0;
    const float sx = sqrtf(sxx), sy = sqrtf(syy);
    if (!(sx >= D.smin && sx <= D.smax && sy >= D.smin && sy <= D.smax)) return 0;
    // the unscattered (m = 0) term is a spike of the window's width; keep the query on the
    // closed form unless that spike is below 1e-4 of the lobe peak: e^-g 8 g sx sy / l^2
    if (-g + logf(8.0f * g * sx * sy / (ell_um * ell_um)) > -9.2f) return 0;
    const float isc = ell_um * rsqrtf(2.0f * g);
    const float vx = (kox - kix) * isc, vy = (koy - kiy) * isc;
    logpeak = logf(ell_um * ell_um / (4.0f * 3.14159265358979f * g));
    if (vx * vx + vy * vy > 64.0f) return 2;
    x[0] = 0.25f * vx;
    x[1] = 0.25f * vy;
    x[2] = kix / k;
    x[3] = kiy / k;
    x[4] = (logf(6.28318530717959f / k) + 0.64f) * (1.0f / 0.28f);
    x[5] = (logf(sx) - 5.05f) * (1.0f / 3.45f);
    x[6] = (logf(sy) - 5.05f) * (1.0f / 3.45f);
    x[7] = (logf(s_um) + 1.84f) * (1.0f / 1.15f);
    x[8] = (logf(ell_um) - 0.46f) * (1.0f / 1.15f);
    x[9] = (logf(g) - 4.38f) * (1.0f / 1.6f);
    return 1;
}

}  // namespace grw
