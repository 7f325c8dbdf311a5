"""FP64 multilayer perceptron (NumPy): the checker of the GPU surrogate's forward pass,
backward pass and Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: 10 inputs -> 4 hidden layers of width 64 with GELU -> 1 output.  GELU is the tanh
form 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).  Weights W[l] have shape [fan_in, fan_out];
a layer computes Y = X @ W + b.
"""

from __future__ import annotations

import math

import numpy as np

SIZES = (10, 64, 64, 64, 64, 1)


C0 = math.sqrt(2.0 / math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(C0 * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(C0 * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * C0 * (1.0 + 3 * 0.044715 * x * x)


def init_params(seed=0, sizes=SIZES):
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b)))
        bs.append(np.zeros(b))
    return Ws, bs


def forward(Ws, bs, X):
    """Returns (output [n, 1], pre-activations list, activations list)."""
    acts = [np.asarray(X, np.float64)]
    pres = []
    h = acts[0]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = h @ W + b
        pres.append(z)
        h = gelu(z) if l < len(Ws) - 1 else z
        acts.append(h)
    return h, pres, acts


def mse_loss(Ws, bs, X, Y):
    out, _, _ = forward(Ws, bs, X)
    r = out[:, 0] - np.asarray(Y, np.float64)
    return float(np.mean(r * r))


def backward(Ws, bs, X, Y):
    """Gradients of mean squared error over the batch: (dW list, db list, loss)."""
    out, pres, acts = forward(Ws, bs, X)
    n = out.shape[0]
    r = out[:, 0] - np.asarray(Y, np.float64)
    loss = float(np.mean(r * r))
    g = (2.0 / n) * r[:, None]
    dWs = [None] * len(Ws)
    dbs = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dWs[l] = acts[l].T @ g
        dbs[l] = g.sum(0)
        if l > 0:
            g = (g @ Ws[l].T) * gelu_grad(pres[l - 1])
    return dWs, dbs, loss


def adam_step(p, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------------------------------
# OCP FP8 E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; largest finite 448,
# smallest subnormal 2^-9) and the quantized forward pass of the FP8 surrogate mode.
# ------------------------------------------------------------------------------------------
E4M3_MAX = 448.0


def e4m3_round(v):
    """Round to the nearest E4M3 value, ties to even; |v| <= 448 is expected (clamped)."""
    v = np.clip(np.asarray(v, np.float64), -E4M3_MAX, E4M3_MAX)
    a = np.abs(v)
    # spacing: 2^-9 below the smallest normal 2^-6, else 2^(floor(log2 a) - 3)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    step = 2.0 ** (e - 3)
    return np.sign(v) * np.round(a / step) * step     # np.round: half to even


def _scale(amax):
    return (amax / E4M3_MAX) if amax > 1e-30 else 0.0


def bf16_round(v):
    """Round float32 values to bfloat16 (8 significant bits, 8 exponent bits), ties to even:
    float32 bit patterns with the low 16 bits cleared."""
    b = np.ascontiguousarray(np.asarray(v, np.float32)).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3_matmul(a, W):
    """The quantized product a @ W of one hidden layer.  Weights per output column (neuron)
    with scale max|W[:, j]| / 448: Wq = E4M3(W / scale) and Wq16 = E4M3(Wq / 16).  Each row
    (query) of a with scale s = max|a| / 448, as two E4M3 terms: hi = E4M3(a / s) and
    lo = E4M3(16 (a / s - hi)).  The product hi Wq + lo Wq16 exact (FP64), then multiplied by
    both scales."""
    a = np.asarray(a, np.float64)
    cmax = np.abs(W).max(axis=0)
    sw = np.where(cmax > 1e-30, cmax / E4M3_MAX, 0.0)
    wq = np.where(sw > 0, e4m3_round(W / np.where(sw > 0, sw, 1.0)), 0.0)
    wq16 = e4m3_round(wq / 16.0)
    amax = np.abs(a).max(axis=1)
    s = np.where(amax > 1e-30, amax / E4M3_MAX, 0.0)
    safe = np.where(s > 0, s, 1.0)
    v = np.where(s[:, None] > 0, a / safe[:, None], 0.0)
    hi = e4m3_round(v)
    lo = e4m3_round(16.0 * (v - hi))
    return (hi @ wq + lo @ wq16) * s[:, None] * sw[None, :]


def forward_e4m3(Ws, bs, X):
    """Forward pass with the FP8 mode's quantization: the input layer on bfloat16 operands
    (inputs and weights rounded from float32 to bfloat16), each hidden layer through
    e4m3_matmul, the output layer unquantized."""
    a = gelu(bf16_round(X) @ bf16_round(Ws[0]) + bs[0])
    for l in range(1, len(Ws) - 1):
        a = gelu(e4m3_matmul(a, Ws[l]) + bs[l])
    return (a @ Ws[-1] + bs[-1])[:, 0]
