"""Training and installation of the learned scattering model (the p_w surrogate).

Every numerical step runs in libgrwave kernels: training samples are drawn and labelled with
the closed-form p_w on the GPU (gr_surrogate_samples), and each optimisation step is one
matrix-core forward/backward pass (gr_mlp_backward) plus an Adam update (gr_adam_step).
PyTorch only holds the device buffers.
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _lib as L

# {g_min, g_max, footprint sigma min (um), footprint sigma max (um)}
DEFAULT_DOMAIN = (16.0, 400.0, 5.0, 5000.0)
SIZES = (10, 64, 64, 64, 64, 1)


def _fp(t):
    return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_float))


def init_params(seed=0):
    """He-normal weights, zero biases, flattened in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b)).ravel())
        parts.append(np.zeros(b))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == L.GR_MLP_PARAMS
    return p


def unflatten(p):
    """Flat parameter vector -> (list of W [fan_in, fan_out], list of b)."""
    p = np.asarray(p, np.float64)
    Ws, bs, o = [], [], 0
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        Ws.append(p[o:o + a * b].reshape(a, b))
        o += a * b
        bs.append(p[o:o + b])
        o += b
    return Ws, bs


class Surrogate:
    """Device-side training helpers bound to one Renderer context."""

    def __init__(self, renderer):
        self.R = renderer
        self.torch = renderer.torch
        self.lib = renderer.lib
        self._ws = None

    def _check(self, rc, what):
        self.R._check(rc, what)

    def workspace(self, n):
        b = C.c_size_t()
        self._check(self.lib.gr_mlp_workspace_size(int(n), C.byref(b)), "gr_mlp_workspace_size")
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = self.torch.empty(int(b.value), dtype=self.torch.uint8, device=self.R.dev)
        return self._ws

    def samples(self, n, seed=4, domain=DEFAULT_DOMAIN, with_queries=False):
        t = self.torch
        x = t.empty((n, 10), dtype=t.float32, device=self.R.dev)
        y = t.empty(n, dtype=t.float32, device=self.R.dev)
        q = t.empty((n, 14), dtype=t.float32, device=self.R.dev) if with_queries else None
        d = (C.c_float * 4)(*domain)
        self._check(self.lib.gr_surrogate_samples(self.R.h, int(n), int(seed), d, _fp(x), _fp(y),
                                                  _fp(q) if q is not None else None),
                    "gr_surrogate_samples")
        return x, y, q

    def forward(self, params, x, dtype=L.GR_BSDF_SURROGATE_BF16):
        """dtype: GR_BSDF_SURROGATE_BF16 or GR_BSDF_SURROGATE_FP8 (E4M3) matrix-core operands."""
        n = x.shape[0]
        y = self.torch.empty(n, dtype=self.torch.float32, device=self.R.dev)
        ws = self.workspace(n)
        self._check(self.lib.gr_mlp_forward(self.R.h, _fp(params), _fp(x), int(n), int(dtype),
                                            C.c_void_p(ws.data_ptr()), _fp(y)), "gr_mlp_forward")
        return y

    def backward(self, params, x, t, grad=None, loss=None):
        n = x.shape[0]
        tt = self.torch
        grad = tt.empty(L.GR_MLP_PARAMS, dtype=tt.float32, device=self.R.dev) if grad is None else grad
        loss = tt.empty(1, dtype=tt.float32, device=self.R.dev) if loss is None else loss
        ws = self.workspace(n)
        self._check(self.lib.gr_mlp_backward(self.R.h, _fp(params), _fp(x), _fp(t), int(n),
                                             C.c_void_p(ws.data_ptr()), _fp(grad), _fp(loss)),
                    "gr_mlp_backward")
        return grad, loss

    def activation(self, x):
        """The network's GELU and its derivative at x (device float), as the kernels compute them."""
        tt = self.torch
        y = tt.empty_like(x)
        dy = tt.empty_like(x)
        self._check(self.lib.gr_mlp_activation(self.R.h, _fp(x), int(x.numel()), _fp(y), _fp(dy)),
                    "gr_mlp_activation")
        return y, dy

    def adam(self, params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._check(self.lib.gr_adam_step(self.R.h, _fp(params), _fp(grad), _fp(m), _fp(v), int(step),
                                          float(lr), float(b1), float(b2), float(eps)), "gr_adam_step")

    def install(self, params, domain=DEFAULT_DOMAIN):
        d = (C.c_float * 4)(*domain)
        self._check(self.lib.gr_set_surrogate(self.R.h, _fp(params), d), "gr_set_surrogate")

    def train(self, n_train=4 << 20, batch=16384, steps=20000, lr=3e-3, lr_final=3e-5, seed=4,
              domain=DEFAULT_DOMAIN, init_seed=0, val_fraction=0.1, log_every=2500):
        """Train on n_train generated samples (last val_fraction held out).  Returns (params
        tensor, history dict)."""
        t = self.torch
        x, y, _ = self.samples(n_train, seed=seed, domain=domain)
        n_val = int(n_train * val_fraction)
        n_tr = n_train - n_val
        xtr, ytr = x[:n_tr], y[:n_tr]
        xva, yva = x[n_tr:], y[n_tr:]
        p = t.tensor(init_params(init_seed), device=self.R.dev)
        m = t.zeros_like(p)
        v = t.zeros_like(p)
        grad = t.empty_like(p)
        loss = t.empty(1, dtype=t.float32, device=self.R.dev)
        hist = {"step": [0], "train_loss": [float("nan")],
                "val_loss": [float(((self.forward(p, xva) - yva) ** 2).mean().item())]}
        nb = max(1, n_tr // batch)
        for s in range(1, steps + 1):
            b = (s - 1) % nb
            xb = xtr[b * batch:(b + 1) * batch]
            yb = ytr[b * batch:(b + 1) * batch]
            self.backward(p, xb, yb, grad, loss)
            frac = (s - 1) / max(1, steps - 1)
            lr_s = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            self.adam(p, grad, m, v, s, lr=lr_s)
            if s % log_every == 0 or s == steps:
                yv = self.forward(p, xva)
                hist["step"].append(s)
                hist["train_loss"].append(float(loss.item()))
                hist["val_loss"].append(float(((yv - yva) ** 2).mean().item()))
        return p, hist
