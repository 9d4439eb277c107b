"""FP64 reference of the alpha-predictor network (not part of the paper).

Oracle (test infrastructure only).

Network: y = w3 . h2 + b3,  h2 = GELU(W2 h1 + b2),  h1 = GELU(W1 x + b1),
x in R^65, widths 128, 128, 1.  GELU(x) = x (1 + erf(x / sqrt 2)) / 2 (exact).
Loss: mean squared error over the batch.  Optimiser: Adam (Kingma & Ba, 2015).

With ``bf16=True`` every operand of every product (weights, inputs,
activations and back-propagated errors entering a matrix product) is first
rounded to bfloat16 with round-to-nearest-even, and the products are summed in
FP64; this is the arithmetic the device runs (BF16 operands, FP32
accumulation) up to the accumulation order.  Biases, GELU and the loss stay
in full precision.  With ``bf16=False`` the network is plain FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

D_IN, D_H = 65, 128
PARAM_SHAPES = (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
                ("w3", (D_H,)), ("b3", (1,)))


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(seed, scale_w=None):
    """He-style uniform init from a seeded PCG64 stream (weights), zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, shape in PARAM_SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) == 2 else D_H
            lim = math.sqrt(6.0 / fan_in) if scale_w is None else scale_w
            p[name] = g.uniform(-lim, lim, size=shape)
    return p


def forward(p, X, bf16=True):
    """X: (B, 65).  Returns (y (B,), cache)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = q(X) @ q(p["W1"]).T + p["b1"]
    h1 = gelu(z1)
    z2 = q(h1) @ q(p["W2"]).T + p["b2"]
    h2 = gelu(z2)
    y = q(h2) @ q(p["w3"]) + p["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, y=y)


def loss(y, t):
    d = np.asarray(y) - np.asarray(t)
    return float(np.mean(d * d))


def backward(p, cache, t, bf16=True):
    """Gradients of the MSE loss with respect to every parameter."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    B = cache["X"].shape[0]
    dy = 2.0 * (cache["y"] - np.asarray(t, dtype=np.float64)) / B          # (B,)
    g = {}
    g["w3"] = q(cache["h2"]).T @ q(dy)
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(q(dy), q(p["w3"]))                                         # (B, 128)
    dz2 = dh2 * gelu_grad(cache["z2"])
    g["W2"] = q(dz2).T @ q(cache["h1"])
    g["b2"] = dz2.sum(axis=0)
    dh1 = q(dz2) @ q(p["W2"])
    dz1 = dh1 * gelu_grad(cache["z1"])
    g["W1"] = q(dz1).T @ q(cache["X"])
    g["b1"] = dz1.sum(axis=0)
    return g


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * grads[k] ** 2
            params[k] = params[k] - self.lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps)
        return params
