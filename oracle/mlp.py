"""FP64 reference of the warm-start network (test infrastructure only).

A fully connected network y = W_L^T(... GELU(W_1^T x + b_1) ...) + b_L, GELU(x) = x Phi(x)
(Hendrycks and Gimpel, 2016), trained on the mean square error with Adam (Kingma and Ba, 2015).
Everything is computed in float64 with plain numpy; with ``bf16_ops=True`` the GEMM operands
(network input, hidden activations, weights, output gradients) are first rounded to bfloat16
(round to nearest even of the float32 value), the precision the learned warm start fixes for its
matrix products.  With ``bf16_ops=False`` nothing is rounded and ``backward`` is the exact gradient
of ``loss`` (pinned by finite differences).

Parameters are one flat array packed per layer l as W_l [dims[l]][dims[l+1]] (row-major) then
b_l [dims[l+1]].
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via the float32 value; returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def n_params(dims) -> int:
    return int(sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1)))


def unpack(dims, params):
    out, o = [], 0
    params = np.asarray(params, np.float64)
    for i in range(len(dims) - 1):
        a, b = dims[i], dims[i + 1]
        W = params[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, params[o:o + b]))
        o += b
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def forward(dims, params, x, bf16_ops=True):
    """Returns y and the cache (GEMM inputs A_l and pre-activations Z_l of every layer)."""
    r = bf16 if bf16_ops else (lambda v: np.asarray(v, np.float64))
    layers = unpack(dims, params)
    A = r(x)
    As, Zs = [], []
    for l, (W, b) in enumerate(layers):
        Z = A @ r(W) + b
        As.append(A)
        Zs.append(Z)
        if l < len(layers) - 1:
            A = r(gelu(Z))
    return Zs[-1], (As, Zs)


def loss(dims, params, x, t, bf16_ops=True) -> float:
    y, _ = forward(dims, params, x, bf16_ops)
    return float(np.mean((y - t) ** 2))


def backward(dims, params, x, t, bf16_ops=True):
    """Gradient of the mean square error (flat, packed like params) and the loss."""
    r = bf16 if bf16_ops else (lambda v: np.asarray(v, np.float64))
    layers = unpack(dims, params)
    y, (As, Zs) = forward(dims, params, x, bf16_ops)
    dZ = r(2.0 * (y - t) / y.size)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (As[l].T @ dZ, dZ.sum(axis=0))
        if l > 0:
            dA = dZ @ r(W).T
            dZ = r(dA * gelu_grad(Zs[l - 1]))
    return pack(grads), float(np.mean((y - t) ** 2))


class Adam:
    """Adam with bias correction; the step count starts at 1."""

    def __init__(self, n, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0

    def step(self, params, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return params - self.lr * mhat / (np.sqrt(vhat) + self.eps)
