"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Multilayer perceptron: ``depth`` hidden layers of ``width`` units with SiLU,
z -> z / (1 + exp(-z)), then a linear output layer.  Parameters are a flat
vector in the library's layout: for each layer W (out x in, row-major) then
b (out).  Written from the definitions (chain rule, Adam as published by
Kingma & Ba, 2015) and pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def layer_dims(n_in, width, depth, n_out):
    dims = []
    for l in range(depth + 1):
        i = n_in if l == 0 else width
        o = n_out if l == depth else width
        dims.append((i, o))
    return dims


def unpack(params, dims):
    out, off = [], 0
    for i, o in dims:
        W = params[off:off + i * o].reshape(o, i)
        off += i * o
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == len(params)
    return out


def n_params(dims):
    return sum(i * o + o for i, o in dims)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, dims):
    """Returns (Y, cache) with cache = list of (input, pre-activation)."""
    layers = unpack(np.asarray(params, np.float64), dims)
    a = np.asarray(X, np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = z if l == len(layers) - 1 else silu(z)
    return a, cache


def backward(params, cache, dY, dims):
    """Gradient of sum(dY * Y) with respect to the parameter vector."""
    layers = unpack(np.asarray(params, np.float64), dims)
    grads = []
    g = np.asarray(dY, np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        a_in, z = cache[l]
        dz = g if l == len(layers) - 1 else g * dsilu(z)
        grads.append((dz.T @ a_in, dz.sum(0)))
        g = dz @ W
    flat = []
    for dW, db in reversed(grads):
        flat += [dW.ravel(), db]
    return np.concatenate(flat)


def mse(Y, T, w=None):
    """L = sum_ij w_j (Y - T)^2 / (n c) and dL/dY."""
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.float64)
    n, c = Y.shape
    w = np.ones(c) if w is None else np.asarray(w, np.float64)
    d = Y - T
    return float((w * d * d).sum() / (n * c)), 2.0 * w * d / (n * c)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    x32 = np.asarray(x, np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
