"""FP64 reference of the warm-start network: dense layers, tanh on hidden layers, linear output,
mean-squared-error loss and its gradient by back-propagation.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Parameters are one flat vector laid out layer
by layer as W_l (row-major [out][in]) then b_l -- the layout the GPU network documents.
"""
from __future__ import annotations

import numpy as np


def unpack(params, dims):
    out, k = [], 0
    for i, o in zip(dims[:-1], dims[1:]):
        W = params[k:k + i * o].reshape(o, i)
        k += i * o
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == len(params)
    return out


def forward(params, dims, x):
    """Activations of every layer (the input first)."""
    acts = [np.asarray(x, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.tanh(z) if l + 1 < len(layers) else z)
    return acts


def gradient(params, dims, x, dy):
    """d(sum dy * y) / d(params) by the chain rule, layer by layer."""
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    acts = forward(params, dims, x)
    grads = []
    d = np.asarray(dy, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        if l + 1 < len(layers):
            d = d * (1.0 - acts[l + 1] ** 2)          # tanh'
        W, _ = layers[l]
        grads.append((d.T @ acts[l], d.sum(axis=0)))
        d = d @ W
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return np.concatenate(flat)


def mse(params, dims, x, target):
    y = forward(params, dims, x)[-1]
    return float(np.mean((y - target) ** 2))


def mse_gradient(params, dims, x, target):
    y = forward(params, dims, x)[-1]
    return gradient(params, dims, x, 2.0 * (y - target) / y.size)
