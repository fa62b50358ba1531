"""FP64 numpy reference of the warm-start MLP -- TEST INFRASTRUCTURE ONLY.

Network: sizes[0] -> ... -> sizes[L], ReLU after hidden layers, linear output,
mean-squared-error loss over all outputs of the batch.  Parameter vector order:
for each layer, W (out x in, row-major) then b (out).  Adam with bias
correction.  Pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def unpack(params, sizes):
    params = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for l in range(len(sizes) - 1):
        ni, no = sizes[l], sizes[l + 1]
        W = params[off:off + no * ni].reshape(no, ni)
        off += no * ni
        b = params[off:off + no]
        off += no
        out.append((W, b))
    assert off == params.size
    return out


def num_params(sizes):
    return sum(sizes[l + 1] * sizes[l] + sizes[l + 1] for l in range(len(sizes) - 1))


def forward(params, sizes, X):
    """Returns (activations [X, h1, ..., hL-1], output)."""
    layers = unpack(params, sizes)
    acts = [np.asarray(X, dtype=np.float64)]
    h = acts[0]
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if l < len(layers) - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return acts, h


def loss_and_grad(params, sizes, X, T):
    layers = unpack(params, sizes)
    acts, out = forward(params, sizes, X)
    B, N = out.shape
    diff = out - np.asarray(T, dtype=np.float64)
    loss = float(np.sum(diff * diff) / (B * N))
    dz = 2.0 * diff / (B * N)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h = acts[l]
        gW = dz.T @ h
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dh = dz @ W
            dz = dh * (h > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(theta, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
