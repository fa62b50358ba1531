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


# ---------------------------------------------------------------------------
# BF16-operand model of the network, with per-element error bounds.
#
# The library computes every product with BF16 operands (the input, the weights, the
# hidden activations and the backpropagated dZ are rounded to bfloat16, round to
# nearest even) and accumulates in FP32; the output, dZ for the bias sums and the
# gradients are FP32.  The functions below take the same BF16 roundings on values
# computed in FP64, and return, next to each result, a bound on how far an FP32
# evaluation of the same formulas (any summation order, at most MAX_SPLIT partial sums
# per product) can lie from it.  Where such an evaluation could round an intermediate
# to a different BF16 neighbour, or flip a ReLU mask, the bound covers the jump.
# ---------------------------------------------------------------------------
U32 = 2.0 ** -24          # unit roundoff of FP32
U64 = 2.0 ** -53
MAX_SPLIT = 16            # partial sums per product (split over the reduction index)


def bf16_round(a):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even), for finite
    values in the FP32 normal range; returned as float64."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)   # rint: round half to even


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def _round_bound(v, e, rnd):
    """Rounding of a value known as v +- e: the rounded oracle value and a bound on
    |rnd(w) - rnd(v)| over all w in [v - e, v + e] (0 where the rounding is unique)."""
    r = rnd(v)
    lo, hi = rnd(v - e), rnd(v + e)
    return r, np.maximum(np.abs(hi - r), np.abs(lo - r))


def forward_backward_bf16(params32, sizes, X32, T32, rnd=bf16_round, exact_forward=False):
    """Forward pass, MSE loss and gradient of the network under the BF16-operand model.

    params32, X32, T32 are the FP32 values the library holds; `rnd` is the operand
    rounding (BF16 by default; the identity gives the plain FP64 network).  With
    exact_forward the caller guarantees that every sum of the forward pass is exactly
    representable in FP32 (for example integer data of small range), so the forward
    values carry no error.  Returns a dict with the
    output `out` and its bound `e_out`, the loss and `e_loss`, the flat gradient `grad`
    (parameter order of `unpack`) and `e_grad`, and `ambiguous` (how many BF16 roundings
    or ReLU masks of the pass the bounds had to treat as undecided)."""
    layers = unpack(np.asarray(params32, np.float32).astype(np.float64), sizes)
    L = len(layers)
    X = np.asarray(X32, np.float32).astype(np.float64)
    T = np.asarray(T32, np.float32).astype(np.float64)
    B = X.shape[0]
    amb = 0
    h = rnd(X)
    e_h = np.zeros_like(h)
    Hs, eHs, Wbs, mask_amb = [h], [e_h], [], []
    for l, (W, b) in enumerate(layers):
        Wb = rnd(W)
        Wbs.append(Wb)
        K = W.shape[1]
        z = h @ Wb.T + b
        mag = np.abs(h) @ np.abs(Wb).T + np.abs(b)
        if exact_forward:
            e = np.zeros_like(z)
        else:
            e = ((_gamma(K + MAX_SPLIT + 1) + K * U64) * mag
                 + (e_h @ np.abs(Wb).T) * (1 + _gamma(K)))
        if l < L - 1:
            r = np.maximum(z, 0.0)
            lo, hi = np.maximum(z - e, 0.0), np.maximum(z + e, 0.0)
            hb = rnd(r)
            e_hb = np.maximum(np.abs(rnd(hi) - hb), np.abs(rnd(lo) - hb))
            amb += int(np.count_nonzero(e_hb))
            mask_amb.append((z - e <= 0.0) & (z + e > 0.0))
            h, e_h = hb, e_hb
            Hs.append(h)
            eHs.append(e_h)
        else:
            out, e_out = z, e
    NO = out.shape[1]
    d = out - T
    e_d = e_out + U32 * (np.abs(d) + e_out)
    loss = float(np.sum(d * d) / (B * NO))
    e_loss = float(np.sum(2.0 * np.abs(d) * e_d + e_d * e_d) / (B * NO)
                   + (B * NO * U64 + U32) * (loss + np.sum(2.0 * np.abs(d) * e_d) / (B * NO)))
    coef = float(np.float32(2.0) / (np.float32(B) * np.float32(NO)))
    g = coef * d
    e_g = coef * e_d + U32 * (np.abs(g) + coef * e_d)
    gb, e_gb = _round_bound(g, e_g, rnd)
    amb += int(np.count_nonzero(e_gb))
    dzf, e_dzf, dzb, e_dzb = g, e_g, gb, e_gb
    grads, e_grads = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        H, e_H, Wb = Hs[l], eHs[l], Wbs[l]
        gW = dzb.T @ H
        e_gW = ((_gamma(B + MAX_SPLIT) + B * U64) * (np.abs(dzb).T @ np.abs(H))
                + np.abs(dzb).T @ e_H + e_dzb.T @ np.abs(H) + e_dzb.T @ e_H)
        gb_ = dzf.sum(axis=0)
        e_gb_ = (_gamma(B + 4) + B * U64) * np.abs(dzf).sum(axis=0) + e_dzf.sum(axis=0)
        grads[l] = (gW, gb_)
        e_grads[l] = (e_gW, e_gb_)
        if l > 0:
            No = Wb.shape[0]
            dH = dzb @ Wb
            e_dH = ((_gamma(No + MAX_SPLIT) + No * U64) * (np.abs(dzb) @ np.abs(Wb))
                    + e_dzb @ np.abs(Wb))
            on = H > 0.0
            ma = mask_amb[l - 1]
            amb += int(np.count_nonzero(ma))
            dz = np.where(on, dH, 0.0)
            e_dz = np.where(ma, np.abs(dH) + e_dH, np.where(on, e_dH, 0.0))
            dzf, e_dzf = dz, e_dz
            dzb, e_dzb = _round_bound(dz, e_dz, rnd)
            amb += int(np.count_nonzero(e_dzb))
    flat = np.concatenate([np.concatenate([a.ravel(), c]) for a, c in grads])
    e_flat = np.concatenate([np.concatenate([a.ravel(), c]) for a, c in e_grads])
    return {"out": out, "e_out": e_out, "loss": loss, "e_loss": e_loss, "grad": flat,
            "e_grad": e_flat, "ambiguous": amb, "hidden": Hs[1:]}


def adam_step_fp32_bound(theta, g, m, v, e_theta, e_m, e_v, lr, b1, b2, eps, step):
    """One bias-corrected Adam step in FP64 (adam_step) with hyperparameters that are
    FP32 values, and bounds on how far an FP32 evaluation of the same step (one rounding
    per operation, from a state known to within e_theta, e_m, e_v) can lie from it.
    Returns (theta, m, v, e_theta, e_m, e_v)."""
    c1, c2 = 1.0 - b1 ** step, 1.0 - b2 ** step
    m2 = b1 * m + (1 - b1) * g
    v2 = b2 * v + (1 - b2) * g * g
    e_m2 = b1 * e_m + 2 * U32 * (b1 * np.abs(m) + (1 - b1) * np.abs(g)) + U32 * np.abs(m2)
    e_v2 = b2 * e_v + 3 * U32 * (b2 * np.abs(v) + (1 - b2) * g * g) + U32 * np.abs(v2)
    mh, vh = m2 / c1, v2 / c2
    # the host forms 1 - b^t in FP32 (pow then a subtraction): 4 roundings relative to c
    e_mh = e_m2 / c1 + 5 * U32 * np.abs(mh) / c1
    e_vh = e_v2 / c2 + 5 * U32 * np.abs(vh) / c2
    sq = np.sqrt(vh)
    e_sq = np.minimum(e_vh / np.maximum(2.0 * sq, 1e-300), np.sqrt(e_vh)) + U32 * sq
    den = sq + eps
    e_den = e_sq + U32 * den
    r = mh / den
    e_r = (e_mh + np.abs(r) * e_den) / np.maximum(den - e_den, 1e-300) + U32 * np.abs(r)
    stp = lr * r
    e_stp = lr * e_r + U32 * np.abs(stp)
    th2 = theta - stp
    e_th2 = e_theta + e_stp + U32 * np.abs(th2)
    return th2, m2, v2, e_th2, e_m2, e_v2
