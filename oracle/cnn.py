"""CPU reference of the learned refinement predictor (not part of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The predictor maps the normalised primitive fields of one patch (plus a halo
of 3 cells) to a per-cell logit of "this cell will be tagged within the next
k steps".  Three valid 3x3 (2D) or 3x3x3 (3D) convolutions with bias, ReLU
after the first two, sigmoid on the output:

    x [cin, n+6, ...] -> conv1 -> relu -> [ch, n+4] -> conv2 -> relu -> [ch, n+2]
      -> conv3 -> [1, n] logits

Loss: binary cross-entropy with logits and a positive-class weight,
    l = -(w y log s(z) + (1 - y) log(1 - s(z))), averaged over all cells.

``bf16=True`` rounds inputs, weights and the activations entering each layer
to bfloat16 (round to nearest even) and accumulates in float32, the
arithmetic of the GPU kernels.  The backward pass is plain FP64 (pinned by
central finite differences in the tests).
"""
from __future__ import annotations

import itertools

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (nearest, ties to even), returned as float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out)


def conv_valid(x: np.ndarray, w: np.ndarray, b: np.ndarray, acc=np.float64) -> np.ndarray:
    """Valid cross-correlation: x [N, Ci, *S], w [Co, Ci, 3, ...] -> [N, Co, *(S-2)]."""
    d = x.ndim - 2
    out_shape = tuple(s - 2 for s in x.shape[2:])
    y = np.zeros((x.shape[0], w.shape[0]) + out_shape, dtype=acc)
    for off in itertools.product(range(3), repeat=d):
        sl = tuple(slice(o, o + s) for o, s in zip(off, out_shape))
        xs = x[(slice(None), slice(None)) + sl].astype(acc)
        wk = w[(slice(None), slice(None)) + off].astype(acc)       # [Co, Ci]
        y += np.einsum("oc,nc...->no...", wk, xs)
    y += b.astype(acc).reshape((1, -1) + (1,) * d)
    return y


def forward(x, params, bf16: bool = False):
    """Logits and the saved activations (a0 input, h1, h2 pre-activations)."""
    W1, b1, W2, b2, W3, b3 = params
    acc = np.float32 if bf16 else np.float64
    r = bf16_round if bf16 else (lambda a: a)
    a0 = r(x)
    z1 = conv_valid(a0, r(W1), b1, acc)
    a1 = r(np.maximum(z1, 0))
    z2 = conv_valid(a1, r(W2), b2, acc)
    a2 = r(np.maximum(z2, 0))
    z3 = conv_valid(a2, r(W3), b3, acc)
    return z3[:, 0], (a0, z1, a1, z2, a2)


def bce_with_logits(z, y, pos_weight: float):
    """Mean weighted BCE and its gradient with respect to the logits."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    # log s(z) = -softplus(-z), log(1 - s(z)) = -softplus(z)
    sp_pos = np.logaddexp(0.0, -z)
    sp_neg = np.logaddexp(0.0, z)
    loss = pos_weight * y * sp_pos + (1.0 - y) * sp_neg
    s = 1.0 / (1.0 + np.exp(-z))
    grad = (pos_weight * y * (s - 1.0) + (1.0 - y) * s) / z.size
    return float(loss.mean()), grad


def _conv_backward(x, w, gy):
    """Gradients of a valid cross-correlation: (dx, dw, db)."""
    d = x.ndim - 2
    out_shape = gy.shape[2:]
    dx = np.zeros_like(x, dtype=np.float64)
    dw = np.zeros_like(w, dtype=np.float64)
    for off in itertools.product(range(3), repeat=d):
        sl = tuple(slice(o, o + s) for o, s in zip(off, out_shape))
        xs = x[(slice(None), slice(None)) + sl]
        gyr = np.moveaxis(gy, 1, 0).reshape(gy.shape[1], -1)
        xr = np.moveaxis(xs, 1, 0).reshape(xs.shape[1], -1)
        dw[(slice(None), slice(None)) + off] += gyr @ xr.T
        dx[(slice(None), slice(None)) + sl] += np.einsum("oc,no...->nc...", w[(slice(None), slice(None)) + off], gy)
    db = gy.sum(axis=tuple(i for i in range(gy.ndim) if i != 1))
    return dx, dw, db


def backward(x, params, y, pos_weight: float):
    """FP64 loss and parameter gradients (same order as params)."""
    W1, b1, W2, b2, W3, b3 = params
    z, (a0, z1, a1, z2, a2) = forward(x, params)
    loss, gz = bce_with_logits(z, y, pos_weight)
    g3 = gz[:, None]
    da2, dW3, db3 = _conv_backward(a2, W3, g3)
    gz2 = da2 * (z2 > 0)
    da1, dW2, db2 = _conv_backward(a1, W2, gz2)
    gz1 = da1 * (z1 > 0)
    _, dW1, db1 = _conv_backward(a0, W1, gz1)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def init_params(c0: int, c1: int, d: int, seed: int):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    k = 3 ** d
    shape1 = (c1, c0) + (3,) * d
    shape2 = (c1, c1) + (3,) * d
    shape3 = (1, c1) + (3,) * d
    W1 = rng.normal(0.0, np.sqrt(2.0 / (c0 * k)), shape1)
    W2 = rng.normal(0.0, np.sqrt(2.0 / (c1 * k)), shape2)
    W3 = rng.normal(0.0, np.sqrt(2.0 / (c1 * k)), shape3)
    return [W1, np.zeros(c1), W2, np.zeros(c1), W3, np.zeros(1)]


def adam_step(params, grads, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected) on FP32 master copies; returns new lists."""
    out_p, out_m, out_v = [], [], []
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for p, g, mi, vi in zip(params, grads, m, v):
        p = np.asarray(p, np.float32)
        g = np.asarray(g, np.float32)
        mi = beta1 * mi + (1.0 - beta1) * g
        vi = beta2 * vi + (1.0 - beta2) * g * g
        mh = mi / c1
        vh = vi / c2
        out_p.append((p - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32))
        out_m.append(mi.astype(np.float32))
        out_v.append(vi.astype(np.float32))
    return out_p, out_m, out_v
