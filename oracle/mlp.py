"""FP64 oracle of the emulator network (test infrastructure only).

The network is a plain multilayer perceptron: widths w_0 -> ... -> w_L,
z_l = a_l W_l^T + b_l, a_{l+1} = silu(z_l) = z_l / (1 + exp(-z_l)) for the
hidden layers, output y = z_{L-1}; loss = mean over batch and outputs of
(y - t)^2; gradients by the chain rule written out layer by layer; Adam
(Kingma & Ba 2015) with beta1 0.9, beta2 0.999, eps 1e-8 and bias correction.

With ``bf16=True`` the operands of the matrix products are BF16 (round to
nearest even, as the device does) while all sums stay FP64: the weights and
the back-propagated deltas are rounded to BF16; in the forward pass each
layer input a enters as the sum of two BF16 values, hi = bf16(a) and
lo = bf16(a - hi) (about 16 significant bits); the weight gradients use the
hi halves.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest BF16 (ties to even), via FP32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_split(x: np.ndarray) -> np.ndarray:
    """hi + lo with hi = bf16(x), lo = bf16(x - hi)."""
    hi = bf16_round(x)
    return hi + bf16_round(np.asarray(x, dtype=np.float64) - hi)


def unpack(params: np.ndarray, widths):
    """Flat parameters (W_0, b_0, W_1, b_1, ...) -> [(W_l, b_l)]."""
    out, off = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = params[off:off + n_in * n_out].reshape(n_out, n_in)
        off += n_in * n_out
        b = params[off:off + n_out]
        off += n_out
        out.append((W, b))
    return out


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, widths, X, bf16=False, keep=False):
    rnd = bf16_round if bf16 else (lambda v: v)
    split = bf16_split if bf16 else (lambda v: v)
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    a = np.asarray(X, dtype=np.float64)
    acts, pres = [], []
    for l, (W, b) in enumerate(layers):
        acts.append(a)
        z = split(a) @ rnd(W).T + b
        pres.append(z)
        a = z * _sigmoid(z) if l + 1 < len(layers) else z
    return (a, acts, pres) if keep else a


def loss_and_grads(params, widths, X, T, bf16=False):
    """Mean-squared error and its gradient with respect to the flat parameters."""
    rnd = bf16_round if bf16 else (lambda v: v)
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    Y, acts, pres = forward(params, widths, X, bf16=bf16, keep=True)
    n = Y.size
    loss = float(np.mean((Y - T) ** 2))
    delta = 2.0 * (Y - T) / n
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dW = rnd(delta).T @ rnd(acts[l])
        db = delta.sum(axis=0)
        grads.append((dW, db))
        if l > 0:
            z = pres[l - 1]
            s = _sigmoid(z)
            delta = (rnd(delta) @ rnd(W)) * (s * (1.0 + z * (1.0 - s)))
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db)
    return loss, np.concatenate(flat)


def adam_step(params, grads, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (params, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * grads
    m2 = b2 * m2 + (1 - b2) * grads * grads
    mh = m1 / (1 - b1 ** t)
    vh = m2 / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2
