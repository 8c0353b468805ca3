"""FP64 reference for the surrogate MLP (test infrastructure only).

Network: dense layers widths[0] -> ... -> widths[L], tanh on hidden layers,
linear output; parameters flat, layer by layer, W_l (widths[l+1] x widths[l],
row-major) then b_l.  Loss: sum w (y - t)^2 / sum w.

With ``bf16=True`` values are rounded to bfloat16 (round to nearest, ties to
even) at the points where the device network stores BF16: the input, the
weights used in products, the hidden activations, and the gradients that
enter products (output-layer gradient and hidden pre-activation gradients).
Everything else is float64.  With ``bf16=False`` the same network is exact
float64 (used for finite-difference checks of the backward pass).
"""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 (ties to even), via float32, returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def layers(params, widths):
    out, off = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = np.asarray(params[off: off + n_in * n_out], dtype=np.float64).reshape(n_out, n_in)
        off += n_in * n_out
        b = np.asarray(params[off: off + n_out], dtype=np.float64)
        off += n_out
        out.append((W, b))
    return out


def forward(params, widths, x, bf16=True):
    q = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    h = q(x)
    acts = [h]
    L = len(widths) - 1
    for l, (W, b) in enumerate(layers(params, widths)):
        z = h @ q(W).T + b
        if l + 1 < L:
            h = q(np.tanh(z))
            acts.append(h)
        else:
            return z, acts


def loss_grad(params, widths, x, t, w=None, bf16=True):
    q = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    y, acts = forward(params, widths, x, bf16)
    t = np.asarray(t, dtype=np.float64)
    w = np.ones_like(t) if w is None else np.asarray(w, dtype=np.float64)
    wsum = w.sum()
    d = y - t
    loss = float((w * d * d).sum() / wsum)
    dz = q(2.0 * w * d / wsum)
    grads = []
    lay = layers(params, widths)
    for l in range(len(lay) - 1, -1, -1):
        W, _ = lay[l]
        gW = dz.T @ acts[l]
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if l > 0:
            dy = dz @ q(W)
            dz = q(dy * (1.0 - acts[l] ** 2))
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.reshape(-1), gb]
    return loss, np.concatenate(flat)


def adam(p, g, m, v, step, lr, b1, b2, eps):
    """One bias-corrected Adam step (Kingma and Ba); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(widths, rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    out = []
    for l in range(len(widths) - 1):
        lim = 1.0 / np.sqrt(widths[l])
        out.append(rng.uniform(-lim, lim, size=widths[l] * widths[l + 1]))
        out.append(np.zeros(widths[l + 1]))
    return np.concatenate(out)
