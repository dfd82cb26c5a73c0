"""FP64 reference of the learned surrogate (TEST INFRASTRUCTURE ONLY).

Network: Fourier features gamma(v) = [sin(2 pi B v), cos(2 pi B v)] of
v = (tx, rx) in [0,1]^4 with a fixed Gaussian B [64][4] (128 inputs), five
ReLU layers of width 256 and a linear head; loss = mean squared error against
y = log(P + eps).  Flat parameter layout: per hidden layer W_l [in][out]
then b_l [256]; then the head w [256] and b [1].

``round_bf16=True`` rounds, to the nearest bfloat16 (ties to even), exactly
the quantities the BF16 training path stores in BF16: the features, the
hidden-layer weights used by the matrix products, the hidden activations, and
the back-propagated pre-activation gradients.  All arithmetic stays FP64.
The backward pass is written out by hand (chain rule through each layer) and
is pinned against autograd and finite differences in tests.
"""
from __future__ import annotations

import numpy as np

WIDTH = 256
IN = 128
HIDDEN = 5


def layout():
    """[(w_off, fan_in, b_off) per hidden layer], head_w, head_b, n_params."""
    out, off = [], 0
    for l in range(HIDDEN):
        fi = IN if l == 0 else WIDTH
        out.append((off, fi, off + fi * WIDTH))
        off += fi * WIDTH + WIDTH
    head_w = off
    head_b = off + WIDTH
    return out, head_w, head_b, head_b + 1


def flatten(layers, head_w, head_b) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts += [np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64).ravel()]
    parts += [np.asarray(head_w, np.float64).ravel(), np.asarray(head_b, np.float64).ravel()]
    return np.concatenate(parts)


def unflatten(p):
    p = np.asarray(p, dtype=np.float64)
    lay, hw, hb, n = layout()
    assert p.size == n
    Ws = [p[o:o + fi * WIDTH].reshape(fi, WIDTH) for o, fi, _ in lay]
    bs = [p[bo:bo + WIDTH] for _, _, bo in lay]
    return Ws, bs, p[hw:hw + WIDTH], p[hb:hb + 1]


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as fp64."""
    return _bf16_exact(x)


def _bf16_exact(x):
    # one rounding: keep 8 significand bits, ties to even
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    scaled = m * 256.0                      # 8 significant bits in the integer part
    r = np.round(scaled)                    # numpy rounds half to even
    return np.ldexp(r / 256.0, e)


def features(v, B, round_bf16=False):
    v = np.asarray(v, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    z = 2.0 * np.pi * (v @ B.T)
    X = np.concatenate([np.sin(z), np.cos(z)], axis=1)
    return _bf16_exact(X) if round_bf16 else X


def forward(v, B, p, round_bf16=False):
    """(yhat [n], cache) with cache = (X list, H list, Ws used)."""
    Ws, bs, w5, b5 = unflatten(p)
    Wq = [_bf16_exact(W) for W in Ws] if round_bf16 else Ws
    X = features(v, B, round_bf16)
    xs, hs = [], []
    for l in range(HIDDEN):
        xs.append(X)
        H = np.maximum(X @ Wq[l] + bs[l], 0.0)
        if round_bf16:
            H = _bf16_exact(H)
        hs.append(H)
        X = H
    yhat = X @ w5 + b5[0]
    return yhat, (xs, hs, Wq)


def loss_and_grads(v, y, B, p, round_bf16=False):
    """MSE loss (1/n) sum (yhat - y)^2 and its gradient (flat), by hand."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    yhat, (xs, hs, Wq) = forward(v, B, p, round_bf16)
    Ws, bs, w5, b5 = unflatten(p)
    d = yhat - y
    loss = float(np.mean(d * d))
    g = 2.0 * d / n                                  # dL/dyhat
    lay, hw, hb, N = layout()
    grad = np.zeros(N)
    H4 = hs[-1]
    grad[hw:hw + WIDTH] = H4.T @ g                   # head weight
    grad[hb] = g.sum()                               # head bias
    dZ = (g[:, None] * w5[None, :]) * (H4 > 0)       # through the last ReLU
    if round_bf16:
        dZ = _bf16_exact(dZ)
    for l in range(HIDDEN - 1, -1, -1):
        o, fi, bo = lay[l]
        grad[bo:bo + WIDTH] = dZ.sum(axis=0)
        grad[o:o + fi * WIDTH] = (xs[l].T @ dZ).ravel()
        if l > 0:
            G = dZ @ Wq[l].T
            dZ = G * (hs[l - 1] > 0)
            if round_bf16:
                dZ = _bf16_exact(dZ)
    return loss, grad


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step with bias correction (t = 1 for the first step)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - (lr / (1 - b1 ** t)) * (m / (np.sqrt(v) / np.sqrt(1 - b2 ** t) + eps))
    return p, m, v
