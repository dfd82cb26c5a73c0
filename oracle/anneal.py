"""FP64 reference of the transmitter optimisation with an annealed sharpness
(TEST INFRASTRUCTURE ONLY; nothing in the product path imports it).

Sec. VII places one transmitter to serve several receivers by maximising
Eq. 8, F(tx) = min_i P_Rx_i(tx), with a gradient method, and raises the
sharpness alpha after every iteration along a geometric progression from 1 to
100 over the iterations (Fig. 5 lists alpha at four iterations).  Here the
loss is L = -F and each iteration takes one Adam step (the paper does not
name its optimiser; Adam with bias correction is the reading used by the GPU
path, followed by a clamp of tx to the box).
"""
from __future__ import annotations

import numpy as np

from . import tracer as T


def alpha_schedule(i, n_iter: int, a_first: float = 1.0, a_last: float = 100.0):
    """alpha at iteration i of n_iter: a_first (a_last / a_first)^(i / (n_iter - 1))."""
    i = np.minimum(np.asarray(i, dtype=np.float64), n_iter - 1)
    return a_first * (a_last / a_first) ** (i / (n_iter - 1))


def adam_step(x, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
              lo: float = 1e-3, hi: float = 1.0 - 1e-3):
    """Adam with bias correction (t = 1 for the first step), then clamp to [lo, hi]."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    xn = x - (lr / (1.0 - b1 ** t)) * (m / (np.sqrt(v) / np.sqrt(1.0 - b2 ** t) + eps))
    return np.clip(xn, lo, hi), m, v


def optimize(walls, rx, tx0, max_order: int, steps: int, lr: float, alphas):
    """Iterations of (L = -min_r P(r) at alpha_i, gradient w.r.t. tx, Adam step).

    ``alphas[i]`` is the sharpness of iteration i.  Returns (tx_hist [steps+1, 2],
    loss_hist [steps]) with loss_hist[i] evaluated at tx_hist[i].
    """
    x = np.asarray(tx0, dtype=np.float64).reshape(2).copy()
    m = np.zeros(2)
    v = np.zeros(2)
    hist = [x.copy()]
    losses = []
    for i in range(steps):
        _, L, _, gt, _ = T.forward_backward(walls, x, rx, max_order, float(alphas[i]), kind="neg_min")
        losses.append(L)
        x, m, v = adam_step(x, gt, m, v, i + 1, lr)
        hist.append(x.copy())
    return np.array(hist), np.array(losses)
