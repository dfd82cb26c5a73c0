"""Tolerance protocol for comparing the FP32 HIP path with the FP64 oracle.

Forward power, per receiver r:
    |P_gpu(r) - P_orc(r)| <= 1e-5 * P_orc(r) + 2 * kappa(r) + ABS_FLOOR
kappa(r) is the largest change of the oracle's P(r) over four runs whose FP32
inputs (walls, tx, rx) are each moved by +-4 FP32 ulps of max(|x|, 1/2) with
seeded random signs.  It measures how strongly P(r) reacts to rounding-sized
changes of positions; with sharpness alpha a position error dx moves a
smoothing argument by alpha*dx/len, so near a shadow edge at alpha = 1000 an
FP32 evaluation cannot hold 1e-5 however it is written.  ABS_FLOOR (1e-30)
covers powers near the bottom of the FP32 range (products of many tiny
factors).

Gradients, per block (tx, walls):
    ||g_gpu - g_orc||_2 <= 1e-3 * ||g_orc||_2
or, where FP32 conditioning does not allow that (sharp shadow edges at large
alpha), ||g_gpu - g_orc||_2 <= 1e-3 ||g_orc||_2 + 2 kappa_g with kappa_g the
largest change of the block's oracle gradient over runs with every FP32 input
moved by +-4 ulps, as for the power.
"""
from __future__ import annotations

import numpy as np

from oracle import tracer as T

ABS_FLOOR = 1e-30
REL = 1e-5
GRAD_REL = 1e-3


def perturb(x: np.ndarray, rng, ulps: int = 4) -> np.ndarray:
    x = np.asarray(x, dtype=np.float32)
    mag = np.maximum(np.abs(x), np.float32(0.5))
    step = np.spacing(mag).astype(np.float64) * ulps
    sign = rng.choice([-1.0, 1.0], size=x.shape)
    return (x.astype(np.float64) + sign * step).astype(np.float32)


def kappa(walls, tx, rx, K, alpha, runs: int = 4, seed: int = 0, P0=None, mode="sigmoid"):
    rng = np.random.default_rng(seed)
    if P0 is None:
        P0 = T.power(walls, tx, rx, K, alpha, mode=mode)
    kap = np.zeros_like(P0)
    for _ in range(runs):
        P = T.power(perturb(walls, rng), perturb(tx, rng), perturb(rx, rng), K, alpha, mode=mode)
        kap = np.maximum(kap, np.abs(P - P0))
    return P0, kap


def check_power(P_gpu, P_orc, kap, label=""):
    P_gpu = np.asarray(P_gpu, dtype=np.float64)
    err = np.abs(P_gpu - P_orc)
    bound = REL * P_orc + 2.0 * kap + ABS_FLOOR
    bad = np.nonzero(err > bound)[0]
    rel = err / np.maximum(P_orc, 1e-300)
    stats = {"max_rel": float(rel.max()) if rel.size else 0.0,
             "frac_within_1e-5": float(np.mean(rel <= REL)) if rel.size else 1.0,
             "n": int(rel.size)}
    assert bad.size == 0, (f"{label}: {bad.size} receivers out of tolerance, e.g. idx {bad[:5]} "
                           f"gpu {P_gpu[bad[:5]]} orc {P_orc[bad[:5]]} kappa {kap[bad[:5]]}; {stats}")
    return stats


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def check_grads(gtx, gw, gtx_o, gw_o, label="", kap=None):
    """kap: optional (kappa_tx, kappa_walls) from grad_kappa."""
    etx = rel_l2(gtx, gtx_o)
    ew = rel_l2(gw, gw_o)
    ktx, kw = (0.0, 0.0) if kap is None else kap
    ntx, nw = float(np.linalg.norm(gtx_o)), float(np.linalg.norm(gw_o))
    assert etx * ntx <= GRAD_REL * ntx + 2 * ktx, \
        f"{label}: tx gradient rel err {etx:.3e} (gpu {gtx}, orc {gtx_o}, kappa {ktx:.3e})"
    assert ew * nw <= GRAD_REL * nw + 2 * kw, f"{label}: wall gradient rel err {ew:.3e} (kappa / norm {kw / nw:.3e})"
    return etx, ew


def grad_kappa(walls, tx, rx, K, alpha, g, runs: int = 2, seed: int = 1, ref=None, mode="sigmoid"):
    """(kappa_tx, kappa_walls): largest L2 change of the oracle's VJP blocks
    (seed g on rx) over runs with every FP32 input moved by +-4 ulps."""
    rng = np.random.default_rng(seed)
    if ref is None:
        gw0, gt0, _ = T.vjp(walls, tx, rx, K, alpha, g, mode=mode)
    else:
        gw0, gt0 = ref
    kt = kw = 0.0
    for _ in range(runs):
        gw, gt, _ = T.vjp(perturb(walls, rng), perturb(tx, rng), perturb(rx, rng), K, alpha, g, mode=mode)
        kt = max(kt, float(np.linalg.norm(gt - gt0)))
        kw = max(kw, float(np.linalg.norm(gw - gw0)))
    return kt, kw
