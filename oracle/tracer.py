"""FP64 CPU oracle of the smoothed image-method ray tracer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the HIP path.

What it computes, following the paper (arXiv 2401.11882):

* Smoothing (Sec. IV, Eq. 3 and Eq. 4): a comparison ``x0 > x1`` becomes
  ``s(x0 - x1; alpha)`` with ``s(x; alpha) = sigmoid(alpha * x)``
  (mode "sigmoid") or the hard sigmoid of Eq. 5-6,
  ``relu6(alpha x + 3) / 6`` (mode "hard_sigmoid").  The unsmoothed
  reference (mode "hard") uses the unit step of Eq. 1 instead.
* Candidates (Sec. V): every ordered sequence of walls of length 0..K with no
  wall repeated back to back (full visibility matrix, box walls included).
* Path in the relaxed scene (Sec. V and Sec. V-B): the image method over
  infinite wall lines.  Images ``I_0 = tx`` and ``I_i`` = mirror of ``I_{i-1}``
  across the line of wall ``sigma_i``; back-trace from ``X_{k+1} = r``: ``X_i``
  is where the line from ``X_{i+1}`` to ``I_i`` meets the line of ``sigma_i``,
  at ``X_i = a + t_i e = X_{i+1} + u_i (I_i - X_{i+1})``.
* Continuous validity (Sec. V-A): each hard check is a comparison, smoothed.
  ``inside(x) = s(x) * s(1 - x)`` (Boolean AND as a product).  Interaction i:
  ``inside(t_i) * inside(u_i)`` (point on its segment, and the point lies
  between the previous point and the image, i.e. a true reflection).
  Obstruction of leg [X_l, X_{l+1}] by wall j (not one of the leg's own end
  walls): the leg meets the wall at leg parameter ``upsilon`` and wall
  parameter ``tau``; the factor is ``1 - inside(tau) * inside(upsilon)``
  (NOT as one minus).  ``V`` is the product of all factors.
* Received power (Eq. 7 with the dyadic coefficient set to the identity, an
  incoherent sum): ``P(r) = sum_paths V / max(|r - I_k|^2, d_min^2)``.
* Objective (Sec. III): ``L = -F``; here ``L_log = -(1/R) sum_r log(P(r)+eps)``,
  ``L_sum = sum_r P(r)``, or ``L_min = -min_r P(r)`` (Eq. 8, Sec. VII).
* Gradients: torch autograd (reverse mode) over the same fp64 expressions, in
  the role the paper gives to automatic differentiation (Sec. I, Sec. III).

Degenerate cases: a zero-length wall cannot mirror (its candidates contribute
0); a back-trace with the line parallel to the wall gives an invalid path
(contribution 0); an obstruction test whose leg is parallel to the wall gives
the factor 1.

Numerics: ``inside`` products are formed as ``exp`` of summed ``logsigmoid``
terms and ``1 - exp(z)`` as ``-expm1(z)``; these are identities of the
definitions above that keep tiny factors (deep shadows) accurate in fp64.
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence

import numpy as np
import torch
import torch.nn.functional as F

DTYPE = torch.float64
DEFAULT_DMIN = 1e-3
DEFAULT_LOG_EPS = 1e-6


# --------------------------------------------------------------------------
# Smoothing functions (Sec. IV)
# --------------------------------------------------------------------------

def unit_step(x):
    """Eq. 1: 1 where x > 0 else 0."""
    return (torch.as_tensor(x, dtype=DTYPE) > 0).to(DTYPE)


def sigmoid(x, alpha):
    """Eq. 3 + Eq. 4: 1 / (1 + exp(-alpha x))."""
    return torch.sigmoid(alpha * torch.as_tensor(x, dtype=DTYPE))


def hard_sigmoid(x, alpha):
    """Eq. 5 + Eq. 6: relu6(alpha x + 3) / 6."""
    z = alpha * torch.as_tensor(x, dtype=DTYPE) + 3.0
    return torch.clamp(z, 0.0, 6.0) / 6.0


def _log_inside(x, alpha):
    """log of s(x) * s(1 - x): smoothed form of the check 0 < x < 1."""
    return F.logsigmoid(alpha * x) + F.logsigmoid(alpha * (1.0 - x))


def _hard_inside(x):
    return ((x > 0) & (x < 1)).to(DTYPE)


def _hs_inside(x, alpha):
    """hard sigmoid(x) * hard sigmoid(1 - x) (Eq. 5-6): the check 0 < x < 1."""
    return hard_sigmoid(x, alpha) * hard_sigmoid(1.0 - x, alpha)


def _cross(u, v):
    return u[..., 0] * v[..., 1] - u[..., 1] * v[..., 0]


# --------------------------------------------------------------------------
# Candidates (Sec. V)
# --------------------------------------------------------------------------

def candidates(n_walls: int, max_order: int) -> list[tuple[int, ...]]:
    """All wall sequences of length 0..K without a wall repeated back to back."""
    out: list[tuple[int, ...]] = [()]
    for k in range(1, max_order + 1):
        for seq in itertools.product(range(n_walls), repeat=k):
            if all(seq[i] != seq[i + 1] for i in range(k - 1)):
                out.append(seq)
    return out


def n_candidates(n_walls: int, max_order: int) -> int:
    return len(candidates(n_walls, max_order)) if n_walls <= 8 else \
        1 + sum(n_walls * (n_walls - 1) ** (k - 1) for k in range(1, max_order + 1))


def _groups(n_walls: int, max_order: int):
    """Candidates grouped by order as LongTensors [C_k, k]."""
    by_k: dict[int, list] = {}
    for seq in candidates(n_walls, max_order):
        by_k.setdefault(len(seq), []).append(seq)
    return {k: torch.tensor(v, dtype=torch.long).reshape(len(v), k) for k, v in by_k.items()}


# --------------------------------------------------------------------------
# Image method (Sec. V, Sec. V-B)
# --------------------------------------------------------------------------

def images(walls, src, seq):
    """Images of ``src`` across the lines of walls seq[:,0], seq[:,1], ...

    walls fp64 [W,4]; src fp64 [2]; seq long [C,k].  Returns (list of k+1
    tensors [C,2], ok [C]) where ok is False when a zero-length wall is used.
    """
    a = walls[:, 0:2]
    e = walls[:, 2:4] - walls[:, 0:2]
    C, k = seq.shape
    out = [src.expand(C, 2)]
    ok = torch.ones(C, dtype=torch.bool)
    for i in range(k):
        A, E = a[seq[:, i]], e[seq[:, i]]
        n = torch.stack([-E[:, 1], E[:, 0]], dim=-1)      # normal of the wall line
        nn = (n * n).sum(-1)
        ok = ok & (nn > 0)
        nn_safe = torch.where(nn > 0, nn, torch.ones_like(nn))
        h = ((out[-1] - A) * n).sum(-1) / nn_safe           # signed distance * |n|
        out.append(out[-1] - 2.0 * h[:, None] * n)
    return out, ok


def _group_terms(walls, tx, rxc, seq, alpha, mode, d_min, want_paths=False):
    """Per-(rx, candidate) contribution for one order group.

    Returns c [Rc, C] (and optionally a dict with points and parameters).
    """
    a = walls[:, 0:2]
    e = walls[:, 2:4] - walls[:, 0:2]
    C, k = seq.shape
    Rc = rxc.shape[0]
    I, ok = images(walls, tx, seq)
    valid = ok[None, :].expand(Rc, C).clone()

    # back-trace: X_{k+1} = r, then X_k .. X_1
    X: list = [None] * (k + 2)
    X[k + 1] = rxc[:, None, :].expand(Rc, C, 2)
    log_f = torch.zeros(Rc, C, dtype=DTYPE)
    f_hard = torch.ones(Rc, C, dtype=DTYPE)
    params = {}
    for i in range(k, 0, -1):
        A, E = a[seq[:, i - 1]][None], e[seq[:, i - 1]][None]
        d = I[i][None] - X[i + 1]
        w = A - X[i + 1]
        den = _cross(d, E)
        nz = den != 0
        den_s = torch.where(nz, den, torch.ones_like(den))
        t = _cross(w, d) / den_s       # position along the wall segment
        u = _cross(w, E) / den_s       # position between X_{i+1} and the image I_i
        valid = valid & nz
        X[i] = A + t[..., None] * E
        if mode == "sigmoid":
            log_f = log_f + _log_inside(t, alpha) + _log_inside(u, alpha)
        elif mode == "hard_sigmoid":
            f_hard = f_hard * _hs_inside(t, alpha) * _hs_inside(u, alpha)
        else:
            f_hard = f_hard * _hard_inside(t) * _hard_inside(u)
        params[i] = (t, u)
    X[0] = tx.expand(Rc, C, 2)

    V = torch.exp(log_f) if mode == "sigmoid" else f_hard
    Wn = walls.shape[0]
    jidx = torch.arange(Wn)
    for l in range(k + 1):
        P0, P1 = X[l], X[l + 1]
        D = (P1 - P0)[:, :, None, :]                    # [Rc,C,1,2]
        w0 = a[None, None] - P0[:, :, None, :]           # [Rc,C,W,2]
        den = _cross(D, e[None, None])                   # [Rc,C,W]
        excl = torch.zeros(C, Wn, dtype=torch.bool)
        if l >= 1:
            excl |= seq[:, l - 1][:, None] == jidx[None]
        if l + 1 <= k:
            excl |= seq[:, l][:, None] == jidx[None]
        use = (den != 0) & ~excl[None]
        den_s = torch.where(den != 0, den, torch.ones_like(den))
        tau = _cross(w0, D) / den_s                      # along wall j
        ups = _cross(w0, e[None, None]) / den_s          # along the leg
        if mode == "sigmoid":
            q = -torch.expm1(_log_inside(tau, alpha) + _log_inside(ups, alpha))
        elif mode == "hard_sigmoid":
            q = 1.0 - _hs_inside(tau, alpha) * _hs_inside(ups, alpha)
        else:
            q = 1.0 - _hard_inside(tau) * _hard_inside(ups)
        q = torch.where(use, q, torch.ones_like(q))
        V = V * torch.prod(q, dim=-1)

    d2 = ((rxc[:, None, :] - I[k][None]) ** 2).sum(-1)
    c = V / torch.clamp(d2, min=d_min * d_min)
    c = torch.where(valid, c, torch.zeros_like(c))
    if want_paths:
        return c, {"X": X, "I": I, "V": V, "valid": valid, "params": params, "d2": d2}
    return c


def _as64(x, requires_grad=False):
    t = torch.as_tensor(np.asarray(x, dtype=np.float64) if not torch.is_tensor(x) else x,
                        dtype=DTYPE).clone()
    if requires_grad:
        t.requires_grad_(True)
    return t


def _chunk_size(n_rx: int, groups, n_walls: int, budget: float = 3e6) -> int:
    widest = max([g.shape[0] for g in groups.values()] + [1])
    return int(max(1, min(n_rx, budget // max(1, widest * max(1, n_walls)))))


# --------------------------------------------------------------------------
# Power map, losses, gradients
# --------------------------------------------------------------------------

def power(walls, tx, rx, max_order: int, alpha: float, mode: str = "sigmoid",
          d_min: float = DEFAULT_DMIN) -> np.ndarray:
    """Received power P(r) for every receiver (fp64 numpy [R])."""
    W = _as64(walls).reshape(-1, 4)
    T = _as64(tx).reshape(2)
    Rx = _as64(rx).reshape(-1, 2)
    groups = _groups(W.shape[0], max_order)
    cs = _chunk_size(Rx.shape[0], groups, W.shape[0])
    out = np.zeros(Rx.shape[0])
    with torch.no_grad():
        for s in range(0, Rx.shape[0], cs):
            rxc = Rx[s:s + cs]
            acc = torch.zeros(rxc.shape[0], dtype=DTYPE)
            for k in sorted(groups):
                acc = acc + _group_terms(W, T, rxc, groups[k], alpha, mode, d_min).sum(1)
            out[s:s + cs] = acc.numpy()
    return out


def loss_value(P, kind: str, log_eps: float = DEFAULT_LOG_EPS) -> float:
    P = np.asarray(P, dtype=np.float64)
    if kind == "sum":
        return float(P.sum())
    if kind == "neg_mean_log":
        return float(-np.mean(np.log(P + log_eps)))
    if kind == "neg_min":
        # Eq. 8 (Sec. VII): F = min over receivers, maximised; as a loss, -F
        return float(-np.min(P))
    raise ValueError(kind)


def loss_seed(P, kind: str, log_eps: float = DEFAULT_LOG_EPS) -> np.ndarray:
    """dL/dP(r) for the two losses."""
    P = np.asarray(P, dtype=np.float64)
    if kind == "sum":
        return np.ones_like(P)
    if kind == "neg_mean_log":
        return -1.0 / (P.size * (P + log_eps))
    if kind == "neg_min":
        # derivative of -min: -1 at the minimiser (the lowest index on a tie)
        g = np.zeros_like(P)
        g[int(np.argmin(P))] = -1.0
        return g
    raise ValueError(kind)


def vjp(walls, tx, rx, max_order: int, alpha: float, g, mode: str = "sigmoid",
        d_min: float = DEFAULT_DMIN):
    """Vector-Jacobian product: sum_r g[r] dP(r)/d(walls, tx, rx).

    Returns (g_walls fp64 [W,4], g_tx [2], g_rx [R,2]).
    """
    W = _as64(walls, True)
    T = _as64(tx, True)
    Rx = _as64(rx).reshape(-1, 2)
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    groups = _groups(W.shape[0], max_order)
    cs = _chunk_size(Rx.shape[0], groups, W.shape[0], budget=1.5e6)
    g_rx = np.zeros((Rx.shape[0], 2))
    for s in range(0, Rx.shape[0], cs):
        gc = torch.as_tensor(g[s:s + cs], dtype=DTYPE)
        if not torch.any(gc != 0):
            continue
        rxc = Rx[s:s + cs].clone().requires_grad_(True)
        acc = torch.zeros(rxc.shape[0], dtype=DTYPE)
        for k in sorted(groups):
            acc = acc + _group_terms(W, T, rxc, groups[k], alpha, mode, d_min).sum(1)
        (acc * gc).sum().backward()
        g_rx[s:s + cs] = rxc.grad.numpy()
    gw = W.grad.numpy().copy() if W.grad is not None else np.zeros(tuple(W.shape))
    gt = T.grad.numpy().copy() if T.grad is not None else np.zeros(2)
    return gw, gt, g_rx


def forward_backward(walls, tx, rx, max_order, alpha, kind="neg_mean_log",
                     log_eps=DEFAULT_LOG_EPS, d_min=DEFAULT_DMIN, rx_weight=None, mode="sigmoid"):
    """Power map, loss, and loss gradients w.r.t. walls and tx.

    ``rx_weight`` (optional 0/1 mask) restricts the gradient to a receiver
    subset while the loss seed keeps the full-map normalisation.
    """
    P = power(walls, tx, rx, max_order, alpha, mode=mode, d_min=d_min)
    L = loss_value(P, kind, log_eps)
    g = loss_seed(P, kind, log_eps)
    if rx_weight is not None:
        g = g * np.asarray(rx_weight, dtype=np.float64)
    gw, gt, grx = vjp(walls, tx, rx, max_order, alpha, g, mode=mode, d_min=d_min)
    return P, L, gw, gt, grx


def path_details(walls, tx, r, max_order, alpha, mode="sigmoid", d_min=DEFAULT_DMIN):
    """Per-candidate details at one receiver (for tests).

    Returns a list of dicts: seq, c, V, points X_1..X_k, their wall and side
    parameters t, u, valid, d2.
    """
    W = _as64(walls).reshape(-1, 4)
    T = _as64(tx).reshape(2)
    Rr = _as64(r).reshape(1, 2)
    out = []
    with torch.no_grad():
        for k, seq in sorted(_groups(W.shape[0], max_order).items()):
            c, info = _group_terms(W, T, Rr, seq, alpha, mode, d_min, want_paths=True)
            for ci in range(seq.shape[0]):
                out.append({
                    "seq": tuple(int(v) for v in seq[ci]),
                    "c": float(c[0, ci]),
                    "V": float(info["V"][0, ci]),
                    "valid": bool(info["valid"][0, ci]),
                    "points": [info["X"][i][0, ci].numpy().copy() for i in range(1, k + 1)],
                    "t": [float(info["params"][i][0][0, ci]) for i in range(1, k + 1)],
                    "u": [float(info["params"][i][1][0, ci]) for i in range(1, k + 1)],
                    "image": info["I"][k][ci].numpy().copy(),
                    "d2": float(info["d2"][0, ci]),
                })
    return out


def work_counts(walls, tx, rx, max_order, alpha, margin: float = 18.0,
                active_log_floor: float = -88.72, cut: float = 0.0):
    """Algorithmic work of the method at these receivers (instrumentation;
    parity unpinned against the paper, which counts no work).

    One rule decides what is credited, with no reference to the order in
    which an implementation visits walls or candidates: a (receiver,
    candidate) pair is *active* when it is valid, its interaction factor F
    (the product of in(t_i) in(u_i)) exceeds exp(active_log_floor) (below, F
    is exactly 0 in FP32, and so is every later product) and, with ``cut`` >
    0, the bound F / max(d^2, d_min^2) of its contribution, known before any
    obstruction test, exceeds cut * P(r).  A pair's back-trace, interaction
    factors and obstruction tests are all credited when it is active and not
    at all otherwise.  Counts:

      * ``path_evals`` and ``interactions`` (k per pair): all pairs;
      * ``active`` and ``active_interactions``: active pairs and their k;
      * ``tests``: obstruction tests of active pairs (a leg is not tested
        against its own end walls);
      * ``unsaturated``: those tests whose leg parameter and wall parameter
        both lie within margin/alpha of [0, 1] (outside, the smoothed factor
        is within 2^-25 of 1 and rounds to 1 in FP32) and whose leg is not
        parallel to the wall.
    """
    W = _as64(walls).reshape(-1, 4)
    T = _as64(tx).reshape(2)
    Rx = _as64(rx).reshape(-1, 2)
    a = W[:, 0:2]
    e = W[:, 2:4] - W[:, 0:2]
    groups = _groups(W.shape[0], max_order)
    cs = max(1, _chunk_size(Rx.shape[0], groups, W.shape[0]) // (max_order + 1))
    band = margin / alpha
    P_all = torch.as_tensor(power(walls, tx, rx, max_order, alpha), dtype=DTYPE) if cut > 0 else None
    out = dict(path_evals=0, interactions=0, active=0, active_interactions=0, tests=0, unsaturated=0)
    nW = W.shape[0]
    jidx = torch.arange(nW)
    with torch.no_grad():
        for s in range(0, Rx.shape[0], cs):
            rxc = Rx[s:s + cs]
            for k, seq in groups.items():
                _, info = _group_terms(W, T, rxc, seq, alpha, "sigmoid", DEFAULT_DMIN, True)
                X = info["X"]
                Cn = seq.shape[0]
                logf = torch.zeros(rxc.shape[0], Cn, dtype=DTYPE)
                for i, (t, u) in info["params"].items():
                    logf = logf + _log_inside(t, alpha) + _log_inside(u, alpha)
                ok = info["valid"] & (logf > active_log_floor)
                if cut > 0:
                    dd = torch.clamp(info["d2"], min=DEFAULT_DMIN * DEFAULT_DMIN)
                    ok = ok & (torch.exp(logf) / dd > cut * P_all[s:s + cs][:, None])
                n_ok = int(ok.sum())
                out["path_evals"] += rxc.shape[0] * Cn
                out["interactions"] += rxc.shape[0] * Cn * k
                out["active"] += n_ok
                out["active_interactions"] += n_ok * k
                for l in range(k + 1):
                    D = (X[l + 1] - X[l])[:, :, None, :]
                    w0 = a[None, None] - X[l][:, :, None, :]
                    den = _cross(D, e[None, None])
                    excl = torch.zeros(Cn, nW, dtype=torch.bool)
                    if l >= 1:
                        excl |= seq[:, l - 1][:, None] == jidx[None]
                    if l + 1 <= k:
                        excl |= seq[:, l][:, None] == jidx[None]
                    use = (~excl[None]) & ok[:, :, None]
                    den_s = torch.where(den != 0, den, torch.ones_like(den))
                    tau = _cross(w0, D) / den_s
                    ups = _cross(w0, e[None, None]) / den_s
                    live = use & (den != 0) & ((tau - 0.5).abs() < 0.5 + band) & \
                        ((ups - 0.5).abs() < 0.5 + band)
                    out["tests"] += int(use.sum())
                    out["unsaturated"] += int(live.sum())
    return out
