"""FP64 CPU oracle of the smoothed image-method tracer in 3D scenes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the HIP path.

The paper states that its framework makes no assumption on the number of
dimensions and that a 3D implementation is straightforward (Sec. VI).  Here the
walls of the 2D method become planar parallelogram panels
``{a + beta (b - a) + gamma (c - a) : beta, gamma in [0, 1]}`` (corner a,
adjacent corners b and c), and every step keeps its 2D meaning:

* images: mirror across the panel's plane, normal n = (b - a) x (c - a)
  (Sec. V, image method);
* back-trace from X_{k+1} = r towards I_i: the line meets the plane at
  X_i = X_{i+1} + u_i (I_i - X_{i+1}); (beta_i, gamma_i) are X_i's panel
  coordinates; the interaction factor is in(beta) in(gamma) in(u) with
  in(x) = s(x) s(1 - x) (Sec. V-A: inside the panel, and a true
  reflection);
* obstruction of a leg [X_l, X_{l+1}] by panel j (not one of the leg's own
  end panels): the leg meets the plane at leg parameter upsilon, the hit
  point has panel coordinates (beta, gamma); factor
  1 - in(upsilon) in(beta) in(gamma);
* power V / max(|r - I_k|^2, d_min^2), P(r) = sum over candidates (Eq. 7
  with identity coefficient); gradients by torch autograd.

Smoothing modes: "sigmoid" (Eq. 3-4, products formed as exp of summed
logsigmoids and 1 - exp(z) as -expm1(z)), "hard_sigmoid" (Eq. 5-6,
relu6(alpha x + 3) / 6, products as written) and "hard" (the unit step of
Eq. 1).  Degenerate cases as in 2D: a zero-area panel gives 0 and never
blocks; a back-trace parallel to a plane gives 0; a leg parallel to a plane
gives the factor 1.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

from .tracer import candidates  # the candidate enumeration is dimension-free (Sec. V)
from .tracer import hard_sigmoid  # Eq. 5-6

DTYPE = torch.float64
DEFAULT_DMIN = 1e-3


def _as64(x, requires_grad=False):
    t = torch.as_tensor(np.asarray(x, dtype=np.float64) if not torch.is_tensor(x) else x, dtype=DTYPE).clone()
    if requires_grad:
        t.requires_grad_(True)
    return t


def _log_inside(x, alpha):
    return F.logsigmoid(alpha * x) + F.logsigmoid(alpha * (1.0 - x))


def _hard_inside(x):
    return ((x > 0) & (x < 1)).to(DTYPE)


def _hs_inside(x, alpha):
    """hard sigmoid(x) * hard sigmoid(1 - x) (Eq. 5-6): the check 0 < x < 1."""
    return hard_sigmoid(x, alpha) * hard_sigmoid(1.0 - x, alpha)


def _dot(u, v):
    return (u * v).sum(-1)


def _groups(n_panels: int, max_order: int):
    by_k: dict[int, list] = {}
    for seq in candidates(n_panels, max_order):
        by_k.setdefault(len(seq), []).append(seq)
    return {k: torch.tensor(v, dtype=torch.long).reshape(len(v), k) for k, v in by_k.items()}


def _panel_coords(w, e1, e2, n, nn):
    """(beta, gamma) of the in-plane vector w = beta e1 + gamma e2."""
    beta = _dot(torch.linalg.cross(w, e2, dim=-1), n) / nn
    gamma = _dot(torch.linalg.cross(e1, w, dim=-1), n) / nn
    return beta, gamma


def _group_terms(panels, tx, rxc, seq, alpha, mode, d_min, want_paths=False):
    a = panels[:, 0:3]
    e1 = panels[:, 3:6] - a
    e2 = panels[:, 6:9] - a
    n = torch.linalg.cross(e1, e2, dim=-1)
    nn = _dot(n, n)
    ok_panel = nn > 0
    nn_s = torch.where(ok_panel, nn, torch.ones_like(nn))
    C, k = seq.shape
    Rc = rxc.shape[0]
    # images
    I = [tx.expand(C, 3)]
    ok = torch.ones(C, dtype=torch.bool)
    for i in range(k):
        j = seq[:, i]
        ok = ok & ok_panel[j]
        h = _dot(I[-1] - a[j], n[j]) / nn_s[j]
        I.append(I[-1] - 2.0 * h[:, None] * n[j])
    valid = ok[None, :].expand(Rc, C).clone()
    # back-trace
    X: list = [None] * (k + 2)
    X[k + 1] = rxc[:, None, :].expand(Rc, C, 3)
    log_f = torch.zeros(Rc, C, dtype=DTYPE)
    f_hard = torch.ones(Rc, C, dtype=DTYPE)
    params = {}
    for i in range(k, 0, -1):
        j = seq[:, i - 1]
        A, N, E1, E2, NN = a[j][None], n[j][None], e1[j][None], e2[j][None], nn_s[j][None]
        d = I[i][None] - X[i + 1]
        den = _dot(d, N)
        nz = den != 0
        den_s = torch.where(nz, den, torch.ones_like(den))
        u = _dot(A - X[i + 1], N) / den_s
        valid = valid & nz
        X[i] = X[i + 1] + u[..., None] * d
        beta, gamma = _panel_coords(X[i] - A, E1, E2, N, NN)
        if mode == "sigmoid":
            log_f = log_f + _log_inside(beta, alpha) + _log_inside(gamma, alpha) + _log_inside(u, alpha)
        elif mode == "hard_sigmoid":
            f_hard = f_hard * _hs_inside(beta, alpha) * _hs_inside(gamma, alpha) * _hs_inside(u, alpha)
        else:
            f_hard = f_hard * _hard_inside(beta) * _hard_inside(gamma) * _hard_inside(u)
        params[i] = (beta, gamma, u)
    X[0] = tx.expand(Rc, C, 3)
    V = torch.exp(log_f) if mode == "sigmoid" else f_hard
    P = panels.shape[0]
    jidx = torch.arange(P)
    for l in range(k + 1):
        P0, P1 = X[l], X[l + 1]
        D = (P1 - P0)[:, :, None, :]                          # [Rc,C,1,3]
        w0 = a[None, None] - P0[:, :, None, :]                # [Rc,C,P,3]
        den = _dot(D, n[None, None])                          # [Rc,C,P]
        excl = torch.zeros(C, P, dtype=torch.bool)
        if l >= 1:
            excl |= seq[:, l - 1][:, None] == jidx[None]
        if l + 1 <= k:
            excl |= seq[:, l][:, None] == jidx[None]
        use = (den != 0) & ~excl[None] & ok_panel[None, None]
        den_s = torch.where(den != 0, den, torch.ones_like(den))
        ups = _dot(w0, n[None, None]) / den_s                 # along the leg
        H = P0[:, :, None, :] + ups[..., None] * D            # hit point on the plane
        beta, gamma = _panel_coords(H - a[None, None], e1[None, None], e2[None, None], n[None, None],
                                    nn_s[None, None])
        if mode == "sigmoid":
            q = -torch.expm1(_log_inside(ups, alpha) + _log_inside(beta, alpha) + _log_inside(gamma, alpha))
        elif mode == "hard_sigmoid":
            q = 1.0 - _hs_inside(ups, alpha) * _hs_inside(beta, alpha) * _hs_inside(gamma, alpha)
        else:
            q = 1.0 - _hard_inside(ups) * _hard_inside(beta) * _hard_inside(gamma)
        q = torch.where(use, q, torch.ones_like(q))
        V = V * torch.prod(q, dim=-1)
    d2 = ((rxc[:, None, :] - I[k][None]) ** 2).sum(-1)
    c = V / torch.clamp(d2, min=d_min * d_min)
    c = torch.where(valid, c, torch.zeros_like(c))
    if want_paths:
        return c, {"X": X, "I": I, "V": V, "valid": valid, "params": params, "d2": d2}
    return c


def _chunk(n_rx, groups, n_panels, budget=2e6):
    widest = max([g.shape[0] for g in groups.values()] + [1])
    return int(max(1, min(n_rx, budget // max(1, widest * max(1, n_panels)))))


def power(panels, tx, rx, max_order: int, alpha: float, mode: str = "sigmoid", d_min: float = DEFAULT_DMIN):
    """Received power P(r) for every receiver (fp64 numpy [R])."""
    Pn = _as64(panels).reshape(-1, 9)
    T = _as64(tx).reshape(3)
    Rx = _as64(rx).reshape(-1, 3)
    groups = _groups(Pn.shape[0], max_order)
    cs = _chunk(Rx.shape[0], groups, Pn.shape[0])
    out = np.zeros(Rx.shape[0])
    with torch.no_grad():
        for s in range(0, Rx.shape[0], cs):
            rxc = Rx[s:s + cs]
            acc = torch.zeros(rxc.shape[0], dtype=DTYPE)
            for k in sorted(groups):
                acc = acc + _group_terms(Pn, T, rxc, groups[k], alpha, mode, d_min).sum(1)
            out[s:s + cs] = acc.numpy()
    return out


def vjp(panels, tx, rx, max_order: int, alpha: float, g, mode: str = "sigmoid", d_min: float = DEFAULT_DMIN):
    """sum_r g[r] dP(r)/d(panels, tx, rx): (g_panels [P,9], g_tx [3], g_rx [R,3])."""
    Pn = _as64(panels, True)
    T = _as64(tx, True)
    Rx = _as64(rx).reshape(-1, 3)
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    groups = _groups(Pn.shape[0], max_order)
    cs = _chunk(Rx.shape[0], groups, Pn.shape[0], budget=1e6)
    g_rx = np.zeros((Rx.shape[0], 3))
    for s in range(0, Rx.shape[0], cs):
        gc = torch.as_tensor(g[s:s + cs], dtype=DTYPE)
        if not torch.any(gc != 0):
            continue
        rxc = Rx[s:s + cs].clone().requires_grad_(True)
        acc = torch.zeros(rxc.shape[0], dtype=DTYPE)
        for k in sorted(groups):
            acc = acc + _group_terms(Pn.reshape(-1, 9), T.reshape(3), rxc, groups[k], alpha, mode, d_min).sum(1)
        (acc * gc).sum().backward()
        g_rx[s:s + cs] = rxc.grad.numpy()
    gp = Pn.grad.numpy().copy() if Pn.grad is not None else np.zeros(tuple(Pn.shape))
    gt = T.grad.numpy().copy() if T.grad is not None else np.zeros(3)
    return gp.reshape(-1, 9), gt, g_rx


def path_details(panels, tx, r, max_order, alpha, mode="sigmoid", d_min=DEFAULT_DMIN):
    """Per-candidate details at one receiver (for tests): seq, c, V, points, image, valid."""
    Pn = _as64(panels).reshape(-1, 9)
    T = _as64(tx).reshape(3)
    Rr = _as64(r).reshape(1, 3)
    out = []
    with torch.no_grad():
        for k, seq in sorted(_groups(Pn.shape[0], max_order).items()):
            c, info = _group_terms(Pn, T, Rr, seq, alpha, mode, d_min, want_paths=True)
            for ci in range(seq.shape[0]):
                out.append({
                    "seq": tuple(int(v) for v in seq[ci]),
                    "c": float(c[0, ci]),
                    "V": float(info["V"][0, ci]),
                    "valid": bool(info["valid"][0, ci]),
                    "points": [info["X"][i][0, ci].numpy().copy() for i in range(1, k + 1)],
                    "image": info["I"][k][ci].numpy().copy(),
                    "d2": float(info["d2"][0, ci]),
                })
    return out


def work_counts(panels, tx, rx, max_order: int, alpha: float, margin: float = 18.0,
                active_log_floor: float = -88.72, cut: float = 0.0):
    """Algorithmic work of the 3D method at these receivers (instrumentation;
    parity unpinned against the paper, which counts no work).

    The rule of the 2D reference's work_counts: a pair is *active* when it is
    valid, its interaction factor F (the product of in(beta) in(gamma) in(u)
    over its interactions) exceeds exp(active_log_floor) and, with ``cut`` >
    0, F / max(d^2, d_min^2) exceeds cut * P(r); its back-trace, interaction
    factors and obstruction tests are credited only then.  Counts:
    ``path_evals``, ``interactions`` (all pairs), ``active``,
    ``active_interactions``, ``tests`` (obstruction tests of active pairs, a
    leg's own end panels excluded) and ``unsaturated`` tests (leg parameter
    and both panel coordinates within margin/alpha of [0, 1], the plane not
    parallel to the leg).
    """
    Pn = _as64(panels).reshape(-1, 9)
    T = _as64(tx).reshape(3)
    Rx = _as64(rx).reshape(-1, 3)
    a = Pn[:, 0:3]
    e1 = Pn[:, 3:6] - a
    e2 = Pn[:, 6:9] - a
    n = torch.linalg.cross(e1, e2, dim=-1)
    nn = _dot(n, n)
    nn_s = torch.where(nn > 0, nn, torch.ones_like(nn))
    groups = _groups(Pn.shape[0], max_order)
    cs = _chunk(Rx.shape[0], groups, Pn.shape[0], budget=1e6)
    band = margin / alpha
    out = dict(path_evals=0, interactions=0, active=0, active_interactions=0, tests=0, unsaturated=0)
    P = Pn.shape[0]
    jidx = torch.arange(P)
    P_all = torch.as_tensor(power(panels, tx, rx, max_order, alpha), dtype=DTYPE) if cut > 0 else None
    with torch.no_grad():
        for s in range(0, Rx.shape[0], cs):
            rxc = Rx[s:s + cs]
            for k, seq in groups.items():
                _, info = _group_terms(Pn, T, rxc, seq, alpha, "sigmoid", DEFAULT_DMIN, want_paths=True)
                X = info["X"]
                Cn = seq.shape[0]
                logf = torch.zeros(rxc.shape[0], Cn, dtype=DTYPE)
                for i, (beta, gamma, u) in info["params"].items():
                    logf = logf + _log_inside(beta, alpha) + _log_inside(gamma, alpha) + _log_inside(u, alpha)
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
                    P0 = X[l]
                    D = (X[l + 1] - P0)[:, :, None, :]
                    w0 = a[None, None] - P0[:, :, None, :]
                    den = _dot(D, n[None, None])
                    excl = torch.zeros(Cn, P, dtype=torch.bool)
                    if l >= 1:
                        excl |= seq[:, l - 1][:, None] == jidx[None]
                    if l + 1 <= k:
                        excl |= seq[:, l][:, None] == jidx[None]
                    use = (~excl[None]) & ok[:, :, None] & (nn[None, None] > 0)
                    den_s = torch.where(den != 0, den, torch.ones_like(den))
                    ups = _dot(w0, n[None, None]) / den_s
                    H = P0[:, :, None, :] + ups[..., None] * D
                    beta, gamma = _panel_coords(H - a[None, None], e1[None, None], e2[None, None], n[None, None],
                                                nn_s[None, None])
                    live = use & (den != 0) & ((ups - 0.5).abs() < 0.5 + band) & \
                        ((beta - 0.5).abs() < 0.5 + band) & ((gamma - 0.5).abs() < 0.5 + band)
                    out["tests"] += int(use.sum())
                    out["unsaturated"] += int(live.sum())
    return out
