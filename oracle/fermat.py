"""FP64 CPU oracle of Fermat path tracing (FPT) with a smoothed convergence check.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the HIP path.

What it computes (arXiv 2401.11882, Sec. V and Sec. V-B).  The image method of
``oracle.tracer`` is one way to place a path's interaction points in the
relaxed scene of infinite wall lines; Sec. V-B names a second, Fermat path
tracing: the points are where the total path length is smallest (Fermat's
principle), found iteratively.  Such a path finder has one discontinuity of its
own, the check that it converged to a valid path, which compares the MPT loss
(zero exactly on a valid path) with zero; smoothed like every other comparison.

For a candidate sigma = (sigma_1..sigma_k) (k <= 2 here):

* X_i = a_i + t_i e_i on the line of wall sigma_i, X_0 = tx, X_{k+1} = r;
  t minimises the length l(t) = sum_l |X_{l+1} - X_l|, a convex function
  (a sum of norms of affine maps of t); damped Newton from t = 1/2, first on
  leg lengths smoothed at their kinks and then on l itself (continuation,
  see DELTA2_STAGES), until the minimum is reached to FP64 precision;
* MPT loss (reading; the paper defers its definition to the MPT paper): the
  squared residual of the law of reflection summed over the interactions,
  L = sum_i |d_out - (d_in - 2 (d_in . n) n)|^2 with d_in, d_out the unit
  directions of the legs into and out of X_i and n the unit normal of the
  wall.  At Fermat's minimum the tangential part vanishes, so L = 0 for a true
  reflection and L = 4 (d . n)^2 for a straight pass through the wall line;
* convergence check "L < eps" smoothed as s((eps - L) / eps) = s(1 - L/eps)
  (dimensionless argument, sharpness alpha as everywhere else; eps = 1e-4:
  the check fails for passes through a wall line steeper than about 0.3
  degrees);
* validity V = prod_i in(t_i) * s(1 - L/eps) * prod over legs and walls not at
  the leg's ends of (1 - in(tau) in(upsilon)), in(x) = s(x) s(1 - x), as in
  the image-method oracle (Sec. V-A), with the legs between the Fermat points;
* contribution V / max(l^2, d_min^2), l the path length; P(r) = sum over
  candidates.

Modes "sigmoid" (Eq. 3-4), "hard_sigmoid" (Eq. 5-6) and "hard" (the unit step
of Eq. 1).  Degenerate cases: a zero-length wall gives no path; a leg of zero
length (a point on the next wall line) gives no path.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

from oracle.tracer import DEFAULT_DMIN, DTYPE, _as64, _cross, _groups

DEFAULT_EPS = 1e-4


def _log_s(z):
    return F.logsigmoid(z)


def _smooth(x, alpha, mode):
    """s(x; alpha) of one comparison x > 0, by mode (as a value, not a log)."""
    if mode == "sigmoid":
        return torch.sigmoid(alpha * x)
    if mode == "hard_sigmoid":
        return torch.clamp(alpha * x + 3.0, 0.0, 6.0) / 6.0
    return (x > 0).to(DTYPE)


def _inside(x, alpha, mode):
    return _smooth(x, alpha, mode) * _smooth(1.0 - x, alpha, mode)


def _legs(A, E, t, tx, rxc):
    """Points X_0..X_{k+1} [Rc, C, k+2, 2] for line parameters t [Rc, C, k]."""
    Rc, C, k = t.shape
    X = A[None] + t[..., None] * E[None]                       # [Rc, C, k, 2]
    X0 = tx.expand(Rc, C, 1, 2)
    Xr = rxc[:, None, None, :].expand(Rc, C, 1, 2)
    return torch.cat([X0, X, Xr], dim=2)


def _length(A, E, t, tx, rxc, delta2=0.0):
    X = _legs(A, E, t, tx, rxc)
    Q = X[:, :, 1:] - X[:, :, :-1]
    return torch.sqrt((Q * Q).sum(-1) + delta2).sum(-1)


# Smoothing of the leg lengths while the minimum is approached: the length
# has a kink where a leg shrinks to zero (a path through the corner of two
# adjacent walls), where Newton's steps stall.  Each leg length |Q| is first
# replaced by sqrt(|Q|^2 + delta^2), smooth and strictly convex, and delta
# is lowered stage by stage to 0, each stage starting from the previous
# minimiser (continuation); the last stage minimises the length itself.
DELTA2_STAGES = (1e-2, 1e-4, 1e-6, 1e-8, 0.0)


def fermat_params(walls, tx, rxc, seq, iters: int = 50, tol: float = 1e-9):
    """Line parameters t [Rc, C, k] minimising the path length: damped Newton
    from t = 1/2 with a halving line search, through the stages of
    DELTA2_STAGES, each until no parameter moves (the minimum reached to FP64
    rounding) or ``iters`` steps; also a flag [Rc, C] that the gradient of the
    length is below tol relative to the wall lengths at the end."""
    a = walls[:, 0:2]
    e = walls[:, 2:4] - walls[:, 0:2]
    C, k = seq.shape
    Rc = rxc.shape[0]
    A, E = a[seq], e[seq]                                        # [C, k, 2]
    t = torch.full((Rc, C, k), 0.5, dtype=DTYPE)
    scale = torch.sqrt((E * E).sum(-1)).clamp(min=1e-300)[None]  # [1, C, k]
    eye = torch.eye(k, dtype=DTYPE)
    # a zero-length wall has no line: its candidates keep t = 1/2 (they give no path)
    degenerate = ((E * E).sum(-1) == 0).any(-1)[None, :, None, None]        # [1, C, 1, 1]
    for d2 in DELTA2_STAGES:
        for _ in range(iters):
            X = _legs(A, E, t, tx, rxc)
            Q = X[:, :, 1:] - X[:, :, :-1]                       # legs [Rc, C, k+1, 2]
            n = torch.sqrt((Q * Q).sum(-1) + d2).clamp(min=1e-300)
            v = Q / n[..., None]
            # dl/dt_i = e_i . (v_{i-1} - v_i): leg i-1 ends at X_i, leg i starts there
            g = (E[None] * (v[:, :, :-1] - v[:, :, 1:])).sum(-1)  # [Rc, C, k]
            if bool((g == 0).all()):
                break
            # Hessian: sum over legs of J^T (I - v v^T) J / n, J = dQ/dt
            ee = (E * E).sum(-1)[None]                            # |e_i|^2
            ve_in = (v[:, :, :-1] * E[None]).sum(-1)              # v_{i-1} . e_i
            ve_out = (v[:, :, 1:] * E[None]).sum(-1)              # v_i . e_i
            H = torch.diag_embed((ee - ve_in ** 2) / n[:, :, :-1] + (ee - ve_out ** 2) / n[:, :, 1:])
            for i in range(k - 1):
                # leg i+1 runs from X_{i+1} (moving with -e_{i+1}) to X_{i+2} (with +e_{i+2})
                vl = v[:, :, i + 1]
                e1, e2 = E[None, :, i], E[None, :, i + 1]
                h = (-(e1 * e2).sum(-1) + (vl * e1).sum(-1) * (vl * e2).sum(-1)) / n[:, :, i + 1]
                H[:, :, i, i + 1] = h
                H[:, :, i + 1, i] = h
            H = H + 1e-14 * H.diagonal(dim1=-2, dim2=-1).sum(-1)[..., None, None] * eye
            H = torch.where(degenerate, eye, H)
            g = torch.where(degenerate[..., 0], torch.zeros_like(g), g)
            step = torch.linalg.solve(H, g[..., None])[..., 0]
            L0 = n.sum(-1) if d2 > 0 else torch.sqrt((Q * Q).sum(-1)).sum(-1)
            lam = torch.ones(Rc, C, dtype=DTYPE)
            acc = torch.zeros(Rc, C, dtype=torch.bool)
            t_prev = t
            for _ in range(60):
                cand = t - lam[..., None] * step
                # near the minimum the length changes below its rounding: accept
                # a step that does not raise it beyond that, so Newton's last
                # steps still land on the minimiser to full precision
                ok = _length(A, E, cand, tx, rxc, d2) <= L0 * (1.0 + 4e-16)
                newly = ok & ~acc
                t = torch.where(newly[..., None], cand, t)
                acc = acc | ok
                if bool(acc.all()):
                    break
                lam = torch.where(acc, lam, 0.5 * lam)
            if bool(((t - t_prev).abs() <= 1e-15 * (1.0 + t.abs())).all()):
                break
    X = _legs(A, E, t, tx, rxc)
    Q = X[:, :, 1:] - X[:, :, :-1]
    u = Q / torch.sqrt((Q * Q).sum(-1)).clamp(min=1e-300)[..., None]
    g = (E[None] * (u[:, :, :-1] - u[:, :, 1:])).sum(-1)
    done = (g.abs() <= tol * scale).all(-1)
    return t, done


def _group_terms(walls, tx, rxc, seq, alpha, mode, d_min, eps, want=False, tc=None):
    """Contributions [Rc, C] of one order group (and details if want); tc =
    (t, converged) precomputed by fermat_params for these receivers, or None."""
    a = walls[:, 0:2]
    e = walls[:, 2:4] - walls[:, 0:2]
    C, k = seq.shape
    Rc = rxc.shape[0]
    ee = (e * e).sum(-1)
    valid = (ee[seq] > 0).all(-1)[None].expand(Rc, C) if k > 0 else torch.ones(Rc, C, dtype=torch.bool)
    if k > 0:
        t, conv = fermat_params(walls, tx, rxc, seq) if tc is None else tc
        X = _legs(a[seq], e[seq], t, tx, rxc)
    else:
        t, conv = torch.zeros(Rc, C, 0, dtype=DTYPE), torch.ones(Rc, C, dtype=torch.bool)
        X = torch.cat([tx.expand(Rc, C, 1, 2), rxc[:, None, None, :].expand(Rc, C, 1, 2)], dim=2)
    Q = X[:, :, 1:] - X[:, :, :-1]
    n = torch.sqrt((Q * Q).sum(-1))
    valid = valid & (n > 0).all(-1)
    u = Q / n.clamp(min=1e-300)[..., None]
    V = torch.ones(Rc, C, dtype=DTYPE)
    L_mpt = torch.zeros(Rc, C, dtype=DTYPE)
    for i in range(k):
        En = e[seq[:, i]]
        nrm = torch.stack([-En[:, 1], En[:, 0]], -1) / torch.sqrt(ee[seq[:, i]]).clamp(min=1e-300)[:, None]
        d_in, d_out = u[:, :, i], u[:, :, i + 1]
        dn = (d_in * nrm[None]).sum(-1)
        rho = d_out - d_in + 2.0 * dn[..., None] * nrm[None]
        L_mpt = L_mpt + (rho * rho).sum(-1)
        V = V * _inside(t[:, :, i], alpha, mode)
    if k > 0:
        V = V * _smooth(1.0 - L_mpt / eps, alpha, mode)
    Wn = walls.shape[0]
    jidx = torch.arange(Wn)
    for l in range(k + 1):
        P0 = X[:, :, l]
        D = Q[:, :, l][:, :, None, :]
        w0 = a[None, None] - P0[:, :, None, :]
        den = _cross(D, e[None, None])
        excl = torch.zeros(C, Wn, dtype=torch.bool)
        if l >= 1:
            excl |= seq[:, l - 1][:, None] == jidx[None]
        if l + 1 <= k:
            excl |= seq[:, l][:, None] == jidx[None]
        use = (den != 0) & ~excl[None]
        den_s = torch.where(den != 0, den, torch.ones_like(den))
        tau = _cross(w0, D) / den_s
        ups = _cross(w0, e[None, None]) / den_s
        if mode == "sigmoid":
            q = -torch.expm1(F.logsigmoid(alpha * tau) + F.logsigmoid(alpha * (1 - tau)) +
                             F.logsigmoid(alpha * ups) + F.logsigmoid(alpha * (1 - ups)))
        else:
            q = 1.0 - _inside(tau, alpha, mode) * _inside(ups, alpha, mode)
        q = torch.where(use, q, torch.ones_like(q))
        V = V * torch.prod(q, dim=-1)
    length = n.sum(-1)
    c = V / torch.clamp(length * length, min=d_min * d_min)
    c = torch.where(valid, c, torch.zeros_like(c))
    if want:
        return c, {"t": t, "X": X, "L_mpt": L_mpt, "length": length, "valid": valid, "converged": conv, "V": V}
    return c


def power(walls, tx, rx, max_order: int, alpha: float, mode: str = "sigmoid", d_min: float = DEFAULT_DMIN,
          eps: float = DEFAULT_EPS) -> np.ndarray:
    """Received power P(r) with Fermat path tracing (fp64 numpy [R])."""
    if max_order > 2:
        raise ValueError("the Fermat oracle covers orders <= 2")
    W = _as64(walls).reshape(-1, 4)
    T = _as64(tx).reshape(2)
    Rx = _as64(rx).reshape(-1, 2)
    groups = _groups(W.shape[0], max_order)
    widest = max(g.shape[0] for g in groups.values())
    # the Newton iterations run over large blocks of receivers, the obstruction
    # tests ([receivers, candidates, walls] tensors) over smaller ones
    big = int(max(1, min(Rx.shape[0], 3e5 // max(1, widest))))
    cs = int(max(1, min(big, 4e5 // max(1, widest * max(1, W.shape[0])))))
    out = np.zeros(Rx.shape[0])
    with torch.no_grad():
        for b in range(0, Rx.shape[0], big):
            rxb = Rx[b:b + big]
            pre = {k: fermat_params(W, T, rxb, groups[k]) for k in groups if k > 0}
            for s in range(0, rxb.shape[0], cs):
                rxc = rxb[s:s + cs]
                acc = torch.zeros(rxc.shape[0], dtype=DTYPE)
                for k in sorted(groups):
                    tc = None if k == 0 else (pre[k][0][s:s + cs], pre[k][1][s:s + cs])
                    acc = acc + _group_terms(W, T, rxc, groups[k], alpha, mode, d_min, eps, tc=tc).sum(1)
                out[b + s:b + s + cs] = acc.numpy()
    return out


def path_details(walls, tx, r, max_order, alpha, mode="sigmoid", d_min=DEFAULT_DMIN, eps=DEFAULT_EPS):
    """Per-candidate details at one receiver: seq, c, points, t, L_mpt, length, converged."""
    W = _as64(walls).reshape(-1, 4)
    T = _as64(tx).reshape(2)
    Rr = _as64(r).reshape(1, 2)
    out = []
    with torch.no_grad():
        for k, seq in sorted(_groups(W.shape[0], max_order).items()):
            c, info = _group_terms(W, T, Rr, seq, alpha, mode, d_min, eps, want=True)
            for ci in range(seq.shape[0]):
                out.append({
                    "seq": tuple(int(v) for v in seq[ci]),
                    "c": float(c[0, ci]),
                    "t": info["t"][0, ci].numpy().copy(),
                    "points": [info["X"][0, ci, i].numpy().copy() for i in range(1, k + 1)],
                    "L_mpt": float(info["L_mpt"][0, ci]),
                    "length": float(info["length"][0, ci]),
                    "valid": bool(info["valid"][0, ci]),
                    "converged": bool(info["converged"][0, ci]),
                })
    return out
