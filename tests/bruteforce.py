"""Brute-force path finder for tiny scenes, independent of the image method.

For a wall sequence (consecutive repeats allowed) the interaction points are
found by Fermat's principle (Sec. V-B names Fermat path tracing as one of the
path finders): minimise the total path length over the wall-LINE parameters
t_i (P_i = a_i + t_i e_i).  The length is a sum of norms of affine maps of t,
hence convex, so damped Newton reaches its unique stationary point.

Hard validity is then decided with orientation predicates, not with the
parametric formulas the oracle uses:
  * each point strictly inside its segment,
  * previous and next points strictly on the same side of the wall line
    (a reflection, not a pass-through),
  * no leg properly crosses another wall (the leg's own end walls excepted).
Receivers where any predicate is within ``amb`` of its decision boundary are
reported as ambiguous so the caller can skip them.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _orient(p, q, r):
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])


def fermat_points(walls, tx, r, seq, iters=100):
    """Minimum-length path over the wall lines: several Newton starts, best kept.

    The length has kinks where a leg shrinks to zero (two adjacent walls
    meeting at a corner); each leg length is smoothed as sqrt(|Q|^2 + 1e-24),
    which moves the minimiser by far less than the 1e-9 checked, and the
    shortest of a few Newton starts is kept.
    """
    best = None
    k = len(seq)
    rng = np.random.default_rng(len(seq) * 7919 + sum(seq))
    starts = [np.full(k, 0.5)] + [rng.uniform(-0.5, 1.5, k) for _ in range(2)]
    for t0 in starts:
        res = _fermat_newton(walls, tx, r, seq, t0, iters)
        if best is None or res[2] < best[2] - 1e-15:
            best = res
    return best


def _fermat_newton(walls, tx, r, seq, t0, iters):
    walls = np.asarray(walls, dtype=np.float64)
    k = len(seq)
    ax = [float(walls[j, 0]) for j in seq]
    ay = [float(walls[j, 1]) for j in seq]
    ex = [float(walls[j, 2] - walls[j, 0]) for j in seq]
    ey = [float(walls[j, 3] - walls[j, 1]) for j in seq]
    tx0, ty0 = float(tx[0]), float(tx[1])
    rx0, ry0 = float(r[0]), float(r[1])
    t = [float(v) for v in t0]
    delta2 = 1e-24    # leg length sqrt(|Q|^2 + delta^2): smooth and strictly convex at |Q| = 0

    def pts(tv):
        return [(tx0, ty0)] + [(ax[i] + tv[i] * ex[i], ay[i] + tv[i] * ey[i]) for i in range(k)] + [(rx0, ry0)]

    def length(tv):
        P = pts(tv)
        return sum(math.sqrt((P[l + 1][0] - P[l][0]) ** 2 + (P[l + 1][1] - P[l][1]) ** 2 + delta2)
                   for l in range(k + 1))

    for _ in range(iters):
        P = pts(t)
        g = np.zeros(k)
        H = np.zeros((k, k))
        for l in range(k + 1):
            qx, qy = P[l + 1][0] - P[l][0], P[l + 1][1] - P[l][1]
            n = math.sqrt(qx * qx + qy * qy + delta2)
            ux, uy = qx / n, qy / n
            # columns of dQ_l/dt: P_{l+1} uses wall index l, P_l uses wall index l-1
            cols = []
            if l + 1 <= k:
                cols.append((l, ex[l], ey[l]))
            if l >= 1:
                cols.append((l - 1, -ex[l - 1], -ey[l - 1]))
            for (i, jx, jy) in cols:
                g[i] += jx * ux + jy * uy
                for (m, kx, ky) in cols:
                    # J_i^T (I - u u^T) J_m / n
                    H[i, m] += (jx * kx + jy * ky - (jx * ux + jy * uy) * (kx * ux + ky * uy)) / n
        if np.linalg.norm(g) < 1e-14:
            break
        step = np.linalg.lstsq(H + 1e-12 * np.trace(H) * np.eye(k), g, rcond=None)[0]
        L0 = length(t)
        lam = 1.0
        while lam > 1e-12 and length([t[i] - lam * step[i] for i in range(k)]) > L0 + 1e-16:
            lam *= 0.5
        t = [t[i] - lam * step[i] for i in range(k)]
    P = pts(t)
    return [np.array(p) for p in P[1:-1]], np.array(t), length(t)


def _seg_cross(p, q, a, b, amb):
    """Strict proper crossing of segments pq and ab; None when ambiguous."""
    d1, d2 = _orient(a, b, p), _orient(a, b, q)
    d3, d4 = _orient(p, q, a), _orient(p, q, b)
    sab = np.linalg.norm(b - a) * max(np.linalg.norm(q - p), 1e-300)
    if min(abs(d1), abs(d2), abs(d3), abs(d4)) < amb * sab:
        # near-touching configuration: undecidable at this tolerance
        if (d1 > 0) != (d2 > 0) and (d3 > 0) != (d4 > 0):
            return None
        if min(abs(d1), abs(d2)) < amb * sab and (d3 > 0) != (d4 > 0):
            return None
        if min(abs(d3), abs(d4)) < amb * sab and (d1 > 0) != (d2 > 0):
            return None
        return False
    return (d1 > 0) != (d2 > 0) and (d3 > 0) != (d4 > 0)


def hard_paths(walls, tx, r, max_order, amb=1e-9):
    """Valid paths at receiver r: dict seq -> (points, length).  None if ambiguous."""
    walls = np.asarray(walls, dtype=np.float64)
    tx = np.asarray(tx, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    W = walls.shape[0]
    out = {}
    for k in range(0, max_order + 1):
        for seq in itertools.product(range(W), repeat=k):
            pts, t, L = fermat_points(walls, tx, r, seq)
            P = [tx] + pts + [r]
            ok = True
            # reflection law first: previous and next points strictly on the same side
            for i in range(k):
                a, b = walls[seq[i], 0:2], walls[seq[i], 2:4]
                s1, s2 = _orient(a, b, P[i]), _orient(a, b, P[i + 2])
                scale = np.linalg.norm(b - a)
                if min(abs(s1), abs(s2)) < 1e-12 * scale:
                    ok = False  # a point on the wall line: not a proper reflection
                elif (s1 > 0) != (s2 > 0):
                    ok = False
            if not ok:
                continue
            for i in range(k):
                if min(abs(t[i]), abs(t[i] - 1.0)) < amb:
                    return None
                if not (0.0 < t[i] < 1.0):
                    ok = False
            if not ok:
                continue
            for l in range(k + 1):
                own = set()
                if l >= 1:
                    own.add(seq[l - 1])
                if l + 1 <= k:
                    own.add(seq[l])
                for j in range(W):
                    if j in own:
                        continue
                    x = _seg_cross(P[l], P[l + 1], walls[j, 0:2], walls[j, 2:4], amb)
                    if x is None:
                        return None
                    if x:
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                out[seq] = (pts, L)
    return out
