"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* values the paper prints (Fig. 2, Fig. 5) -- tests/golden/paper_figures.txt
* the smoothing contract C1-C4 and Eq. 2 (Sec. IV-A)
* closed forms: free-space LOS, LOS inside the box with hand-derived
  crossing parameters, one reflection on a long wall (image distance)
* reciprocity of image distances (mirrors are involutive isometries)
* alpha -> infinity convergence to the hard-indicator result (Eq. 2)
* brute force on tiny scenes with an independent Fermat path finder and
  orientation predicates
* zero-gradient removal inside a hard shadow (Sec. I, Sec. VII)
* translation / rotation / scaling invariants of the gradient
* autograd vs central finite differences
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

import bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()[:2]
                vals[k] = float(v)
    return vals


# ---------------------------------------------------------------- smoothing

def test_smoothing_values_printed_in_fig2():
    g = _golden()
    for alpha in (0.5, 1.0, 10.0, 100.0, 1000.0):
        assert float(T.sigmoid(1.0 / alpha, alpha)) == pytest.approx(g["sigmoid_at_one_over_alpha"], rel=1e-14)
        assert float(T.hard_sigmoid(0.0, alpha)) == pytest.approx(g["hard_sigmoid_at_zero"], abs=0)
        assert float(T.hard_sigmoid(3.0 / alpha, alpha)) == pytest.approx(g["hard_sigmoid_at_three_over_alpha"], rel=1e-15)
        assert float(T.hard_sigmoid(-3.0 / alpha, alpha)) == 0.0


@pytest.mark.parametrize("fn", [T.sigmoid, T.hard_sigmoid])
def test_smoothing_contract_c1_to_c4(fn):
    x = torch.linspace(-5, 5, 2001, dtype=torch.float64)
    for alpha in (0.3, 1.0, 7.0, 100.0):
        s = fn(x, alpha)
        assert torch.all((s >= 0) & (s <= 1))                               # range [0, 1]
        assert float(fn(-1e6, alpha)) == pytest.approx(0.0, abs=1e-12)      # C1
        assert float(fn(1e6, alpha)) == pytest.approx(1.0, abs=1e-12)
        assert torch.all(s[1:] >= s[:-1])                                   # C2
        assert float(fn(0.0, alpha)) == 0.5                                 # C3
        assert torch.allclose(s - 0.5, 0.5 - fn(-x, alpha), atol=1e-15)     # C4
    # Eq. 2: pointwise limit is the unit step of Eq. 1 (x != 0)
    xs = torch.tensor([-0.3, -1e-3, 1e-3, 0.2], dtype=torch.float64)
    assert torch.allclose(fn(xs, 1e7), T.unit_step(xs), atol=1e-12)


def test_alpha_schedule_fig5():
    g = _golden()
    n = int(g["alpha_schedule_n"])
    sched = np.geomspace(g["alpha_schedule_lo"], g["alpha_schedule_hi"], n)
    for i in (20, 40, 60, 80):
        assert round(sched[i], 2) == pytest.approx(g[f"alpha_schedule_i{i}"], abs=1e-9)


# ---------------------------------------------------------------- candidates

def test_candidate_counts():
    assert len(T.candidates(5, 1)) == 6
    assert len(T.candidates(68, 2)) == 4625
    assert T.n_candidates(36, 3) == 45397
    assert WL.n_candidates(36, 3) == 45397 and WL.n_candidates(68, 2) == 4625
    # brute force: filter all W^k sequences
    for W, K in [(3, 3), (4, 2), (1, 3), (0, 2)]:
        n = sum(1 for k in range(K + 1) for s in np.ndindex(*([W] * k)) if all(s[i] != s[i + 1] for i in range(k - 1)))
        assert len(T.candidates(W, K)) == n == WL.n_candidates(W, K)


# ---------------------------------------------------------------- closed forms

def test_free_space_los():
    rx = WL.rx_grid(8)
    tx = np.array([0.3, 0.55], np.float32)
    P = T.power(np.zeros((0, 4), np.float32), tx, rx, 0, 100.0)
    d2 = ((rx.astype(np.float64) - tx.astype(np.float64)) ** 2).sum(1)
    np.testing.assert_allclose(P, 1.0 / np.maximum(d2, 1e-6), rtol=1e-14)
    # the d_min floor
    P = T.power(np.zeros((0, 4), np.float32), rx[5], rx[5:6], 0, 100.0)
    assert P[0] == pytest.approx(1e6)


def _sig(z):
    return 0.5 * (1.0 + math.tanh(0.5 * z))


def _inside(x, alpha):
    return _sig(alpha * x) * _sig(alpha * (1.0 - x))


def test_los_inside_box_closed_form():
    """K=0 with the 4 box walls: each wall's crossing parameters written by hand."""
    alpha = 100.0
    tx = np.array([0.37, 0.61])
    rng = np.random.default_rng(0)
    rx = rng.uniform(0.0, 1.0, (200, 2))
    rx = np.concatenate([rx, [[0.999, 0.5], [0.5, 0.0005], [0.0007, 0.0009]]])
    P = T.power(WL.BOX_WALLS, tx, rx, 0, alpha)
    for m, r in enumerate(rx):
        Dx, Dy = r[0] - tx[0], r[1] - tx[1]
        Vm = 1.0
        # bottom y=0 running x: 0 -> 1 ; top y=1 running x: 1 -> 0
        for yc, x0, x1 in ((0.0, 0.0, 1.0), (1.0, 1.0, 0.0)):
            if Dy != 0:
                ups = (yc - tx[1]) / Dy
                xc = tx[0] + ups * Dx
                tau = (xc - x0) / (x1 - x0)
                Vm *= 1.0 - _inside(tau, alpha) * _inside(ups, alpha)
        # right x=1 running y: 0 -> 1 ; left x=0 running y: 1 -> 0
        for xcst, y0, y1 in ((1.0, 0.0, 1.0), (0.0, 1.0, 0.0)):
            if Dx != 0:
                ups = (xcst - tx[0]) / Dx
                yc = tx[1] + ups * Dy
                tau = (yc - y0) / (y1 - y0)
                Vm *= 1.0 - _inside(tau, alpha) * _inside(ups, alpha)
        ref = Vm / max(Dx * Dx + Dy * Dy, 1e-6)
        assert P[m] == pytest.approx(ref, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("alpha", [10.0, 100.0, 1000.0])
def test_single_reflection_long_wall(alpha):
    """One wall (-1e3,0)->(1e3,0), tx and rx above it: the order-1 path has the
    mirror distance and closed-form t, u (Sec. V-B image method)."""
    wall = np.array([[-1e3, 0.0, 1e3, 0.0]])
    tx = np.array([0.3, 0.2])
    rng = np.random.default_rng(1)
    rx = np.stack([rng.uniform(-0.5, 1.5, 64), rng.uniform(0.05, 1.0, 64)], 1)
    P = T.power(wall, tx, rx, 1, alpha)
    mirror = np.array([tx[0], -tx[1]])
    for m, r in enumerate(rx):
        # LOS leg vs the wall: leg parameter where y = 0, wall parameter of that x
        ups = (0.0 - tx[1]) / (r[1] - tx[1])
        xc = tx[0] + ups * (r[0] - tx[0])
        q = 1.0 - _inside((xc + 1e3) / 2e3, alpha) * _inside(ups, alpha)
        los = q / np.sum((r - tx) ** 2)
        u = r[1] / (r[1] + tx[1])
        X = r[0] + u * (tx[0] - r[0])
        t = (X + 1e3) / 2e3
        refl = _inside(t, alpha) * _inside(u, alpha) / np.sum((r - mirror) ** 2)
        assert P[m] == pytest.approx(los + refl, rel=1e-12)
        # alpha -> infinity: both paths fully valid
    P_hard = T.power(wall, tx, rx, 1, alpha, mode="hard")
    ref = 1.0 / np.sum((rx - tx) ** 2, 1) + 1.0 / np.sum((rx - mirror) ** 2, 1)
    np.testing.assert_allclose(P_hard, ref, rtol=1e-13)


def test_fake_reflection_through_wall_is_rejected():
    """A wall between tx and rx must not give a reflection (side test u in (0,1)).

    tx (0.3,0.5), rx (0.8,0.6), wall x=0.5 for y in [0.2,0.8]: the image method
    gives t = 1/6 (on the segment) but u = 3 (not between rx and the image).
    """
    walls = np.array([[0.5, 0.2, 0.5, 0.8]])
    det = T.path_details(walls, [0.3, 0.5], [0.8, 0.6], 1, 100.0)
    refl = [d for d in det if d["seq"] == (0,)][0]
    assert refl["V"] < 1e-80
    los = [d for d in det if d["seq"] == ()][0]
    assert los["V"] < 1e-10          # LOS crosses the wall well inside both segments


# ---------------------------------------------------------------- reciprocity

def test_image_distance_reciprocity():
    s = WL.scene_random_box(2, 6, 4, 3, 100.0, seed=3)
    W = torch.tensor(s.walls, dtype=torch.float64)
    tx = torch.tensor(s.tx, dtype=torch.float64)
    rng = np.random.default_rng(2)
    for _ in range(5):
        r = torch.tensor(rng.uniform(0, 1, 2))
        for seq in T.candidates(W.shape[0], 3):
            if not seq:
                continue
            S = torch.tensor([seq], dtype=torch.long)
            Rv = torch.tensor([seq[::-1]], dtype=torch.long)
            I, _ = T.images(W, tx, S)
            J, _ = T.images(W, r, Rv)
            d1 = torch.linalg.norm(r - I[-1][0])
            d2 = torch.linalg.norm(tx - J[-1][0])
            assert float(abs(d1 - d2)) <= 1e-13 * float(d1)


# ---------------------------------------------------------------- brute force

def test_bruteforce_fermat_matches_hard_oracle():
    """Tiny scenes: valid path sets, points and hard power agree with Fermat brute force."""
    checked = 0
    for seed, n_int, K in [(0, 1, 2), (1, 2, 2), (2, 3, 1), (3, 2, 2)]:
        s = WL.scene_random_box(2, n_int, 6, K, 100.0, seed=seed)
        for m in range(0, s.n_rx, 3):
            r = s.rx[m].astype(np.float64)
            bf = BF.hard_paths(s.walls, s.tx, r, K)
            if bf is None:
                continue
            det = T.path_details(s.walls, s.tx, r, K, 100.0, mode="hard")
            orc_valid = {d["seq"]: d for d in det if d["valid"] and d["V"] == 1.0}
            # sequences with a wall repeated back to back are never valid
            assert all(all(q[i] != q[i + 1] for i in range(len(q) - 1)) for q in bf)
            assert set(bf) == set(orc_valid), (seed, m)
            for seq, (pts, L) in bf.items():
                d = orc_valid[seq]
                for p_bf, p_or in zip(pts, d["points"]):
                    np.testing.assert_allclose(p_bf, p_or, atol=1e-9)
                assert math.sqrt(d["d2"]) == pytest.approx(L, rel=1e-10)   # image distance = path length
            P_bf = sum(1.0 / max(L * L, 1e-6) for _, L in bf.values())
            P_or = T.power(s.walls, s.tx, r[None], K, 100.0, mode="hard")[0]
            assert P_or == pytest.approx(P_bf, rel=1e-10)
            checked += 1
    assert checked > 20


# ---------------------------------------------------------------- alpha -> inf

def test_alpha_limit_converges_to_hard():
    s = WL.scene_random_box(2, 4, 12, 2, 100.0, seed=5)
    P_hard = T.power(s.walls, s.tx, s.rx, 2, 1.0, mode="hard")
    errs = []
    for alpha in (1e2, 1e3, 1e4, 1e6):
        P = T.power(s.walls, s.tx, s.rx, 2, alpha)
        errs.append(np.abs(P - P_hard) / np.maximum(P_hard, 1e-300))
    # error shrinks with alpha and is negligible for almost every receiver at 1e6
    assert np.median(errs[1]) < np.median(errs[0])
    assert np.median(errs[3]) < 1e-12
    assert np.mean(errs[3] < 1e-9) > 0.95


# ---------------------------------------------------------------- gradients

def test_zero_gradient_removed_in_shadow():
    """LOS only, box + one segment: in the hard shadow dP/dtx is 0; smoothed it is not,
    and moving tx along it raises the received power."""
    walls = np.concatenate([WL.BOX_WALLS, [[0.4, 0.3, 0.6, 0.7]]]).astype(np.float32)
    tx = np.array([0.2, 0.5])
    rx = np.array([[0.8, 0.5], [0.75, 0.45]])
    P_hard = T.power(walls, tx, rx, 0, 1.0, mode="hard")
    assert np.all(P_hard == 0.0)
    _, gt_h, _ = T.vjp(walls, tx, rx, 0, 1.0, np.ones(2), mode="hard")
    assert np.all(gt_h == 0.0)
    _, gt, _ = T.vjp(walls, tx, rx, 0, 10.0, np.ones(2))
    assert np.linalg.norm(gt) > 0
    step = 1e-3 * gt / np.linalg.norm(gt)
    assert T.power(walls, tx + step, rx, 0, 10.0).sum() > T.power(walls, tx, rx, 0, 10.0).sum()


def _all_points_and_grads(s, K, alpha, g):
    gw, gt, grx = T.vjp(s.walls, s.tx, s.rx, K, alpha, g)
    pts = np.concatenate([s.walls.reshape(-1, 2), s.tx.reshape(1, 2), s.rx]).astype(np.float64)
    grads = np.concatenate([gw.reshape(-1, 2), gt.reshape(1, 2), grx])
    return pts, grads


def test_gradient_invariants():
    s = WL.scene_random_box(2, 5, 5, 2, 30.0, seed=7)
    P = T.power(s.walls, s.tx, s.rx, 2, 30.0)
    g = np.random.default_rng(0).uniform(0.5, 1.5, s.n_rx)
    pts, gr = _all_points_and_grads(s, 2, 30.0, g)
    scale = np.abs(gr).sum()
    np.testing.assert_allclose(gr.sum(0), 0.0, atol=1e-11 * scale)                       # translation
    rot = (pts[:, 0] * gr[:, 1] - pts[:, 1] * gr[:, 0]).sum()
    assert abs(rot) < 1e-11 * scale                                                       # rotation
    assert (pts * gr).sum() == pytest.approx(-2.0 * (g * P).sum(), rel=1e-10)            # scaling


@pytest.mark.parametrize("alpha", [10.0, 100.0])
def test_autograd_matches_central_differences(alpha):
    s = WL.scene_random_box(2, 3, 4, 2, alpha, seed=11)
    rx = s.rx.astype(np.float64)
    g = np.linspace(0.5, 1.5, len(rx))
    gw, gt, _ = T.vjp(s.walls, s.tx, rx, 2, alpha, g)

    def f(walls, tx):
        return float(np.dot(g, T.power(walls, tx, rx, 2, alpha)))

    def cd(fun, x0, h):
        return (fun(x0 + h) - fun(x0 - h)) / (2 * h)

    def rich(fun, x0, h):   # Richardson extrapolation of central differences
        return (4 * cd(fun, x0, h / 2) - cd(fun, x0, h)) / 3

    walls = s.walls.astype(np.float64)
    tx = s.tx.astype(np.float64)
    for i in range(2):
        def ft(x, i=i):
            t2 = tx.copy(); t2[i] = x
            return f(walls, t2)
        assert gt[i] == pytest.approx(rich(ft, tx[i], 1e-3 / alpha), rel=1e-6, abs=1e-9 * np.abs(gt).max())
    rng = np.random.default_rng(3)
    for _ in range(6):
        j, c = int(rng.integers(0, walls.shape[0])), int(rng.integers(0, 4))

        def fw(x, j=j, c=c):
            w2 = walls.copy(); w2[j, c] = x
            return f(w2, tx)
        assert gw[j, c] == pytest.approx(rich(fw, walls[j, c], 1e-3 / alpha), rel=1e-5, abs=1e-7 * np.abs(gw).max())


def test_loss_seed_matches_finite_difference():
    P = np.array([1e-3, 2.0, 0.5, 1e-8])
    for kind in ("sum", "neg_mean_log"):
        g = T.loss_seed(P, kind)
        for i in range(len(P)):
            h = 1e-3 if kind == "sum" else 1e-5 * (P[i] + 1e-6)
            Pp, Pm = P.copy(), P.copy()
            Pp[i] += h; Pm[i] -= h
            fd = (T.loss_value(Pp, kind) - T.loss_value(Pm, kind)) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-6)


def test_degenerate_inputs():
    # zero-length wall: its candidates contribute nothing, it never blocks
    walls = np.array([[0.5, 0.5, 0.5, 0.5], [0.0, 0.0, 1.0, 0.0]])
    rx = np.array([[0.2, 0.3], [0.9, 0.1]])
    tx = np.array([0.6, 0.4])
    P = T.power(walls, tx, rx, 2, 100.0)
    P_ref = T.power(walls[1:], tx, rx, 2, 100.0)
    np.testing.assert_allclose(P, P_ref, rtol=1e-14)
    # no receivers
    assert T.power(walls, tx, np.zeros((0, 2)), 2, 100.0).shape == (0,)
