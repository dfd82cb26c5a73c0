"""Pins of the FP64 reference of the 3D (parallelogram-panel) tracer.

* A 2D scene extruded into vertical panels, with the transmitter and the
  receivers at half height, keeps every path in that plane with the vertical
  panel coordinate 1/2, where in(1/2) = s(alpha/2)^2 = 1 to 1e-21 at
  alpha = 100: the 3D power and gradients equal the (separately pinned) 2D
  reference's.
* Reflection off a large floor: the image-distance closed form.
* Valid paths obey the law of reflection at every point, and their length
  equals the image distance.
* alpha -> infinity tends to the unit-step model; autograd vs central
  differences; degenerate panels.
"""
import numpy as np
import pytest

from oracle import tracer as T2
from oracle import tracer3d as T3
from paper_2401_11882_amd import workloads as WL


@pytest.mark.parametrize("K", [0, 1, 2])
def test_extruded_2d_scene_matches_2d(K):
    s = WL.scene_random_box(2, 5, 6, K, 100.0, seed=40 + K)
    e = WL.extrude(s)
    P2 = T2.power(s.walls, s.tx, s.rx, K, 100.0)
    P3 = T3.power(e.panels, e.tx, e.rx, K, 100.0)
    np.testing.assert_allclose(P3, P2, rtol=1e-10, atol=1e-300)
    P2h = T2.power(s.walls, s.tx, s.rx, K, 1.0, mode="hard")
    P3h = T3.power(e.panels, e.tx, e.rx, K, 1.0, mode="hard")
    np.testing.assert_allclose(P3h, P2h, rtol=1e-12)


def test_extruded_gradients_match_2d():
    s = WL.scene_random_box(2, 4, 4, 2, 100.0, seed=7)
    e = WL.extrude(s)
    g = np.ones(s.n_rx)
    gw2, gt2, grx2 = T2.vjp(s.walls, s.tx, s.rx, 2, 100.0, g)
    gp3, gt3, grx3 = T3.vjp(e.panels, e.tx, e.rx, 2, 100.0, g)
    np.testing.assert_allclose(gt3[:2], gt2, rtol=1e-8, atol=1e-10 * np.abs(gt2).max())
    np.testing.assert_allclose(grx3[:, :2], grx2, rtol=1e-8, atol=1e-10 * np.abs(grx2).max())
    # panel corners a = (ax, ay, 0), b = (bx, by, 0), c = (ax, ay, H): chain to the 2D endpoints
    ga = gp3[:, 0:2] + gp3[:, 6:8]
    gb = gp3[:, 3:5]
    np.testing.assert_allclose(np.concatenate([ga, gb], 1), gw2, rtol=1e-7, atol=1e-9 * np.abs(gw2).max())


def test_floor_reflection_closed_form():
    floor = np.array([[-10, -10, 0, 10, -10, 0, -10, 10, 0]], np.float64)
    tx = np.array([0.2, 0.3, 0.5])
    rx = np.array([[0.7, 0.6, 0.25], [0.1, 0.9, 1.5]])
    P = T3.power(floor, tx, rx, 1, 100.0)
    img = np.array([0.2, 0.3, -0.5])
    ref = 1.0 / ((rx - tx) ** 2).sum(1) + 1.0 / ((rx - img) ** 2).sum(1)
    # the smoothed factors differ from 1 by at most e^-25 (u = 3/4 for the second receiver)
    np.testing.assert_allclose(P, ref, rtol=1e-10)


def test_law_of_reflection_and_path_length():
    s = WL.scene3d_room(8, 4, 4, 2, 100.0, seed=3)
    checked = 0
    for m in range(0, s.n_rx, 2):
        r = s.rx[m].astype(np.float64)
        for d in T3.path_details(s.panels, s.tx, r, 2, 1.0, mode="hard"):
            if not d["valid"] or d["V"] != 1.0 or not d["seq"]:
                continue
            pts = [s.tx.astype(np.float64)] + d["points"] + [r]
            for i, j in enumerate(d["seq"]):
                a, b, c = (s.panels[j].astype(np.float64).reshape(3, 3))
                n = np.cross(b - a, c - a)
                n /= np.linalg.norm(n)
                din = pts[i + 1] - pts[i]
                dout = pts[i + 2] - pts[i + 1]
                din /= np.linalg.norm(din)
                dout /= np.linalg.norm(dout)
                np.testing.assert_allclose(dout, din - 2.0 * np.dot(din, n) * n, atol=1e-9)
                assert abs(np.dot(pts[i + 1] - a, n)) < 1e-12
            L = sum(np.linalg.norm(pts[i + 1] - pts[i]) for i in range(len(pts) - 1))
            assert L == pytest.approx(np.sqrt(d["d2"]), rel=1e-11)
            checked += 1
    assert checked >= 10


def test_large_alpha_tends_to_unit_step():
    s = WL.scene3d_room(8, 3, 6, 2, 100.0, seed=5)
    Ph = T3.power(s.panels, s.tx, s.rx, 2, 1.0, mode="hard")
    P = T3.power(s.panels, s.tx, s.rx, 2, 1e7)
    rel = np.abs(P - Ph) / np.maximum(Ph, 1e-300)
    assert np.mean(rel < 1e-9) > 0.95


@pytest.mark.parametrize("alpha", [10.0, 100.0])
def test_autograd_matches_central_differences(alpha):
    s = WL.scene3d_room(8, 3, 2, 1, alpha, seed=11)
    g = np.ones(s.n_rx)
    gp, gt, _ = T3.vjp(s.panels, s.tx, s.rx, 1, alpha, g)

    def f(pan, tx):
        return T3.power(pan, tx, s.rx, 1, alpha).sum()

    h = 1e-6   # smoothing lengths are panel size / alpha >= 2e-3: truncation ~ (h / 2e-3)^2
    tx = s.tx.astype(np.float64)
    for c in range(3):
        tp, tm = tx.copy(), tx.copy()
        tp[c] += h
        tm[c] -= h
        fd = (f(s.panels, tp) - f(s.panels, tm)) / (2 * h)
        assert gt[c] == pytest.approx(fd, rel=2e-5, abs=1e-7 * np.abs(gt).max())
    pan = s.panels.astype(np.float64)
    for j, c in [(6, 0), (7, 4), (8, 8), (2, 1), (0, 2)]:
        pp, pm = pan.copy(), pan.copy()
        pp[j, c] += h
        pm[j, c] -= h
        fd = (f(pp, tx) - f(pm, tx)) / (2 * h)
        assert gp[j, c] == pytest.approx(fd, rel=2e-5, abs=1e-7 * np.abs(gp).max())


def test_degenerate_panels():
    # a zero-area panel between tx and rx neither reflects nor blocks
    flat = np.array([[0.5, 0.4, 0.3, 0.5, 0.6, 0.3, 0.5, 0.5, 0.3]], np.float64)   # b - a parallel to c - a
    tx = np.array([0.2, 0.5, 0.3])
    rx = np.array([[0.8, 0.5, 0.3]])
    P = T3.power(flat, tx, rx, 1, 100.0)
    assert P[0] == pytest.approx(1.0 / 0.36, rel=1e-12)


# --- hard-sigmoid smoothing (Eq. 5-6) in 3D ---------------------------------

HS = "hard_sigmoid"


@pytest.mark.parametrize("K", [0, 1, 2])
def test_hard_sigmoid_extruded_matches_2d(K):
    """At half height the vertical panel coordinate is 1/2, where
    hs(alpha / 2)^2 = 1 exactly for alpha >= 6: the 2D hard-sigmoid reference."""
    s = WL.scene_random_box(2, 5, 6, K, 30.0, seed=60 + K)
    e = WL.extrude(s)
    P2 = T2.power(s.walls, s.tx, s.rx, K, 30.0, mode=HS)
    P3 = T3.power(e.panels, e.tx, e.rx, K, 30.0, mode=HS)
    np.testing.assert_allclose(P3, P2, rtol=1e-12, atol=1e-300)


def test_hard_sigmoid_blocked_and_partial_closed_forms():
    alpha = 50.0
    tx = np.array([0.2, 0.5, 0.5])
    rx = np.array([[0.8, 0.5, 0.5]])
    d2 = 0.36
    # a square panel x = 0.5 centred on the line of sight: in(.) = 1 for every coordinate, factor exactly 0
    centred = np.array([[0.5, 0.25, 0.25, 0.5, 0.75, 0.25, 0.5, 0.25, 0.75]])
    assert T3.power(centred, tx, rx, 0, alpha, mode=HS)[0] == 0.0
    # the same panel shifted so that the crossing has beta = -1/alpha: in(beta) = hs(-1) = 1/3, factor 2/3
    shifted = centred.copy()
    shifted[0, 1::3] += 0.25 + 0.5 / alpha   # y of a, b, c: beta = (0.5 - y_a) / 0.5 = -1/alpha
    P = T3.power(shifted, tx, rx, 0, alpha, mode=HS)[0]
    assert P == pytest.approx((2.0 / 3.0) / d2, rel=1e-12)


def test_hard_sigmoid_large_alpha_tends_to_unit_step():
    s = WL.scene3d_room(8, 3, 6, 2, 100.0, seed=5)
    Ph = T3.power(s.panels, s.tx, s.rx, 2, 1.0, mode="hard")
    P = T3.power(s.panels, s.tx, s.rx, 2, 1e9, mode=HS)
    rel = np.abs(P - Ph) / np.maximum(Ph, 1e-300)
    assert np.mean(rel < 1e-9) > 0.95


@pytest.mark.parametrize("alpha", [20.0, 50.0])
def test_hard_sigmoid_autograd_matches_central_differences(alpha):
    s = WL.scene3d_room(8, 3, 2, 1, alpha, seed=12)
    g = np.ones(s.n_rx)
    gp, gt, _ = T3.vjp(s.panels, s.tx, s.rx, 1, alpha, g, mode=HS)

    def f(pan, tx):
        return T3.power(pan, tx, s.rx, 1, alpha, mode=HS).sum()

    h = 1e-7   # piecewise linear factors: exact away from the kinks
    tx = s.tx.astype(np.float64)
    for c in range(3):
        tp, tm = tx.copy(), tx.copy()
        tp[c] += h
        tm[c] -= h
        fd = (f(s.panels, tp) - f(s.panels, tm)) / (2 * h)
        assert gt[c] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(gt).max())
    pan = s.panels.astype(np.float64)
    for j, c in [(6, 0), (7, 4), (8, 8), (2, 1), (0, 2)]:
        pp, pm = pan.copy(), pan.copy()
        pp[j, c] += h
        pm[j, c] -= h
        fd = (f(pp, tx) - f(pm, tx)) / (2 * h)
        assert gp[j, c] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(gp).max())
