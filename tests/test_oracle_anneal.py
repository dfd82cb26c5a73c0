"""Pins of the FP64 reference of the transmitter-placement application (Sec. VII).

* the alpha schedule against the values printed in the Fig. 5 caption
  (tests/golden/paper_figures.txt);
* the min-objective seed (Eq. 8) against finite differences of the loss;
* line-of-sight reciprocity P(a -> b) = P(b -> a) (the leg parameter enters
  only through in(x) = s(ax) s(a(1-x)), symmetric under x -> 1 - x);
* the first Adam step in closed form (each coordinate moves by lr sign(g));
* the paper's qualitative claim: from a start inside the zero-gradient region
  the unsmoothed objective gives no step at all, while the annealed one
  reaches the optimum.
"""
import os

import numpy as np
import pytest

from oracle import anneal as A
from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_schedule_matches_fig5_caption():
    g = _golden()
    n = int(g["alpha_schedule_n"])
    for i in (20, 40, 60, 80):
        a = A.alpha_schedule(i, n, g["alpha_schedule_lo"], g["alpha_schedule_hi"])
        assert round(float(a), 2) == pytest.approx(g[f"alpha_schedule_i{i}"], abs=1e-9)
    a = A.alpha_schedule(np.arange(n + 5), n)
    assert a[0] == 1.0 and a[n - 1] == pytest.approx(100.0, rel=1e-15)
    assert np.all(np.diff(a[:n]) > 0) and np.all(a[n:] == a[n - 1])
    # constant ratio between iterations: a geometric progression
    r = a[1:n] / a[:n - 1]
    assert np.allclose(r, r[0], rtol=1e-12)


def test_min_objective_seed_matches_finite_difference():
    P = np.array([2.0, 1e-3, 0.5, 7.0])
    g = T.loss_seed(P, "neg_min")
    assert T.loss_value(P, "neg_min") == -1e-3
    for i in range(P.size):
        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (T.loss_value(Pp, "neg_min") - T.loss_value(Pm, "neg_min")) / (2 * h)
        assert g[i] == pytest.approx(fd, abs=1e-9)
    # a tie seeds the lowest index only
    g = T.loss_seed(np.array([3.0, 1.0, 1.0]), "neg_min")
    assert list(g) == [0.0, -1.0, 0.0]


@pytest.mark.parametrize("alpha", [1.0, 10.0, 100.0])
def test_line_of_sight_reciprocity(alpha):
    s = WL.placement_problem(3, 4)
    pts = WL.random_points(6, 7, 12).astype(np.float64)
    for a, b in zip(pts[:6], pts[6:]):
        p_ab = T.power(s.walls, a, b[None], 0, alpha)[0]
        p_ba = T.power(s.walls, b, a[None], 0, alpha)[0]
        assert p_ab == pytest.approx(p_ba, rel=1e-12)


def test_first_adam_step_is_lr_sign():
    x = np.array([0.3, 0.6])
    g = np.array([-2.5e-3, 40.0])
    xn, m, v = A.adam_step(x, g, np.zeros(2), np.zeros(2), 1, 0.01)
    np.testing.assert_allclose(xn - x, -0.01 * np.sign(g), rtol=1e-5)
    # clamp to the box
    xn, _, _ = A.adam_step(np.array([0.0015, 0.9985]), np.array([1.0, -1.0]), np.zeros(2), np.zeros(2), 1, 0.01)
    assert list(xn) == [1e-3, 1.0 - 1e-3]


def _hard_objective(s, t):
    return float(np.min(T.power(s.walls, np.asarray(t, np.float64), s.rx, 0, 1.0, mode="hard")))


def test_annealing_leaves_the_zero_gradient_region():
    """Problem 7 with two receivers starts where one receiver is shadowed: the
    unsmoothed objective is 0 with a zero gradient there, so Adam does not move;
    annealing alpha from 1 to 100 over 100 iterations reaches the optimum found
    by a 64 x 64 scan of the unsmoothed objective (Sec. VII, Fig. 4-5)."""
    s = WL.placement_problem(7, 2)
    assert _hard_objective(s, s.tx) == 0.0
    h_hard, _ = A.optimize(s.walls, s.rx, s.tx, 0, 100, 0.01, np.full(100, 1e6))
    assert np.array_equal(h_hard[-1], s.tx.astype(np.float64))
    h, losses = A.optimize(s.walls, s.rx, s.tx, 0, 100, 0.01, A.alpha_schedule(np.arange(100), 100))
    g = (np.arange(64) + 0.5) / 64
    G = np.stack(np.meshgrid(g, g, indexing="xy"), -1).reshape(-1, 2)
    # reciprocity: the objective over tx positions from each receiver's view
    F = np.min(np.stack([T.power(s.walls, s.rx[i], G, 0, 1.0, mode="hard") for i in range(2)]), 0)
    assert _hard_objective(s, h[-1]) >= 0.95 * F.max()
