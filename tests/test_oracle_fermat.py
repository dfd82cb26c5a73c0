"""Pins of the Fermat-path-tracing oracle (oracle/fermat.py, Sec. V-B) that do
not go through its own Newton iteration:

* closed forms on one long wall: a true reflection sits at the specular point
  with the mirror-image length and a zero MPT loss; a pass-through sits where
  the straight segment crosses the wall line, with MPT loss 4 (d . n)^2;
* against the image method (itself pinned in test_oracle_pins.py): on every
  true reflection of small random scenes the Fermat points equal the image
  method's, and so does the contribution wherever the image method's side
  factors in(u) are 1;
* against brute force: the returned parameters are a minimum of the path
  length (no grid point and no small move is shorter) on orders 1 and 2;
* the smoothing limit: the sigmoid version tends to the unit-step version as
  alpha grows (Eq. 2).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import fermat as FM
from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

LONG = np.array([[-1e3, 0.0, 1e3, 0.0]])


def test_single_reflection_closed_form():
    tx, r = np.array([0.3, 0.4]), np.array([0.8, 0.1])
    d = {x["seq"]: x for x in FM.path_details(LONG, tx, r, 1, 100.0)}
    X = d[(0,)]["points"][0]
    assert X[0] == pytest.approx((tx[0] * r[1] + r[0] * tx[1]) / (tx[1] + r[1]), abs=1e-12)
    assert X[1] == 0.0
    assert d[(0,)]["length"] == pytest.approx(math.hypot(r[0] - tx[0], r[1] + tx[1]), rel=1e-14)
    assert d[(0,)]["L_mpt"] < 1e-20
    # power: LOS unobstructed (the only wall is the reflector), reflection factor in(t) s(1)
    c_los = 1.0 / ((r - tx) ** 2).sum()
    t = (X[0] + 1e3) / 2e3
    a = 100.0
    s = lambda z: 1.0 / (1.0 + math.exp(-a * z))  # noqa: E731
    c_ref = s(t) * s(1 - t) * s(1.0 - d[(0,)]["L_mpt"] / FM.DEFAULT_EPS) / d[(0,)]["length"] ** 2
    assert FM.power(LONG, tx, r[None], 1, a)[0] == pytest.approx(c_los + c_ref, rel=1e-12)


def test_pass_through_closed_form():
    tx, r = np.array([0.3, 0.4]), np.array([0.8, -0.2])
    d = {x["seq"]: x for x in FM.path_details(LONG, tx, r, 1, 100.0)}
    X = d[(0,)]["points"][0]
    assert X[0] == pytest.approx(tx[0] + (r[0] - tx[0]) * tx[1] / (tx[1] - r[1]), abs=1e-12)
    u = (r - tx) / np.linalg.norm(r - tx)
    assert d[(0,)]["L_mpt"] == pytest.approx(4 * u[1] ** 2, rel=1e-12)
    assert d[(0,)]["length"] == pytest.approx(np.linalg.norm(r - tx), rel=1e-14)
    # the check fails (its argument is 1 - L / eps, about -2.4e4 here): the
    # pass-through contributes nothing at alpha = 100, and the LOS leg crosses
    # the long wall in its middle, so almost nothing arrives
    assert d[(0,)]["c"] < 1e-300
    assert FM.power(LONG, tx, r[None], 1, 100.0)[0] < 1e-12


@pytest.mark.parametrize("seed,K", [(1, 2), (2, 2), (3, 1)])
def test_matches_image_method_on_true_reflections(seed, K):
    alpha = 100.0
    s = WL.scene_random_box(2, 3, 4, K, alpha, seed=seed)
    n_refl = n_equal = 0
    for r in s.rx:
        di = T.path_details(s.walls, s.tx, r, K, alpha)
        df = FM.path_details(s.walls, s.tx, r, K, alpha)
        for a, b in zip(di, df):
            assert a["seq"] == b["seq"]
            if len(a["seq"]) == 0:
                assert b["c"] == pytest.approx(a["c"], rel=1e-13, abs=1e-300)
                continue
            true_refl = a["valid"] and all(0.0 < u < 1.0 for u in a["u"])
            if not true_refl:
                continue
            n_refl += 1
            # same points (Fermat's minimum of a true reflection is the specular point)
            assert np.abs(np.array(a["points"]) - np.array(b["points"])).max() < 1e-9
            assert b["L_mpt"] < 1e-16
            # same contribution where the image method's side factors are 1 in FP64
            if all(min(u, 1 - u) * alpha > 40.0 for u in a["u"]):
                n_equal += 1
                assert b["c"] == pytest.approx(a["c"], rel=1e-7, abs=1e-300)   # deep shadows amplify 1e-15 moves
    assert n_refl > 20 and n_equal > 10


def _length(walls, tx, r, seq, t):
    P = [np.asarray(tx, float)] + [walls[j, :2] + ti * (walls[j, 2:] - walls[j, :2]) for j, ti in zip(seq, t)] + \
        [np.asarray(r, float)]
    return sum(np.linalg.norm(P[i + 1] - P[i]) for i in range(len(P) - 1))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_minimum_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    walls = np.concatenate([WL.BOX_WALLS, rng.uniform(0.1, 0.9, (2, 4))]).astype(np.float64)
    tx, r = rng.uniform(0.05, 0.95, 2), rng.uniform(0.05, 0.95, 2)
    grid = np.linspace(-1.0, 2.0, 121)
    for seq in [(4,), (0,), (4, 5), (1, 4), (2, 0)]:
        d = {x["seq"]: x for x in FM.path_details(walls, tx, r, len(seq), 100.0)}[seq]
        t = np.asarray(d["t"])
        L = _length(walls, tx, r, seq, t)
        assert L == pytest.approx(d["length"], rel=1e-13)
        best = min(_length(walls, tx, r, seq, g) for g in itertools.product(grid, repeat=len(seq)))
        assert L <= best + 1e-12
        for i in range(len(seq)):
            for h in (1e-4, -1e-4):
                tt = t.copy()
                tt[i] += h
                assert _length(walls, tx, r, seq, tt) >= L - 1e-15


def test_alpha_to_infinity_tends_to_unit_step():
    s = WL.scene_random_box(2, 2, 4, 2, 100.0, seed=4)
    P_hard = FM.power(s.walls, s.tx, s.rx, 2, 1.0, mode="hard")
    errs = [np.abs(FM.power(s.walls, s.tx, s.rx, 2, a) - P_hard).max() for a in (1e2, 1e4, 1e6)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1e-3 * P_hard.max()
