"""The algorithmic work model (oracle instrumentation), pinned two ways that do
not go through the oracle's own vectorised code:

* closed form: with the cut, the FP32-zero floor and the saturation band all
  switched off, every pair is active and every test counts, so the counts are
  the enumeration itself -- sum_k n_k ((k+1) W - 2k) obstruction tests
  (each of the k+1 legs skips its own end walls: 2k exclusions) and
  sum_k k n_k interactions over sum_k n_k candidates, n_k = W (W-1)^(k-1);
  199.0 tests and 1.985 interactions per path evaluation on the 68-wall,
  order-2 benchmark scene;
* brute force: a plain-Python loop over (receiver, candidate) pairs on tiny
  scenes, written here from the definitions (images, back-trace, smoothed
  factors, the rule for active pairs), reproduces active pairs, their interactions,
  tests and unsaturated tests exactly.

Plus: the cut only removes work, and the stored model holds the figures the
benchmark reads.
"""
import json
import math
import os

import pytest

from oracle import tracer as T
from oracle import tracer3d as T3
from paper_2401_11882_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ----------------------------------------------------------------- closed form

def _enumeration(W, K):
    n = [1] + [W * (W - 1) ** (k - 1) for k in range(1, K + 1)]
    C = sum(n)
    tests = sum(n[k] * ((k + 1) * W - 2 * k) for k in range(K + 1))
    inter = sum(k * n[k] for k in range(K + 1))
    return C, tests, inter


def test_closed_form_counts_benchmark_scene():
    s = WL.scene_64(alpha=100.0)
    R = 3
    c = T.work_counts(s.walls, s.tx, s.rx[[0, 30000, 65535]], 2, 100.0, margin=math.inf,
                      active_log_floor=-math.inf, cut=0.0)
    C, tests, inter = _enumeration(68, 2)
    assert C == 4625 and tests == 920380 and inter == 9180
    assert c["path_evals"] == R * C
    assert c["active"] == R * C and c["active_interactions"] == c["interactions"] == R * inter
    assert c["tests"] == c["unsaturated"] == R * tests
    assert tests / C == pytest.approx(199.0, abs=2e-3)
    assert inter / C == pytest.approx(1.985, abs=1e-3)


@pytest.mark.parametrize("K", [0, 1, 2, 3])
def test_closed_form_counts_all_orders(K):
    s = WL.scene_random_box(2, 3, 4, K, 100.0, seed=5)
    W = s.walls.shape[0]
    c = T.work_counts(s.walls, s.tx, s.rx[:5], K, 100.0, margin=math.inf, active_log_floor=-math.inf)
    C, tests, inter = _enumeration(W, K)
    assert c["path_evals"] == 5 * C and c["active"] == 5 * C
    assert c["tests"] == c["unsaturated"] == 5 * tests
    assert c["interactions"] == c["active_interactions"] == 5 * inter


def test_closed_form_counts_3d():
    s = WL.scene3d_room(2, 3, 2, 2, 100.0, seed=4)
    P = s.panels.shape[0]
    c = T3.work_counts(s.panels, s.tx, s.rx[:3], 2, 100.0, margin=math.inf, active_log_floor=-math.inf)
    C, tests, inter = _enumeration(P, 2)
    assert c["path_evals"] == 3 * C and c["active"] == 3 * C
    assert c["tests"] == c["unsaturated"] == 3 * tests
    assert c["interactions"] == 3 * inter


# ----------------------------------------------------------------- brute force

def _log_sig(z):
    return -math.log1p(math.exp(-z)) if z >= 0 else z - math.log1p(math.exp(z))


def _log_in(x, alpha):
    return _log_sig(alpha * x) + _log_sig(alpha * (1.0 - x))


def _cx(u, v):
    return u[0] * v[1] - u[1] * v[0]


def _sub(p, q):
    return (p[0] - q[0], p[1] - q[1])


def _seqs(W, K):
    out = [()]
    for k in range(1, K + 1):
        prev = [s for s in out if len(s) == k - 1]
        out += [s + (j,) for s in prev for j in range(W) if not s or s[-1] != j]
    return out


def _brute(walls, tx, rxs, K, alpha, margin=18.0, floor=-88.72, cut=0.0, d_min=1e-3):
    W = len(walls)
    A = [(float(w[0]), float(w[1])) for w in walls]
    E = [(float(w[2] - w[0]), float(w[3] - w[1])) for w in walls]
    tx = (float(tx[0]), float(tx[1]))
    band = margin / alpha
    per_rx = []
    for r in rxs:
        r = (float(r[0]), float(r[1]))
        rows = []
        for seq in _seqs(W, K):
            k = len(seq)
            img = [tx]
            valid = True
            for j in seq:
                n = (-E[j][1], E[j][0])
                nn = n[0] * n[0] + n[1] * n[1]
                if nn == 0:
                    valid = False
                    nn = 1.0
                h = ((img[-1][0] - A[j][0]) * n[0] + (img[-1][1] - A[j][1]) * n[1]) / nn
                img.append((img[-1][0] - 2 * h * n[0], img[-1][1] - 2 * h * n[1]))
            X = [None] * (k + 2)
            X[k + 1] = r
            logf = 0.0
            for i in range(k, 0, -1):
                j = seq[i - 1]
                d = _sub(img[i], X[i + 1])
                w = _sub(A[j], X[i + 1])
                den = _cx(d, E[j])
                if den == 0:
                    valid = False
                    den = 1.0
                t = _cx(w, d) / den
                u = _cx(w, E[j]) / den
                X[i] = (A[j][0] + t * E[j][0], A[j][1] + t * E[j][1])
                logf += _log_in(t, alpha) + _log_in(u, alpha)
            X[0] = tx
            V = math.exp(logf)
            tests = []          # (in band) per obstruction test
            for l in range(k + 1):
                D = _sub(X[l + 1], X[l])
                own = set()
                if l >= 1:
                    own.add(seq[l - 1])
                if l + 1 <= k:
                    own.add(seq[l])
                for j in range(W):
                    if j in own:
                        continue
                    den = _cx(D, E[j])
                    w0 = _sub(A[j], X[l])
                    if den == 0:
                        tests.append(False)
                        continue
                    tau = _cx(w0, D) / den
                    ups = _cx(w0, E[j]) / den
                    V *= -math.expm1(_log_in(tau, alpha) + _log_in(ups, alpha))
                    tests.append(abs(tau - 0.5) < 0.5 + band and abs(ups - 0.5) < 0.5 + band)
            d2 = (r[0] - img[k][0]) ** 2 + (r[1] - img[k][1]) ** 2
            c = V / max(d2, d_min * d_min) if valid else 0.0
            rows.append((k, valid, logf, c, tests, d2))
        per_rx.append(rows)
    out = dict(path_evals=0, interactions=0, active=0, active_interactions=0, tests=0, unsaturated=0)
    for rows in per_rx:
        P = sum(row[3] for row in rows)
        for k, valid, logf, c, tests, d2 in rows:
            out["path_evals"] += 1
            out["interactions"] += k
            if valid and logf > floor and (cut <= 0 or math.exp(logf) / max(d2, d_min * d_min) > cut * P):
                out["active"] += 1
                out["active_interactions"] += k
                out["tests"] += len(tests)
                out["unsaturated"] += sum(tests)
    return out


@pytest.mark.parametrize("alpha,cut", [(100.0, 0.0), (100.0, 2.0 ** -24 / 37), (100.0, 1e-3), (10.0, 1e-4),
                                       (1000.0, 2.0 ** -24 / 37)])
def test_brute_force_reproduces_counts(alpha, cut):
    s = WL.scene_random_box(2, 2, 4, 2, alpha, seed=11)        # box + 2 segments: 6 walls, 37 candidates
    rx = s.rx[::3]
    got = T.work_counts(s.walls, s.tx, rx, 2, alpha, cut=cut)
    ref = _brute(s.walls, s.tx, rx, 2, alpha, cut=cut)
    assert got == ref
    assert 0 < ref["active"] < ref["path_evals"]
    assert 0 < ref["unsaturated"] < ref["tests"]


def test_brute_force_reproduces_counts_order3():
    s = WL.scene_random_box(4, 1, 4, 3, 100.0, seed=2)         # box + 1 segment: 5 walls, 106 candidates
    rx = s.rx[::5]
    cut = 2.0 ** -24 / 106
    assert T.work_counts(s.walls, s.tx, rx, 3, 100.0, cut=cut) == _brute(s.walls, s.tx, rx, 3, 100.0, cut=cut)


# ----------------------------------------------------------------- cut and stored model

def _check_cut_monotone(count):
    base = count(0.0)
    tiny = count(1e-300)
    cut = count(2.0 ** -24 / 4625)
    big = count(1e-6)
    for k in ("path_evals", "interactions"):
        assert tiny[k] == base[k] == cut[k] == big[k]
    for k in ("active", "active_interactions", "tests", "unsaturated"):
        assert big[k] <= cut[k] <= tiny[k] <= base[k]
    assert big["active"] < base["active"]


def test_cut_only_removes_work_2d():
    s = WL.scene_random_box(2, 6, 4, 2, 100.0, seed=3)
    _check_cut_monotone(lambda c: T.work_counts(s.walls, s.tx, s.rx, 2, 100.0, cut=c))


def test_cut_only_removes_work_3d():
    s = WL.scene3d_room(2, 4, 3, 2, 100.0, seed=3)
    _check_cut_monotone(lambda c: T3.work_counts(s.panels, s.tx, s.rx, 2, 100.0, cut=c))


def test_stored_model_matches_its_weights():
    with open(os.path.join(ROOT, "bench_work_model.json")) as f:
        m = json.load(f)
    assert m["cut_total"] == pytest.approx(2.0 ** -24)
    from oracle.count_work import WEIGHTS, WEIGHTS_3D, model, n_candidates
    assert m["weights"] == WEIGHTS and m["scene3d"]["weights"] == WEIGHTS_3D
    assert n_candidates(68, 2) == 4625 and n_candidates(38, 2) == 1445
    for key, W, sec in (("100", WEIGHTS, m["per_alpha"]), ("100", WEIGHTS_3D, m["scene3d"]["per_alpha"])):
        rec = sec[key]
        again = model(rec["counts"], W)
        assert again["fwd_flops_per_path_eval"] == pytest.approx(rec["fwd_flops_per_path_eval"])
        assert again["bwd_flops_per_path_eval"] == pytest.approx(rec["bwd_flops_per_path_eval"])
        assert 0 < rec["per_path_eval"]["active"] < 1
        assert rec["counts"]["interactions"] / rec["counts"]["path_evals"] == pytest.approx(
            (68 + 2 * 4556) / 4625 if sec is m["per_alpha"] else (38 + 2 * 38 * 37) / 1445)
