"""The algorithmic work model (oracle instrumentation): the contribution cut
only removes work, a vanishing cut removes none, and the stored model holds
the figures the benchmark reads."""
import json
import os

import numpy as np
import pytest

from oracle import tracer as T
from oracle import tracer3d as T3
from paper_2401_11882_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_cut_monotone(count):
    base = count(0.0)
    tiny = count(1e-300)
    cut = count(2.0 ** -24 / 4625)
    big = count(1e-6)
    for k in ("path_evals", "interactions", "active", "active_interactions"):
        assert tiny[k] == base[k]
    for k in ("path_evals", "interactions"):
        assert cut[k] == base[k] == big[k]
    for k in ("active", "active_interactions", "unsaturated"):
        assert big[k] <= cut[k] <= base[k]
    assert cut["unsaturated"] <= tiny["unsaturated"] <= base["unsaturated"]
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
    assert n_candidates(68, 2) == 4625 and n_candidates(38, 2) == 1445
    for key, W, sec in (("100", WEIGHTS, m["per_alpha"]), ("100", WEIGHTS_3D, m["scene3d"]["per_alpha"])):
        rec = sec[key]
        again = model(rec["counts"], W)
        assert again["fwd_flops_per_path_eval"] == pytest.approx(rec["fwd_flops_per_path_eval"])
        assert again["bwd_flops_per_path_eval"] == pytest.approx(rec["bwd_flops_per_path_eval"])
        assert 0 < rec["per_path_eval"]["active"] < 1
