"""Transmitter placement (Sec. VII): min objective, schedule, Adam on points and
the annealed loop, HIP path against the FP64 reference."""
import numpy as np
import pytest
import torch

from oracle import anneal as A
from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

import parity_util as PU

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2401_11882_amd import batched, placement, tracer
    return batched, placement, tracer


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.mark.parametrize("alpha", [1.0, 6.43, 100.0])
@pytest.mark.parametrize("n_rx", [2, 4])
def test_min_loss_single_scene_vs_oracle(alpha, n_rx):
    _, _, tr = _mods()
    p = WL.placement_problem(11, n_rx)
    sc = tr.Scene(_dev(p.walls), _dev(p.tx), _dev(p.rx), 0, alpha)
    P, L, gtx, gw, _ = tr.forward_backward(sc, loss="neg_min")
    P_o, L_o, gw_o, gt_o, _ = T.forward_backward(p.walls, p.tx, p.rx, 0, alpha, kind="neg_min")
    _, kap = PU.kappa(p.walls, p.tx, p.rx, 0, alpha, P0=P_o)
    PU.check_power(P.cpu().numpy(), P_o, kap, "placement")
    assert float(L) == pytest.approx(L_o, rel=1e-5)
    PU.check_grads(gtx.cpu().numpy(), gw.cpu().numpy(), gt_o, gw_o, "min loss")


def test_min_loss_grid_scene_and_seed():
    """Many receivers and reflections: the seed is -1 at the lowest minimiser only."""
    _, _, tr = _mods()
    s = WL.scene_random_box(2, 8, 16, 2, 30.0, seed=21)
    sc = tr.Scene(_dev(s.walls), _dev(s.tx), _dev(s.rx), 2, s.alpha, grid_nx=16)
    P, L, seed = tr.forward(sc, loss="neg_min", want_seed=True)
    Pc = P.cpu().numpy()
    am = int(np.argmin(Pc))
    assert float(L) == -float(Pc[am])
    ref = np.zeros_like(Pc)
    ref[am] = -1.0
    assert np.array_equal(seed.cpu().numpy(), ref)
    _, L2, gtx, gw, _ = tr.forward_backward(sc, loss="neg_min")
    P_o, L_o, gw_o, gt_o, _ = T.forward_backward(s.walls, s.tx, s.rx, 2, s.alpha, kind="neg_min")
    assert int(np.argmin(P_o)) == am
    assert float(L2) == pytest.approx(L_o, rel=1e-5)
    PU.check_grads(gtx.cpu().numpy(), gw.cpu().numpy(), gt_o, gw_o, "min loss grid")


def test_min_loss_batched_matches_single():
    batched, _, tr = _mods()
    probs = [WL.placement_problem(k, 2 + k % 3) for k in range(9)]
    for p in probs:
        p.alpha = 10.0
    plan = batched.BatchPlan(probs, 0)
    P, L, gtx, gw = [t.clone() for t in plan.run(loss="neg_min")]
    for k, p in enumerate(probs):
        rs, ws = plan.scene_slice(k)
        sc = tr.Scene(_dev(p.walls), _dev(p.tx), _dev(p.rx), 0, 10.0)
        P1, L1, g1, w1, _ = tr.forward_backward(sc, loss="neg_min")
        torch.testing.assert_close(P[rs], P1, rtol=2e-6, atol=0)
        assert float(L[k]) == pytest.approx(float(L1), rel=2e-6)
        assert PU.rel_l2(gtx[k].cpu().numpy(), g1.cpu().numpy()) < 1e-5
        assert PU.rel_l2(gw[ws].cpu().numpy(), w1.cpu().numpy()) < 1e-5
    plan.close()


def test_min_loss_batched_rejects_large_scene():
    batched, _, tr = _mods()
    s = WL.scene_random_box(2, 3, 16, 0, 10.0, seed=1)     # 256 receivers
    plan = batched.BatchPlan([s], 0)
    from paper_2401_11882_amd._lib import DrtError
    with pytest.raises(DrtError):
        plan.run(loss="neg_min")
    plan.close()


def test_alpha_schedule_kernel():
    _, _, tr = _mods()
    out = torch.empty(300, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for i in (0, 1, 20, 40, 60, 80, 99, 130):
        step.fill_(i)
        tr.alpha_schedule(step, 100, 1.0, 100.0, out)
        ref = float(A.alpha_schedule(i, 100))
        assert torch.all(out == out[0])
        assert float(out[0]) == pytest.approx(ref, rel=2e-6)


def test_adam_points_matches_reference():
    _, _, tr = _mods()
    rng = np.random.default_rng(3)
    n = 700
    x = rng.uniform(0.1, 0.9, (n, 2))
    m = np.zeros((n, 2))
    v = np.zeros((n, 2))
    xd, md, vd = _dev(x), torch.zeros(n, 2, device="cuda"), torch.zeros(n, 2, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in range(1, 6):
        g = rng.normal(0, 1, (n, 2)) * 10.0 ** rng.uniform(-3, 2, (n, 1))
        x, m, v = A.adam_step(x, g, m, v, t, 0.01)
        tr.adam_points(xd, _dev(g), md, vd, step, lr=0.01)
        np.testing.assert_allclose(xd.cpu().numpy(), x, rtol=0, atol=2e-6)
    assert int(step) == 5


def test_annealed_loop_matches_reference():
    """100 annealed iterations, three problems at once, graph-replayed: each
    trajectory stays within 2e-2 of the FP64 reference at every iteration and
    reaches the same unsmoothed objective class."""
    _, placement, _ = _mods()
    probs = [WL.placement_problem(7, 2), WL.placement_problem(4, 3), WL.placement_problem(9, 4)]
    res = placement.optimize(probs, steps=100, lr=0.01)
    hist = res["tx_hist"].cpu().numpy()
    for k, p in enumerate(probs):
        h_o, L_o = A.optimize(p.walls, p.rx, p.tx, 0, 100, 0.01, A.alpha_schedule(np.arange(100), 100))
        err = np.abs(hist[:, k] - h_o).max()
        assert err < 2e-2, (k, err)
        F_gpu = float(np.min(T.power(p.walls, hist[-1, k].astype(np.float64), p.rx, 0, 1.0, mode="hard")))
        F_orc = float(np.min(T.power(p.walls, h_o[-1], p.rx, 0, 1.0, mode="hard")))
        assert (F_gpu > 0) == (F_orc > 0)
        assert F_gpu == pytest.approx(F_orc, rel=5e-2)
    np.testing.assert_allclose(res["loss_hist"].cpu().numpy()[0],
                               [T.loss_value(T.power(p.walls, p.tx, p.rx, 0, 1.0), "neg_min") for p in probs],
                               rtol=1e-5)


def test_unsmoothed_start_in_shadow_does_not_move():
    _, placement, _ = _mods()
    p = WL.placement_problem(7, 2)
    res = placement.optimize([p], steps=50, lr=0.01, fixed_alpha=placement.HARD_ALPHA)
    assert torch.equal(res["tx"].cpu()[0], torch.tensor(p.tx))
    ann = placement.optimize([p], steps=100, lr=0.01, use_graph=False)
    F = placement.objective([p], ann["tx"])
    ref = placement.grid_optimum([p], 64)
    assert float(F[0]) >= 0.95 * float(ref[0])


def test_grid_optimum_matches_reference():
    _, placement, _ = _mods()
    probs = [WL.placement_problem(k, 3) for k in range(4)]
    best = placement.grid_optimum(probs, 32, alpha=30.0).cpu().numpy()
    g = WL.rx_grid(32).astype(np.float64)
    for k, p in enumerate(probs):
        F = np.min(np.stack([T.power(p.walls, p.rx[i], g, 0, 30.0) for i in range(3)]), 0)
        assert best[k] == pytest.approx(F.max(), rel=1e-5)


def test_study_small():
    _, placement, _ = _mods()
    out = placement.study(n_per_count=32, rx_counts=(2, 3), grid_n=64)
    for n_rx, r in out.items():
        assert 0.0 <= r["annealed_success"] <= 1.0 and 0.0 <= r["unsmoothed_success"] <= 1.0
        print("placement study", n_rx, r)
