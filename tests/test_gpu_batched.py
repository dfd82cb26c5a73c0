"""Batched persistent launch: parity with single-scene launches and the oracle."""
import os

import numpy as np
import pytest
import torch

from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

import parity_util as PU

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2401_11882_amd import batched, tracer
    return batched, tracer


def _single(tr, s, loss="neg_mean_log"):
    dev = torch.device("cuda")
    sc = tr.Scene(torch.tensor(s.walls, device=dev), torch.tensor(s.tx, device=dev), torch.tensor(s.rx, device=dev),
                  s.max_order, s.alpha, grid_nx=s.grid_n)
    return [t.clone() for t in tr.forward_backward(sc, loss=loss)[:4]]


def _small_mixed():
    """Uneven small scenes: different wall counts, grid sizes, a ragged receiver list, alphas."""
    out = []
    for i, (n_int, n, alpha) in enumerate([(3, 8, 100.0), (7, 16, 30.0), (1, 8, 1000.0), (5, 0, 100.0), (0, 8, 100.0)]):
        s = WL.scene_random_box(3, n_int, max(n, 1), 2, alpha, seed=100 + i)
        if n == 0:
            s.rx = WL.random_points(3, i, 77)
            s.grid_n = 0
        out.append(s)
    return out


def test_batched_small_vs_oracle():
    batched, tr = _mods()
    scenes = _small_mixed()
    plan = batched.BatchPlan(scenes, 2)
    P, L, gtx, gw = [t.cpu().numpy() for t in plan.run()]
    for s_i, s in enumerate(scenes):
        rs, ws = plan.scene_slice(s_i)
        P_o, L_o, gw_o, gt_o, _ = T.forward_backward(s.walls, s.tx, s.rx, 2, s.alpha)
        _, kap = PU.kappa(s.walls, s.tx, s.rx, 2, s.alpha, P0=P_o)
        PU.check_power(P[rs], P_o, kap, f"batched scene {s_i}")
        assert L[s_i] == pytest.approx(L_o, rel=1e-5)
        PU.check_grads(gtx[s_i], gw[ws], gt_o, gw_o, f"batched scene {s_i}")
    plan.close()


def test_batched_matches_single_scene_launches():
    batched, tr = _mods()
    scenes = WL.batch_scenes(12, side_cap=32)
    plan = batched.BatchPlan(scenes, 2)
    P, L, gtx, gw = [t.clone() for t in plan.run()]
    for s_i, s in enumerate(scenes):
        rs, ws = plan.scene_slice(s_i)
        P1, L1, g1, w1 = _single(tr, s)
        torch.testing.assert_close(P[rs], P1, rtol=2e-6, atol=0)
        torch.testing.assert_close(L[s_i:s_i + 1], L1, rtol=2e-6, atol=0)
        assert PU.rel_l2(gtx[s_i].cpu().numpy(), g1.cpu().numpy()) < 1e-5
        assert PU.rel_l2(gw[ws].cpu().numpy(), w1.cpu().numpy()) < 1e-5
    plan.close()


def test_batched_deterministic_and_graph_replay():
    batched, tr = _mods()
    scenes = WL.batch_scenes(16, side_cap=16)
    plan = batched.BatchPlan(scenes, 2)
    a = [t.clone() for t in plan.run()]
    b = [t.clone() for t in plan.run()]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in plan.out:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(plan.out, a):
            assert torch.equal(x, y), f"replay {rep}"
        _ = float(plan.out[1].sum())
    plan.close()


@pytest.mark.parametrize("nw", [4, 8, 16])
def test_every_launch_shape_agrees_when_workgroups_take_several_items(nw):
    """One workgroup per CU, more items than workgroups: each wavefront slot is
    reused for several items, and its recorded contributions and leg boxes
    must be the current item's.  Repeated runs are bitwise equal and match
    the default launch shape."""
    batched, tr = _mods()
    scenes = WL.batch_scenes(24, side_cap=32)
    plan = batched.BatchPlan(scenes, 2)
    ref = [t.clone() for t in plan.run()]
    for cc, tw in ((1, 8), (4, 16)):
        plan.set_config(nw=nw, cchunk=cc, blocks_per_cu=1, tile_w=tw)
        a = [t.clone() for t in plan.run()]
        b = [t.clone() for t in plan.run()]
        for x, y, z in zip(a, b, ref):
            assert torch.equal(x, y)
            torch.testing.assert_close(x, z, rtol=1e-5, atol=1e-6 * float(z.abs().max()))
    assert plan.info()["items"] > 256
    plan.close()


def test_batched_screen_exact():
    batched, tr = _mods()
    scenes = _small_mixed() + WL.batch_scenes(8, side_cap=32)
    out = {}
    try:
        for on in (True, False):
            tr.set_screen(on)
            plan = batched.BatchPlan(scenes, 2)
            out[on] = [t.clone() for t in plan.run()]
            plan.close()
    finally:
        tr.set_screen(True)
    for x, y in zip(out[True], out[False]):
        assert torch.equal(x, y)


def test_batched_cut_within_bound():
    """Batched contribution cut: power within 2^-24 P (+ FP32 rounding) of the
    uncut power, gradients to FP32 accuracy."""
    batched, tr = _mods()
    scenes = _small_mixed() + WL.batch_scenes(8, side_cap=32)
    out = {}
    try:
        for on in (True, False):
            tr.set_cut(on)
            plan = batched.BatchPlan(scenes, 2)
            out[on] = [t.clone() for t in plan.run()]
            plan.close()
    finally:
        tr.set_cut(True)
    P_cut, P_all = out[True][0].double(), out[False][0].double()
    assert bool((P_cut <= P_all * (1 + 1e-6)).all())
    assert float(((P_all - P_cut).abs() / P_all.clamp_min(1e-30)).max()) <= 2.0 ** -24 + 2e-6
    for x, y in zip(out[True][1:], out[False][1:]):
        if x.numel() == 0:
            continue
        torch.testing.assert_close(x, y, rtol=1e-4, atol=1e-5 * float(y.abs().max()))


def test_batched_cache_overflow_reevaluates():
    """A contribution cache too small for the lists: the wavefronts that
    overflow re-evaluate their share in the adjoint.  Power and loss are
    bitwise those of a plan with room for every list; gradients agree to FP32
    accuracy (re-evaluation bounds P(r) for the cut by its own running sum)."""
    batched, tr = _mods()
    scenes = _small_mixed() + WL.batch_scenes(6, side_cap=32)
    ref_plan = batched.BatchPlan(scenes, 2)
    ref = [t.clone() for t in ref_plan.run()]
    ref_plan.close()
    try:
        tr.set_cache_limit(8 << 20)
        plan = batched.BatchPlan(scenes, 2)
        cap = plan.info()["cache_cap"]
        out = [t.clone() for t in plan.run()]
        plan.close()
    finally:
        tr.set_cache_limit(32 << 30)
    assert 0 < cap < 64
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    for x, y in zip(out[2:], ref[2:]):
        torch.testing.assert_close(x, y, rtol=1e-5, atol=1e-6 * float(y.abs().max()))


def test_autotune_and_cache(tmp_path):
    batched, tr = _mods()
    scenes = WL.batch_scenes(24, side_cap=32)
    ref_plan = batched.BatchPlan(scenes, 2)
    ref = [t.clone() for t in ref_plan.run()]
    ref_plan.close()
    cache = str(tmp_path / "tune.txt")
    plan = batched.BatchPlan(scenes, 2)
    best = plan.autotune(cache_path=cache)
    out = plan.run()
    for x, y in zip(out, ref):
        torch.testing.assert_close(x, y, rtol=1e-5, atol=1e-6 * float(y.abs().max()))
    plan.close()
    assert os.path.getsize(cache) > 0
    plan2 = batched.BatchPlan(scenes, 2, tune_cache=cache)
    assert plan2.config() == best
    plan2.close()


def test_full_batch_512_sampled():
    """512 scenes, 8..128 interior segments, 64^2..256^2 receivers, order <= 2, alpha 100:
    one launch; sampled receivers of sampled scenes vs the oracle, two scenes vs single launches."""
    batched, tr = _mods()
    scenes = WL.batch_scenes(512)
    plan = batched.BatchPlan(scenes, 2)
    info = plan.info()
    assert info["items"] == sum((s.n_rx + 63) // 64 for s in scenes)
    P, L, gtx, gw = [t.cpu() for t in plan.run()]
    assert torch.isfinite(P).all() and torch.isfinite(gw).all() and torch.isfinite(gtx).all()
    rng = np.random.default_rng(5)
    for s_i in rng.choice(512, size=4, replace=False):
        s = scenes[s_i]
        rs, ws = plan.scene_slice(s_i)
        idx = rng.choice(s.n_rx, size=6, replace=False)
        P_o, kap = PU.kappa(s.walls, s.tx, s.rx[idx], 2, s.alpha)
        PU.check_power(P[rs].numpy()[idx], P_o, kap, f"scene {s_i}")
    for s_i in (0, 511):
        s = scenes[s_i]
        rs, ws = plan.scene_slice(s_i)
        P1, L1, g1, w1 = [t.cpu() for t in _single(tr, s)]
        torch.testing.assert_close(P[rs], P1, rtol=2e-6, atol=0)
        assert PU.rel_l2(gtx[s_i].numpy(), g1.numpy()) < 1e-5
        assert PU.rel_l2(gw[ws].numpy(), w1.numpy()) < 1e-5
    # the two cheapest scenes in full against the oracle: every receiver's
    # power, the scene's loss and its gradients (tx and every wall endpoint)
    cost = [s.n_rx * WL.n_candidates(s.walls.shape[0], 2) for s in scenes]
    for s_i in np.argsort(cost)[:2]:
        s = scenes[s_i]
        rs, ws = plan.scene_slice(s_i)
        P_o, L_o, gw_o, gt_o, _ = T.forward_backward(s.walls, s.tx, s.rx, 2, s.alpha)
        _, kap = PU.kappa(s.walls, s.tx, s.rx, 2, s.alpha, P0=P_o, runs=2)
        st = PU.check_power(P[rs].numpy(), P_o, kap, f"scene {s_i} (full)")
        assert float(L[s_i]) == pytest.approx(L_o, rel=1e-5, abs=1e-5)
        PU.check_grads(gtx[s_i].numpy(), gw[ws].numpy(), gt_o, gw_o, f"scene {s_i} (full)")
        print(f"batched scene {s_i}: {s.walls.shape[0]} walls, {s.n_rx} rx, {st}", flush=True)
    plan.close()


def test_plan_rejects_scenes_beyond_the_lds_budget():
    batched, tr = _mods()
    from paper_2401_11882_amd._lib import DrtError
    big = WL.scene_random_box(3, 1000, 8, 1, 100.0, seed=1)      # 1004 walls
    with pytest.raises(DrtError):
        batched.BatchPlan([big], 1)
    ok = WL.scene_random_box(3, 900, 8, 1, 100.0, seed=1)        # 904 walls: fits at 4 wavefronts
    plan = batched.BatchPlan([ok], 1)
    assert plan.config()["nw"] == 4
    with pytest.raises(DrtError):
        plan.set_config(nw=16)
    P, L, gtx, gw = plan.run()
    assert torch.isfinite(P).all() and torch.isfinite(gw).all()
    plan.close()
