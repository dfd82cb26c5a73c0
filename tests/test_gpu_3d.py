"""3D scenes of parallelogram panels: the HIP kernels against the FP64 reference
(oracle/tracer3d.py), and an extruded 2D scene against the 2D reference."""
import numpy as np
import pytest
import torch

from oracle import tracer as T
from oracle import tracer3d as T3
from paper_2401_11882_amd import workloads as WL

import parity_util as PU

pytestmark = pytest.mark.gpu


def _tr3():
    from paper_2401_11882_amd import tracer3d
    return tracer3d


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _scene(s, rx=None, grid=True):
    rx_np = s.rx if rx is None else rx
    return _tr3().Scene3(_dev(s.panels), _dev(s.tx), _dev(rx_np), s.max_order, s.alpha,
                         grid_nx=(s.grid_n if (grid and rx is None) else 0))


def kappa3(panels, tx, rx, K, alpha, runs=4, seed=0, P0=None):
    """Rounding sensitivity of the reference power (as parity_util.kappa, for panels)."""
    rng = np.random.default_rng(seed)
    if P0 is None:
        P0 = T3.power(panels, tx, rx, K, alpha)
    kap = np.zeros_like(P0)
    for _ in range(runs):
        P = T3.power(PU.perturb(panels, rng), PU.perturb(tx, rng), PU.perturb(rx, rng), K, alpha)
        kap = np.maximum(kap, np.abs(P - P0))
    return P0, kap


def test_free_space_and_single_mirror_closed_forms():
    tr = _tr3()
    tx = np.array([0.2, 0.3, 0.4], np.float32)
    rx = np.array([[0.7, 0.6, 0.5], [0.2, 0.3, 0.4005]], np.float32)
    sc = tr.Scene3(_dev(np.zeros((0, 9))), _dev(tx), _dev(rx), 2, 100.0)
    P = tr.forward(sc)[0].cpu().numpy()
    d2 = ((rx.astype(np.float64) - tx) ** 2).sum(1)
    np.testing.assert_allclose(P, 1.0 / np.maximum(d2, 1e-6), rtol=2e-6)
    # a large mirror z = 0 far from every edge: LOS + one reflection off the floor
    floor = np.array([[-5, -5, 0, 5, -5, 0, -5, 5, 0]], np.float32)
    sc = tr.Scene3(_dev(floor), _dev(tx), _dev(rx[:1]), 1, 100.0)
    P = float(tr.forward(sc)[0][0])
    img = tx.astype(np.float64) * np.array([1, 1, -1])
    want = 1.0 / d2[0] + 1.0 / ((rx[0] - img) ** 2).sum()
    assert P == pytest.approx(want, rel=2e-6)


@pytest.mark.parametrize("K", [0, 1, 2, 3])
@pytest.mark.parametrize("alpha", [10.0, 100.0, 1000.0])
def test_room_scenes_all_orders(K, alpha):
    tr = _tr3()
    s = WL.scene3d_room(9, 2 if K < 3 else 0, 16, K, alpha, seed=40 + K)
    sc = _scene(s)
    P, L, gtx, gp, grx = tr.forward_backward(sc, loss="neg_mean_log", want_rx=True)
    P_o, kap = kappa3(s.panels, s.tx, s.rx, K, alpha)
    PU.check_power(P.cpu().numpy(), P_o, kap, f"3D K={K}")
    L_o = -np.mean(np.log(P_o + 1e-6))
    assert float(L) == pytest.approx(L_o, rel=1e-5)
    g = -1.0 / (s.n_rx * (P_o + 1e-6))
    gp_o, gt_o, grx_o = T3.vjp(s.panels, s.tx, s.rx, K, alpha, g)
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, f"3D K={K}")
    assert PU.rel_l2(grx.cpu().numpy(), grx_o) <= PU.GRAD_REL, "receiver gradients"


def test_extruded_2d_scene_matches_the_2d_reference():
    """Vertical panels of height 1 with every point at half height: each path
    stays in that plane and the height coordinate sits at 1/2, where
    in(1/2) = s(alpha/2)^2 = 1 to FP32 precision at alpha = 100."""
    s2 = WL.scene_random_box(3, 4, 16, 2, 100.0, seed=5)
    s3 = WL.extrude(s2)
    tr = _tr3()
    sc = tr.Scene3(_dev(s3.panels), _dev(s3.tx), _dev(s3.rx), 2, 100.0)
    P = tr.forward(sc)[0].cpu().numpy()
    P_o, kap = PU.kappa(s2.walls, s2.tx, s2.rx, 2, 100.0)
    PU.check_power(P, P_o, kap, "extruded")


def test_full_size_scene_sampled():
    """Room + 32 rectangles, 256 x 256 receivers, order <= 2, in the bench's
    launch shape: sampled receivers against the reference, and gradients of a
    loss over a sampled receiver subset."""
    tr = _tr3()
    s = WL.scene3d_32()
    sc = _scene(s)
    P, L, seed = tr.forward(sc, loss="neg_mean_log", want_seed=True)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.choice(s.n_rx, 62, replace=False), [0, s.n_rx - 1]]))
    P_o, kap = kappa3(s.panels, s.tx, s.rx[idx], 2, s.alpha)
    PU.check_power(P.cpu().numpy()[idx], P_o, kap, "scene3d_32")
    w = np.zeros(s.n_rx, np.float32)
    w[idx[:24]] = 1.0
    g = seed * _dev(w)
    gtx, gp, grx = tr.backward(sc, g, want_rx=True)
    gp_o, gt_o, grx_o = T3.vjp(s.panels, s.tx, s.rx[idx[:24]], 2, s.alpha, seed.cpu().numpy()[idx[:24]])
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, "scene3d_32")
    assert PU.rel_l2(grx.cpu().numpy()[idx[:24]], grx_o) <= PU.GRAD_REL, "receiver gradients"
    rest = np.setdiff1d(np.arange(s.n_rx), idx[:24])
    assert torch.count_nonzero(grx[torch.as_tensor(rest, device="cuda")]) == 0


def test_degenerate_panel_and_ragged_receivers():
    """A zero-area panel neither reflects nor blocks; 100 receivers (a ragged
    last tile) without grid order."""
    tr = _tr3()
    s = WL.scene3d_room(9, 3, 16, 2, 50.0, seed=3)
    pan = s.panels.copy()
    pan[7, 6:9] = pan[7, 0:3] + 2.0 * (pan[7, 3:6] - pan[7, 0:3])   # c on the line a-b: zero area
    rx = np.random.default_rng(1).uniform(0.05, 0.95, (100, 3)).astype(np.float32)
    sc = tr.Scene3(_dev(pan), _dev(s.tx), _dev(rx), 2, 50.0)
    P, L, gtx, gp = tr.forward_backward(sc, loss="sum")
    P_o, kap = kappa3(pan, s.tx, rx, 2, 50.0)
    PU.check_power(P.cpu().numpy(), P_o, kap, "degenerate")
    assert float(L) == pytest.approx(P_o.sum(), rel=1e-5)
    gp_o, gt_o, _ = T3.vjp(pan, s.tx, rx, 2, 50.0, np.ones(100))
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, "degenerate")
    assert np.all(gp.cpu().numpy()[7] == 0.0)


def test_min_loss_seed_and_reuse_are_exact():
    tr = _tr3()
    s = WL.scene3d_room(9, 4, 16, 2, 100.0, seed=11)
    sc = _scene(s)
    P, L, seed = tr.forward(sc, loss="neg_min", want_seed=True)
    Pn = P.cpu().numpy()
    m = int(np.argmin(Pn))
    assert float(L) == -float(Pn[m])
    sd = seed.cpu().numpy()
    assert sd[m] == -1.0 and np.count_nonzero(sd) == 1
    g1 = tr.backward(sc, seed, reuse_forward=True)
    g0 = tr.backward(sc, seed, reuse_forward=False)
    # re-evaluation bounds P(r) for the contribution cut by its own wavefront's
    # running sum, so it may keep a few terms below 2^-24 P / C that the
    # forward dropped: equal to FP32 accuracy
    for a, b in zip(g0, g1):
        torch.testing.assert_close(a, b, rtol=1e-6, atol=1e-6 * float(b.abs().max()))
    from paper_2401_11882_amd import tracer as tr2
    tr2.set_cut(False)
    try:
        g1 = tr.backward(sc, seed, reuse_forward=False)
        tr.forward(sc, loss="neg_min", want_seed=True)
        g0 = tr.backward(sc, seed, reuse_forward=True)
    finally:
        tr2.set_cut(True)
    for a, b in zip(g0, g1):   # without the cut both paths sum the same terms: bitwise equal
        assert torch.equal(a, b)
    # deterministic: a second identical call is bitwise identical
    P2, L2, gtx2, gp2 = tr.forward_backward(sc, loss="neg_mean_log")
    P3, L3, gtx3, gp3 = tr.forward_backward(sc, loss="neg_mean_log")
    assert torch.equal(P2, P3) and torch.equal(gtx2, gtx3) and torch.equal(gp2, gp3)


def test_empty_receiver_set():
    tr = _tr3()
    s = WL.scene3d_room(9, 2, 16, 1, 100.0)
    sc = tr.Scene3(_dev(s.panels), _dev(s.tx), _dev(np.zeros((0, 3))), 1, 100.0)
    P, L, gtx, gp = tr.forward_backward(sc, loss="sum")
    assert P.numel() == 0 and float(L) == 0.0
    assert torch.count_nonzero(gtx) == 0 and torch.count_nonzero(gp) == 0


@pytest.mark.parametrize("alpha", [10.0, 100.0])
def test_panel_culling_changes_no_bit(alpha):
    """Culled (panel, leg) pairs are ones whose factor is exactly 1 in every
    lane: with culling off (the process-wide screen switch) every output is
    bitwise the same."""
    from paper_2401_11882_amd import tracer as tr
    tr3 = _tr3()
    s = WL.scene3d_room(9, 12, 16, 2, alpha, seed=21)
    sc = _scene(s)
    on = tr3.forward_backward(sc, loss="neg_mean_log")
    tr.set_screen(False)
    try:
        off = tr3.forward_backward(sc, loss="neg_mean_log")
    finally:
        tr.set_screen(True)
    for a, b in zip(on, off):
        assert torch.equal(a, b)


@pytest.mark.parametrize("alpha", [10.0, 100.0, 1000.0])
def test_contribution_cut_within_bound_3d(alpha):
    """3D contribution cut: the power stays within 2^-24 P(r) (+ FP32
    rounding) of the uncut power and never above it; gradients (tx, panels,
    receivers) agree to FP32 accuracy.  The overflow path of the contribution
    cache (re-evaluation) is covered too."""
    from paper_2401_11882_amd import tracer as tr
    tr3 = _tr3()
    s = WL.scene3d_room(9, 12, 16, 2, alpha, seed=21)
    sc = _scene(s)
    res = {}
    try:
        for on in (True, False):
            tr.set_cut(on)
            res[on] = [t.clone() for t in tr3.forward_backward(sc, loss="neg_mean_log", want_rx=True)]
        tr.set_cut(True)
        tr.set_cache_limit(1 << 16)   # most wavefronts overflow and re-evaluate
        res["reeval"] = [t.clone() for t in tr3.forward_backward(sc, loss="neg_mean_log", want_rx=True)]
    finally:
        tr.set_cut(True)
        tr.set_cache_limit(32 << 30)
    Pc, Pe = res[True][0].double(), res[False][0].double()
    assert bool((Pc <= Pe * (1 + 1e-6)).all())
    assert float(((Pe - Pc).abs() / Pe.clamp_min(1e-30)).max()) <= 2.0 ** -24 + 2e-6
    assert torch.equal(res["reeval"][0], res[True][0])
    for other in (res[False], res["reeval"]):
        for x, y in zip(res[True][2:], other[2:]):
            torch.testing.assert_close(x, y, rtol=1e-4, atol=1e-5 * float(y.abs().max()))


def test_maximum_panel_count_sampled():
    """DRT3_MAX_PANELS panels (room + 250 rectangles, four 64-panel batches in
    the culling masks), order <= 1, a 16 x 16 grid: sampled receivers and a
    sampled-loss gradient against the reference."""
    tr = _tr3()
    s = WL.scene3d_room(9, 250, 16, 1, 100.0, seed=77)
    assert s.n_panels == 256
    sc = _scene(s)
    P, L, seed = tr.forward(sc, loss="neg_mean_log", want_seed=True)
    idx = np.random.default_rng(3).choice(s.n_rx, 24, replace=False)
    P_o, kap = kappa3(s.panels, s.tx, s.rx[idx], 1, 100.0)
    PU.check_power(P.cpu().numpy()[idx], P_o, kap, "256 panels")
    w = np.zeros(s.n_rx, np.float32)
    w[idx[:12]] = 1.0
    gtx, gp = tr.backward(sc, seed * _dev(w), reuse_forward=False)
    gp_o, gt_o, _ = T3.vjp(s.panels, s.tx, s.rx[idx[:12]], 1, 100.0, seed.cpu().numpy()[idx[:12]])
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, "256 panels")
    # the adjoint from the recorded contributions and masks gives the same gradients
    P2, L2, seed2 = tr.forward(sc, loss="neg_mean_log", want_seed=True)
    g2 = tr.backward(sc, seed2 * _dev(w), reuse_forward=True)
    assert torch.equal(g2[0], gtx) and torch.equal(g2[1], gp)


def test_graph_capture_replay_matches_eager():
    """The 3D forward + adjoint captured once into a HIP graph and replayed
    with the transmitter moved between replays: every replay equals the eager
    call on the same inputs."""
    tr = _tr3()
    s = WL.scene3d_room(9, 6, 16, 2, 100.0, seed=5)
    pan, rx = _dev(s.panels), _dev(s.rx)
    tx = _dev(s.tx)
    sc = tr.Scene3(pan, tx, rx, 2, 100.0, grid_nx=16)
    out = (torch.empty(s.n_rx, device="cuda"), torch.empty(1, device="cuda"), torch.empty(3, device="cuda"),
           torch.empty(s.n_panels, 9, device="cuda"))
    tr.forward_backward(sc, loss="neg_mean_log", out=out)   # workspace allocated outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            tr.forward_backward(sc, loss="neg_mean_log", out=out)
    torch.cuda.synchronize()
    shifts = [(0.0, 0.0, 0.0), (0.05, -0.03, 0.02), (-0.1, 0.04, -0.05)]
    for i, d in enumerate(shifts):
        tx.copy_(_dev(s.tx) + _dev(np.array(d)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in out]
        _ = (tx * 2).sum().item()   # unrelated eager work between replays
        want = tr.forward_backward(sc, loss="neg_mean_log")
        for a, b in zip(got, want):
            assert torch.equal(a, b), f"replay {i}"


# --- hard-sigmoid smoothing (Eq. 5-6) ---------------------------------------

def _scene_hs(s, alpha):
    return _tr3().Scene3(_dev(s.panels), _dev(s.tx), _dev(s.rx), s.max_order, alpha, grid_nx=s.grid_n,
                         smoothing="hard_sigmoid")


def kappa3_hs(panels, tx, rx, K, alpha, runs=4, seed=0):
    rng = np.random.default_rng(seed)
    P0 = T3.power(panels, tx, rx, K, alpha, mode="hard_sigmoid")
    kap = np.zeros_like(P0)
    for _ in range(runs):
        P = T3.power(PU.perturb(panels, rng), PU.perturb(tx, rng), PU.perturb(rx, rng), K, alpha,
                     mode="hard_sigmoid")
        kap = np.maximum(kap, np.abs(P - P0))
    return P0, kap


@pytest.mark.parametrize("K", [0, 1, 2, 3])
@pytest.mark.parametrize("alpha", [10.0, 50.0])
def test_hard_sigmoid_room_scenes_all_orders(K, alpha):
    tr = _tr3()
    s = WL.scene3d_room(9, 2 if K < 3 else 0, 16, K, alpha, seed=50 + K)
    sc = _scene_hs(s, alpha)
    P, L, gtx, gp = tr.forward_backward(sc, loss="neg_mean_log")
    P_o, kap = kappa3_hs(s.panels, s.tx, s.rx, K, alpha)
    PU.check_power(P.cpu().numpy(), P_o, kap, f"3D hard K={K}")
    L_o = -np.mean(np.log(P_o + 1e-6))
    assert float(L) == pytest.approx(L_o, rel=1e-5, abs=1e-5 * float(np.mean(np.abs(np.log(P_o + 1e-6)))))
    g = -1.0 / (s.n_rx * (P_o + 1e-6))
    gp_o, gt_o, _ = T3.vjp(s.panels, s.tx, s.rx, K, alpha, g, mode="hard_sigmoid")
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, f"3D hard K={K}")


def test_hard_sigmoid_full_size_sampled():
    tr = _tr3()
    s = WL.scene3d_32()
    sc = _scene_hs(s, 100.0)
    P, L, seed = tr.forward(sc, loss="neg_mean_log", want_seed=True)
    rng = np.random.default_rng(8)
    idx = np.unique(np.concatenate([rng.choice(s.n_rx, 62, replace=False), [0, s.n_rx - 1]]))
    P_o, kap = kappa3_hs(s.panels, s.tx, s.rx[idx], 2, 100.0)
    PU.check_power(P.cpu().numpy()[idx], P_o, kap, "scene3d_32 hard")
    w = np.zeros(s.n_rx, np.float32)
    w[idx[:24]] = 1.0
    gtx, gp = tr.backward(sc, seed * _dev(w))
    gp_o, gt_o, _ = T3.vjp(s.panels, s.tx, s.rx[idx[:24]], 2, 100.0, seed.cpu().numpy()[idx[:24]],
                           mode="hard_sigmoid")
    PU.check_grads(gtx.cpu().numpy(), gp.cpu().numpy(), gt_o, gp_o, "scene3d_32 hard")


def test_hard_sigmoid_screen_and_culling_change_no_bit():
    from paper_2401_11882_amd import tracer as tr
    tr3 = _tr3()
    s = WL.scene3d_room(9, 12, 16, 2, 30.0, seed=23)
    sc = _scene_hs(s, 30.0)
    on = tr3.forward_backward(sc, loss="neg_mean_log")
    tr.set_screen(False)
    try:
        off = tr3.forward_backward(sc, loss="neg_mean_log")
    finally:
        tr.set_screen(True)
    for a, b in zip(on, off):
        assert torch.equal(a, b)
