"""Fermat path tracing on the GPU (drt_forward_fermat, Sec. V-B) against the
FP64 Fermat oracle (oracle/fermat.py), and against the GPU image method on
receivers where the two path finders agree in exact arithmetic."""
import numpy as np
import pytest
import torch

from oracle import fermat as FM
from oracle import tracer as T
from paper_2401_11882_amd import workloads as WL

import parity_util as PU

pytestmark = pytest.mark.gpu


def _tr():
    from paper_2401_11882_amd import tracer
    return tracer


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _scene(walls, tx, rx, K, alpha, grid_n=0, smoothing="sigmoid"):
    return _tr().Scene(_dev(walls), _dev(tx), _dev(rx), K, alpha, grid_nx=grid_n, smoothing=smoothing)


def _kappa(walls, tx, rx, K, alpha, mode="sigmoid", runs=4, seed=0, P0=None):
    """As parity_util.kappa, for the Fermat oracle: the largest change of P(r)
    over runs with every FP32 input moved by +-4 ulps of max(|x|, 1/2)."""
    rng = np.random.default_rng(seed)
    if P0 is None:
        P0 = FM.power(walls, tx, rx, K, alpha, mode=mode)
    kap = np.zeros_like(P0)
    for _ in range(runs):
        P = FM.power(PU.perturb(walls, rng), PU.perturb(tx, rng), PU.perturb(rx, rng), K, alpha, mode=mode)
        kap = np.maximum(kap, np.abs(P - P0))
    return P0, kap


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("alpha", [10.0, 100.0, 1000.0])
def test_small_scene_full_map(K, alpha):
    """Box + 4 segments, 16x16 receivers: every receiver against the oracle."""
    s = WL.scene_random_box(2, 4, 16, K, alpha, seed=13)
    P, L = _tr().forward_fermat(_scene(s.walls, s.tx, s.rx, K, alpha, s.grid_n), loss="neg_mean_log")
    P_o, kap = _kappa(s.walls, s.tx, s.rx, K, alpha)
    st = PU.check_power(P.cpu().numpy(), P_o, kap, f"fermat K={K} alpha={alpha}")
    print(f"fermat K={K} alpha={alpha}", st, flush=True)
    assert float(L) == pytest.approx(-np.mean(np.log(P_o + 1e-6)), rel=1e-5, abs=1e-5)


def test_single_segment_scene_hard_sigmoid():
    s = WL.scene_single_segment()
    P, _ = _tr().forward_fermat(_scene(s.walls, s.tx, s.rx, 1, 50.0, s.grid_n, "hard_sigmoid"))
    P_o, kap = _kappa(s.walls, s.tx, s.rx, 1, 50.0, mode="hard_sigmoid")
    st = PU.check_power(P.cpu().numpy(), P_o, kap, "fermat hard sigmoid")
    print("fermat hard sigmoid", st, flush=True)


def test_benchmark_scene_sampled():
    """Box + 64 segments, 256^2 receivers, order <= 2, alpha 100: 32 receivers
    (16 consecutive receivers of one row plus 16 random ones) against the oracle."""
    s = WL.scene_64(alpha=100.0)
    P, _ = _tr().forward_fermat(_scene(s.walls, s.tx, s.rx, 2, 100.0, s.grid_n))
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(16) + 256 * 100 + 64, rng.choice(s.n_rx, 16, replace=False)]))
    P_o, kap = _kappa(s.walls, s.tx, s.rx[idx], 2, 100.0, runs=2)
    st = PU.check_power(P.cpu().numpy()[idx], P_o, kap, "fermat benchmark scene")
    print("fermat benchmark scene", st, flush=True)


def test_equals_image_method_where_the_finders_agree():
    """On receivers where the oracle's Fermat and image-method powers agree to
    1e-12 (every contributing path is a true reflection away from the side
    test's band, or the two smoothings give the same factors), the GPU's two
    finders agree to FP32 accuracy."""
    alpha = 1000.0
    s = WL.scene_random_box(2, 4, 32, 2, alpha, seed=17)
    sc = _scene(s.walls, s.tx, s.rx, 2, alpha, s.grid_n)
    Pf, _ = _tr().forward_fermat(sc)
    Pi, _, _ = _tr().forward(sc)
    Pf_o = FM.power(s.walls, s.tx, s.rx, 2, alpha)
    Pi_o = T.power(s.walls, s.tx, s.rx, 2, alpha)
    same = np.abs(Pf_o - Pi_o) <= 1e-12 * Pi_o
    assert same.mean() > 0.5, same.mean()
    _, kap = PU.kappa(s.walls, s.tx, s.rx[same], 2, alpha, P0=Pi_o[same])
    a, b = Pf.cpu().numpy()[same].astype(np.float64), Pi.cpu().numpy()[same].astype(np.float64)
    bad = np.abs(a - b) > 2e-5 * b + 4 * kap + 1e-30
    assert not bad.any(), (np.nonzero(bad)[0][:5], a[bad][:5], b[bad][:5])
    print(f"finders agree on {same.sum()} of {same.size} receivers; max rel diff {np.max(np.abs(a - b) / b):.2e}",
          flush=True)


def test_edge_cases():
    tr = _tr()
    from paper_2401_11882_amd import _lib
    s = WL.scene_random_box(2, 3, 4, 2, 100.0, seed=2)
    # order 3 is not offered
    with pytest.raises(_lib.DrtError) as ei:
        tr.forward_fermat(_scene(s.walls, s.tx, s.rx, 3, 100.0))
    assert ei.value.code == _lib.DRT_ENOTSUP
    # empty receivers
    P, L = tr.forward_fermat(tr.Scene(_dev(s.walls), _dev(s.tx), torch.zeros(0, 2, device="cuda"), 2, 100.0),
                             loss="sum")
    assert P.numel() == 0 and float(L) == 0.0
    # ragged receivers and a zero-length wall
    walls = np.concatenate([s.walls, [[0.5, 0.5, 0.5, 0.5]]]).astype(np.float32)
    rx = WL.random_points(2, 9, 100)
    P, _ = tr.forward_fermat(_scene(walls, s.tx, rx, 2, 100.0))
    assert torch.isfinite(P).all()
    P_o, kap = _kappa(walls, s.tx, rx, 2, 100.0, runs=2)
    PU.check_power(P.cpu().numpy(), P_o, kap, "fermat ragged + zero-length wall")
