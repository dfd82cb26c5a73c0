"""BF16-MFMA surrogate kernels vs the FP64 reference (rounded where the GPU stores BF16)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2401_11882_amd import workloads as WL

import parity_util as PU

pytestmark = pytest.mark.gpu


def _S():
    from paper_2401_11882_amd import surrogate
    return surrogate


def _net(max_batch=4096):
    S = _S()
    return S, S.Surrogate(WL.fourier_matrix(0), S.init_params(0), max_batch=max_batch)


def _inputs(n, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return v, y


# Tolerance model.  Both sides round the same quantities to BF16, but from
# FP32 (GPU) or FP64 (reference) values, so an occasional BF16 rounding lands
# one step apart and propagates.  The scale of that effect is measured on the
# reference itself: the same inputs moved by one FP32 ulp (random sign) give a
# second reference run, and the GPU must stay within a small multiple of that
# spread (plus an FP32-accumulation floor).

def _ulp_perturbed(v, seed):
    rng = np.random.default_rng(seed)
    return (v.astype(np.float64) + rng.choice([-1.0, 1.0], v.shape) * np.spacing(v.astype(np.float32))).astype(np.float32)


def test_forward_matches_reference():
    S, net = _net()
    v, _ = _inputs(4096 + 64 * 3 + 5)          # several chunks and a ragged tail
    yg = net.forward(torch.tensor(v).cuda()).cpu().numpy().astype(np.float64)
    B, p = WL.fourier_matrix(0), S.init_params(0)
    yo, _ = M.forward(v, B, p, round_bf16=True)
    yp, _ = M.forward(_ulp_perturbed(v, 7), B, p, round_bf16=True)
    scale = 1 + np.abs(yo).max()
    e_g, e_p = np.abs(yg - yo), np.abs(yp - yo)
    assert np.median(e_g) < 1e-5 * scale
    thr = 1e-4 * scale
    assert np.mean(e_g > thr) <= 3 * np.mean(e_p > thr) + 0.01, (np.mean(e_g > thr), np.mean(e_p > thr))
    assert e_g.max() <= 3 * e_p.max() + thr, (e_g.max(), e_p.max())
    net.close()


def test_gradients_match_reference():
    S, net = _net()
    v, y = _inputs(2048, seed=1)
    g, loss = net.grads(torch.tensor(v).cuda(), torch.tensor(y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    B, p = WL.fourier_matrix(0), S.init_params(0)
    lo, go = M.loss_and_grads(v, y, B, p, round_bf16=True)
    _, gp = M.loss_and_grads(_ulp_perturbed(v, 8), y, B, p, round_bf16=True)
    assert float(loss) == pytest.approx(lo, rel=1e-4)
    lay, hw, hb, n = M.layout()
    blocks = [(o, o + fi * 256) for o, fi, _ in lay] + [(bo, bo + 256) for _, _, bo in lay] + [(hw, hw + 256), (hb, hb + 1)]
    for a, b in blocks:
        e_g, e_p = PU.rel_l2(g[a:b], go[a:b]), PU.rel_l2(gp[a:b], go[a:b])
        print(f"block [{a},{b}): gpu {e_g:.2e} reference spread {e_p:.2e}")
        assert e_g <= 3 * e_p + 2e-3, (a, b, e_g, e_p)
    net.close()


def test_train_step_is_adam_on_the_gradients():
    """Three consecutive steps, each against torch's Adam given the library's
    gradients at the current parameters (the bias corrections use the device
    step count, which the training pass advances)."""
    S, net = _net()
    v, y = _inputs(1024, seed=2)
    vd, yd = torch.tensor(v).cuda(), torch.tensor(y).cuda()
    pt = torch.tensor(net.params().astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3)
    for step in range(3):
        g, _ = net.grads(vd, yd)
        net.train_step(vd, yd, 1e-3)
        pt.grad = torch.tensor(g.cpu().numpy().astype(np.float64))
        opt.step()
        np.testing.assert_allclose(net.params().astype(np.float64), pt.detach().numpy(), rtol=1e-5, atol=1e-7,
                                   err_msg=f"after step {step + 1}")
    net.close()


def test_train_step_on_row_indices_equals_gathered_rows():
    """drt_mlp_train_step_rows on an index list = drt_mlp_train_step on the gathered rows, bitwise."""
    S, a = _net()
    _, b = _net()
    v, y = _inputs(3000, seed=4)
    vd, yd = torch.tensor(v).cuda(), torch.tensor(y).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    rows = torch.randperm(3000, device="cuda", generator=g)[:1024].to(torch.int32).contiguous()
    for step in range(2):
        la = a.train_step(vd, yd, 1e-3, rows=rows).clone()
        lb = b.train_step(vd.index_select(0, rows.long()).contiguous(),
                          yd.index_select(0, rows.long()).contiguous(), 1e-3).clone()
        assert torch.equal(la, lb), (step, float(la), float(lb))
    np.testing.assert_array_equal(a.params(), b.params())
    a.close()
    b.close()


@pytest.mark.parametrize("n_rx", [1024, 300, 100, 1])
def test_scan_is_mean_of_forward(n_rx):
    # 1024: whole 128-row tiles per transmitter (per-tile sums); 300, 100, 1:
    # tiles that span 2, 3 or 128 transmitters (per-row outputs, then means)
    S, net = _net(max_batch=8192)
    rx_np = WL.rx_grid(32)[:n_rx]
    tx = torch.tensor(WL.rx_grid(4)).cuda()          # 16 transmitters
    rx = torch.tensor(rx_np).cuda()
    F = net.scan(tx, rx).cpu().numpy()
    pairs = torch.cat([tx.repeat_interleave(rx.shape[0], 0), rx.repeat(tx.shape[0], 1)], 1).contiguous()
    yh = net.forward(pairs).cpu().numpy().reshape(16, n_rx)
    np.testing.assert_allclose(F, yh.astype(np.float64).mean(1), rtol=1e-5, atol=1e-6)
    # and against the reference for two transmitters
    for t in (0, 9):
        v = np.concatenate([np.repeat(WL.rx_grid(4)[t:t + 1], n_rx, 0), rx_np], 1)
        yo, _ = M.forward(v, WL.fourier_matrix(0), S.init_params(0), round_bf16=True)
        assert F[t] == pytest.approx(yo.mean(), abs=1e-3 * (1 + abs(yo.mean())))
    net.close()


def test_datagen_targets_match_tracer():
    """Training data: log(P + eps) from the batched tracer equals the single-scene tracer's."""
    S = _S()
    from paper_2401_11882_amd import tracer as tr
    s = WL.scene_64()
    v, y, txs = S.generate_data(s.walls, 8, 512, 100.0, 2, seed=3)
    assert v.shape == (8 * 512, 4) and y.shape == (8 * 512,)
    vn = v.cpu().numpy()
    for i in (0, 7):
        rows = slice(i * 512, (i + 1) * 512)
        sc = tr.Scene(torch.tensor(s.walls).cuda(), torch.tensor(txs[i]).cuda(), v[rows, 2:4].contiguous(), 2, 100.0)
        P, _, _ = tr.forward(sc)
        np.testing.assert_allclose(y[rows].cpu().numpy(), np.log(P.cpu().numpy().astype(np.float64) + 1e-6),
                                   rtol=1e-5, atol=1e-5)
        np.testing.assert_array_equal(vn[rows, 0:2], np.repeat(txs[i:i + 1], 512, 0))


def test_datagen_targets_match_oracle():
    """Training data against the FP64 oracle: y = log(P + 1e-6) of the batched
    forward (scattered receivers, the 68-wall scene, order <= 2, alpha 100)
    for 2 transmitters x 256 receivers, within the image of the power bound
    through the log plus FP32 rounding of the log."""
    S = _S()
    from oracle import tracer as T
    s = WL.scene_64()
    v, y, txs = S.generate_data(s.walls, 4, 256, 100.0, 2, seed=7)
    vn, yn = v.cpu().numpy(), y.cpu().numpy().astype(np.float64)
    for i in (0, 3):
        rows = slice(i * 256, (i + 1) * 256)
        rx = vn[rows, 2:4]
        P_o, kap = PU.kappa(s.walls, txs[i], rx, 2, 100.0)
        y_o = np.log(P_o + 1e-6)
        bound = (PU.REL * P_o + 2 * kap + PU.ABS_FLOOR) / (P_o + 1e-6) + 4e-7 * np.maximum(1.0, np.abs(y_o))
        err = np.abs(yn[rows] - y_o)
        assert np.all(err <= bound), (i, np.nonzero(err > bound)[0][:5], err.max())
        print(f"tx {i}: max |y - y_oracle| {err.max():.2e}, median {np.median(err):.2e}", flush=True)


def test_training_reduces_loss():
    S = _S()
    s = WL.scene_64()
    v, y, _ = S.generate_data(s.walls, 64, 1024, 100.0, 2, seed=4)
    net = S.Surrogate(WL.fourier_matrix(0), S.init_params(0), max_batch=8192)
    hist = S.train(net, v, y, epochs=12, batch=8192, lr=2e-3)
    assert hist[-1] < 0.5 * hist[0], hist
    net.close()


def test_surrogate_guided_search_gain():
    """Full study on the 64-segment scene: 1e7 tracer-generated samples, BF16
    training, then reaching F >= F* + log 0.99 with and without the surrogate."""
    S = _S()
    r = S.experiment(seed=0)
    print({k: r[k] for k in ("datagen_s", "train_s", "heldout_rmse", "heldout_max_abs", "F_star", "speedup",
                             "speedup_lower_bound", "exact_step_ratio", "surrogate_end_to_end_s",
                             "break_even_searches")}, r["plain"], r["surrogate"])
    assert r["samples"] == 2442 * 4096
    assert r["heldout_rmse"] < 0.5 * r["target_std"]
    assert r["heldout_max_abs"] >= r["heldout_rmse"]
    assert r["surrogate"]["reached"]
    # the surrogate path needs fewer exact-tracer steps and less time than the plain one
    assert r["exact_step_ratio"] > 1.0
    sp = r["speedup"] if r["speedup"] is not None else r["speedup_lower_bound"]
    assert sp > 1.0
    # its estimate of the objective is reported in log-power units at both points
    assert np.isfinite(r["surrogate"]["abs_err_top"]) and np.isfinite(r["surrogate"]["abs_err_best"])
