"""Pins of the FP64 surrogate reference (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2401_11882_amd import workloads as WL


def _params():
    layers = WL.mlp_init(0)
    hidden = [(W.astype(np.float64), b.astype(np.float64)) for W, b in layers[:-1]]
    hw, hb = layers[-1]
    return M.flatten(hidden, hw[:, 0], hb)


def test_parameter_count_and_layout():
    lay, hw, hb, n = M.layout()
    assert n == 296449
    assert [fi for _, fi, _ in lay] == [128, 256, 256, 256, 256]
    p = _params()
    assert p.size == n
    Ws, bs, w5, b5 = M.unflatten(p)
    np.testing.assert_array_equal(Ws[0], WL.mlp_init(0)[0][0])


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(20000).astype(np.float32) * 10
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x.astype(np.float64)), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_features_closed_form():
    B = WL.fourier_matrix(0)
    v = np.zeros((1, 4))
    X = M.features(v, B)
    np.testing.assert_allclose(X[0, :64], 0.0, atol=1e-15)
    np.testing.assert_allclose(X[0, 64:], 1.0, atol=1e-15)
    v = np.array([[0.25, 0.0, 0.0, 0.0]])
    Bu = np.zeros((64, 4)); Bu[:, 0] = np.arange(64)
    X = M.features(v, Bu)   # sin(2 pi f / 4)
    np.testing.assert_allclose(X[0, :64], np.sin(np.pi * np.arange(64) / 2), atol=1e-12)


def test_manual_backward_matches_autograd_and_fd():
    rng = np.random.default_rng(1)
    B = WL.fourier_matrix(0).astype(np.float64)
    p = _params()
    v = rng.uniform(0, 1, (64, 4))
    y = rng.standard_normal(64)
    loss, g = M.loss_and_grads(v, y, B, p)
    # autograd on the same definition
    lay, hw, hb, n = M.layout()
    pt = torch.tensor(p, requires_grad=True)
    X = torch.tensor(M.features(v, B))
    for o, fi, bo in lay:
        X = torch.relu(X @ pt[o:o + fi * 256].reshape(fi, 256) + pt[bo:bo + 256])
    yh = X @ pt[hw:hw + 256] + pt[hb]
    lt = torch.mean((yh - torch.tensor(y)) ** 2)
    lt.backward()
    assert float(lt) == pytest.approx(loss, rel=1e-13)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(g).max())
    # central differences on a few coordinates
    for i in rng.choice(n, 8, replace=False):
        h = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[i] += h; pm[i] -= h
        fd = (M.loss_and_grads(v, y, B, pp)[0] - M.loss_and_grads(v, y, B, pm)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(10)
    m = np.zeros(10); v = np.zeros(10)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-3)
    for t in range(1, 6):
        g = rng.standard_normal(10)
        p, m, v = M.adam(p, g, m, v, t, 3e-3)
        opt.zero_grad(); pt.grad = torch.tensor(g); opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12)


def test_rounded_path_stays_close_to_exact():
    rng = np.random.default_rng(3)
    B = WL.fourier_matrix(0).astype(np.float64)
    p = _params()
    v = rng.uniform(0, 1, (256, 4))
    y0, _ = M.forward(v, B, p)
    y1, _ = M.forward(v, B, p, round_bf16=True)
    assert np.max(np.abs(y1 - y0)) < 0.05 * (1 + np.max(np.abs(y0)))
