"""Transmitter optimisation by gradient steps on the smoothed power map.

Sec. III frames the problem as minimising L = -F over parameters (here the
transmitter position) with a gradient method; Sec. VII optimises the
transmitter position.  One step = the fused forward + adjoint
(drt_forward_backward) followed by an Adam update of tx (drt_adam_tx), both
on the device; the step is captured once in a HIP graph and replayed, with
no host synchronisation until the end.  The per-step loss and transmitter
are recorded on the device.
"""
from __future__ import annotations

import torch

from . import tracer as tr


def optimize_tx(walls: torch.Tensor, tx0: torch.Tensor, rx: torch.Tensor, max_order: int, alpha: float,
                steps: int = 200, lr: float = 1e-2, grid_nx: int = 0, loss: str = "neg_mean_log",
                lo: float = 1e-3, hi: float = 1.0 - 1e-3, use_graph: bool = True, state=None):
    """Returns dict(tx [2], tx_hist [steps+1, 2], loss_hist [steps], state) (device tensors).

    loss_hist[i] is the loss at tx_hist[i]; tx_hist[i+1] is tx after step i.
    ``state`` (the dict returned by a previous call: Adam moments and step
    count) continues an earlier run instead of starting Adam afresh.
    """
    dev = tx0.device
    tx = tx0.detach().clone().float().contiguous()
    if state is None:
        state = {"m": torch.zeros(2, device=dev), "v": torch.zeros(2, device=dev),
                 "step": torch.zeros(1, dtype=torch.int32, device=dev)}
    m, v, step = state["m"], state["v"], state["step"]
    step0 = step.clone()
    tx_hist = torch.zeros(steps + 1, 2, device=dev)
    loss_hist = torch.zeros(steps, device=dev)
    tx_hist[0] = tx
    sc = tr.Scene(walls, tx, rx, max_order, alpha, grid_nx=grid_nx)
    out = (torch.empty(sc.n_rx, device=dev), torch.empty(1, device=dev), torch.empty(2, device=dev),
           torch.empty(sc.n_walls, 4, device=dev), None)

    def one_step():
        tr.forward_backward(sc, loss=loss, out=out)
        idx = (step - step0).long()
        loss_hist.index_copy_(0, idx, out[1])
        tr.adam_tx(tx, out[2], m, v, step, lr=lr, lo=lo, hi=hi)
        tx_hist.index_copy_(0, idx + 1, tx.view(1, 2))

    if not use_graph:
        for _ in range(steps):
            one_step()
        return {"tx": tx, "tx_hist": tx_hist, "loss_hist": loss_hist, "state": state}

    # workspace and kernels warmed outside the capture, then state reset
    tr.forward_backward(sc, loss=loss, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            one_step()
    torch.cuda.current_stream().wait_stream(side)
    # capture does not execute: state is still the initial one
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return {"tx": tx, "tx_hist": tx_hist, "loss_hist": loss_hist, "state": state}
