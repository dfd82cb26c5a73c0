"""PyTorch-facing binding of the 3D tracer (argument marshalling only).

Scenes of planar parallelogram panels (corner a and its neighbours b, c);
every number is computed by the kernels in libdrt.so behind the drt3_* calls.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import Drt3Scene, check, lib
from .tracer import DEFAULT_DMIN, DEFAULT_LOG_EPS, _dev_f32, _ptr, stream_handle


class Scene3:
    """Device-resident 3D scene: panels [P,9] = (a, b, c), tx [3], rx [R,3]."""

    def __init__(self, panels, tx, rx, max_order: int, alpha: float, d_min: float = DEFAULT_DMIN,
                 grid_nx: int = 0, smoothing: str = "sigmoid"):
        self.panels = _dev_f32(panels, "panels", (9,)) if panels.numel() else panels
        self.tx = _dev_f32(tx, "tx")
        if self.tx.numel() != 3:
            raise ValueError("tx must hold 3 floats")
        self.rx = _dev_f32(rx, "rx", (3,))
        dev = self.tx.device
        for t, nm in ((self.panels, "panels"), (self.rx, "rx")):
            if t.numel() and t.device != dev:
                raise ValueError(f"{nm} is on {t.device}, tx on {dev}")
        self.max_order = int(max_order)
        self.alpha = float(alpha)
        self.d_min = float(d_min)
        self.grid_nx = int(grid_nx)
        self.smoothing = _lib.SMOOTHING[smoothing]
        self.device = dev

    @property
    def n_panels(self):
        return int(self.panels.shape[0]) if self.panels.numel() else 0

    @property
    def n_rx(self):
        return int(self.rx.shape[0])

    def c_struct(self) -> Drt3Scene:
        return Drt3Scene(
            panels_dev=self.panels.data_ptr() if self.n_panels else None, n_panels=self.n_panels,
            tx_dev=self.tx.data_ptr(),
            rx_dev=self.rx.data_ptr() if self.n_rx else None, n_rx=self.n_rx, rx_grid_nx=self.grid_nx,
            max_order=self.max_order, alpha=self.alpha, smoothing=self.smoothing, d_min=self.d_min)


_WS: dict = {}


def workspace(sc: Drt3Scene, device) -> tuple[torch.Tensor, int]:
    n = ctypes.c_size_t(0)
    check(lib().drt3_workspace_size(ctypes.byref(sc), ctypes.byref(n)))
    key = (str(device),)
    buf = _WS.get(key)
    if buf is None or buf.numel() < n.value:
        buf = torch.empty(max(n.value, 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf, int(n.value)


def forward(scene: Scene3, loss: str = "none", log_eps: float = DEFAULT_LOG_EPS, want_seed: bool = False,
            stream=None):
    """P(r) [R]; plus the loss scalar (and dL/dP) when loss != 'none'."""
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    P = torch.empty(scene.n_rx, dtype=torch.float32, device=scene.device)
    L = torch.empty(1, dtype=torch.float32, device=scene.device) if loss != "none" else None
    seed = torch.empty_like(P) if (want_seed and loss != "none") else None
    check(lib().drt3_forward(ctypes.byref(sc), _lib.LOSS[loss], float(log_eps), _ptr(P), _ptr(L), _ptr(seed),
                             _ptr(ws), nbytes, stream_handle(stream)))
    return P, L, seed


def backward(scene: Scene3, grad_power: torch.Tensor, reuse_forward: bool = False, want_rx: bool = False,
             stream=None):
    """(dL/dtx [3], dL/dpanels [P,9]) for a given dL/dP, and dL/drx [R,3] when want_rx."""
    _dev_f32(grad_power, "grad_power")
    if grad_power.numel() != scene.n_rx:
        raise ValueError("grad_power must have one entry per receiver")
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    gtx = torch.empty(3, dtype=torch.float32, device=scene.device)
    gp = torch.empty(scene.n_panels, 9, dtype=torch.float32, device=scene.device)
    grx = torch.empty(scene.n_rx, 3, dtype=torch.float32, device=scene.device) if want_rx else None
    flags = _lib.DRT_BWD_REUSE_FORWARD if reuse_forward else 0
    check(lib().drt3_backward(ctypes.byref(sc), _ptr(grad_power), flags, _ptr(gtx),
                              _ptr(gp if scene.n_panels else None), _ptr(grx), _ptr(ws), nbytes,
                              stream_handle(stream)))
    return (gtx, gp, grx) if want_rx else (gtx, gp)


def forward_backward(scene: Scene3, loss: str = "neg_mean_log", log_eps: float = DEFAULT_LOG_EPS, out=None,
                     want_rx: bool = False, stream=None):
    """(P, L, dL/dtx, dL/dpanels), plus dL/drx [R,3] when want_rx, in one call; ``out`` may hold
    those tensors preallocated."""
    if loss == "none":
        raise ValueError("forward_backward needs a loss")
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    if out is None:
        dev = scene.device
        out = (torch.empty(scene.n_rx, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.float32, device=dev),
               torch.empty(3, dtype=torch.float32, device=dev),
               torch.empty(scene.n_panels, 9, dtype=torch.float32, device=dev))
        if want_rx:
            out = out + (torch.empty(scene.n_rx, 3, dtype=torch.float32, device=dev),)
    P, L, gtx, gp = out[:4]
    grx = out[4] if len(out) > 4 else None
    check(lib().drt3_forward_backward(ctypes.byref(sc), _lib.LOSS[loss], float(log_eps), _ptr(P), _ptr(L),
                                      _ptr(gtx), _ptr(gp if scene.n_panels else None), _ptr(grx), _ptr(ws),
                                      nbytes, stream_handle(stream)))
    return out
