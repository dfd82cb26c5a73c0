"""PyTorch-facing binding of the HIP tracer (argument marshalling only).

Every number is computed by the kernels in libdrt.so; this module checks
tensor types/devices, keeps one workspace per device and passes raw device
pointers and the current HIP stream through the C ABI.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import DrtScene, check, lib

DEFAULT_DMIN = 1e-3
DEFAULT_LOG_EPS = 1e-6


def _dev_f32(x: torch.Tensor, name: str, shape_tail=None) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device, got {x.device}")
    if x.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(x.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected [*, {', '.join(map(str, shape_tail))}]")
    return x


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def stream_handle(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Scene:
    """Device-resident scene description (walls [W,4], tx [2], rx [R,2]).

    rx=None with grid_nx, grid_ny > 0 leaves the receivers to the library:
    the cell centres of a grid_nx x grid_ny grid over [0,1]^2 (no receiver
    array is passed)."""

    def __init__(self, walls, tx, rx, max_order: int, alpha: float, d_min: float = DEFAULT_DMIN,
                 grid_nx: int = 0, smoothing: str = "sigmoid", grid_ny: int = 0):
        self.walls = _dev_f32(walls, "walls", (4,)) if walls.numel() else walls
        self.tx = _dev_f32(tx, "tx")
        if self.tx.numel() != 2:
            raise ValueError("tx must hold 2 floats")
        dev = self.tx.device
        if rx is None:
            if grid_nx <= 0 or grid_ny <= 0:
                raise ValueError("rx=None needs grid_nx > 0 and grid_ny > 0")
            self.rx = None
            self._n_rx = int(grid_nx) * int(grid_ny)
        else:
            self.rx = _dev_f32(rx, "rx", (2,))
            self._n_rx = int(self.rx.shape[0])
        for t, nm in ((self.walls, "walls"), (self.rx, "rx")):
            if t is not None and t.numel() and t.device != dev:
                raise ValueError(f"{nm} is on {t.device}, tx on {dev}")
        self.max_order = int(max_order)
        self.alpha = float(alpha)
        self.d_min = float(d_min)
        self.grid_nx = int(grid_nx)
        self.smoothing = _lib.SMOOTHING[smoothing]
        self.device = dev

    @property
    def n_walls(self):
        return int(self.walls.shape[0]) if self.walls.numel() else 0

    @property
    def n_rx(self):
        return self._n_rx

    def c_struct(self) -> DrtScene:
        return DrtScene(
            walls_dev=self.walls.data_ptr() if self.n_walls else None, n_walls=self.n_walls,
            tx_dev=self.tx.data_ptr(),
            rx_dev=self.rx.data_ptr() if (self.rx is not None and self.n_rx) else None, n_rx=self.n_rx,
            rx_grid_nx=self.grid_nx,
            max_order=self.max_order, alpha=self.alpha, smoothing=self.smoothing, d_min=self.d_min)


_WS: dict = {}


def workspace(sc: DrtScene, device) -> tuple[torch.Tensor, int]:
    n = ctypes.c_size_t(0)
    check(lib().drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)))
    key = (str(device),)
    buf = _WS.get(key)
    if buf is None or buf.numel() < n.value:
        buf = torch.empty(max(n.value, 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf, int(n.value)


def num_candidates(n_walls: int, max_order: int) -> int:
    c = ctypes.c_int64(0)
    check(lib().drt_num_candidates(int(n_walls), int(max_order), ctypes.byref(c)))
    return int(c.value)


def valu_peak() -> tuple[float, float]:
    """(sustained FP32 FMA TFLOP/s, v_exp_f32 1e12 lane-ops/s) of the current device (diagnostic)."""
    f, e = ctypes.c_double(0.0), ctypes.c_double(0.0)
    check(lib().drt_valu_peak(ctypes.byref(f), ctypes.byref(e)))
    return float(f.value), float(e.value)


def set_launch_config(nw: int = 0, cchunk: int = 0) -> None:
    check(lib().drt_set_launch_config(int(nw), int(cchunk)))


def set_cache_limit(nbytes: int) -> None:
    check(lib().drt_set_cache_limit(int(nbytes)))


def set_screen(enabled: bool) -> None:
    """Candidate screen on/off (process-wide; on by default)."""
    check(lib().drt_set_screen(1 if enabled else 0))


def set_cut(enabled: bool) -> None:
    """Contribution cut on/off (process-wide; on by default); see drt_set_cut."""
    check(lib().drt_set_cut(1 if enabled else 0))


def cache_lists(scene: Scene) -> list[list[int]]:
    """Per wavefront slot, the candidates the last seeded forward recorded as
    nonzero (None for a slot that overflowed); reads the shared workspace."""
    sc = scene.c_struct()
    ws, _ = workspace(sc, scene.device)
    v = [ctypes.c_int64(0) for _ in range(4)]
    check(lib().drt_cache_layout(ctypes.byref(sc), *[ctypes.byref(x) for x in v]))
    slots, cap, off_idx, off_n = (int(x.value) for x in v)
    if cap == 0:
        return []
    idx = ws[off_idx:off_idx + 4 * slots * cap].view(torch.int32).view(slots, cap).cpu()
    cnt = ws[off_n:off_n + 4 * slots].view(torch.int32).cpu()
    return [None if int(n) < 0 else idx[s, :int(n)].tolist() for s, n in enumerate(cnt)]


def forward(scene: Scene, loss: str = "none", log_eps: float = DEFAULT_LOG_EPS,
            want_seed: bool = False, stream=None):
    """P(r) [R]; plus the loss scalar (and dL/dP) when loss != 'none'."""
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    P = torch.empty(scene.n_rx, dtype=torch.float32, device=scene.device)
    L = torch.empty(1, dtype=torch.float32, device=scene.device) if loss != "none" else None
    seed = torch.empty_like(P) if (want_seed and loss != "none") else None
    check(lib().drt_forward(ctypes.byref(sc), _lib.LOSS[loss], float(log_eps), _ptr(P), _ptr(L),
                            _ptr(seed), _ptr(ws), nbytes, stream_handle(stream)))
    return P, L, seed


def forward_fermat(scene: Scene, loss: str = "none", log_eps: float = DEFAULT_LOG_EPS, max_iter: int = 16,
                   conv_eps: float = 1e-4, stream=None):
    """P(r) [R] (and the loss scalar) with Fermat path tracing in place of the
    image method (drt_forward_fermat; orders <= 2)."""
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    P = torch.empty(scene.n_rx, dtype=torch.float32, device=scene.device)
    L = torch.empty(1, dtype=torch.float32, device=scene.device) if loss != "none" else None
    check(lib().drt_forward_fermat(ctypes.byref(sc), int(max_iter), float(conv_eps), _lib.LOSS[loss],
                                   float(log_eps), _ptr(P), _ptr(L), _ptr(ws), nbytes, stream_handle(stream)))
    return P, L


def backward(scene: Scene, grad_power: torch.Tensor, want_rx: bool = False, reuse_forward: bool = False,
             stream=None):
    """(dL/dtx [2], dL/dwalls [W,4], dL/drx [R,2] or None) for a given dL/dP.

    reuse_forward=True starts from the contributions the last forward() on
    this same scene recorded in the shared workspace (see drt_backward)."""
    _dev_f32(grad_power, "grad_power")
    if grad_power.numel() != scene.n_rx:
        raise ValueError("grad_power must have one entry per receiver")
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    gtx = torch.empty(2, dtype=torch.float32, device=scene.device)
    gw = torch.empty(scene.n_walls, 4, dtype=torch.float32, device=scene.device)
    grx = torch.empty(scene.n_rx, 2, dtype=torch.float32, device=scene.device) if want_rx else None
    flags = _lib.DRT_BWD_REUSE_FORWARD if reuse_forward else 0
    check(lib().drt_backward(ctypes.byref(sc), _ptr(grad_power), flags, _ptr(gtx), _ptr(gw if scene.n_walls else None),
                             _ptr(grx), _ptr(ws), nbytes, stream_handle(stream)))
    return gtx, gw, grx


def forward_backward(scene: Scene, loss: str = "neg_mean_log", log_eps: float = DEFAULT_LOG_EPS,
                     want_rx: bool = False, out=None, stream=None):
    """Power map, loss, and its gradients in one call.

    ``out`` may hold preallocated tensors (P, L, gtx, gw, grx) to reuse, e.g.
    inside a captured HIP graph.
    """
    if loss == "none":
        raise ValueError("forward_backward needs a loss")
    sc = scene.c_struct()
    ws, nbytes = workspace(sc, scene.device)
    if out is None:
        dev = scene.device
        out = (torch.empty(scene.n_rx, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.float32, device=dev),
               torch.empty(2, dtype=torch.float32, device=dev),
               torch.empty(scene.n_walls, 4, dtype=torch.float32, device=dev),
               torch.empty(scene.n_rx, 2, dtype=torch.float32, device=dev) if want_rx else None)
    P, L, gtx, gw, grx = out
    check(lib().drt_forward_backward(ctypes.byref(sc), _lib.LOSS[loss], float(log_eps), _ptr(P), _ptr(L),
                                     _ptr(gtx), _ptr(gw if scene.n_walls else None), _ptr(grx),
                                     _ptr(ws), nbytes, stream_handle(stream)))
    return out


def forward_backward_noalloc(scene: Scene, loss: str = "neg_mean_log", log_eps: float = DEFAULT_LOG_EPS,
                             want_rx: bool = False, out=None, stream=None):
    """As forward_backward, through drt_forward_backward_noalloc: the library's
    per-device scratch array serves as the workspace (no workspace tensor).
    Calls that overlap on one device race; ``out`` as in forward_backward."""
    if loss == "none":
        raise ValueError("forward_backward needs a loss")
    sc = scene.c_struct()
    if out is None:
        dev = scene.device
        out = (torch.empty(scene.n_rx, dtype=torch.float32, device=dev),
               torch.empty(1, dtype=torch.float32, device=dev),
               torch.empty(2, dtype=torch.float32, device=dev),
               torch.empty(scene.n_walls, 4, dtype=torch.float32, device=dev),
               torch.empty(scene.n_rx, 2, dtype=torch.float32, device=dev) if want_rx else None)
    P, L, gtx, gw, grx = out
    check(lib().drt_forward_backward_noalloc(ctypes.byref(sc), _lib.LOSS[loss], float(log_eps), _ptr(P), _ptr(L),
                                             _ptr(gtx), _ptr(gw if scene.n_walls else None), _ptr(grx),
                                             stream_handle(stream)))
    return out


def adam_tx(tx, grad, m, v, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8, lo=1e-3, hi=1.0 - 1e-3,
            stream=None) -> None:
    for t, nm in ((tx, "tx"), (grad, "grad"), (m, "m"), (v, "v")):
        _dev_f32(t, nm)
    if step.dtype != torch.int32 or step.device.type != "cuda":
        raise ValueError("step must be an int32 GPU tensor")
    check(lib().drt_adam_tx(_ptr(tx), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), lr, b1, b2, eps, lo, hi,
                            stream_handle(stream)))


def adam_points(x, grad, m, v, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8, lo=1e-3, hi=1.0 - 1e-3,
                stream=None) -> None:
    """Adam + clamp on x [n, 2] (all points share the int32 step counter)."""
    for t, nm in ((x, "x"), (grad, "grad"), (m, "m"), (v, "v")):
        _dev_f32(t, nm)
        if t.shape != x.shape:
            raise ValueError(f"{nm} shape {tuple(t.shape)} differs from x {tuple(x.shape)}")
    if x.dim() != 2 or x.shape[1] != 2:
        raise ValueError("x must be [n, 2]")
    if step.dtype != torch.int32 or step.device.type != "cuda":
        raise ValueError("step must be an int32 GPU tensor")
    check(lib().drt_adam_points(int(x.shape[0]), _ptr(x), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), lr, b1, b2,
                                eps, lo, hi, stream_handle(stream)))


def alpha_schedule(step, n_iter: int, a_first: float, a_last: float, out: torch.Tensor, stream=None) -> None:
    """out[:] = a_first (a_last / a_first)^(min(step, n_iter-1) / (n_iter-1)), step read on the device."""
    _dev_f32(out, "out")
    if step.dtype != torch.int32 or step.device.type != "cuda":
        raise ValueError("step must be an int32 GPU tensor")
    check(lib().drt_alpha_schedule(_ptr(step), int(n_iter), float(a_first), float(a_last), _ptr(out),
                                   int(out.numel()), stream_handle(stream)))


class SmoothedPower(torch.autograd.Function):
    """P(r) as a differentiable function of (walls, tx, rx); adjoint in HIP."""

    @staticmethod
    def forward(ctx, walls, tx, rx, max_order, alpha, d_min=DEFAULT_DMIN, grid_nx=0):
        scene = Scene(walls.detach(), tx.detach(), rx.detach(), max_order, alpha, d_min, grid_nx)
        P, _, _ = forward(scene)
        ctx.scene = scene
        ctx.need_rx = rx.requires_grad
        return P

    @staticmethod
    def backward(ctx, gP):
        gtx, gw, grx = backward(ctx.scene, gP.contiguous().float(), want_rx=ctx.need_rx)
        return gw, gtx, grx, None, None, None, None


def smoothed_power(walls, tx, rx, max_order, alpha, d_min=DEFAULT_DMIN, grid_nx=0):
    return SmoothedPower.apply(walls, tx, rx, max_order, alpha, d_min, grid_nx)
