"""PyTorch-facing binding of the batched persistent launch (marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import DrtBatch, DrtBatchShape, DrtPlanConfig, check, lib
from .tracer import DEFAULT_DMIN, DEFAULT_LOG_EPS, _ptr, stream_handle


class BatchPlan:
    """Many scenes (walls, tx, receivers, alpha each) traced in one launch.

    ``scenes``: sequence of objects with ``walls`` [W,4], ``tx`` [2], ``rx``
    [R,2] (numpy float32), ``grid_n`` (0 if not a grid) and ``alpha``.
    """

    def __init__(self, scenes, max_order: int, device="cuda", d_min: float = DEFAULT_DMIN,
                 tune_cache: str | None = None, smoothing: str = "sigmoid"):
        self.device = torch.device(device)
        self.n_scenes = len(scenes)
        self.max_order = int(max_order)
        self.n_walls = np.array([s.walls.shape[0] for s in scenes], dtype=np.int32)
        self.n_rx = np.array([s.rx.shape[0] for s in scenes], dtype=np.int32)
        self.grid_nx = np.array([getattr(s, "grid_n", 0) or 0 for s in scenes], dtype=np.int32)
        self.wall_off = np.concatenate([[0], np.cumsum(self.n_walls)]).astype(np.int64)
        self.rx_off = np.concatenate([[0], np.cumsum(self.n_rx)]).astype(np.int64)
        W = np.concatenate([s.walls for s in scenes]).astype(np.float32) if self.wall_off[-1] else \
            np.zeros((0, 4), np.float32)
        self.walls = torch.tensor(W, device=self.device).reshape(-1, 4).contiguous()
        self.tx = torch.tensor(np.stack([s.tx for s in scenes]).astype(np.float32), device=self.device)
        self.rx = torch.tensor(np.concatenate([s.rx for s in scenes]).astype(np.float32),
                               device=self.device).reshape(-1, 2).contiguous()
        self.alpha = torch.tensor(np.array([s.alpha for s in scenes], dtype=np.float32), device=self.device)
        self.d_min = float(d_min)
        self.smoothing = _lib.SMOOTHING[smoothing]
        shape = DrtBatchShape(self.n_scenes,
                              self.n_walls.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              self.n_rx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              self.grid_nx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              self.max_order)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().drt_plan_create(ctypes.byref(shape), tune_cache.encode() if tune_cache else None,
                                        ctypes.byref(h)))
        self._h = h
        self.out = self._alloc()

    def _alloc(self):
        dev = self.device
        return (torch.empty(int(self.rx_off[-1]), dtype=torch.float32, device=dev),
                torch.empty(self.n_scenes, dtype=torch.float32, device=dev),
                torch.empty(self.n_scenes, 2, dtype=torch.float32, device=dev),
                torch.empty(int(self.wall_off[-1]), 4, dtype=torch.float32, device=dev))

    def _batch(self) -> DrtBatch:
        return DrtBatch(self.walls.data_ptr() if self.walls.numel() else None, self.tx.data_ptr(),
                        self.rx.data_ptr() if self.rx.numel() else None, self.alpha.data_ptr(), self.d_min,
                        self.smoothing)

    def run(self, loss: str = "neg_mean_log", log_eps: float = DEFAULT_LOG_EPS, stream=None):
        """(power [sum R], loss [S], grad_tx [S,2], grad_walls [sum W,4]) in the plan's own buffers.

        loss='none' computes the power maps only (the other outputs are left as they were)."""
        P, L, gtx, gw = self.out
        b = self._batch()
        check(lib().drt_batched_forward_backward(self._h, ctypes.byref(b), _lib.LOSS[loss], float(log_eps),
                                                 _ptr(P), _ptr(L), _ptr(gtx), _ptr(gw if gw.numel() else None),
                                                 stream_handle(stream)))
        return self.out

    def autotune(self, loss: str = "neg_mean_log", log_eps: float = DEFAULT_LOG_EPS, cache_path: str | None = None):
        P, L, gtx, gw = self.out
        b = self._batch()
        check(lib().drt_batched_autotune(self._h, ctypes.byref(b), _lib.LOSS[loss], float(log_eps), _ptr(P),
                                         _ptr(L), _ptr(gtx), _ptr(gw if gw.numel() else None),
                                         cache_path.encode() if cache_path else None, stream_handle()))
        return self.config()

    def config(self) -> dict:
        c = DrtPlanConfig()
        check(lib().drt_plan_get_config(self._h, ctypes.byref(c)))
        return {"nw": c.nw, "cchunk": c.cchunk, "blocks_per_cu": c.blocks_per_cu, "tile_w": c.tile_w}

    def set_config(self, nw=8, cchunk=1, blocks_per_cu=0, tile_w=8) -> None:
        c = DrtPlanConfig(nw, cchunk, blocks_per_cu, tile_w)
        check(lib().drt_plan_set_config(self._h, ctypes.byref(c)))

    def info(self) -> dict:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        check(lib().drt_plan_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"items": a.value, "path_evals": b.value, "cache_cap": c.value}

    def scene_slice(self, s: int):
        return (slice(int(self.rx_off[s]), int(self.rx_off[s + 1])),
                slice(int(self.wall_off[s]), int(self.wall_off[s + 1])))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().drt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
