"""ctypes loader for libdrt.so, the HIP library behind include/drt.h.

There is no CPU fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdrt.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "drt.h")

c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t

DRT_OK, DRT_EINVAL, DRT_EWORKSPACE, DRT_ENOTSUP, DRT_EHIP = 0, -1, -2, -3, -4
DRT_SIGMOID = 0
DRT_HARD_SIGMOID = 1
SMOOTHING = {"sigmoid": DRT_SIGMOID, "hard_sigmoid": DRT_HARD_SIGMOID}
DRT_BWD_REUSE_FORWARD = 1
LOSS = {"none": 0, "sum": 1, "neg_mean_log": 2, "neg_min": 3}


class DrtScene(ctypes.Structure):
    _fields_ = [
        ("walls_dev", c_void_p), ("n_walls", c_int32),
        ("tx_dev", c_void_p),
        ("rx_dev", c_void_p), ("n_rx", c_int32), ("rx_grid_nx", c_int32),
        ("max_order", c_int32), ("alpha", c_float), ("smoothing", c_int32), ("d_min", c_float),
    ]


class Drt3Scene(ctypes.Structure):
    _fields_ = [
        ("panels_dev", c_void_p), ("n_panels", c_int32),
        ("tx_dev", c_void_p),
        ("rx_dev", c_void_p), ("n_rx", c_int32), ("rx_grid_nx", c_int32),
        ("max_order", c_int32), ("alpha", c_float), ("smoothing", c_int32), ("d_min", c_float),
    ]


class DrtBatchShape(ctypes.Structure):
    _fields_ = [("n_scenes", c_int32), ("n_walls", ctypes.POINTER(c_int32)), ("n_rx", ctypes.POINTER(c_int32)),
                ("rx_grid_nx", ctypes.POINTER(c_int32)), ("max_order", c_int32)]


class DrtBatch(ctypes.Structure):
    _fields_ = [("walls_dev", c_void_p), ("tx_dev", c_void_p), ("rx_dev", c_void_p), ("alpha_dev", c_void_p),
                ("d_min", c_float), ("smoothing", c_int32)]


class DrtPlanConfig(ctypes.Structure):
    _fields_ = [("nw", c_int32), ("cchunk", c_int32), ("blocks_per_cu", c_int32), ("tile_w", c_int32)]


class DrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_SIGS = {
    "drt_abi_version": ([], c_int32),
    "drt_status_string": ([c_int32], ctypes.c_char_p),
    "drt_last_error": ([], ctypes.c_char_p),
    "drt_num_candidates": ([c_int32, c_int32, ctypes.POINTER(ctypes.c_int64)], c_int32),
    "drt_set_launch_config": ([c_int32, c_int32], c_int32),
    "drt_workspace_size": ([ctypes.POINTER(DrtScene), ctypes.POINTER(c_size_t)], c_int32),
    "drt_forward": ([ctypes.POINTER(DrtScene), c_int32, c_float, c_void_p, c_void_p, c_void_p,
                     c_void_p, c_size_t, c_void_p], c_int32),
    "drt_backward": ([ctypes.POINTER(DrtScene), c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_size_t, c_void_p], c_int32),
    "drt_set_cache_limit": ([ctypes.c_int64], c_int32),
    "drt_set_screen": ([c_int32], c_int32),
    "drt_set_cut": ([c_int32], c_int32),
    "drt_cache_layout": ([ctypes.POINTER(DrtScene), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], c_int32),
    "drt_forward_backward": ([ctypes.POINTER(DrtScene), c_int32, c_float, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "drt_forward_backward_noalloc": ([ctypes.POINTER(DrtScene), c_int32, c_float, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
    "drt_forward_fermat": ([ctypes.POINTER(DrtScene), c_int32, c_float, c_int32, c_float, c_void_p, c_void_p,
                            c_void_p, c_size_t, c_void_p], c_int32),
    "drt_adam_tx": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float,
                     c_float, c_float, c_float, c_void_p], c_int32),
    "drt_adam_points": ([c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float,
                         c_float, c_float, c_float, c_void_p], c_int32),
    "drt_alpha_schedule": ([c_void_p, c_int32, c_float, c_float, c_void_p, c_int32, c_void_p], c_int32),
    "drt_plan_create": ([ctypes.POINTER(DrtBatchShape), ctypes.c_char_p, ctypes.POINTER(c_void_p)], c_int32),
    "drt_plan_destroy": ([c_void_p], c_int32),
    "drt_plan_get_config": ([c_void_p, ctypes.POINTER(DrtPlanConfig)], c_int32),
    "drt_plan_set_config": ([c_void_p, ctypes.POINTER(DrtPlanConfig)], c_int32),
    "drt_plan_info": ([c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                       ctypes.POINTER(c_int32)], c_int32),
    "drt_batched_forward_backward": ([c_void_p, ctypes.POINTER(DrtBatch), c_int32, c_float, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p], c_int32),
    "drt_batched_autotune": ([c_void_p, ctypes.POINTER(DrtBatch), c_int32, c_float, c_void_p, c_void_p,
                              c_void_p, c_void_p, ctypes.c_char_p, c_void_p], c_int32),
    "drt_mlp_num_params": ([ctypes.POINTER(ctypes.c_int64)], c_int32),
    "drt_mlp_create": ([c_void_p, c_void_p, c_int32, ctypes.POINTER(c_void_p)], c_int32),
    "drt_mlp_destroy": ([c_void_p], c_int32),
    "drt_mlp_get_params": ([c_void_p, c_void_p], c_int32),
    "drt_mlp_set_params": ([c_void_p, c_void_p], c_int32),
    "drt_mlp_grads": ([c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p], c_int32),
    "drt_mlp_train_step": ([c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_float, c_void_p, c_void_p], c_int32),
    "drt_mlp_train_step_rows": ([c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_float, c_void_p,
                                 c_void_p], c_int32),
    "drt_mlp_forward": ([c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p], c_int32),
    "drt_mlp_scan": ([c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p], c_int32),
    "drt_log_targets": ([c_void_p, ctypes.c_int64, c_float, c_void_p, c_void_p], c_int32),
    "drt_valu_peak": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], c_int32),
    "drt3_workspace_size": ([ctypes.POINTER(Drt3Scene), ctypes.POINTER(c_size_t)], c_int32),
    "drt3_forward": ([ctypes.POINTER(Drt3Scene), c_int32, c_float, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_size_t, c_void_p], c_int32),
    "drt3_backward": ([ctypes.POINTER(Drt3Scene), c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                       c_void_p, c_size_t, c_void_p], c_int32),
    "drt3_forward_backward": ([ctypes.POINTER(Drt3Scene), c_int32, c_float, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
}

_lib = None


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drt3?_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2401_11882_amd.build`")
        # torch first: its HIP runtime (same soname) is then the one the library binds to
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != DRT_OK:
        L = lib()
        raise DrtError(rc, f"{L.drt_status_string(rc).decode()}: {L.drt_last_error().decode()}")
