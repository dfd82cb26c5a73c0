"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import math
import os

import pytest

from paper_2401_11882_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libdrt.so not built")

BOGUS = 0x7F0000001000  # never dereferenced: every call below fails validation first


def _scene(**kw):
    d = dict(walls_dev=BOGUS, n_walls=5, tx_dev=BOGUS, rx_dev=BOGUS, n_rx=1024, rx_grid_nx=32,
             max_order=1, alpha=100.0, smoothing=0, d_min=1e-3)
    d.update(kw)
    return _lib.DrtScene(**d)


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = _lib.header_symbols()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._SIGS), "binding signatures out of sync with include/drt.h"


def test_version_and_status_strings():
    L = _lib.lib()
    assert L.drt_abi_version() == 2
    for code in (0, -1, -2, -3, -4):
        assert L.drt_status_string(code)
    assert L.drt_status_string(-99) == b"unknown status"


def test_num_candidates():
    L = _lib.lib()
    c = ctypes.c_int64()
    for W, K, n in [(5, 1, 6), (68, 2, 4625), (36, 3, 45397), (0, 3, 1), (1, 3, 2), (2, 3, 7)]:
        assert L.drt_num_candidates(W, K, ctypes.byref(c)) == 0
        assert c.value == n
    assert L.drt_num_candidates(5, 4, ctypes.byref(c)) == _lib.DRT_EINVAL
    assert L.drt_num_candidates(-1, 1, ctypes.byref(c)) == _lib.DRT_EINVAL


def test_cache_limit_changes_workspace():
    L = _lib.lib()
    sc = _scene(n_walls=68, n_rx=65536, rx_grid_nx=256, max_order=2)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(a)) == 0
    assert L.drt_set_cache_limit(0) == 0
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(b)) == 0
    assert L.drt_set_cache_limit(32 << 30) == 0
    # full cache: 1024 tiles x 8 wavefronts x 579 entries x 260 bytes
    assert a.value - b.value >= 1024 * 8 * 579 * 260


def test_workspace_size_host_only():
    L = _lib.lib()
    n = ctypes.c_size_t()
    sc = _scene()
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == 0
    assert n.value > 0 and n.value % 256 == 0
    big = _scene(n_walls=68, n_rx=65536, rx_grid_nx=256, max_order=2)
    m = ctypes.c_size_t()
    assert L.drt_workspace_size(ctypes.byref(big), ctypes.byref(m)) == 0
    assert m.value > n.value


@pytest.mark.parametrize("field,value,code", [
    ("alpha", 0.0, _lib.DRT_EINVAL),
    ("alpha", -1.0, _lib.DRT_EINVAL),
    ("alpha", math.inf, _lib.DRT_EINVAL),
    ("alpha", math.nan, _lib.DRT_EINVAL),
    ("d_min", 0.0, _lib.DRT_EINVAL),
    ("max_order", 4, _lib.DRT_EINVAL),
    ("max_order", -1, _lib.DRT_EINVAL),
    ("n_walls", -1, _lib.DRT_EINVAL),
    ("n_walls", 4096, _lib.DRT_EINVAL),
    ("n_rx", -5, _lib.DRT_EINVAL),
    ("rx_grid_nx", 12, _lib.DRT_EINVAL),
    ("rx_grid_nx", 48, _lib.DRT_EINVAL),
    ("smoothing", 2, _lib.DRT_ENOTSUP),
    ("walls_dev", None, _lib.DRT_EINVAL),
    ("tx_dev", None, _lib.DRT_EINVAL),
])
def test_scene_validation(field, value, code):
    L = _lib.lib()
    sc = _scene(**{field: value})
    n = ctypes.c_size_t()
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == code
    assert L.drt_last_error()
    rc = L.drt_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, None, BOGUS, 1 << 30, None)
    assert rc == code


def test_call_validation_before_launch():
    L = _lib.lib()
    sc = _scene()
    n = ctypes.c_size_t()
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == 0
    # workspace missing / too small
    assert L.drt_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, None, None, n.value, None) == _lib.DRT_EWORKSPACE
    assert L.drt_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, None, BOGUS, n.value - 1, None) == _lib.DRT_EWORKSPACE
    # bad loss kind / eps
    assert L.drt_forward(ctypes.byref(sc), 7, 1e-6, BOGUS, None, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    assert L.drt_forward(ctypes.byref(sc), 2, 0.0, BOGUS, None, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    # missing outputs
    assert L.drt_forward(ctypes.byref(sc), 0, 1e-6, None, None, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    assert L.drt_backward(ctypes.byref(sc), BOGUS, 0, None, BOGUS, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    assert L.drt_backward(ctypes.byref(sc), None, 0, BOGUS, BOGUS, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    assert L.drt_backward(ctypes.byref(sc), BOGUS, 4, BOGUS, BOGUS, None, BOGUS, n.value, None) == _lib.DRT_EINVAL
    assert L.drt_set_cache_limit(-1) == _lib.DRT_EINVAL
    assert L.drt_forward_backward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, BOGUS, BOGUS, None, BOGUS, n.value,
                                  None) == _lib.DRT_EINVAL
    # adam arguments
    assert L.drt_adam_tx(BOGUS, BOGUS, BOGUS, BOGUS, BOGUS, 0.0, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == _lib.DRT_EINVAL
    assert L.drt_adam_tx(BOGUS, BOGUS, BOGUS, BOGUS, BOGUS, 1e-2, 1.0, 0.999, 1e-8, 0.0, 1.0, None) == _lib.DRT_EINVAL
    assert L.drt_adam_tx(BOGUS, BOGUS, BOGUS, BOGUS, None, 1e-2, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == _lib.DRT_EINVAL
    assert L.drt_adam_tx(BOGUS, BOGUS, BOGUS, BOGUS, BOGUS, 1e-2, 0.9, 0.999, 1e-8, 1.0, 0.0, None) == _lib.DRT_EINVAL
    assert L.drt_adam_points(0, BOGUS, BOGUS, BOGUS, BOGUS, BOGUS, 1e-2, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == _lib.DRT_EINVAL
    # schedule arguments
    assert L.drt_alpha_schedule(BOGUS, 1, 1.0, 100.0, BOGUS, 4, None) == _lib.DRT_EINVAL
    assert L.drt_alpha_schedule(BOGUS, 100, 0.0, 100.0, BOGUS, 4, None) == _lib.DRT_EINVAL
    assert L.drt_alpha_schedule(BOGUS, 100, 1.0, 100.0, BOGUS, 0, None) == _lib.DRT_EINVAL
    assert L.drt_alpha_schedule(None, 100, 1.0, 100.0, BOGUS, 4, None) == _lib.DRT_EINVAL
    # surrogate steps: a NULL handle, or a NULL row list, is rejected on the host
    assert L.drt_mlp_train_step(None, BOGUS, BOGUS, 64, 1e-3, None, None) == _lib.DRT_EINVAL
    assert L.drt_mlp_train_step_rows(None, BOGUS, BOGUS, BOGUS, 64, 1e-3, None, None) == _lib.DRT_EINVAL
    # the min loss needs a receiver; an unknown smoothing is not supported
    empty = _scene(n_rx=0, rx_dev=None, rx_grid_nx=0)
    assert L.drt_forward(ctypes.byref(empty), 3, 1e-6, None, BOGUS, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt_set_screen(2) == _lib.DRT_EINVAL
    assert L.drt_set_cut(-1) == _lib.DRT_EINVAL
    # launch config knob
    assert L.drt_set_launch_config(3, 0) == _lib.DRT_EINVAL
    assert L.drt_set_launch_config(0, -1) == _lib.DRT_EINVAL
    assert L.drt_set_launch_config(0, 0) == 0


def test_plan_create_validation():
    L = _lib.lib()
    h = ctypes.c_void_p()
    W = (ctypes.c_int32 * 2)(10, 12)
    R = (ctypes.c_int32 * 2)(64, 100)
    bad = (ctypes.c_int32 * 2)(10, -3)
    assert L.drt_plan_create(None, None, ctypes.byref(h)) == _lib.DRT_EINVAL
    assert L.drt_plan_create(ctypes.byref(_lib.DrtBatchShape(0, W, R, None, 2)), None, ctypes.byref(h)) == _lib.DRT_EINVAL
    assert L.drt_plan_create(ctypes.byref(_lib.DrtBatchShape(2, W, R, None, 4)), None, ctypes.byref(h)) == _lib.DRT_EINVAL
    assert L.drt_plan_create(ctypes.byref(_lib.DrtBatchShape(2, bad, R, None, 2)), None, ctypes.byref(h)) == _lib.DRT_EINVAL
    assert L.drt_plan_create(ctypes.byref(_lib.DrtBatchShape(2, W, None, None, 2)), None, ctypes.byref(h)) == _lib.DRT_EINVAL
    assert h.value is None
    assert L.drt_plan_destroy(None) == 0
    assert L.drt_batched_forward_backward(None, None, 2, 1e-6, None, None, None, None, None) == _lib.DRT_EINVAL
    assert L.drt_plan_get_config(None, None) == _lib.DRT_EINVAL


def _scene3(**kw):
    d = dict(panels_dev=BOGUS, n_panels=8, tx_dev=BOGUS, rx_dev=BOGUS, n_rx=1024, rx_grid_nx=32,
             max_order=2, alpha=100.0, smoothing=0, d_min=1e-3)
    d.update(kw)
    return _lib.Drt3Scene(**d)


@pytest.mark.parametrize("field,value,code", [
    ("alpha", 0.0, _lib.DRT_EINVAL),
    ("alpha", math.nan, _lib.DRT_EINVAL),
    ("d_min", -1.0, _lib.DRT_EINVAL),
    ("max_order", 4, _lib.DRT_EINVAL),
    ("n_panels", -1, _lib.DRT_EINVAL),
    ("n_panels", 257, _lib.DRT_EINVAL),
    ("n_rx", -1, _lib.DRT_EINVAL),
    ("rx_grid_nx", 12, _lib.DRT_EINVAL),
    ("smoothing", 2, _lib.DRT_ENOTSUP),
    ("panels_dev", None, _lib.DRT_EINVAL),
    ("tx_dev", None, _lib.DRT_EINVAL),
])
def test_scene3_validation(field, value, code):
    L = _lib.lib()
    sc = _scene3(**{field: value})
    n = ctypes.c_size_t()
    assert L.drt3_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == code
    assert L.drt_last_error()
    assert L.drt3_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, None, BOGUS, 1 << 30, None) == code
    assert L.drt3_backward(ctypes.byref(sc), BOGUS, 0, BOGUS, BOGUS, None, BOGUS, 1 << 30, None) == code
    assert L.drt3_forward_backward(ctypes.byref(sc), 2, 1e-6, BOGUS, None, BOGUS, BOGUS, None, BOGUS, 1 << 30,
                                   None) == code


def test_scene3_call_validation_before_launch():
    L = _lib.lib()
    sc = _scene3()
    n = ctypes.c_size_t()
    assert L.drt3_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == 0
    assert n.value > 0
    # the largest scene fits its accumulators in LDS
    assert L.drt3_workspace_size(ctypes.byref(_scene3(n_panels=256)), ctypes.byref(n)) == 0
    assert L.drt3_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, None, None, n.value, None) == _lib.DRT_EWORKSPACE
    assert L.drt3_forward(ctypes.byref(sc), 7, 1e-6, BOGUS, None, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_forward(ctypes.byref(sc), 2, 0.0, BOGUS, None, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_forward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, BOGUS, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_backward(ctypes.byref(sc), BOGUS, 4, BOGUS, BOGUS, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_backward(ctypes.byref(sc), BOGUS, 0, None, BOGUS, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_backward(ctypes.byref(sc), BOGUS, 0, BOGUS, None, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL
    assert L.drt3_forward_backward(ctypes.byref(sc), 0, 1e-6, BOGUS, None, BOGUS, BOGUS, None, BOGUS, 1 << 30,
                                   None) == _lib.DRT_EINVAL
    empty = _scene3(n_rx=0, rx_dev=None, rx_grid_nx=0)
    assert L.drt3_forward(ctypes.byref(empty), 3, 1e-6, None, BOGUS, None, BOGUS, 1 << 30, None) == _lib.DRT_EINVAL


def test_valu_peak_rejects_null_outputs():
    L = _lib.lib()
    d = ctypes.c_double()
    assert L.drt_valu_peak(None, ctypes.byref(d)) == _lib.DRT_EINVAL
    assert L.drt_valu_peak(ctypes.byref(d), None) == _lib.DRT_EINVAL


def test_noalloc_validation_before_any_device_call():
    """The allocation-free entry point checks its arguments and the scratch
    size on the host: these calls fail before the first HIP call."""
    L = _lib.lib()
    sc = _scene()
    # loss_kind NONE, NULL outputs
    assert L.drt_forward_backward_noalloc(ctypes.byref(sc), 0, 1e-6, BOGUS, None, BOGUS, BOGUS, None,
                                          None) == _lib.DRT_EINVAL
    assert L.drt_forward_backward_noalloc(ctypes.byref(sc), 2, 1e-6, None, None, BOGUS, BOGUS, None,
                                          None) == _lib.DRT_EINVAL
    assert L.drt_forward_backward_noalloc(ctypes.byref(sc), 2, 1e-6, BOGUS, None, None, BOGUS, None,
                                          None) == _lib.DRT_EINVAL
    assert L.drt_forward_backward_noalloc(None, 2, 1e-6, BOGUS, None, BOGUS, BOGUS, None, None) == _lib.DRT_EINVAL
    # gradient partials of 16,384 tiles x 4,098 columns exceed the 64 MiB scratch
    big = _scene(n_walls=1024, n_rx=1 << 20, rx_grid_nx=1024, max_order=1)
    assert L.drt_forward_backward_noalloc(ctypes.byref(big), 2, 1e-6, BOGUS, None, BOGUS, BOGUS, None,
                                          None) == _lib.DRT_EINVAL
    msg = L.drt_last_error().decode()
    assert "allocation-free" in msg and "drt_forward_backward" in msg


def test_receiver_grid_needs_a_row_length():
    """rx_dev == NULL selects the library's receiver grid, which needs rx_grid_nx."""
    L = _lib.lib()
    n = ctypes.c_size_t()
    sc = _scene(rx_dev=None, rx_grid_nx=0)
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == _lib.DRT_EINVAL
    sc = _scene(rx_dev=None, rx_grid_nx=32)
    assert L.drt_workspace_size(ctypes.byref(sc), ctypes.byref(n)) == 0
