"""Host-side helpers of the study code that run without a GPU."""
import numpy as np
import torch

from paper_2401_11882_amd.surrogate import z_order_dev


def _morton_reference(ix: int, iy: int, bits: int) -> int:
    """Bit b of x goes to bit 2b, bit b of y to bit 2b + 1."""
    code = 0
    for b in range(bits):
        code |= ((ix >> b) & 1) << (2 * b)
        code |= ((iy >> b) & 1) << (2 * b + 1)
    return code


def test_z_order_interleaves_the_quantised_coordinates():
    rng = np.random.default_rng(3)
    p = rng.uniform(0.0, 1.0, (500, 2)).astype(np.float32)
    p[0] = (0.0, 0.0)
    p[1] = (1.0, 1.0)  # clamped to the last cell
    codes = z_order_dev(torch.tensor(p)).numpy()
    for (x, y), c in zip(p, codes):
        ix = min(int(np.float32(x) * np.float32(65536.0)), 65535)
        iy = min(int(np.float32(y) * np.float32(65536.0)), 65535)
        assert int(c) == _morton_reference(ix, iy, 16)


def test_z_order_keeps_sorted_tiles_compact():
    # 4096 uniform points in Z-order: blocks of 64 consecutive points cover a
    # small patch each, unlike blocks of the drawn order
    rng = np.random.default_rng(4)
    p = rng.uniform(0.0, 1.0, (4096, 2)).astype(np.float32)
    order = torch.argsort(z_order_dev(torch.tensor(p)), stable=True).numpy()
    tiles = p[order].reshape(64, 64, 2)
    extent = (tiles.max(axis=1) - tiles.min(axis=1)).mean()
    drawn = p.reshape(64, 64, 2)
    assert extent < 0.35 < (drawn.max(axis=1) - drawn.min(axis=1)).mean()
