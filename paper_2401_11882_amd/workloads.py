"""Seeded synthetic inputs for the smoothed image-method tracer.

This module only draws numbers: scene geometry, transmitter positions,
receiver grids and the random tensors of the learned surrogate. It holds none
of the tracer's arithmetic, so both the FP64 oracle and the HIP path read the
exact same FP32 arrays from it.

Scene family (the paper's experiments use small synthetic 2D layouts, Sec. VI
and Sec. VII; no public dataset exists, so these stand in):

* The unit-square box is always present as walls 0..3 (bottom, right, top,
  left), each running counter-clockwise.
* Interior segments: centre ~ U[0,1]^2, length ~ U(0.05, 0.3), angle ~ U[0, pi),
  computed in FP64 and rounded once to FP32. Segments may cross each other or
  poke out of the box.
* The single-segment scene uses endpoints ~ U[0.2, 0.8]^2.
* The transmitter is drawn ~ U[0,1]^2 right after any scene-level draws.
* Receivers sit at the centres of an N x N grid of cells of the unit square,
  index m = j*N + i for the cell (i, j).

Every generator takes ``numpy.random.default_rng([11882, config, scene])`` so a
(config, scene) pair always gives the same arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 11882

BOX_WALLS = np.array(
    [[0.0, 0.0, 1.0, 0.0],
     [1.0, 0.0, 1.0, 1.0],
     [1.0, 1.0, 0.0, 1.0],
     [0.0, 1.0, 0.0, 0.0]], dtype=np.float32)


def rng_for(config: int, scene: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(config), int(scene)])


def rx_grid(n: int) -> np.ndarray:
    """Cell centres of an n x n grid on [0,1]^2, float32 [n*n, 2], m = j*n + i."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    xs, ys = np.meshgrid(c, c, indexing="xy")  # ys varies along rows (j), xs along columns (i)
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float32)


def random_segments(rng: np.random.Generator, n: int,
                    len_lo: float = 0.05, len_hi: float = 0.3) -> np.ndarray:
    """n segments drawn as (cx, cy, length, angle), returned as float32 [n, 4] = ax, ay, bx, by."""
    out = np.empty((n, 4), dtype=np.float64)
    for s in range(n):
        cx, cy = rng.uniform(0.0, 1.0), rng.uniform(0.0, 1.0)
        ln = rng.uniform(len_lo, len_hi)
        ang = rng.uniform(0.0, math.pi)
        hx, hy = 0.5 * ln * math.cos(ang), 0.5 * ln * math.sin(ang)
        out[s] = (cx - hx, cy - hy, cx + hx, cy + hy)
    return out.astype(np.float32)


@dataclasses.dataclass
class Scene:
    walls: np.ndarray      # float32 [W, 4]
    tx: np.ndarray         # float32 [2]
    rx: np.ndarray         # float32 [R, 2]
    grid_n: int            # receivers form a grid_n x grid_n grid (0 if not a grid)
    max_order: int
    alpha: float

    @property
    def n_walls(self) -> int:
        return int(self.walls.shape[0])

    @property
    def n_rx(self) -> int:
        return int(self.rx.shape[0])


def n_candidates(n_walls: int, max_order: int) -> int:
    """Count of ordered wall sequences of length 0..K with no wall repeated back to back."""
    total, term = 1, 0
    for k in range(1, max_order + 1):
        term = n_walls if k == 1 else term * (n_walls - 1)
        total += term
    return total


def scene_single_segment(seed: int = 0, grid_n: int = 32, alpha: float = 100.0) -> Scene:
    """Box + one interior segment with endpoints ~U[0.2,0.8]^2, order <= 1."""
    rng = rng_for(1, seed)
    tx = rng.uniform(0.0, 1.0, 2)
    seg = rng.uniform(0.2, 0.8, 4)
    walls = np.concatenate([BOX_WALLS, seg[None, :].astype(np.float32)], axis=0)
    return Scene(walls, tx.astype(np.float32), rx_grid(grid_n), grid_n, 1, alpha)


def scene_random_box(config: int, n_interior: int, grid_n: int, max_order: int,
                     alpha: float, seed: int = 0) -> Scene:
    rng = rng_for(config, seed)
    tx = rng.uniform(0.0, 1.0, 2)
    segs = random_segments(rng, n_interior)
    walls = np.concatenate([BOX_WALLS, segs], axis=0)
    return Scene(walls, tx.astype(np.float32), rx_grid(grid_n), grid_n, max_order, alpha)


def scene_64(seed: int = 0, grid_n: int = 256, alpha: float = 100.0) -> Scene:
    """Box + 64 segments, 256 x 256 receivers, order <= 2 (4,625 wall sequences)."""
    return scene_random_box(2, 64, grid_n, 2, alpha, seed)


def scene_32_order3(seed: int = 0, grid_n: int = 512, alpha: float = 100.0) -> Scene:
    """Box + 32 segments, 512 x 512 receivers, order <= 3 (45,397 wall sequences)."""
    return scene_random_box(4, 32, grid_n, 3, alpha, seed)


def batch_scenes(n_scenes: int = 512, lo: int = 8, hi: int = 128,
                 sides=(64, 128, 256), alpha: float = 100.0,
                 side_cap: int | None = None) -> list[Scene]:
    """Many scenes of uneven size: interior count ~U{lo..hi}, grid side ~U{sides}, order <= 2.

    ``side_cap`` shrinks every grid to at most that side (for quick tests); the
    geometry draws are unchanged.
    """
    out = []
    for s in range(n_scenes):
        rng = rng_for(3, s)
        n_int = int(rng.integers(lo, hi + 1))
        side = int(sides[int(rng.integers(0, len(sides)))])
        tx = rng.uniform(0.0, 1.0, 2)
        segs = random_segments(rng, n_int)
        walls = np.concatenate([BOX_WALLS, segs], axis=0)
        if side_cap is not None:
            side = min(side, side_cap)
        out.append(Scene(walls, tx.astype(np.float32), rx_grid(side), side, 2, alpha))
    return out


def placement_problem(scene: int, n_rx: int, alpha: float = 1.0) -> Scene:
    """One transmitter-placement problem (Sec. VII): box + 2..5 interior segments
    of length U(0.2, 0.5), n_rx receivers ~U[0.05, 0.95]^2 and a start
    position tx ~U[0.05, 0.95]^2; line of sight only (order 0), as in the
    paper's example.  Receivers are scattered (grid_n = 0)."""
    rng = rng_for(6, 1000 * int(n_rx) + int(scene))
    n_int = int(rng.integers(2, 6))
    segs = random_segments(rng, n_int, 0.2, 0.5)
    walls = np.concatenate([BOX_WALLS, segs], axis=0)
    rx = rng.uniform(0.05, 0.95, (n_rx, 2)).astype(np.float32)
    tx = rng.uniform(0.05, 0.95, 2).astype(np.float32)
    return Scene(walls, tx, rx, 0, 0, alpha)


# --- 3D scenes: parallelogram panels [P][9] = corner a, adjacent corners b, c ---

ROOM_PANELS = np.array(
    [[0, 0, 0, 1, 0, 0, 0, 1, 0],    # floor z = 0
     [0, 0, 1, 0, 1, 1, 1, 0, 1],    # ceiling z = 1
     [0, 0, 0, 0, 1, 0, 0, 0, 1],    # x = 0
     [1, 0, 0, 1, 0, 1, 1, 1, 0],    # x = 1
     [0, 0, 0, 0, 0, 1, 1, 0, 0],    # y = 0
     [0, 1, 0, 1, 1, 0, 0, 1, 1]],   # y = 1
    dtype=np.float32)


@dataclasses.dataclass
class Scene3D:
    panels: np.ndarray     # float32 [P, 9]
    tx: np.ndarray         # float32 [3]
    rx: np.ndarray         # float32 [R, 3]
    grid_n: int            # receivers form a grid_n x grid_n grid at one height (0 if not)
    max_order: int
    alpha: float

    @property
    def n_panels(self) -> int:
        return int(self.panels.shape[0])

    @property
    def n_rx(self) -> int:
        return int(self.rx.shape[0])


def random_panels(rng: np.random.Generator, n: int, len_lo: float = 0.05, len_hi: float = 0.3) -> np.ndarray:
    """n rectangles: centre ~U[0,1]^3, normal uniform on the sphere, side lengths
    ~U(len_lo, len_hi), in-plane angle ~U[0, 2 pi); float32 [n, 9]."""
    out = np.empty((n, 9), dtype=np.float64)
    for s in range(n):
        c = rng.uniform(0.0, 1.0, 3)
        nrm = rng.normal(0.0, 1.0, 3)
        nrm /= np.linalg.norm(nrm)
        l1, l2 = rng.uniform(len_lo, len_hi, 2)
        th = rng.uniform(0.0, 2.0 * np.pi)
        ref = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        t1 = np.cross(nrm, ref)
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(nrm, t1)
        u = np.cos(th) * t1 + np.sin(th) * t2
        v = np.cross(nrm, u)
        e1, e2 = l1 * u, l2 * v
        a = c - 0.5 * (e1 + e2)
        out[s] = np.concatenate([a, a + e1, a + e2])
    return out.astype(np.float32)


def rx_plane(n: int, z: float) -> np.ndarray:
    """Cell centres of an n x n grid of [0,1]^2 at height z, float32 [n*n, 3], m = j*n + i."""
    xy = rx_grid(n).astype(np.float64)
    return np.concatenate([xy, np.full((xy.shape[0], 1), z)], axis=1).astype(np.float32)


def scene3d_room(config: int, n_panels: int, grid_n: int, max_order: int, alpha: float, seed: int = 0,
                 z: float = 0.5) -> Scene3D:
    """Unit-cube room (6 panels) + n random rectangles; tx ~U[0.1, 0.9]^3;
    receivers on an n x n grid at height z."""
    rng = rng_for(config, seed)
    tx = rng.uniform(0.1, 0.9, 3)
    panels = np.concatenate([ROOM_PANELS, random_panels(rng, n_panels)], axis=0)
    return Scene3D(panels, tx.astype(np.float32), rx_plane(grid_n, z), grid_n, max_order, alpha)


def scene3d_32(seed: int = 0, grid_n: int = 256, alpha: float = 100.0) -> Scene3D:
    """Room + 32 rectangles, 256 x 256 receivers at mid-height, order <= 2 (1,445 panel sequences)."""
    return scene3d_room(8, 32, grid_n, 2, alpha, seed)


def extrude(s: Scene, height: float = 1.0) -> Scene3D:
    """The 2D scene as vertical panels of the given height, tx and receivers at
    half height: every path stays in that plane."""
    W = s.walls.astype(np.float64)
    z0 = np.zeros((W.shape[0], 1))
    a = np.concatenate([W[:, 0:2], z0], axis=1)
    b = np.concatenate([W[:, 2:4], z0], axis=1)
    c = np.concatenate([W[:, 0:2], z0 + height], axis=1)
    h = np.full((s.rx.shape[0], 1), 0.5 * height)
    return Scene3D(np.concatenate([a, b, c], axis=1).astype(np.float32),
                   np.array([s.tx[0], s.tx[1], 0.5 * height], np.float32),
                   np.concatenate([s.rx.astype(np.float64), h], axis=1).astype(np.float32),
                   0, s.max_order, s.alpha)


def random_points(config: int, scene: int, n: int) -> np.ndarray:
    """n points ~U[0,1]^2 as float32 [n, 2] (transmitter starts, sampled receivers)."""
    rng = rng_for(config, 1000 + scene)
    return rng.uniform(0.0, 1.0, (n, 2)).astype(np.float32)


# --- learned surrogate: the random tensors it needs -------------------------

MLP_WIDTHS = (128, 256, 256, 256, 256, 256, 1)


def fourier_matrix(seed: int = 0, n_freq: int = 64, in_dim: int = 4,
                   sigma: float = 4.0) -> np.ndarray:
    """Fixed Gaussian frequency matrix B ~ N(0, sigma^2), float32 [n_freq, in_dim]."""
    rng = rng_for(5, 2000 + seed)
    return (sigma * rng.standard_normal((n_freq, in_dim))).astype(np.float32)


def mlp_init(seed: int = 0, widths=MLP_WIDTHS) -> list[tuple[np.ndarray, np.ndarray]]:
    """He-uniform weights W_l float32 [in, out] and zero biases, seeded."""
    rng = rng_for(5, 3000 + seed)
    layers = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        lim = math.sqrt(6.0 / fi)
        w = rng.uniform(-lim, lim, (fi, fo)).astype(np.float32)
        b = np.zeros((fo,), dtype=np.float32)
        layers.append((w, b))
    return layers
