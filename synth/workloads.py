"""Workload recipes: the synthetic grids and stencil weights of the paper's
evaluation families (1D heat, 2D heat / 5-point star, 2D 9-point box and the
asymmetric "general box", 3D heat / 7-point star, 3D 27-point box; evaluation
section, Table 1) at the sizes this library is measured on.

Everything is drawn from counter-based SplitMix64 streams:

* stream 0: initial grid values, uniform [0, 1), element i = flat row-major
  index;
* stream 1: random stencil weights (one stencil per workload);
* stream 2: batched grid sides, s = clamp(floor(64 * 16**U), 64, 1024);
* stream 3: batched stencil kind, 5-point star if U < 0.5 else 9-point box;
* stream 4: batched per-grid weights, 9 draws per grid at offset 9*i.

Random positive weights are raw = 1 - U in (0, 1], divided by their exactly
rounded sum (math.fsum).  FP32 workloads feed every consumer the FP32-rounded
weights widened back to FP64, so the FP64 oracle and the FP32 kernels see the
same operator.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .splitmix import uniform_f32, uniform_f64

SEED = 2103
STREAM_GRID = 0
STREAM_WEIGHTS = 1
STREAM_BATCH_SIDES = 2
STREAM_BATCH_KIND = 3
STREAM_BATCH_WEIGHTS = 4

STAR = 0
BOX = 1


def grid_f32(shape, seed: int = SEED, stream: int = STREAM_GRID) -> np.ndarray:
    n = int(np.prod(shape))
    return uniform_f32(seed, stream, n).reshape(shape)


def grid_f64(shape, seed: int = SEED, stream: int = STREAM_GRID) -> np.ndarray:
    n = int(np.prod(shape))
    return uniform_f64(seed, stream, n).reshape(shape)


def to_f32_exact(w) -> np.ndarray:
    """FP32-rounded weights widened back to FP64 (exact)."""
    return np.asarray(w, dtype=np.float64).astype(np.float32).astype(np.float64)


def _normalise(raw: np.ndarray) -> np.ndarray:
    s = math.fsum(float(v) for v in raw.ravel())
    return raw / s


def random_positive_weights(dim: int, radius: int = 1, seed: int = SEED,
                            stream: int = STREAM_WEIGHTS, offset: int = 0,
                            mask: np.ndarray | None = None) -> np.ndarray:
    """Dense (2r+1)^dim FP64 weights, positive on ``mask`` (all points if
    None), drawn in row-major order of the masked points, summing to 1."""
    side = 2 * radius + 1
    shape = (side,) * dim
    if mask is None:
        mask = np.ones(shape, dtype=bool)
    k = int(mask.sum())
    raw = 1.0 - uniform_f64(seed, stream, k, offset)
    w = np.zeros(shape, dtype=np.float64)
    w[mask] = _normalise(raw)
    return w


def star_mask(dim: int, radius: int = 1) -> np.ndarray:
    side = 2 * radius + 1
    idx = np.indices((side,) * dim) - radius
    nonzero_axes = (idx != 0).sum(axis=0)
    return nonzero_axes <= 1


def heat1d_weights() -> np.ndarray:
    return np.array([0.25, 0.5, 0.25], dtype=np.float64)


def star2d_weights(center: float, neighbour: float) -> np.ndarray:
    w = np.zeros((3, 3), dtype=np.float64)
    w[1, 1] = center
    w[0, 1] = w[2, 1] = w[1, 0] = w[1, 2] = neighbour
    return w


def star3d_weights(center: float, neighbour: float) -> np.ndarray:
    w = np.zeros((3, 3, 3), dtype=np.float64)
    w[1, 1, 1] = center
    for axis in range(3):
        for d in (0, 2):
            idx = [1, 1, 1]
            idx[axis] = d
            w[tuple(idx)] = neighbour
    return w


@dataclass
class Workload:
    name: str
    dim: int
    shape: tuple
    dtype: str            # "f32" | "f64"
    T: int
    shape_kind: int       # STAR | BOX
    weights: np.ndarray   # dense FP64 (already FP32-exact for f32 workloads)
    folds: tuple = (1,)
    note: str = ""
    extra: dict = field(default_factory=dict)


def _make_workloads(seed: int = SEED) -> dict:
    wl = {}
    wl["heat1d"] = Workload(
        "heat1d", 1, (1_000_000,), "f64", 100, STAR, heat1d_weights(), (1,),
        "1D 3-point heat (0.25, 0.5, 0.25), N=1e6, FP64, T=100, plain sweep")
    wl["star2d"] = Workload(
        "star2d", 2, (8192, 8192), "f32", 1000, STAR,
        to_f32_exact(star2d_weights(0.6, 0.1)), (1, 2, 4),
        "2D 5-point star (0.6; 0.1 x4), 8192^2 FP32, T=1000; plain, fold m=2, m=4")
    wl["star3d"] = Workload(
        "star3d", 3, (512, 512, 512), "f32", 200, STAR,
        to_f32_exact(star3d_weights(0.4, 0.1)), (1, 2),
        "3D 7-point star (0.4; 0.1 x6), 512^3 FP32, T=200; plain, fold m=2")
    wl["box3d"] = Workload(
        "box3d", 3, (512, 512, 512), "f32", 200, BOX,
        to_f32_exact(random_positive_weights(3, 1, seed, STREAM_WEIGHTS)), (1, 2),
        "3D 27-point random positive box, 512^3 FP32, T=200; plain, fold m=2")
    wl["box2d"] = Workload(
        "box2d", 2, (16384, 16384), "f32", 400, BOX,
        to_f32_exact(random_positive_weights(2, 1, seed, STREAM_WEIGHTS)), (1, 4, 8),
        "2D 9-point random positive box, 16384^2 FP32, T=400; plain, fold m=4 "
        "(9x9) and m=8 (17x17), vector and BF16x3 MFMA")
    # Table 1: 1D5P (a 5-point 1D box, radius 2), 10,240,000 points x 1000
    wl["box1d5p"] = Workload(
        "box1d5p", 1, (10_240_000,), "f64", 1000, BOX,
        random_positive_weights(1, 2, seed, STREAM_WEIGHTS, offset=64), (1,),
        "1D 5-point random positive box (1D5P), N=10,240,000, FP64, T=1000, plain sweep")
    # the star2d workload with zero Dirichlet boundaries (the paper states no
    # boundary; zero ghosts are the reading measured beside the periodic one)
    wl["star2d_dirichlet"] = Workload(
        "star2d_dirichlet", 2, (8192, 8192), "f32", 1000, STAR,
        to_f32_exact(star2d_weights(0.6, 0.1)), (1, 2, 4),
        "2D 5-point star (0.6; 0.1 x4), 8192^2 FP32, T=1000, zero Dirichlet boundaries; "
        "plain, fold m=2, m=4", {"boundary": "zero"})
    # the 2D star in FP64 (the paper's precision), plain and folded
    wl["star2d_f64"] = Workload(
        "star2d_f64", 2, (8192, 8192), "f64", 1000, STAR, star2d_weights(0.6, 0.1), (1, 2),
        "2D 5-point star (0.6; 0.1 x4), 8192^2 FP64, T=1000; plain, fold m=2")
    # the paper's worked example (Section 3.3): the unit 9-point box, here
    # normalised (each weight fl32(1/9)), whose folds are rank one
    wl["unitbox2d"] = Workload(
        "unitbox2d", 2, (16384, 16384), "f32", 400, BOX,
        to_f32_exact(np.full((3, 3), 1.0 / 9.0)), (1, 4, 8),
        "2D unit 9-point box (each weight 1/9), 16384^2 FP32, T=400; plain, fold m=4 "
        "and m=8, dense, separable (rank one) and BF16x3 MFMA")
    # the unit box in 3D (each weight fl32(1/27)): a product of three 1D
    # weights, folded or not
    wl["unitbox3d"] = Workload(
        "unitbox3d", 3, (512, 512, 512), "f32", 200, BOX,
        to_f32_exact(np.full((3, 3, 3), 1.0 / 27.0)), (1, 2),
        "3D unit 27-point box (each weight 1/27), 512^3 FP32, T=200; plain and fold m=2, "
        "dense and separable (a product of three 1D weights)")
    return wl


WORKLOADS = _make_workloads()

# Table 1's nonlinear benchmarks (plain only: a max or a counting rule
# cannot be folded).  APOP: option values over N asset prices, 3-point
# stencil with a discount (weights sum 0.999), floored by the put payoff
# max(0.6 - x/N, 0), starting from the payoff.  Game of Life: 5000^2 cells,
# each alive with probability 1/2.
APOP = dict(n=10_240_000, T=1000, weights=np.array([0.3, 0.45, 0.249]))
LIFE = dict(shape=(5000, 5000), T=1000)


def apop_payoff(n: int) -> np.ndarray:
    return np.maximum(0.6 - np.arange(n, dtype=np.float64) / n, 0.0)


def life_cells(shape, seed: int = SEED) -> np.ndarray:
    u = uniform_f64(seed, STREAM_GRID, int(np.prod(shape)))
    return (u < 0.5).astype(np.uint8).reshape(shape)


def batched_recipe(count: int = 4096, seed: int = SEED, lo: int = 64, hi: int = 1024):
    """Sides, kinds and FP32-exact weights of the batched workload.

    Returns (sides[count] int64, kinds[count] in {STAR, BOX},
    weights: list of dense 3x3 FP64 arrays)."""
    u_side = uniform_f64(seed, STREAM_BATCH_SIDES, count)
    sides = np.floor(lo * (hi / lo) ** u_side).astype(np.int64)
    sides = np.clip(sides, lo, hi)
    u_kind = uniform_f64(seed, STREAM_BATCH_KIND, count)
    kinds = np.where(u_kind < 0.5, STAR, BOX).astype(np.int64)
    smask = star_mask(2, 1)
    bmask = np.ones((3, 3), dtype=bool)
    weights = []
    for i in range(count):
        mask = smask if kinds[i] == STAR else bmask
        w = random_positive_weights(2, 1, seed, STREAM_BATCH_WEIGHTS, 9 * i, mask)
        weights.append(to_f32_exact(w))
    return sides, kinds, weights
