"""Seeded synthetic workloads for the immersed Newmark IMEX time stepper.

This module only *describes* inputs: mesh sizes, hole layouts, source
positions, the excitation signal f_t sampled at the step times, and seeded
random initial fields.  It contains none of the method's arithmetic (no
basis functions, quadrature, assembly or time integration), so both the GPU
path and the CPU oracle can take their inputs from here without sharing any
computation.

The layouts stand in for the paper's perforated plate (Section "Perforated
plate": ten circular holes with centres and radii drawn from uniform
distributions, the source on the hole-free strip on the left) and its
voided 3D example (Section "Three-dimensional example"), whose geometry file
is not published.  All materials are uniform with homogeneous Neumann
boundaries, as in both examples.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Workload:
    """One immersed wave problem on an axis-aligned box of Cartesian cells.

    The physical domain is the box minus the union of open balls
    ``|x - centre_j| < radius_j`` (circles in 2D, spheres in 3D).
    """

    name: str
    dim: int
    n_cells: Sequence[int]                # cells per direction (len == dim)
    p: int                                # GLL order
    extent: Sequence[float] = (1.0, 1.0, 1.0)
    rho: float = 1.0
    c: float = 1.0
    alpha_f: float = 1e-5                 # fictitious-domain density scaling
    tree_depth: int = 3                   # space-tree depth on cut cells
    hole_centers: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    hole_radii: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0,)))
    source: Sequence[float] = (0.1, 0.5, 0.5)
    source_freq: float = 10.0             # Ricker centre frequency [Hz]
    cfl: float = 0.9                      # safety factor on the uncut-cell step
    steps: int = 200
    explicit_fp: int = 64                 # 64 or 32 (the implicit block is FP64)
    forced_cut: Optional[np.ndarray] = None  # cell ids treated as cut even if uncut
    cut_mass: str = "consistent"          # mass of cut cells: "consistent" or "hrz" (lumped)

    @property
    def n_holes(self) -> int:
        return int(len(self.hole_radii))

    @property
    def h(self) -> List[float]:
        return [self.extent[k] / self.n_cells[k] for k in range(self.dim)]

    @property
    def grid_nodes(self) -> List[int]:
        return [self.n_cells[k] * self.p + 1 for k in range(self.dim)]

    @property
    def n_grid(self) -> int:
        return int(np.prod(self.grid_nodes))


def ricker(t: np.ndarray, fs: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 fs^2 tau^2) exp(-pi^2 fs^2 tau^2), tau = t - t0.

    The default delay t0 = 1.5 / fs makes f_t(0) ~ -1e-8, so the zero
    initial state is consistent with the forcing to that level.
    """
    if t0 is None:
        t0 = 1.5 / fs
    a = (math.pi * fs * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ft_table(dt: float, n_steps: int, fs: float, start_step: int = 0) -> np.ndarray:
    """f_t(t_n) for n = start_step .. start_step + n_steps (n_steps + 1 values)."""
    n = np.arange(start_step, start_step + n_steps + 1, dtype=np.float64)
    return ricker(n * dt, fs)


def random_field(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal vector (for initial states in tests)."""
    return np.random.default_rng(seed).standard_normal(n)


def _holes_2d(rng, n, x_range=(0.2, 1.0), y_range=(0.0, 1.0), r_range=(0.03, 0.08)):
    xc = rng.uniform(*x_range, size=n)
    yc = rng.uniform(*y_range, size=n)
    r = rng.uniform(*r_range, size=n)
    return np.stack([xc, yc], axis=1), r


def _voids_3d(rng, n, r_range=(0.02, 0.06)):
    xc = rng.uniform(0.0, 1.0, size=n)
    yc = rng.uniform(0.0, 1.0, size=n)
    zc = rng.uniform(0.2, 1.0, size=n)
    r = rng.uniform(*r_range, size=n)
    return np.stack([xc, yc, zc], axis=1), r


def config1() -> Workload:
    """16x16 cells, p=4, one centred hole r=0.2, depth 3, 200 FP64 steps."""
    return Workload(name="plate16_p4_1hole", dim=2, n_cells=(16, 16), p=4,
                    tree_depth=3, hole_centers=np.array([[0.5, 0.5]]),
                    hole_radii=np.array([0.2]), source=(0.1, 0.5),
                    steps=200, explicit_fp=64)


def config2(seed: int = 2, explicit_fp: int = 64) -> Workload:
    """128x128 cells, p=4, 12 seeded holes r ~ U(0.03, 0.08), 5000 steps."""
    rng = np.random.default_rng(seed)
    c, r = _holes_2d(rng, 12)
    return Workload(name="plate128_p4_12holes", dim=2, n_cells=(128, 128), p=4,
                    tree_depth=3, hole_centers=c, hole_radii=r, source=(0.1, 0.5),
                    steps=5000, explicit_fp=explicit_fp)


def config3(seed: int = 3, n: int = 64, n_voids: int = 40, explicit_fp: int = 64) -> Workload:
    """n^3 hex cells at p=3, seeded spherical voids r ~ U(0.02, 0.06), depth 2."""
    rng = np.random.default_rng(seed)
    c, r = _voids_3d(rng, n_voids)
    return Workload(name=f"cube{n}_p3_{n_voids}voids", dim=3, n_cells=(n, n, n), p=3,
                    tree_depth=2, hole_centers=c, hole_radii=r,
                    source=(0.5, 0.5, 0.0), steps=2000, explicit_fp=explicit_fp)


def config5(seed: int = 5, n: int = 48, n_voids: int = 60) -> Workload:
    """n^3 hex cells at p=4 with seeded voids (implicit block ~5% of dofs)."""
    rng = np.random.default_rng(seed)
    c, r = _voids_3d(rng, n_voids)
    return Workload(name=f"cube{n}_p4_{n_voids}voids", dim=3, n_cells=(n, n, n), p=4,
                    tree_depth=2, hole_centers=c, hole_radii=r,
                    source=(0.5, 0.5, 0.0), steps=2500, explicit_fp=64)


def cube_replica(w: Workload, n: int, seed: int) -> Workload:
    """A reduced replica of a voided cube: n^3 cells of the same size h (the
    box shrinks to n h per side), the same order, tree depth and radius range
    of the voids, and a void count that keeps the number of voids per unit
    volume (rounded, at least two); voids placed as in the full cube (x, y
    uniform, z uniform over the upper 80 %), the source at the centre of the
    bottom face."""
    ext = n * w.h[0]
    n_voids = max(2, int(round(w.n_holes * (n / w.n_cells[0]) ** 3)))
    rng = np.random.default_rng(seed)
    xc = rng.uniform(0.0, ext, size=n_voids)
    yc = rng.uniform(0.0, ext, size=n_voids)
    zc = rng.uniform(0.2 * ext, ext, size=n_voids)
    r = rng.uniform(float(w.hole_radii.min()), float(w.hole_radii.max()), size=n_voids)
    return dataclasses.replace(w, name=f"{w.name}_replica{n}", n_cells=(n, n, n), extent=(ext, ext, ext),
                               hole_centers=np.stack([xc, yc, zc], axis=1), hole_radii=r,
                               source=(0.5 * ext, 0.5 * ext, 0.0))


def config3_replica(n: int = 24, seed: int = 33) -> Workload:
    """Replica of the 64^3 p = 3 cube (40 voids): 24^3 cells by default, two voids."""
    return cube_replica(config3(), n, seed)


def config5_replica(n: int = 12, seed: int = 58) -> Workload:
    """Replica of the 48^3 p = 4 cube (60 voids): 12^3 cells by default, two voids."""
    return cube_replica(config5(), n, seed)


def config4_instances(n_instances: int = 64, base_seed: int = 4000) -> List[Workload]:
    """Uneven 2D instances: N ~ U{32..128}, p ~ U{2..6}, 1..12 holes."""
    out = []
    for i in range(n_instances):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.integers(32, 129))
        p = int(rng.integers(2, 7))
        nh = int(rng.integers(1, 13))
        c, r = _holes_2d(rng, nh, x_range=(0.2, 1.0))
        xs = float(rng.uniform(0.02, 0.10))
        ys = float(rng.uniform(0.1, 0.9))
        out.append(Workload(name=f"inst{i}_n{n}_p{p}_h{nh}", dim=2, n_cells=(n, n), p=p,
                            tree_depth=3, hole_centers=c, hole_radii=r,
                            source=(xs, ys), steps=1000, explicit_fp=32))
    return out


def fully_implicit(w: Workload) -> Workload:
    """The same problem with every cell in the implicit block: no d dofs, so
    the IMEX step is the trapezoidal Newmark rule on all dofs (the fully
    implicit comparator of Section "Time Integration")."""
    return dataclasses.replace(w, name=w.name + "_fully_implicit",
                               forced_cut=np.arange(int(np.prod(w.n_cells)), dtype=np.int64))


def small_2d(n=(5, 4), p=3, holes=((0.55, 0.45, 0.23),), depth=2, source=(0.1, 0.3),
             name="small2d") -> Workload:
    """Small ragged 2D case for fast tests (holes given as (x, y, r))."""
    hc = np.array([[h[0], h[1]] for h in holes]).reshape(-1, 2)
    hr = np.array([h[2] for h in holes], dtype=np.float64)
    return Workload(name=name, dim=2, n_cells=tuple(n), p=p, tree_depth=depth,
                    hole_centers=hc, hole_radii=hr, source=source, steps=50)


def small_3d(n=(4, 3, 5), p=2, holes=((0.5, 0.45, 0.55, 0.3),), depth=1,
             source=(0.1, 0.2, 0.15), name="small3d") -> Workload:
    """Small ragged 3D case for fast tests (holes given as (x, y, z, r))."""
    hc = np.array([[h[0], h[1], h[2]] for h in holes]).reshape(-1, 3)
    hr = np.array([h[3] for h in holes], dtype=np.float64)
    return Workload(name=name, dim=3, n_cells=tuple(n), p=p, tree_depth=depth,
                    hole_centers=hc, hole_radii=hr, source=source, steps=30)


def mlp_init(inputs_: int, hidden: int, outputs: int, seed: int, out_scale: float = 0.1) -> np.ndarray:
    """Seeded initial parameters of the learned preconditioner, packed FP32
    [W1 (hidden x inputs) | b1 | W2 (hidden x hidden) | b2 | W3 (outputs x hidden) | b3]:
    He-normal hidden layers, a small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((hidden, inputs_)) * np.sqrt(2.0 / inputs_)
    w2 = rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)
    w3 = rng.standard_normal((outputs, hidden)) * np.sqrt(2.0 / hidden) * out_scale
    parts = [w1.ravel(), np.zeros(hidden), w2.ravel(), np.zeros(hidden), w3.ravel(), np.zeros(outputs)]
    return np.concatenate(parts).astype(np.float32)


def mlp_unpack(params: np.ndarray, inputs_: int, hidden: int, outputs: int):
    """The six parameter arrays of a packed vector (views, FP32)."""
    shapes = [(hidden, inputs_), (hidden,), (hidden, hidden), (hidden,), (outputs, hidden), (outputs,)]
    out, k = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(params[k:k + n].reshape(sh))
        k += n
    assert k == len(params)
    return out
