"""Seeded synthetic inputs for the HRKAN training step (numpy only).

This module holds no arithmetic of the method: it only describes the
workloads (network shape, PDE instance, point counts, precision) and draws the
collocation points, boundary/initial targets and N(0, 0.1^2) weights from a
seeded generator. Both the GPU binding's users and the CPU oracle's users take
their inputs from here.

Point recipe (the paper draws interior points uniformly at random and places
boundary points evenly, Sec. 4.1 and 4.2):
  * interior: i.i.d. uniform over the domain;
  * boundary/initial: cell-centred, evenly spaced along each edge
    (x_i = lo + (i + 1/2) * len / count), no duplicated corners.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

POISSON2D = 0
BURGERS1D = 1
LINEAR2D = 2

SEED_BASE = 2409142480


@dataclasses.dataclass(frozen=True)
class Net:
    widths: tuple
    G: int
    k: int = 3
    m: int = 4
    lo: float = -1.0
    hi: float = 1.0
    order: int = 2        # jet order along each input coordinate

    @property
    def n_layers(self) -> int:
        return len(self.widths) - 1

    @property
    def n_basis(self) -> int:
        return self.G + self.k

    def weight_shapes(self):
        nb = self.n_basis
        return [(self.widths[l] * nb, self.widths[l + 1]) for l in range(self.n_layers)]

    @property
    def n_params(self) -> int:
        return sum(a * b for a, b in self.weight_shapes())


@dataclasses.dataclass(frozen=True)
class Pde:
    kind: int
    nu: float = 0.0
    alpha: float = 0.05
    adv: float = 1.0
    # LINEAR2D: c0 u + sum_k cx[k-1] d^k u/dx^k + sum_k cy[k-1] d^k u/dy^k = f,
    # f making sin(pi x) sin(pi y) the solution (zero on the square's edges)
    c0: float = 0.0
    cx: tuple = ()
    cy: tuple = ()

    @property
    def orders(self):
        """Highest derivative order along x and y that the residual needs."""
        if self.kind == POISSON2D:
            return 2, 2
        if self.kind == BURGERS1D:
            return 2, 1
        ox = max([k + 1 for k, c in enumerate(self.cx) if c != 0.0], default=0)
        oy = max([k + 1 for k, c in enumerate(self.cy) if c != 0.0], default=0)
        return ox, oy


@dataclasses.dataclass
class Problem:
    """One training-step instance: weights, points and targets (float64)."""
    net: Net
    pde: Pde
    W: List[np.ndarray]
    x_int: np.ndarray      # [n_int, 2]
    x_bc: np.ndarray       # [n_bc, 2]
    g_bc: np.ndarray       # [n_bc]

    @property
    def n_int(self) -> int:
        return self.x_int.shape[0]

    @property
    def n_bc(self) -> int:
        return self.x_bc.shape[0]

    def rounded(self, dtype) -> "Problem":
        """The same instance with every array rounded once to dtype and held
        as float64 (what the oracle is given for a run in that dtype)."""
        f = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)
        return Problem(self.net, self.pde, [f(w) for w in self.W], f(self.x_int),
                       f(self.x_bc), f(self.g_bc))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    net: Net
    pde: Pde
    n_int: int
    n_bc: int
    dtype: str            # "f64", "f32", "bf16"
    seed: int
    grid_points: bool = False   # c1: tensor grid instead of random interior
    n_instances: int = 1
    recipe: str = ""            # "burgers_paper": the paper's own Burgers points and targets


def _cell_centred(lo: float, hi: float, n: int) -> np.ndarray:
    if n <= 0:
        return np.zeros(0)
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * ((hi - lo) / n)


def weights(net: Net, rng: np.random.Generator, std: float = 0.1) -> List[np.ndarray]:
    return [rng.standard_normal(s) * std for s in net.weight_shapes()]


def poisson_points(n_int: int, n_bc: int, rng: np.random.Generator, grid: bool = False):
    """Interior of [-1,1]^2 and its four edges (targets 0)."""
    if grid:
        side = int(round(math.sqrt(n_int)))
        assert side * side == n_int
        c = _cell_centred(-1.0, 1.0, side)
        X, Y = np.meshgrid(c, c, indexing="ij")
        x_int = np.stack([X.ravel(), Y.ravel()], axis=1)
    else:
        x_int = rng.uniform(-1.0, 1.0, size=(n_int, 2))
    per = n_bc // 4
    assert per * 4 == n_bc
    c = _cell_centred(-1.0, 1.0, per)
    one = np.ones(per)
    x_bc = np.concatenate([
        np.stack([-one, c], 1), np.stack([one, c], 1),
        np.stack([c, -one], 1), np.stack([c, one], 1)], axis=0)
    return x_int, x_bc, np.zeros(n_bc)


def burgers_points(n_int: int, n_bc: int, rng: np.random.Generator):
    """Interior of [-1,1]x[0,1]; half of the extra points on the initial line
    t = 0 with target -sin(pi x), a quarter on each wall x = -1, x = +1 with
    target 0."""
    x = rng.uniform(-1.0, 1.0, size=n_int)
    t = rng.uniform(0.0, 1.0, size=n_int)
    x_int = np.stack([x, t], axis=1)
    n_ic = n_bc // 2
    n_w = n_bc // 4
    assert n_ic + 2 * n_w == n_bc
    xi = _cell_centred(-1.0, 1.0, n_ic)
    tw = _cell_centred(0.0, 1.0, n_w)
    one = np.ones(n_w)
    x_bc = np.concatenate([
        np.stack([xi, np.zeros(n_ic)], 1),
        np.stack([-one, tw], 1), np.stack([one, tw], 1)], axis=0)
    g = np.concatenate([-np.sin(np.pi * xi), np.zeros(2 * n_w)])
    return x_int, x_bc, g


def burgers_paper_points(n_int: int, n_bc: int, rng: np.random.Generator):
    """The paper's Burgers instance after its change of variable (Sec. 4.2):
    interior of [0,2.5]^2; a third of the extra points on the initial line
    t = 0 with target 1/cosh(4x - 5), a third on each wall x = 0, x = 2.5
    with target 0."""
    x = rng.uniform(0.0, 2.5, size=n_int)
    t = rng.uniform(0.0, 2.5, size=n_int)
    x_int = np.stack([x, t], axis=1)
    k = n_bc // 3
    assert 3 * k == n_bc
    xi = _cell_centred(0.0, 2.5, k)
    tw = _cell_centred(0.0, 2.5, k)
    x_bc = np.concatenate([
        np.stack([xi, np.zeros(k)], 1),
        np.stack([np.zeros(k), tw], 1), np.stack([np.full(k, 2.5), tw], 1)], axis=0)
    g = np.concatenate([1.0 / np.cosh(4.0 * xi - 5.0), np.zeros(2 * k)])
    return x_int, x_bc, g


NU_BURGERS = 0.01 / math.pi

WORKLOADS = {
    # Poisson, [2,8,1], G=5, 32x32 cell-centred interior + 4x32 edges, FP64
    "poisson_c1": Workload("poisson_c1", Net((2, 8, 1), G=5), Pde(POISSON2D),
                           1024, 128, "f64", SEED_BASE + 0, grid_points=True),
    # Burgers nu=0.01/pi, [2,32,32,1], G=10, 65,536 + 4,096 points, FP32
    "burgers_c2": Workload("burgers_c2", Net((2, 32, 32, 1), G=10), Pde(BURGERS1D, NU_BURGERS),
                           65536, 4096, "f32", SEED_BASE + 1),
    # Poisson, [2,64,64,64,1], G=16, 262,144 + 4x4,096 points, FP32
    "poisson_c3": Workload("poisson_c3", Net((2, 64, 64, 64, 1), G=16), Pde(POISSON2D),
                           262144, 16384, "f32", SEED_BASE + 2),
    # Burgers, [2,128,128,128,1], G=20, 1,048,576 + 65,536 points, BF16 contraction
    "burgers_c4": Workload("burgers_c4", Net((2, 128, 128, 128, 1), G=20), Pde(BURGERS1D, NU_BURGERS),
                           1048576, 65536, "bf16", SEED_BASE + 3),
    # 256 Burgers instances, [2,32,32,1], G=10, uneven point counts, FP32
    "burgers_batched_c5": Workload("burgers_batched_c5", Net((2, 32, 32, 1), G=10),
                                   Pde(BURGERS1D, NU_BURGERS), 0, 0, "f32", SEED_BASE + 4,
                                   n_instances=256),
    # the paper's Poisson training run (Sec. 4.1): [2,2,1], g=5, 960 random
    # interior points, 30 evenly spaced points per edge, FP32
    "poisson_paper": Workload("poisson_paper", Net((2, 2, 1), G=5), Pde(POISSON2D),
                              960, 120, "f32", SEED_BASE + 5),
    # the paper's Burgers instance (Sec. 4.2) on [0,2.5]^2: u_t + u u_x / 4 -
    # nu / 16 u_xx with nu = 0.001, [2,3,3,3,1], g=7 on the same range,
    # 10,000 + 100 initial + 2 x 100 wall points, FP32
    "burgers_paper": Workload("burgers_paper", Net((2, 3, 3, 3, 1), G=7, lo=0.0, hi=2.5),
                              Pde(BURGERS1D, 0.001 / 16.0, adv=0.25), 10000, 300, "f32",
                              SEED_BASE + 6, recipe="burgers_paper"),
    # fourth derivatives (Sec. 3: larger m for higher derivatives):
    # u_xxxx + u_yyyy = f on [-1,1]^2, [2,16,16,1], g=8, m=6 (the basis is
    # C^5, so the gradient's v^(5) is continuous), 8,192 + 4 x 256 points, FP64
    "linear_o4": Workload("linear_o4", Net((2, 16, 16, 1), G=8, m=6, order=4),
                          Pde(LINEAR2D, alpha=1e-4, cx=(0, 0, 0, 1), cy=(0, 0, 0, 1)),
                          8192, 1024, "f64", SEED_BASE + 7),
    # a fifth derivative, the case Sec. 3 names, with its m = 6:
    # u_y + u_xxxxx = f on [-1,1]^2, [2,8,8,1], g=6, 4,096 + 4 x 128 points, FP64
    "linear_o5": Workload("linear_o5", Net((2, 8, 8, 1), G=6, m=6, order=5),
                          Pde(LINEAR2D, alpha=1e-6, cx=(0, 0, 0, 0, 1), cy=(1,)),
                          4096, 512, "f64", SEED_BASE + 8),
}


def make_problem(wl: Workload, n_int: Optional[int] = None, n_bc: Optional[int] = None,
                 seed: Optional[int] = None, pde: Optional[Pde] = None) -> Problem:
    """Draw one instance of a workload (optionally with other point counts)."""
    seed = wl.seed if seed is None else seed
    n_int = wl.n_int if n_int is None else n_int
    n_bc = wl.n_bc if n_bc is None else n_bc
    rw = np.random.default_rng([seed, 1])
    rx = np.random.default_rng([seed, 2])
    W = weights(wl.net, rw)
    pde = wl.pde if pde is None else pde
    if pde.kind in (POISSON2D, LINEAR2D):
        x_int, x_bc, g = poisson_points(n_int, n_bc, rx, grid=wl.grid_points and n_int == wl.n_int)
    elif wl.recipe == "burgers_paper":
        x_int, x_bc, g = burgers_paper_points(n_int, n_bc, rx)
    else:
        x_int, x_bc, g = burgers_points(n_int, n_bc, rx)
    return Problem(wl.net, pde, W, x_int, x_bc, g)


def batched_instances(wl: Workload, n_instances: Optional[int] = None,
                      lo: int = 4096, hi: int = 65536) -> List[Problem]:
    """Independent Burgers instances with log-uniform nu in [1e-3, 1e-1] and
    interior counts uniform in [lo, hi] (boundary = interior/16, rounded to a
    multiple of 4)."""
    n = wl.n_instances if n_instances is None else n_instances
    rs = np.random.default_rng([wl.seed, 3])
    out = []
    for i in range(n):
        n_int = int(rs.integers(lo, hi + 1))
        n_bc = max(4, (n_int // 16) // 4 * 4)
        nu = float(10.0 ** rs.uniform(-3.0, -1.0))
        out.append(make_problem(wl, n_int=n_int, n_bc=n_bc, seed=wl.seed + 1000 * (i + 1),
                                pde=Pde(BURGERS1D, nu)))
    return out
