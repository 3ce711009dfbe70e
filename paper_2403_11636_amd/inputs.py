"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws obstacle geometries and random
vectors and names the problem configurations. The paper's channel benchmark grids (adaptive, from
p4est) are not available, so the workloads are Cartesian background grids on the unit box with
seeded, non-overlapping disc / sphere obstacles of the sizes listed below.

Boundary condition codes per face, in the order x-, x+, y-, y+, z-, z+:
    0 = Dirichlet no-slip (w = 0), 1 = Dirichlet parabolic inflow (amplitude ubar), 2 = Neumann
    do-nothing (h = 0).
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

NOSLIP, INFLOW, NEUMANN = 0, 1, 2
CACHE_INVERSE, CACHE_MATRIX, CACHE_NONE = 0, 1, 2


@dataclasses.dataclass
class Problem:
    """One finite cell Stokes problem on the unit box [0,1]^d."""

    dim: int
    n_cells: int                 # finest-level cells per axis
    n_levels: int                # levels of the hierarchy (finest has n_cells, each coarser halves)
    balls: np.ndarray            # (n_balls, 4): centre x, y, z (0 in 2D), radius
    bcs: Tuple[int, ...]         # 6 face codes
    eta: float = 1.0
    alpha_fict: float = 1e-8
    nitsche_beta: float = 20.0
    quad_depth: int = 3
    ubar: float = 0.3
    force: int = 0               # 0 = none, 1 = manufactured body force
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    name: str = ""
    immersed_nitsche: int = 0    # 1: obstacle surfaces are no-slip Dirichlet boundaries (Nitsche)

    @property
    def n_nodes(self) -> int:
        return (self.n_cells + 1) ** self.dim

    @property
    def n_dofs(self) -> int:
        return (self.dim + 1) * self.n_nodes

    def level_cells(self, level: int) -> int:
        return self.n_cells >> (self.n_levels - 1 - level)

    def level_dofs(self, level: int) -> int:
        return (self.dim + 1) * (self.level_cells(level) + 1) ** self.dim


def place_balls(rng: np.random.Generator, dim: int, count: int, rmin: float, rmax: float,
                lo: float = 0.1, hi: float = 0.9, max_tries: int = 100000) -> np.ndarray:
    """Rejection-sample `count` non-overlapping balls: centres U[lo,hi]^dim, radii U[rmin,rmax]."""
    out: List[List[float]] = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place the requested obstacles")
        c = rng.uniform(lo, hi, size=dim)
        r = rng.uniform(rmin, rmax)
        ok = True
        for b in out:
            if np.linalg.norm(c - np.asarray(b[:dim])) <= r + b[3]:
                ok = False
                break
        if ok:
            cc = [0.0, 0.0, 0.0]
            cc[:dim] = c.tolist()
            out.append(cc + [float(r)])
    return np.asarray(out, dtype=np.float64).reshape(-1, 4)


def config1(n_cells: int = 32, n_levels: int = 3) -> Problem:
    """2D, one disc (0.5, 0.5) r = 0.2, manufactured body force, no-slip walls, V(2,2)."""
    balls = np.array([[0.5, 0.5, 0.0, 0.2]])
    return Problem(dim=2, n_cells=n_cells, n_levels=n_levels, balls=balls,
                   bcs=(NOSLIP,) * 6, force=1, name=f"2d_disc_manufactured_{n_cells}")


def config2(seed: int = 0, n_cells: int = 512, n_levels: int = 7) -> Problem:
    """2D channel-like box: 20 seeded discs r ~ U[0.02,0.06], inflow left, do-nothing right."""
    rng = np.random.default_rng(seed)
    balls = place_balls(rng, 2, 20, 0.02, 0.06)
    return Problem(dim=2, n_cells=n_cells, n_levels=n_levels, balls=balls,
                   bcs=(INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP),
                   name=f"2d_20discs_{n_cells}_seed{seed}")


def config3(seed: int = 0, n_cells: int = 64, n_levels: int = 5) -> Problem:
    """3D box: 40 seeded porous spheres r ~ U[0.04,0.1], inflow x-, do-nothing x+, no-slip else."""
    rng = np.random.default_rng(seed)
    balls = place_balls(rng, 3, 40, 0.04, 0.1)
    return Problem(dim=3, n_cells=n_cells, n_levels=n_levels, balls=balls,
                   bcs=(INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP),
                   name=f"3d_40spheres_{n_cells}_seed{seed}")


def batch_problem(seed: int) -> Problem:
    """One problem of the batching workload: 2D, n = 32 m cells per axis with m ~ U{2..8} (64..256),
    6 levels (coarsest 2..8 cells), 1..12 seeded discs r ~ U[0.02, 0.06], alpha_f in
    {1e-6, 1e-8, 1e-10}, inflow left, do-nothing right, no-slip top/bottom."""
    rng = np.random.default_rng(1000 + seed)
    n_cells = 32 * int(rng.integers(2, 9))
    n_balls = int(rng.integers(1, 13))
    alpha = float((1e-6, 1e-8, 1e-10)[int(rng.integers(0, 3))])
    balls = place_balls(rng, 2, n_balls, 0.02, 0.06)
    return Problem(dim=2, n_cells=n_cells, n_levels=6, balls=balls, alpha_fict=alpha,
                   bcs=(INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP),
                   name=f"2d_batch_{n_cells}_{n_balls}discs_seed{seed}")


def small_problem(dim: int, n_cells: int, n_levels: int, seed: int, n_balls: int = 2,
                  rmin: float = 0.08, rmax: float = 0.18, bcs=None, alpha_fict: float = 1e-8,
                  force: int = 1) -> Problem:
    """Small seeded problem for parity tests: a few balls, mixed walls."""
    rng = np.random.default_rng(seed)
    balls = place_balls(rng, dim, n_balls, rmin, rmax, lo=0.25, hi=0.75) if n_balls else np.zeros((0, 4))
    if bcs is None:
        bcs = (INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP)
    return Problem(dim=dim, n_cells=n_cells, n_levels=n_levels, balls=balls, bcs=tuple(bcs),
                   alpha_fict=alpha_fict, force=force,
                   name=f"{dim}d_small_{n_cells}_seed{seed}")


EDGE_CASES = ("inflow_wall", "corner", "two_in_cell")


def edge_problem(dim: int, n_cells: int, n_levels: int, case: str, alpha_fict: float = 1e-8) -> Problem:
    """Obstacles where the seeded generators never put them (their centres keep a margin from the
    walls and from each other):
      * "inflow_wall": a ball crossing the x- (inflow) face, inflow / do-nothing / no-slip walls;
      * "corner": a ball covering the corner x = y (= z) = 0 of an all no-slip box;
      * "two_in_cell": two balls whose gap of 0.02 lies inside one cell of a 16-cell-per-axis grid,
        so that cell (and the coarser cells around it) is cut by both."""
    z = 0.5 if dim == 3 else 0.0
    if case == "inflow_wall":
        balls = [[0.03, 0.47, z, 0.11]]
        bcs = (INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP)
    elif case == "corner":
        balls = [[0.03, 0.04, 0.03 if dim == 3 else 0.0, 0.13]]
        bcs = (NOSLIP,) * 6
    elif case == "two_in_cell":
        balls = [[0.40, 0.53, z, 0.10], [0.62, 0.53, z, 0.10]]
        bcs = (INFLOW, NEUMANN, NOSLIP, NOSLIP, NOSLIP, NOSLIP)
    else:
        raise ValueError(f"unknown edge case {case!r}")
    return Problem(dim=dim, n_cells=n_cells, n_levels=n_levels, balls=np.asarray(balls, dtype=np.float64),
                   bcs=bcs, alpha_fict=alpha_fict, force=1, name=f"{dim}d_edge_{case}_{n_cells}")


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 vector."""
    return np.random.default_rng(seed).standard_normal(n)
