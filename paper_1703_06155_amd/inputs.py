"""Seeded synthetic inputs for the cube-grid volume-integral-equation workloads.

This module only draws geometry, contrasts and right-hand sides.  It holds none
of the solver's arithmetic (no kernel entries, no factorization): both the HIP
path and the CPU oracle consume what it produces.

The workloads stand in for the paper's SWG-meshed dielectric bodies (Sec. VI),
whose meshes are not available: cells of a uniform grid with edge h carry one
unknown each, the wavelength is 1 (k = 2*pi) and h = lambda/10 as in the
paper's mesh size (Sec. VI-B).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WAVENUMBER = 2.0 * math.pi
CELL = 0.1


def cube_grid(nx: int, ny: int, nz: int, h: float = CELL) -> np.ndarray:
    """Cell centres of an nx*ny*nz grid, cell (ix,iy,iz) at index (ix*ny+iy)*nz+iz."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return (pts + 0.5) * h


def contrast(n: int, seed: int) -> np.ndarray:
    """Per-cell contrast chi ~ U[0.5, 1.5] from numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(0.5, 1.5, n)


def directions(m: int, seed: int) -> np.ndarray:
    """m unit vectors uniform on the sphere (normalised Gaussian draws)."""
    d = np.random.default_rng(seed).standard_normal((m, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def plane_waves(points: np.ndarray, dirs: np.ndarray, k: float = WAVENUMBER) -> np.ndarray:
    """Incident plane waves exp(-j k d.r), one column per direction (N x m, complex128)."""
    phase = points @ np.asarray(dirs, dtype=np.float64).reshape(-1, 3).T
    return np.exp(-1j * k * phase)


def fibonacci_sphere(m: int, centre, radius: float) -> np.ndarray:
    """m nearly uniform observation points on a sphere (Fibonacci lattice)."""
    i = np.arange(m) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / m)
    theta = math.pi * (1.0 + 5.0 ** 0.5) * i
    xyz = np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], 1)
    return np.asarray(centre, dtype=np.float64) + radius * xyz


@dataclass
class Problem:
    """One synthetic VIE problem: geometry, contrast, solver parameters and RHS."""
    name: str
    grid: tuple
    points: np.ndarray
    chi: np.ndarray
    k: float
    h: float
    leaf: int
    eta: float
    eps: float
    rhs: np.ndarray          # N x nrhs complex128, user order
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.points.shape[0]


def make_problem(name: str, grid, leaf: int, eps: float, eta: float = 1.0,
                 chi_seed: int = 0, nrhs: int = 1, rhs_seed: int | None = None) -> Problem:
    """Cube-grid problem; nrhs=1 gives b = exp(-j k z), otherwise random plane waves."""
    nx, ny, nz = grid
    pts = cube_grid(nx, ny, nz)
    chi = contrast(pts.shape[0], chi_seed)
    if nrhs == 1 and rhs_seed is None:
        rhs = plane_waves(pts, np.array([[0.0, 0.0, 1.0]]))
    else:
        rhs = plane_waves(pts, directions(nrhs, 3 if rhs_seed is None else rhs_seed))
    return Problem(name, tuple(grid), pts, chi, WAVENUMBER, CELL, leaf, eta, eps, rhs)


def config(idx: int, nrhs: int = 1) -> Problem:
    """The five benchmark configurations (small correctness case, headline case, ...)."""
    if idx == 0:
        return make_problem("cube16_leaf32_eps1e-6", (16, 16, 16), 32, 1e-6)
    if idx == 1:
        return make_problem("cube32_leaf64_eps1e-4", (32, 32, 32), 64, 1e-4, nrhs=nrhs)
    if idx == 2:
        return make_problem("cube64_leaf64_eps1e-4", (64, 64, 64), 64, 1e-4)
    if idx == 4:
        return make_problem("cube48_leaf32_eps1e-6", (48, 48, 48), 32, 1e-6)
    raise ValueError("config 3 is a batch: use batch_problems()")


def batch_problems(count: int = 64, nrhs: int = 16, sides=(12, 32), leaf: int = 48) -> list:
    """Independent box problems with sides U{sides[0]..sides[1]}, problem p seeded 1000+p."""
    out = []
    for p in range(count):
        rng = np.random.default_rng(1000 + p)
        grid = tuple(int(v) for v in rng.integers(sides[0], sides[1] + 1, size=3))
        pts = cube_grid(*grid)
        chi = rng.uniform(0.5, 1.5, pts.shape[0])
        dirs = rng.standard_normal((nrhs, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        out.append(Problem(f"box{p}_{grid[0]}x{grid[1]}x{grid[2]}", grid, pts, chi,
                           WAVENUMBER, CELL, leaf, 1.0, 1e-4, plane_waves(pts, dirs)))
    return out


def rod(nz: int, nxy: int = 4, leaf: int = 32, eps: float = 1e-4) -> Problem:
    """Quasi-1-D rod nxy x nxy x nz (0.4 lambda square cross-section at h = lambda/10)."""
    return make_problem(f"rod{nxy}x{nxy}x{nz}", (nxy, nxy, nz), leaf, eps)
