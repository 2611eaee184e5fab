"""Per-cell input fields of the benchmark problems (input generator only).

Every field is evaluated at the mean of a tetrahedron's four vertex positions
(the point the paper stores cell data at) and returned in user cell order.
The paper's streamer initial pulse is an ``exp(-r^2/sigma^2)`` Gaussian; the
benchmark problem uses the same form on the unit cube.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .meshgen import CubeMesh


def _cell_points(mesh: CubeMesh) -> np.ndarray:
    return mesh.xyz[mesh.tets].mean(axis=1)


def gaussian_field(mesh: CubeMesh, center=(0.5, 0.5, 0.5),
                   sigma: float = 0.1) -> np.ndarray:
    p = _cell_points(mesh) - np.asarray(center, np.float64)
    return np.exp(-np.einsum("ij,ij->i", p, p) / (sigma * sigma))


def rotating_velocity(mesh: CubeMesh) -> np.ndarray:
    """V = (sin(pi y), sin(pi z), sin(pi x)) per cell, float64 [Nc, 3]."""
    p = _cell_points(mesh)
    return np.stack([np.sin(np.pi * p[:, 1]), np.sin(np.pi * p[:, 2]),
                     np.sin(np.pi * p[:, 0])], axis=1)


def mms_exact(mesh: CubeMesh) -> np.ndarray:
    """Manufactured potential sin(pi x) sin(pi y) sin(pi z) per cell."""
    p = _cell_points(mesh)
    return np.prod(np.sin(np.pi * p), axis=1)


def mms_source(mesh: CubeMesh) -> np.ndarray:
    """f = Laplacian of the manufactured potential, per cell."""
    return -3.0 * np.pi ** 2 * mms_exact(mesh)


@dataclass(frozen=True)
class ProblemFields:
    u0: np.ndarray          # scalar initial value per cell
    vel: np.ndarray         # velocity per cell [Nc, 3]
    diffusivity: float
    cfl: float


def problem_fields(mesh: CubeMesh, center=(0.5, 0.5, 0.5), sigma=0.1,
                   diffusivity=1e-3, cfl=0.4) -> ProblemFields:
    """Convection-diffusion benchmark problem: Gaussian pulse in a rotating
    velocity field, zero-flux walls."""
    return ProblemFields(u0=gaussian_field(mesh, center, sigma),
                         vel=rotating_velocity(mesh),
                         diffusivity=float(diffusivity), cfl=float(cfl))


@dataclass(frozen=True)
class BatchMember:
    n: int                  # hexes per side (6 n^3 cells)
    seed: int
    diffusivity: float
    center: tuple


def batch_recipe(count=64, seed=4242, lo=5e4, hi=2e6):
    """Batched benchmark: `count` cube meshes with cell counts log-uniform in
    [lo, hi] (n = round(cbrt(N / 6)) clamped to the range), diffusivity
    uniform in [1e-4, 1e-2], Gaussian centre uniform in [0.3, 0.7]^3; mesh k
    uses seed 1000 + k."""
    rng = np.random.default_rng(seed)
    nlo = int(np.ceil(np.cbrt(lo / 6.0)))
    nhi = int(np.floor(np.cbrt(hi / 6.0)))
    out = []
    for k in range(count):
        N = np.exp(rng.uniform(np.log(lo), np.log(hi)))
        n = int(np.clip(round(np.cbrt(N / 6.0)), nlo, nhi))
        D = float(rng.uniform(1e-4, 1e-2))
        c = tuple(float(x) for x in rng.uniform(0.3, 0.7, 3))
        out.append(BatchMember(n=n, seed=1000 + k, diffusivity=D, center=c))
    return out
