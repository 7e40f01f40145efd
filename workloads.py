"""Seeded synthetic inputs for the free-space Stokes sums.

This module only draws random numbers; it holds none of the summation
method's arithmetic, so both the CPU reference under ``oracle/`` and the
GPU path may use it.

Workloads (positions, strengths) follow the sums evaluated in the paper
(Section 2, eqs. def_stokeslet/def_stresslet/def_rotlet) and the uniform
random systems of its Results section; the configurations named below are
the ones this project measures.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "uniform_cube",
    "sphere_surface",
    "gaussian_blobs",
    "normal_strengths",
    "uniform_strengths",
    "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed``."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_cube(n: int, seed: int, lo: float = 0.0, L: float = 1.0) -> np.ndarray:
    """``n`` points i.i.d. uniform in ``[lo, lo+L)^3`` as an ``(n, 3)`` float64 array."""
    return lo + L * rng(seed).random((n, 3))


def sphere_surface(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """``n`` points uniform on the unit sphere and their outward unit normals."""
    z = rng(seed).standard_normal((n, 3))
    x = z / np.linalg.norm(z, axis=1, keepdims=True)
    return x, x.copy()


def gaussian_blobs(n: int, seed: int, nblobs: int = 64, sigma: float = 0.02,
                   centre_lo: float = 0.1, centre_hi: float = 0.9) -> np.ndarray:
    """``n`` points in ``nblobs`` isotropic Gaussian clusters of width ``sigma``.

    Centres are uniform in ``[centre_lo, centre_hi)^3``; points are assigned to
    blobs round-robin so every blob holds ``n // nblobs`` or one more points.
    """
    g = rng(seed)
    centres = centre_lo + (centre_hi - centre_lo) * g.random((nblobs, 3))
    which = np.arange(n) % nblobs
    return centres[which] + sigma * g.standard_normal((n, 3))


def normal_strengths(n: int, seed: int, batch: int | None = None) -> np.ndarray:
    """Strength vectors with i.i.d. N(0,1) components: ``(n,3)`` or ``(batch,n,3)``."""
    shape = (n, 3) if batch is None else (batch, n, 3)
    return rng(seed).standard_normal(shape)


def uniform_strengths(n: int, seed: int, batch: int | None = None) -> np.ndarray:
    """Strength vectors with i.i.d. U[-1,1] components (the paper's Results setup)."""
    shape = (n, 3) if batch is None else (batch, n, 3)
    return 2.0 * rng(seed).random(shape) - 1.0


# Measured configurations: id -> description.  Seeds: positions 1000+id,
# strengths 2000+id(+b for batch member b), adjoint weights 3000+id.
CONFIGS = {
    1: dict(kernel="stokeslet", n=1000, positions="uniform", dtype="f64", tol=1e-6),
    2: dict(kernel="stokeslet", n=100_000, positions="uniform", dtype="f32|f64", tol=1e-6),
    3: dict(kernel="stresslet", n=200_000, positions="sphere", dtype="f32", tol=1e-6),
    4: dict(kernel="rotlet", n=1_000_000, positions="uniform", dtype="f32", tol=1e-6, batch=16),
    5: dict(kernel="stokeslet", n=4_000_000, positions="blobs", dtype="f32", tol=1e-6, adjoint=True),
    0: dict(kernel="stokeslet", n=1_000_000, positions="uniform", dtype="f32|f64", tol=1e-6, adjoint=True),
}
