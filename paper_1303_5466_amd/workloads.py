"""Seeded synthetic inputs for the Nystrom systems this library solves.

This module only draws inputs: grid coordinates, the identity-term
coefficient a(x), and right-hand sides.  It holds none of the solver's
arithmetic (no kernel values, no quadrature, no factorisation), so both the
HIP path and the CPU reference may take their inputs from here.

Grid convention (Sec. 5, general formulation): cell-centred points on the
unit square, x_ij = ((i + 1/2) h, (j + 1/2) h), h = 1/n, point index
p = i * ny + j with i the x index.
"""
from __future__ import annotations

import numpy as np


def grid_points(nx: int, ny: int | None = None) -> np.ndarray:
    """(nx*ny, 2) float64 cell-centred grid on [0, nx*h] x [0, ny*h], h = 1/max(nx, ny)."""
    ny = nx if ny is None else ny
    h = 1.0 / max(nx, ny)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    return np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h], axis=1)


def coef_const(points: np.ndarray) -> np.ndarray:
    """a(x) = 1."""
    return np.ones(points.shape[0])


def coef_sine(points: np.ndarray) -> np.ndarray:
    """a(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y)."""
    x, y = points[:, 0], points[:, 1]
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)


def coef_bumps(points: np.ndarray, rng: np.random.Generator, nbumps: int = 4,
               amp: float = 0.3) -> np.ndarray:
    """a(x) = 1 + amp * sum of nbumps Gaussian bumps, centres ~ U[0,1]^2,
    widths ~ U(0.05, 0.25)."""
    c = rng.uniform(0.0, 1.0, size=(nbumps, 2))
    s = rng.uniform(0.05, 0.25, size=nbumps)
    a = np.ones(points.shape[0])
    for b in range(nbumps):
        d2 = ((points - c[b]) ** 2).sum(axis=1)
        a += amp * np.exp(-d2 / (2 * s[b] ** 2))
    return a


def contrast_bump(points: np.ndarray, amp: float = 0.5, width: float = 0.15,
                  centre=(0.5, 0.5)) -> np.ndarray:
    """b(x) = amp * exp(-|x - centre|^2 / (2 width^2)) (scattering contrast)."""
    d2 = ((points - np.asarray(centre)) ** 2).sum(axis=1)
    return amp * np.exp(-d2 / (2 * width ** 2))


def rhs_uniform(n_points: int, nrhs: int, seed: int) -> np.ndarray:
    """(n_points, nrhs) column-major-friendly RHS ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(nrhs, n_points)).T)


def rhs_normal(n_points: int, nrhs: int, seed: int) -> np.ndarray:
    """(n_points, nrhs) RHS ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((nrhs, n_points)).T)


def shuffled(points: np.ndarray, seed: int):
    """A random permutation of the points (the solver accepts any point order)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(points.shape[0])
    return points[perm], perm


# Named workloads: grid side, coefficient, RHS recipe, tolerance.
WORKLOADS = {
    "laplace64": dict(n=64, coef="const", nrhs=1, rhs="uniform", seed=0, tol=1e-10),
    "laplace256": dict(n=256, coef="sine", nrhs=16, rhs="normal", seed=1, tol=1e-10),
    "laplace512": dict(n=512, coef="sine", nrhs=4, rhs="normal", seed=2, tol=1e-10),
}


def make_batch(n_inst: int = 64, seed: int = 3, side_lo: int = 32, side_hi: int = 256):
    """Many independent square grids of uneven size (side ~ U{side_lo..side_hi}),
    each with Gaussian-bump coefficients and one N(0,1) right-hand side.
    Returns (list of points, list of a, list of f, tol)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=n_inst)
    pts, coefs, rhs = [], [], []
    for n in sides:
        p = grid_points(int(n))
        pts.append(p)
        coefs.append(coef_bumps(p, rng))
        rhs.append(rng.standard_normal(p.shape[0]))
    return pts, coefs, rhs, 1e-8


def make_workload(name: str):
    """Return (points, a, f, tol) for a named workload."""
    w = WORKLOADS[name]
    pts = grid_points(w["n"])
    a = coef_const(pts) if w["coef"] == "const" else coef_sine(pts)
    gen = rhs_uniform if w["rhs"] == "uniform" else rhs_normal
    f = gen(pts.shape[0], w["nrhs"], w["seed"])
    return pts, a, f, w["tol"]


def rhs_complex_normal(n_points: int, nrhs: int, seed: int) -> np.ndarray:
    """(n_points, nrhs) complex RHS, real and imaginary parts ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nrhs, n_points)) + 1j * rng.standard_normal((nrhs, n_points))
    return np.ascontiguousarray(z.T)


# Served scattering workload: the Lippmann-Schwinger operator with the
# Helmholtz kernel at wavenumber 20 and a Gaussian contrast bump (amplitude
# 0.5, width 0.15, centred), grids of side 128 to 1024
SCATTER_K = 20.0
SCATTER_SIDES = (128, 256, 512, 1024)
