"""Nystrom discretisation of a(x) s(x) + int b(x) K(|x-y|) c(y) s(y) dy = f(x).

TEST INFRASTRUCTURE ONLY (see package docstring).

Follows Sec. 5 ("General formulation"): on a regular grid with spacing h,
    A_ij = a(x_i) delta_ij + h^2 b(x_i) K(|x_i - x_j|) c(x_j),   i != j.
The paper does not say how the singular diagonal entry is formed for the
Laplace kernel; the reading used here is that the diagonal carries the exact
integral of the kernel over the point's own square cell (an O(h^2) quantity),
    A_ii = a(x_i) + b(x_i) c(x_i) * int_{cell_i} K(|x_i - y|) dy.

Kernels (Sec. 2.2 and Sec. 5.3):
    Laplace    K(r) = (1/2pi) log r
    Helmholtz  G(r) = (i/4) H0^(1)(k r)   (outgoing fundamental solution of
               -Lap - k^2; the sign printed in Sec. 5.3 is read as a misprint,
               since the scattering derivation of Sec. 5.4 needs this one)
The scattering (Lippmann-Schwinger) operator of Sec. 5.4 is the special case
a = 1, b = c = sqrt(contrast).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sps


# ----------------------------------------------------------------------------
# Kernels
# ----------------------------------------------------------------------------
def laplace_kernel(r):
    """K(r) = log(r) / (2 pi) (Sec. 2.2, equivalent-density paragraph)."""
    return np.log(r) / (2.0 * np.pi)


def helmholtz_kernel(r, k):
    """G(r) = (i/4) H0^(1)(k r)."""
    return 0.25j * sps.hankel1(0, k * r)


def kernel(r, kind="laplace", k=0.0):
    if kind == "laplace":
        return laplace_kernel(r)
    if kind == "helmholtz":
        return helmholtz_kernel(r, k)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Self-cell integrals int_{[-h/2,h/2]^2} K(|y|) dy
# ----------------------------------------------------------------------------
def self_cell_laplace(h: float) -> float:
    """Exact integral of (1/2pi) log|y| over the square cell of side h centred
    at the origin.  Scaling y = h u gives h^2 (log h + J) / (2 pi) with
    J = int_{[-1/2,1/2]^2} log|u| du = -log(2)/2 - 3/2 + pi/4 (integrating over
    the eight triangles cut by the diagonals in polar coordinates)."""
    J = -0.5 * math.log(2.0) - 1.5 + math.pi / 4.0
    return h * h * (math.log(h) + J) / (2.0 * math.pi)


def _gauss_legendre(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def self_cell_helmholtz(h: float, k: float, nq: int = 24) -> complex:
    """int over the centred cell of (i/4) H0^(1)(k|y|) dy.

    G(r) = -(1/2pi) log r + R(r) with R bounded and smooth in r (its leading
    behaviour is r^2 log r), so the integral is the closed-form Laplace term
    with a minus sign plus a Gauss-Legendre quadrature of R over the eight
    triangles of the cell in polar coordinates (r from 0 to h/(2 cos t))."""
    lap = -self_cell_laplace(h)
    t, wt = _gauss_legendre(nq, 0.0, np.pi / 4)
    total = 0.0 + 0.0j
    for tt, ww in zip(t, wt):
        rmax = h / (2.0 * np.cos(tt))
        r, wr = _gauss_legendre(nq, 0.0, rmax)
        g = 0.25j * sps.hankel1(0, k * r) + np.log(r) / (2.0 * np.pi)
        total += ww * np.sum(wr * r * g)
    return lap + 8.0 * total


def self_cell(h, kind="laplace", k=0.0):
    if kind == "laplace":
        return self_cell_laplace(h)
    return self_cell_helmholtz(h, k)


# ----------------------------------------------------------------------------
# Dense assembly
# ----------------------------------------------------------------------------
def grid_spacing(points: np.ndarray) -> float:
    xs = np.unique(points[:, 0])
    ys = np.unique(points[:, 1])
    d = np.concatenate([np.diff(xs), np.diff(ys)])
    return float(np.median(d))


def assemble(points, a=None, kind="laplace", k=0.0, bvec=None, rows=None, cols=None):
    """Dense (sub)matrix A(rows, cols) of the Nystrom system.

    bvec, if given, is the scattering contrast: entries become
    sqrt(b_i) h^2 G sqrt(b_j) off the diagonal and 1 + b_i int_cell G on it.
    """
    n_pts = points.shape[0]
    h = grid_spacing(points)
    rows = np.arange(n_pts) if rows is None else np.asarray(rows)
    cols = np.arange(n_pts) if cols is None else np.asarray(cols)
    a = np.ones(n_pts) if a is None else np.asarray(a)
    P = points[rows]
    Q = points[cols]
    r = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1))
    same = rows[:, None] == cols[None, :]
    r = np.where(same, 1.0, r)
    Kv = h * h * kernel(r, kind, k)
    sc = self_cell(h, kind, k)
    if bvec is not None:
        sb = np.sqrt(np.asarray(bvec))
        Kv = sb[rows][:, None] * Kv * sb[cols][None, :]
        diag = 1.0 + bvec[rows] * sc
    else:
        diag = a[rows] + sc
    Kv = np.where(same, 0.0, Kv)
    return Kv + np.where(same, diag[:, None], 0.0)


# ----------------------------------------------------------------------------
# Exact products u = A s without forming A
# ----------------------------------------------------------------------------
def matvec_direct(points, s, a=None, kind="laplace", k=0.0, bvec=None, block=2048):
    """u = A s by a blocked direct sum over all pairs (exact, O(N^2))."""
    n_pts = points.shape[0]
    s = np.asarray(s)
    vec = s.ndim == 1
    S = s.reshape(n_pts, -1)
    out = np.zeros(S.shape, dtype=np.result_type(S.dtype, complex if kind == "helmholtz" else float))
    for i0 in range(0, n_pts, block):
        rows = np.arange(i0, min(n_pts, i0 + block))
        for j0 in range(0, n_pts, block):
            cols = np.arange(j0, min(n_pts, j0 + block))
            out[rows] += assemble(points, a, kind, k, bvec, rows, cols) @ S[cols]
    return out[:, 0] if vec else out


def _grid_index(points):
    """(ix, iy, nx, ny, h) for points on a regular grid."""
    h = grid_spacing(points)
    x0 = points[:, 0].min()
    y0 = points[:, 1].min()
    ix = np.rint((points[:, 0] - x0) / h).astype(np.int64)
    iy = np.rint((points[:, 1] - y0) / h).astype(np.int64)
    return ix, iy, int(ix.max()) + 1, int(iy.max()) + 1, h


def matvec_fft(points, s, a=None, kind="laplace", k=0.0, bvec=None):
    """u = A s by FFT convolution with the kernel on grid offsets.

    The off-diagonal part of A is h^2 K(h |(di, dj)|), a function of the grid
    offset only, so A s is a 2-D aperiodic convolution; it is evaluated with a
    zero-padded (2nx) x (2ny) FFT.  Exact up to FFT rounding."""
    n_pts = points.shape[0]
    ix, iy, nx, ny, h = _grid_index(points)
    s = np.asarray(s)
    vec = s.ndim == 1
    S = s.reshape(n_pts, -1)
    a = np.ones(n_pts) if a is None else np.asarray(a)
    Px, Py = 2 * nx, 2 * ny
    di = np.arange(Px)
    di = np.where(di < nx, di, di - Px)
    dj = np.arange(Py)
    dj = np.where(dj < ny, dj, dj - Py)
    r = h * np.sqrt(di[:, None] ** 2 + dj[None, :] ** 2)
    r[0, 0] = 1.0
    Kt = h * h * kernel(r, kind, k)
    Kt[0, 0] = 0.0
    Khat = np.fft.fft2(Kt)
    sc = self_cell(h, kind, k)
    if bvec is not None:
        sb = np.sqrt(np.asarray(bvec))
    out = np.zeros(S.shape, dtype=complex if (kind == "helmholtz" or np.iscomplexobj(S)) else float)
    for c in range(S.shape[1]):
        col = S[:, c] * (sb if bvec is not None else 1.0)
        g = np.zeros((Px, Py), dtype=complex)
        g[ix, iy] = col
        conv = np.fft.ifft2(np.fft.fft2(g) * Khat)[ix, iy]
        if bvec is not None:
            u = sb * conv + (1.0 + bvec * sc) * S[:, c]
        else:
            u = conv + (a + sc) * S[:, c]
        out[:, c] = u if np.iscomplexobj(out) else u.real
    return out[:, 0] if vec else out
