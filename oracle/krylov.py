"""Restarted GMRES on the exact matrix-vector product.

TEST INFRASTRUCTURE ONLY (see package docstring).

For grids too large to assemble A (N = 262144 needs 550 GB) the exact
discrete solution is obtained iteratively: GMRES(restart) with the FFT
convolution product of `nystrom.matvec_fft`, run to a relative residual far
below the solver's target.  Plain modified Gram-Schmidt Arnoldi with Givens
rotations (Saad and Schultz, 1986).
"""
from __future__ import annotations

import numpy as np

from . import nystrom


def gmres(matvec, b, tol=1e-13, restart=50, maxiter=2000, x0=None):
    """Solve M x = b for one right-hand side; returns (x, rel_residual, iters)."""
    b = np.asarray(b)
    dt = np.result_type(b.dtype, float)
    x = np.zeros_like(b, dtype=dt) if x0 is None else np.array(x0, dtype=dt)
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0.0, 0
    it = 0
    while it < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            return x, beta / bn, it
        V = np.zeros((restart + 1, b.size), dtype=dt)
        H = np.zeros((restart + 1, restart), dtype=dt)
        cs = np.zeros(restart, dtype=dt)
        sn = np.zeros(restart, dtype=dt)
        g = np.zeros(restart + 1, dtype=dt)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(restart):
            w = matvec(V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = np.conj(cs[j]) * H[j, j] + np.conj(sn[j]) * H[j + 1, j]
            H[j + 1, j] = 0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_used = j + 1
            if abs(g[j + 1]) / bn <= tol * 0.5:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + V[:j_used].T @ y
    r = b - matvec(x)
    return x, np.linalg.norm(r) / bn, it


def solve(points, f, a=None, kind="laplace", k=0.0, bvec=None, tol=1e-13, restart=50):
    """sigma = A^{-1} f column by column with the exact FFT product."""
    F = np.asarray(f).reshape(points.shape[0], -1)
    out = np.zeros(F.shape, dtype=complex if (kind == "helmholtz" or np.iscomplexobj(F)) else float)
    info = []
    for c in range(F.shape[1]):
        mv = lambda v: nystrom.matvec_fft(points, v, a, kind, k, bvec)
        x, res, its = gmres(mv, F[:, c], tol=tol, restart=restart)
        out[:, c] = x
        info.append((res, its))
    return (out[:, 0] if np.asarray(f).ndim == 1 else out), info
