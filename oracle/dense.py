"""Exact discrete solution by dense LU with partial pivoting.

TEST INFRASTRUCTURE ONLY (see package docstring).

The solver approximates sigma = A^{-1} f for the dense Nystrom matrix of
Sec. 5 (General formulation); this module computes that sigma directly
(LAPACK getrf/getrs through SciPy), the plain definition the compressed
inverse is measured against.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import nystrom


def solve(points, f, a=None, kind="laplace", k=0.0, bvec=None):
    """sigma = A^{-1} f with A assembled densely (float64 / complex128)."""
    A = nystrom.assemble(points, a, kind, k, bvec)
    lu = sla.lu_factor(A, overwrite_a=True, check_finite=False)
    return sla.lu_solve(lu, f, check_finite=False)


def rel_error(x, ref):
    """max over columns of |x - ref| / |ref| (2-norms)."""
    x = np.asarray(x).reshape(ref.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    return float(max(np.linalg.norm(x[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c])
                     for c in range(ref.shape[1])))
