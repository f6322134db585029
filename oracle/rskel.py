"""The paper's compressed inverse, written out in its own order and notation.

TEST INFRASTRUCTURE ONLY (see package docstring).

Steps, each following the passage cited:
  tree        binary tree of boxes by bisection of a regular grid (Sec. 2.2)
  skeletons   I_i = I^sk_c1 u I^sk_c2 (leaves: all points); I_i^sk = points of
              I_i within m layers of the box boundary, I_i^rs the rest
              (Sec. 3.1, "Structure of skeleton sets in 2D")
  T_i         K(Z, X^sk) T = K(Z, X^rs) with Z the m grid layers just outside
              the box (Sec. 3.1; Sec. 3.3.2 and the remark after Algorithm 3
              for the rectangular least-squares case), solved through a
              column-pivoted QR truncated at tol * |R_11| (the ID of Sec. 2.1)
  R_i, L_i    R_i = [I T] Pi^T, L_i = R_i^T for symmetric A (Sec. 2.2 remark)
  inverse     Algorithm 1 (HSS inversion): F_i, E_i = (R F^{-1} L)^{-1},
              R~, D~, L~; direct inversion at the top
  apply       A^{-1} = D~ + L~ (A~^{l-1})^{-1} R~ applied recursively
              (Sec. 2.4, telescoping inverse), the dense-block form of
              Algorithm 6

Readings where the paper is silent (each listed in the design notes):
  * grid cell-centred, h = 1/max(nx, ny); leaves at most `leaf` points a
    side, every box split the same number of times per dimension (longer side
    first, x on ties), children low half first;
  * the layer rule is applied at the leaves too;
  * the proxy ring keeps all (a+2m)(b+2m) - ab nodes, including nodes outside
    the domain, and the rectangular system is solved in least squares;
  * m = 1 for tol >= 1e-6, m = 2 for 1e-11 <= tol < 1e-6, m = 3 below.
  * for a scaled kernel sqrt(b_i) G sqrt(b_j) the interpolation of the
    unscaled G is rescaled: T = diag(1/sqrt b_sk) T_G diag(sqrt b_rs).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import nystrom


def layers_for_tol(tol: float) -> int:
    if tol >= 1e-6:
        return 1
    if tol >= 1e-11:
        return 2
    return 3


def n_splits(side: int, leaf: int) -> int:
    """Smallest d with ceil(side / 2^d) <= leaf."""
    d = 0
    while -(-side // (1 << d)) > leaf:
        d += 1
    return d


@dataclass
class Box:
    x0: int
    x1: int
    y0: int
    y1: int
    depth: int
    children: list = field(default_factory=list)
    parent: "Box | None" = None
    # filled by skeletonisation
    act: np.ndarray | None = None     # global point indices of I_i
    sk: np.ndarray | None = None      # positions (into act) of I_i^sk
    rs: np.ndarray | None = None      # positions (into act) of I_i^rs
    T: np.ndarray | None = None
    R: np.ndarray | None = None
    # filled by Algorithm 1
    E: np.ndarray | None = None
    Dt: np.ndarray | None = None
    Lt: np.ndarray | None = None
    Rt: np.ndarray | None = None
    Ft: np.ndarray | None = None

    @property
    def shape(self):
        return (self.x1 - self.x0, self.y1 - self.y0)


def build_tree(nx: int, ny: int, leaf: int = 8) -> tuple[Box, list[list[Box]]]:
    """Binary tree by bisection (Sec. 2.2).  Returns the root and the boxes
    grouped by depth (0 = root)."""
    sx, sy = n_splits(nx, leaf), n_splits(ny, leaf)
    # global split schedule: the dimension with the longer remaining segment
    sched = []
    dx = dy = 0
    while dx < sx or dy < sy:
        lx = -(-nx // (1 << dx))
        ly = -(-ny // (1 << dy))
        if dx < sx and (dy >= sy or lx >= ly):
            sched.append(0)
            dx += 1
        else:
            sched.append(1)
            dy += 1
    root = Box(0, nx, 0, ny, 0)
    levels = [[root]]
    for d, dim in enumerate(sched):
        nxt = []
        for b in levels[-1]:
            if dim == 0:
                xm = b.x0 + (b.x1 - b.x0) // 2
                c = [Box(b.x0, xm, b.y0, b.y1, d + 1), Box(xm, b.x1, b.y0, b.y1, d + 1)]
            else:
                ym = b.y0 + (b.y1 - b.y0) // 2
                c = [Box(b.x0, b.x1, b.y0, ym, d + 1), Box(b.x0, b.x1, ym, b.y1, d + 1)]
            for cc in c:
                cc.parent = b
            b.children = c
            nxt.extend(c)
        levels.append(nxt)
    return root, levels


def interface_step(k: float, h: float, ppw: float) -> int:
    """Spacing in grid cells of the interface skeleton points for ppw points
    per wavelength 2 pi / k (Sec. 5.3, skeleton structure of the Helmholtz
    kernel); at least one cell."""
    return max(1, int(np.floor(2.0 * np.pi / (k * h * ppw))))


def skeleton_mask(b: Box, i, j, m: int, step: int = 0):
    """Which points (grid indices i, j) of box b's active set are skeleton:
    the m layers next to its boundary (Sec. 3.1), and with step > 0 also the
    points of the two grid lines on either side of the cut between its
    children whose distance past the boundary layers, along the cut, is
    step // 2 modulo step (a few points per wavelength on the interface,
    Sec. 5.3)."""
    d = np.minimum.reduce([i - b.x0, b.x1 - 1 - i, j - b.y0, b.y1 - 1 - j])
    sk = d < m
    if step > 0 and b.children:
        c1, c2 = b.children
        if c1.x1 == c2.x0:                       # cut across x
            line = (i == c1.x1 - 1) | (i == c1.x1)
            along, length = j - b.y0, b.y1 - b.y0
        else:                                    # cut across y
            line = (j == c1.y1 - 1) | (j == c1.y1)
            along, length = i - b.x0, b.x1 - b.x0
        past = np.minimum(along, length - 1 - along) - m
        sk = sk | (line & (past >= 0) & (past % step == step // 2))
    return sk


def index_sets(nx: int, ny: int, leaf: int, m: int, step: int = 0):
    """Active, skeleton and residual sets of every box (Sec. 3.1), without any
    kernel arithmetic.  Points are numbered p = i * ny + j.  Returns the tree
    levels with b.act (global ids), b.sk and b.rs (positions into b.act);
    step > 0 adds interface points (skeleton_mask)."""
    root, levels = build_tree(nx, ny, leaf)
    for depth in range(len(levels) - 1, -1, -1):
        for b in levels[depth]:
            if not b.children:
                ii, jj = np.meshgrid(np.arange(b.x0, b.x1), np.arange(b.y0, b.y1), indexing="ij")
                b.act = (ii * ny + jj).ravel()
            else:
                c1, c2 = b.children
                b.act = np.concatenate([c1.act[c1.sk], c2.act[c2.sk]])
            i, j = b.act // ny, b.act % ny
            msk = skeleton_mask(b, i, j, m, step)
            b.sk = np.nonzero(msk)[0]
            b.rs = np.nonzero(~msk)[0]
    return root, levels


class RSkel:
    """Dense-block recursive-skeletonisation inverse of the Nystrom matrix."""

    def __init__(self, points, a=None, tol=1e-10, leaf=8, layers=None,
                 kind="laplace", k=0.0, bvec=None, ppw=0.0):
        self.points = np.asarray(points, dtype=float)
        self.N = self.points.shape[0]
        self.a = np.ones(self.N) if a is None else np.asarray(a, dtype=float)
        self.tol = tol
        self.m = layers_for_tol(tol) if layers is None else layers
        self.kind, self.k, self.bvec = kind, k, bvec
        ix, iy, nx, ny, h = nystrom._grid_index(self.points)
        self.nx, self.ny, self.h = nx, ny, h
        self.ix, self.iy = ix, iy
        self.gid = np.full((nx, ny), -1, dtype=np.int64)
        self.gid[ix, iy] = np.arange(self.N)
        self.x0 = self.points[:, 0].min() - 0.5 * h
        self.y0 = self.points[:, 1].min() - 0.5 * h
        # interface skeleton points per wavelength (Helmholtz only)
        self.step = interface_step(k, h, ppw) if kind == "helmholtz" and ppw > 0 else 0
        self.root, self.levels = build_tree(nx, ny, leaf)
        self.dtype = complex if kind == "helmholtz" else float
        self.T_cache = {}
        self._skeletonise()
        self._invert()

    # -- matrix entries ------------------------------------------------------
    def A(self, rows, cols):
        return nystrom.assemble(self.points, self.a, self.kind, self.k, self.bvec, rows, cols)

    def K(self, P, Q):
        """Plain kernel K(|p - q|) between coordinate arrays."""
        r = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1))
        return nystrom.kernel(r, self.kind, self.k)

    # -- skeletons (Sec. 3.1) ----------------------------------------------
    def _in_layers(self, b: Box, idx):
        return skeleton_mask(b, self.ix[idx], self.iy[idx], self.m, self.step)

    def _proxy(self, b: Box):
        """Z: grid nodes within m layers outside the box (may lie outside the domain)."""
        m = self.m
        zi, zj = np.meshgrid(np.arange(b.x0 - m, b.x1 + m), np.arange(b.y0 - m, b.y1 + m),
                             indexing="ij")
        zi, zj = zi.ravel(), zj.ravel()
        out = ~((zi >= b.x0) & (zi < b.x1) & (zj >= b.y0) & (zj < b.y1))
        return np.stack([self.x0 + (zi[out] + 0.5) * self.h, self.y0 + (zj[out] + 0.5) * self.h], 1)

    def interp(self, b: Box, Xsk, Xrs):
        """T with K(Z, X^sk) T = K(Z, X^rs): truncated column-pivoted QR least
        squares (ID of Sec. 2.1 with the proxy acceleration of Sec. 2.2)."""
        Z = self._proxy(b)
        Ks = self.K(Z, Xsk)
        Kr = self.K(Z, Xrs)
        return truncated_qrcp_lstsq(Ks, Kr, self.tol)

    def _skeletonise(self):
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if not b.children:
                    ii, jj = np.meshgrid(np.arange(b.x0, b.x1), np.arange(b.y0, b.y1), indexing="ij")
                    b.act = self.gid[ii.ravel(), jj.ravel()]
                else:
                    c1, c2 = b.children
                    b.act = np.concatenate([c1.act[c1.sk], c2.act[c2.sk]])
                if b is self.root:
                    continue
                msk = self._in_layers(b, b.act)
                b.sk = np.nonzero(msk)[0]
                b.rs = np.nonzero(~msk)[0]
                k, r = len(b.sk), len(b.rs)
                Xsk = self.points[b.act[b.sk]]
                Xrs = self.points[b.act[b.rs]]
                T = self.interp(b, Xsk, Xrs) if r else np.zeros((k, 0))
                if self.bvec is not None and r:
                    sb = np.sqrt(self.bvec)
                    T = (1.0 / sb[b.act[b.sk]])[:, None] * T * sb[b.act[b.rs]][None, :]
                b.T = T
                R = np.zeros((k, k + r), dtype=self.dtype)
                R[:, b.sk] = np.eye(k)
                R[:, b.rs] = T
                b.R = R

    # -- Algorithm 1 -------------------------------------------------------
    def _invert(self):
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if not b.children:
                    F = self.A(b.act, b.act).astype(self.dtype)
                else:
                    c1, c2 = b.children
                    s1, s2 = c1.act[c1.sk], c2.act[c2.sk]
                    k1 = len(s1)
                    F = np.zeros((len(b.act), len(b.act)), dtype=self.dtype)
                    F[:k1, k1:] = self.A(s1, s2)
                    F[k1:, :k1] = self.A(s2, s1)
                    F[:k1, :k1] += c1.E
                    F[k1:, k1:] += c2.E
                if b is self.root:
                    b.Ft = np.linalg.inv(F)
                    continue
                Finv = np.linalg.inv(F)
                R = b.R
                L = R.T
                E = np.linalg.inv(R @ Finv @ L)
                b.E = E
                b.Rt = E @ R @ Finv
                b.Dt = Finv @ (np.eye(F.shape[0]) - L @ b.Rt)
                b.Lt = Finv @ L @ E

    # -- compressed forward product (Sec. 2.3, the factorization of A itself) --
    def forward_matvec(self, x):
        """y ~ A x through the skeletonization alone, in O(N) work: the block
        of A between two distinct boxes i, j is L_i A(sk_i, sk_j) R_j (the
        interpolation of Sec. 2.1 holds for every point outside a box), so A =
        D + L A~ R with D the leaf blocks and A~ the kernel on the skeletons,
        which telescopes up the tree.  Up: skeleton charges x^_b = R_b x_b
        (x_b the box's active vector, its children's charges).  Across: at
        every box above the leaves, each child's skeleton receives the kernel
        block to its sibling's skeleton times the sibling's charges.  Down:
        the potential y^_b on a skeleton spreads to the active points as
        L_b y^_b = R_b^T y^_b and into the children; leaves add their own
        dense block A(I_i, I_i) x_i."""
        x = np.asarray(x)
        X = x.reshape(self.N, -1).astype(np.result_type(x.dtype, self.dtype))
        charge = {}
        for depth in range(len(self.levels) - 1, 0, -1):
            for b in self.levels[depth]:
                if not b.children:
                    v = X[b.act]
                else:
                    v = np.concatenate([charge[id(c)] for c in b.children])
                charge[id(b)] = b.R @ v
        pot = {id(b): np.zeros_like(charge[id(b)]) for lev in self.levels[1:] for b in lev}
        for lev in self.levels:
            for b in lev:
                if b.children:
                    c1, c2 = b.children
                    s1, s2 = c1.act[c1.sk], c2.act[c2.sk]
                    pot[id(c1)] += self.A(s1, s2) @ charge[id(c2)]
                    pot[id(c2)] += self.A(s2, s1) @ charge[id(c1)]
        Y = np.zeros_like(X)
        for depth in range(1, len(self.levels)):
            for b in self.levels[depth]:
                spread = b.R.T @ pot[id(b)]          # on the active points
                if not b.children:
                    Y[b.act] = spread + self.A(b.act, b.act) @ X[b.act]
                else:
                    k1 = len(b.children[0].sk)
                    pot[id(b.children[0])] += spread[:k1]
                    pot[id(b.children[1])] += spread[k1:]
        if len(self.levels) == 1:                   # a single box: no compression
            Y = self.A(self.root.act, self.root.act) @ X
        return Y[:, 0] if x.ndim == 1 else Y

    # -- apply: A^{-1} f = D~ f + L~ (A~^{l-1})^{-1} R~ f --------------------
    def solve(self, f):
        f = np.asarray(f)
        F2 = f.reshape(self.N, -1).astype(np.result_type(f.dtype, self.dtype))
        rhs = {}
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if not b.children:
                    fb = F2[b.act]
                else:
                    fb = np.concatenate([rhs[id(c)][1] for c in b.children])
                if b is self.root:
                    rhs[id(b)] = (fb, None)
                else:
                    rhs[id(b)] = (fb, b.Rt @ fb)
        out = np.zeros_like(F2)
        phi = {id(self.root): self.root.Ft @ rhs[id(self.root)][0]}
        for depth in range(len(self.levels)):
            for b in self.levels[depth]:
                sol = phi[id(b)]
                if b is not self.root:
                    sol = b.Dt @ rhs[id(b)][0] + b.Lt @ sol
                if not b.children:
                    out[b.act] = sol
                else:
                    k1 = len(b.children[0].sk)
                    phi[id(b.children[0])] = sol[:k1]
                    phi[id(b.children[1])] = sol[k1:]
        return out[:, 0] if f.ndim == 1 else out


def truncated_qrcp_lstsq(Ks, Kr, tol):
    """min ||Ks T - Kr|| through Ks P = Q R (column pivoting, LAPACK geqp3),
    keeping the leading rho columns with |R_jj| > tol |R_11|:
    T = P [R11^{-1} Q1^* Kr ; 0]."""
    Q, R, piv = sla.qr(Ks, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    rho = int(np.sum(d > tol * d[0])) if d.size else 0
    k = Ks.shape[1]
    T = np.zeros((k, Kr.shape[1]), dtype=np.result_type(Ks.dtype, Kr.dtype))
    if rho:
        C = Q[:, :rho].conj().T @ Kr
        T[piv[:rho]] = sla.solve_triangular(R[:rho, :rho], C)
    return T
