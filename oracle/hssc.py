"""Compressed-block (HSS-C) inverse: the fast arithmetic of Sec. 3.3.

TEST INFRASTRUCTURE ONLY (see package docstring).

Above a skeleton size k_cut (remark at the end of Sec. 4.3) the per-box
blocks of the inverse are kept compressed instead of dense:

  HSS1D       a matrix on points ordered along a curve (a box's skeleton ring
              in cyclic order, or an interface strip along its direction),
              kept on a binary tree of contiguous ranges: dense diagonal
              blocks at the leaves, every off-diagonal sibling block as a
              low-rank product U V^T (weak admissibility).
  LR          a low-rank product U V^T.

Operations (Sec. 3.3.1), each written as its definition:
  hss1d_compress     entries of an operator -> HSS1D (off-diagonal blocks by
                     truncated SVD at the absolute threshold eps)
  hss1d_invert       HSS1D inverse by the recursive Woodbury identity on the
                     2 x 2 block form of every node (children inverted first,
                     the node's coupling as a low-rank update)
  hss1d_sum          A + B on one tree, generators concatenated, then
                     hss1d_recompress (every sum is followed by a
                     recompression, remark in Sec. 3.3.1)
  hss1d_split/merge  restriction to, or block-diagonal union of, point sets,
                     re-treed on the target order
  lr_to_hss1d        U V^T in HSS1D form
  rand_id            randomized interpolative decomposition of an operator
                     given by its products (Gaussian test matrix, blocks of 16
                     samples until the residual estimate is below eps)
  inter_lowrank      Algorithm 3: T = U V^T from the column ID of K(Z, X^rs)
  build_finv         Algorithm 4: (F^rs)^-1, F^{s<-r}, F^{r<-s} and the inverse
                     Schur complement (S^rs)^-1
  apply_finv         F^-1 u from those four blocks (block elimination of the
                     residual part first)
  build_e            Algorithm 5: E^-1 = phi_ss + T phi_rs + phi_sr T^T +
                     T phi_rr T^T (the dimensionally consistent reading of the
                     index-garbled formula of Sec. 3.2), recompressed, summed
                     with (S^rs)^-1 and inverted
  solve              Algorithm 6 with APPLY_Finv, the LR interpolation and the
                     HSS1D E of every compressed box

Readings (the paper defers the HSS1D internals to other work):
  * HSS1D here is the weak-admissibility form with a low-rank pair per
    sibling block (no nested bases): the same operations, a log factor more
    storage than nested generators;
  * truncations are absolute, at eps = tol * 0.1 (blocks of these matrices
    have norms of order one);
  * skeleton rings are ordered by angle around the box centre, interface
    strips by the coordinate along the interface;
  * the least-squares solve with K(Z, X^sk) in Algorithm 3 is the truncated
    pivoted QR of the dense-block path (the fast HSS least squares of the
    remark after Algorithm 3 computes the same T up to tol);
  * the root (and every box with k <= k_cut) is handled by the dense-block
    Algorithm 1, exactly as in rskel.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import nystrom
from .rskel import RSkel, truncated_qrcp_lstsq


# ----------------------------------------------------------------------------
# low-rank pairs
# ----------------------------------------------------------------------------
def recompress(U, V, eps):
    """U V^T -> U' V'^T of smallest rank with spectral error <= eps (QR of
    both factors, SVD of the small core)."""
    if U.shape[1] == 0 or U.shape[0] == 0 or V.shape[0] == 0:
        return U[:, :0], V[:, :0]
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    X, s, Yh = np.linalg.svd(Ru @ Rv.T)
    q = int(np.sum(s > eps))
    return Qu @ (X[:, :q] * s[:q]), Qv @ Yh[:q].T


def truncated_svd(B, eps):
    """Dense block -> U V^T with spectral error <= eps."""
    if B.size == 0:
        return B[:, :0], B.T[:, :0]
    X, s, Yh = np.linalg.svd(B, full_matrices=False)
    q = int(np.sum(s > eps))
    return X[:, :q] * s[:q], Yh[:q].T


def rand_id(matvec, rmatvec, m, n, eps, rng, block=16, dtype=float):
    """Randomized column ID of an m x n operator (Sec. 3.3.1): Y = Omega^T A
    grows in blocks of 16 Gaussian samples until a further block adds a
    residual below eps; the pivoted QR of Y gives the column skeleton J and
    T with A ~ A[:, J] [I T] Pi^T.  Returns (J, T, rest) with rest the
    non-skeleton columns in order."""
    Y = np.zeros((0, n), dtype=dtype)
    while True:
        Om = rng.standard_normal((m, block))
        Z = rmatvec(Om).T                     # block x n  = Om^T A
        if Y.shape[0]:
            # residual of the new samples against the row space of Y
            Q, _ = np.linalg.qr(Y.T)
            res = Z.T - Q @ (Q.T.conj() @ Z.T)
            Y = np.vstack([Y, Z])
            if np.linalg.norm(res, 2) <= eps or Y.shape[0] >= n:
                break
        else:
            Y = Z
            if Y.shape[0] >= n:
                break
    Q, R, piv = sla.qr(Y, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    # samples are Gaussian combinations of rows: scale the threshold by the
    # sample size (|Omega^T A| ~ sqrt(l) |A| for a column direction)
    q = int(np.sum(d > eps * np.sqrt(Y.shape[0]))) if d.size else 0
    J = piv[:q]
    rest = piv[q:]
    T = sla.solve_triangular(R[:q, :q], R[:q, q:]) if q else np.zeros((0, n - q))
    return J, T, rest


# ----------------------------------------------------------------------------
# HSS1D
# ----------------------------------------------------------------------------
def _tree(n, leaf):
    """Balanced bisection of [0, n) into contiguous ranges; node = [lo, hi,
    left, right] (children -1 at leaves).  Node 0 is the root."""
    nodes = [[0, n, -1, -1]]
    stack = [0]
    while stack:
        i = stack.pop()
        lo, hi = nodes[i][0], nodes[i][1]
        if hi - lo > leaf:
            mid = lo + (hi - lo) // 2
            nodes[i][2] = len(nodes)
            nodes.append([lo, mid, -1, -1])
            nodes[i][3] = len(nodes)
            nodes.append([mid, hi, -1, -1])
            stack += [nodes[i][2], nodes[i][3]]
    return nodes


class HSS1D:
    """Matrix on an ordered point set (global ids `ids`): dense leaves D,
    low-rank sibling blocks A[R1, R2] = U12 V12^T, A[R2, R1] = U21 V21^T."""

    def __init__(self, ids, leaf, eps, dtype=float):
        self.ids = np.asarray(ids)
        self.n = len(self.ids)
        self.leaf = leaf
        self.eps = eps
        self.dtype = dtype
        self.nodes = _tree(self.n, leaf)
        self.D = {}
        self.G = {}      # internal node -> (U12, V12, U21, V21)

    def ranges(self, i):
        lo, hi, a, b = self.nodes[i]
        return (lo, hi) if a < 0 else ((self.nodes[a][0], self.nodes[a][1]), (self.nodes[b][0], self.nodes[b][1]))

    def max_rank(self):
        return max([max(g[0].shape[1], g[2].shape[1]) for g in self.G.values()] + [0])

    def matvec(self, X):
        X = np.asarray(X)
        vec = X.ndim == 1
        X = X.reshape(self.n, -1)
        Y = np.zeros((self.n, X.shape[1]), dtype=np.result_type(self.dtype, X.dtype))
        for i, (lo, hi, a, b) in enumerate(self.nodes):
            if a < 0:
                Y[lo:hi] += self.D[i] @ X[lo:hi]
            else:
                (l1, h1), (l2, h2) = self.ranges(i)
                U12, V12, U21, V21 = self.G[i]
                Y[l1:h1] += U12 @ (V12.T @ X[l2:h2])
                Y[l2:h2] += U21 @ (V21.T @ X[l1:h1])
        return Y[:, 0] if vec else Y

    def rmatvec(self, X):
        """A^T X (plain transpose, also for complex entries)."""
        X = np.asarray(X)
        vec = X.ndim == 1
        X = X.reshape(self.n, -1)
        Y = np.zeros((self.n, X.shape[1]), dtype=np.result_type(self.dtype, X.dtype))
        for i, (lo, hi, a, b) in enumerate(self.nodes):
            if a < 0:
                Y[lo:hi] += self.D[i].T @ X[lo:hi]
            else:
                (l1, h1), (l2, h2) = self.ranges(i)
                U12, V12, U21, V21 = self.G[i]
                Y[l2:h2] += V12 @ (U12.T @ X[l1:h1])
                Y[l1:h1] += V21 @ (U21.T @ X[l2:h2])
        return Y[:, 0] if vec else Y

    def dense(self):
        return self.matvec(np.eye(self.n, dtype=self.dtype))

    def entries(self, P, Q):
        """Dense block A[P, Q] (positions), assembled from the representation."""
        out = np.zeros((len(P), len(Q)), dtype=self.dtype)
        P = np.asarray(P)
        Q = np.asarray(Q)
        for i, (lo, hi, a, b) in enumerate(self.nodes):
            if a < 0:
                pi = (P >= lo) & (P < hi)
                qi = (Q >= lo) & (Q < hi)
                if pi.any() and qi.any():
                    out[np.ix_(pi, qi)] += self.D[i][np.ix_(P[pi] - lo, Q[qi] - lo)]
            else:
                (l1, h1), (l2, h2) = self.ranges(i)
                U12, V12, U21, V21 = self.G[i]
                p1 = (P >= l1) & (P < h1)
                p2 = (P >= l2) & (P < h2)
                q1 = (Q >= l1) & (Q < h1)
                q2 = (Q >= l2) & (Q < h2)
                if p1.any() and q2.any():
                    out[np.ix_(p1, q2)] += U12[P[p1] - l1] @ V12[Q[q2] - l2].T
                if p2.any() and q1.any():
                    out[np.ix_(p2, q1)] += U21[P[p2] - l2] @ V21[Q[q1] - l1].T
        return out


def hss1d_compress(ids, entry, leaf, eps, dtype=float):
    """HSS1D_Compress: HSS1D of the operator whose entries between positions
    P and Q of `ids` are entry(P, Q); each off-diagonal sibling block by a
    truncated SVD at eps."""
    H = HSS1D(ids, leaf, eps, dtype)
    for i, (lo, hi, a, b) in enumerate(H.nodes):
        if a < 0:
            r = np.arange(lo, hi)
            H.D[i] = np.asarray(entry(r, r), dtype=dtype)
        else:
            (l1, h1), (l2, h2) = H.ranges(i)
            r1, r2 = np.arange(l1, h1), np.arange(l2, h2)
            U12, V12 = truncated_svd(np.asarray(entry(r1, r2), dtype=dtype), eps)
            U21, V21 = truncated_svd(np.asarray(entry(r2, r1), dtype=dtype), eps)
            H.G[i] = (U12, V12, U21, V21)
    return H


def lr_to_hss1d(ids, U, V, leaf, eps):
    """LR_to_HSS1D: U V^T (rows and columns on `ids`) in HSS1D form."""
    dtype = np.result_type(U.dtype, V.dtype)
    H = HSS1D(ids, leaf, eps, dtype)
    for i, (lo, hi, a, b) in enumerate(H.nodes):
        if a < 0:
            H.D[i] = U[lo:hi] @ V[lo:hi].T
        else:
            (l1, h1), (l2, h2) = H.ranges(i)
            U12, V12 = recompress(U[l1:h1], V[l2:h2], eps)
            U21, V21 = recompress(U[l2:h2], V[l1:h1], eps)
            H.G[i] = (U12, V12, U21, V21)
    return H


def hss1d_recompress(H):
    """HSS1D_Recompress: every sibling pair brought to its eps-rank."""
    for i, (U12, V12, U21, V21) in H.G.items():
        H.G[i] = recompress(U12, V12, H.eps) + recompress(U21, V21, H.eps)
    return H


def hss1d_sum(A, B):
    """HSS1D_Sum on one order and tree, followed by a recompression."""
    assert np.array_equal(A.ids, B.ids) and A.leaf == B.leaf
    C = HSS1D(A.ids, A.leaf, min(A.eps, B.eps), np.result_type(A.dtype, B.dtype))
    for i in A.D:
        C.D[i] = A.D[i] + B.D[i]
    for i in A.G:
        a, b = A.G[i], B.G[i]
        C.G[i] = (np.hstack([a[0], b[0]]), np.hstack([a[1], b[1]]),
                  np.hstack([a[2], b[2]]), np.hstack([a[3], b[3]]))
    return hss1d_recompress(C)


def add_lowrank(H, U, V):
    """H + U V^T on H's order and tree (LR_to_HSS1D + HSS1D_Sum)."""
    return hss1d_sum(H, lr_to_hss1d(H.ids, U, V, H.leaf, H.eps))


def hss1d_split(H, positions, leaf=None):
    """HSS1D_Split: the diagonal block of H on a subset of its positions (in
    the given order), as an HSS1D on its own tree."""
    pos = np.asarray(positions)
    return hss1d_compress(H.ids[pos], lambda P, Q: H.entries(pos[P], pos[Q]), leaf or H.leaf, H.eps, H.dtype)


def hss1d_invert(H):
    """HSS1D_Invert: recursive Woodbury.  For a node with children ranges R1,
    R2, A = diag(A11, A22) + Ub Vt^T with Ub = diag(U12, U21) and
    Vt = [[0, V21], [V12, 0]]; then A^-1 = D^-1 - P M^-1 Q^T, P = D^-1 Ub,
    Q = D^-T Vt, M = I + Vt^T P, whose diagonal blocks are the children's
    inverses plus a low-rank term and whose sibling blocks are low rank."""
    dt = H.dtype

    def rec(i):
        lo, hi, a, b = H.nodes[i]
        if a < 0:
            sub = HSS1D(H.ids[lo:hi], H.leaf, H.eps, dt)
            sub.D[0] = np.linalg.inv(H.D[i])
            return sub
        inv1, inv2 = rec(a), rec(b)
        U12, V12, U21, V21 = H.G[i]
        q1, q2 = U12.shape[1], U21.shape[1]
        P1 = inv1.matvec(U12)                 # A11^-1 U12
        P2 = inv2.matvec(U21)                 # A22^-1 U21
        Q1 = inv1.rmatvec(V21)                # A11^-T V21
        Q2 = inv2.rmatvec(V12)                # A22^-T V12
        M = np.eye(q1 + q2, dtype=np.result_type(dt, P1.dtype))
        M[:q1, q1:] = V12.T @ P2
        M[q1:, :q1] = V21.T @ P1
        Mi = np.linalg.inv(M)
        # diagonal blocks: A11^-1 - P1 Mi[q1, q2] Q1^T, A22^-1 - P2 Mi[q2, q1] Q2^T
        if q1 and q2:
            inv1 = add_lowrank(inv1, -P1 @ Mi[:q1, q1:], Q1)
            inv2 = add_lowrank(inv2, -P2 @ Mi[q1:, :q1], Q2)
        out = HSS1D(H.ids[lo:hi], H.leaf, H.eps, dt)
        # graft the children's trees below a new root
        _graft(out, inv1, inv2)
        G12 = recompress(-P1 @ Mi[:q1, :q1], Q2, H.eps)
        G21 = recompress(-P2 @ Mi[q1:, q1:], Q1, H.eps)
        out.G[0] = G12 + G21
        return out

    return rec(0)


def _graft(out, left, right):
    """Copy the leaves and sibling blocks of two sub-HSS1Ds into out, whose
    tree (same bisection) has them as the root's children."""
    a, b = out.nodes[0][2], out.nodes[0][3]

    def copy(src, si, di):
        lo, hi, sa, sb = src.nodes[si]
        if sa < 0:
            out.D[di] = src.D[si]
            return
        out.G[di] = src.G[si]
        copy(src, sa, out.nodes[di][2])
        copy(src, sb, out.nodes[di][3])

    copy(left, 0, a)
    copy(right, 0, b)


# ----------------------------------------------------------------------------
# the compressed-block inverse
# ----------------------------------------------------------------------------
class HSSC(RSkel):
    """Algorithm 1 with the compressed blocks of Sec. 3.3 for every box whose
    skeleton has more than k_cut points (dense blocks below, as in rskel)."""

    def __init__(self, points, a=None, tol=1e-10, leaf=8, layers=None, k_cut=64, hss_leaf=32,
                 kind="laplace", k=0.0, bvec=None, seed=0):
        self.k_cut = k_cut
        self.hss_leaf = hss_leaf
        self.eps = 0.1 * tol
        self.rng = np.random.default_rng(seed)
        self.stats = {"compressed_boxes": 0, "max_rank": 0}
        super().__init__(points, a, tol, leaf, layers, kind, k, bvec)

    # ---- orderings -------------------------------------------------------
    def _ring_order(self, b, ids):
        """Skeleton ids of box b ordered cyclically (angle about its centre)."""
        P = self.points[ids]
        cx = self.x0 + 0.5 * (b.x0 + b.x1) * self.h
        cy = self.y0 + 0.5 * (b.y0 + b.y1) * self.h
        ang = np.arctan2(P[:, 1] - cy, P[:, 0] - cx)
        rad = np.hypot(P[:, 0] - cx, P[:, 1] - cy)
        return ids[np.lexsort((rad, ang))]

    def _line_order(self, b, ids):
        """Interface ids of box b ordered along the interface between its
        children (the split line), then across it."""
        c1 = b.children[0]
        split_x = c1.x1 != b.x1
        P = self.points[ids]
        along, across = (P[:, 1], P[:, 0]) if split_x else (P[:, 0], P[:, 1])
        return ids[np.lexsort((across, along))]

    def compressed(self, b):
        return b is not self.root and b.children and len(b.sk) > self.k_cut

    # ---- INTER_LOWRANK (Algorithm 3) ----------------------------------------
    def inter_lowrank(self, b, Xsk, Xrs):
        """T = U V^T: column ID of K(Z, X^rs) (RAND_ID), then
        U = K(Z, X^sk)^+ K(Z, X^rs[:, J]) and V^T[:, J] = I, V^T[:, rest] = T_rp."""
        Z = self._proxy(b)
        Ks = self.K(Z, Xsk)
        Kr = self.K(Z, Xrs)
        scale = np.linalg.norm(Kr, 2)
        J, Trp, rest = rand_id(lambda X: Kr @ X, lambda Y: Kr.T @ Y, Kr.shape[0], Kr.shape[1],
                               self.tol * scale, self.rng, dtype=Kr.dtype)
        U = truncated_qrcp_lstsq(Ks, Kr[:, J], self.tol)
        V = np.zeros((Kr.shape[1], len(J)), dtype=np.result_type(U.dtype, Trp.dtype))
        V[J] = np.eye(len(J))
        V[rest] = Trp.T
        return U, V

    # ---- entries of F_i on its children's skeletons ------------------------
    def _F_entries(self, b):
        """entry(P, Q) for global-id arrays: the children's E where both ids
        belong to one child, the kernel where they do not (Algorithm 1, line 5)."""
        c1, c2 = b.children
        own_c = np.full(self.N, -1)
        own_p = np.full(self.N, -1)
        for ci, c in enumerate((c1, c2)):
            own_c[c.E_ids] = ci
            own_p[c.E_ids] = np.arange(len(c.E_ids))

        def entry(Pg, Qg):
            Pg = np.asarray(Pg)
            Qg = np.asarray(Qg)
            out = self.A(Pg, Qg).astype(self.dtype)
            for ci, c in enumerate((c1, c2)):
                pm = own_c[Pg] == ci
                qm = own_c[Qg] == ci
                if pm.any() and qm.any():
                    out[np.ix_(pm, qm)] = c.E_entries(own_p[Pg[pm]], own_p[Qg[qm]])
            return out
        return entry

    # ---- BUILD_Finv (Algorithm 4) and BUILD_E (Algorithm 5) ----------------
    def _compressed_box(self, b):
        entry = self._F_entries(b)
        S_ids = self._ring_order(b, b.act[b.sk])
        R_ids = self._line_order(b, b.act[b.rs])
        L, eps = self.hss_leaf, self.eps
        # (i)-(ii) split the children's E into boundary and interface parts,
        # merge them and add the compressed sibling interactions: F^sk, F^rs
        Fsk = hss1d_compress(S_ids, lambda P, Q: entry(S_ids[P], S_ids[Q]), L, eps, self.dtype)
        Frs = hss1d_compress(R_ids, lambda P, Q: entry(R_ids[P], R_ids[Q]), L, eps, self.dtype)
        # (iii) (F^rs)^-1
        Frs_inv = hss1d_invert(Frs)
        # (iv) F^{s<-r} by a randomized ID; F^{r<-s} is its transpose (symmetric F)
        Bsr = entry(S_ids, R_ids)
        scale = max(np.linalg.norm(Bsr, 2), 1e-300)
        J, Tb, rest = rand_id(lambda X: Bsr @ X, lambda Y: Bsr.T @ Y, len(S_ids), len(R_ids), eps, self.rng,
                              dtype=Bsr.dtype)
        Ub = Bsr[:, J]
        Vb = np.zeros((len(R_ids), len(J)), dtype=Bsr.dtype)
        Vb[J] = np.eye(len(J))
        Vb[rest] = Tb.T
        # (v) S^rs = F^sk - F^{s<-r} (F^rs)^-1 F^{r<-s}, then its inverse
        W = Frs_inv.matvec(Vb)                            # (F^rs)^-1 Vb
        core = Vb.T @ W                                   # Vb^T (F^rs)^-1 Vb
        Srs = add_lowrank(Fsk, -Ub @ core, Ub)
        Srs_inv = hss1d_invert(Srs)
        # BUILD_E: T = U_T V_T^T on (S_ids, R_ids) order
        T_U, T_V = b.T_lr
        W1 = Frs_inv.rmatvec(T_V)                         # (F^rs)^-T V_T
        W2 = Frs_inv.rmatvec(Vb)                          # (F^rs)^-T Vb
        G1 = W1.T @ Vb                                    # V_T^T (F^rs)^-1 Vb
        Z = Srs_inv.rmatvec(Ub)                           # (S^rs)^-T Ub
        X = -G1 @ Z.T                                     # V_T^T phi_rs
        C = W1.T @ T_V + G1 @ (Z.T @ Ub) @ (W2.T @ T_V)   # V_T^T phi_rr V_T
        UE = np.hstack([T_U, X.T])
        VE = np.hstack([(X + C @ T_U.T).T, T_U])
        UE, VE = recompress(UE, VE, eps)
        Einv = add_lowrank(Srs_inv, UE, VE)
        E = hss1d_invert(Einv)
        b.E_hss = E
        b.E_ids = S_ids
        b.E_entries = E.entries
        b.blocks = dict(S_ids=S_ids, R_ids=R_ids, Frs_inv=Frs_inv, Ub=Ub, Vb=Vb, Srs_inv=Srs_inv)
        self.stats["compressed_boxes"] += 1
        self.stats["max_rank"] = max(self.stats["max_rank"], E.max_rank(), Srs_inv.max_rank(),
                                     Frs_inv.max_rank(), Ub.shape[1], T_U.shape[1])

    def apply_finv(self, b, us, ur):
        """APPLY_Finv: F^-1 [u_s; u_r] with the residual part eliminated first:
        x_s = (S^rs)^-1 (u_s - F^{s<-r} (F^rs)^-1 u_r), x_r = (F^rs)^-1 (u_r - F^{r<-s} x_s)."""
        k = b.blocks
        y = k["Frs_inv"].matvec(ur)
        xs = k["Srs_inv"].matvec(us - k["Ub"] @ (k["Vb"].T @ y))
        xr = k["Frs_inv"].matvec(ur - k["Vb"] @ (k["Ub"].T @ xs))
        return xs, xr

    # ---- the build --------------------------------------------------------
    def _skeletonise(self):
        super()._skeletonise()
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if self.compressed(b):
                    S_ids = self._ring_order(b, b.act[b.sk])
                    R_ids = self._line_order(b, b.act[b.rs])
                    U, V = self.inter_lowrank(b, self.points[S_ids], self.points[R_ids])
                    if self.bvec is not None:
                        # T of sqrt(b) G sqrt(b) from T of G (as in rskel)
                        sb = np.sqrt(self.bvec)
                        U = U / sb[S_ids][:, None]
                        V = V * sb[R_ids][:, None]
                    b.T_lr = (U, V)

    def _invert(self):
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if self.compressed(b):
                    self._compressed_box(b)
                    continue
                # dense-block box (Algorithm 1), its children's E read from
                # their representation
                if not b.children:
                    F = self.A(b.act, b.act).astype(self.dtype)
                else:
                    F = self._F_entries(b)(b.act, b.act)
                if b is self.root:
                    b.Ft = np.linalg.inv(F)
                    continue
                Finv = np.linalg.inv(F)
                R = b.R
                Lm = R.T
                E = np.linalg.inv(R @ Finv @ Lm)
                b.E = E
                b.Rt = E @ R @ Finv
                b.Dt = Finv @ (np.eye(F.shape[0]) - Lm @ b.Rt)
                b.Lt = Finv @ Lm @ E
                sk_ids = b.act[b.sk]
                if b.parent is not None and self.compressed(b.parent):
                    # a dense E entering a compressed parent: HSS1D_Compress it
                    order = self._ring_order(b, sk_ids)
                    pos = {int(g): i for i, g in enumerate(sk_ids)}
                    perm = np.array([pos[int(g)] for g in order])
                    Ed = E[np.ix_(perm, perm)]
                    H = hss1d_compress(order, lambda P, Q: Ed[np.ix_(P, Q)], self.hss_leaf, self.eps, self.dtype)
                    b.E_ids = order
                    b.E_entries = H.entries
                else:
                    b.E_ids = sk_ids
                    b.E_entries = (lambda EE: (lambda P, Q: EE[np.ix_(P, Q)]))(E)

    # ---- Algorithm 6 --------------------------------------------------------
    def solve(self, f):
        f = np.asarray(f)
        F2 = f.reshape(self.N, -1).astype(np.result_type(f.dtype, self.dtype))
        up = {}          # box -> (u in act order, up-vector in E_ids order, extra)
        for depth in range(len(self.levels) - 1, -1, -1):
            for b in self.levels[depth]:
                if not b.children:
                    u = F2[b.act]
                else:
                    u = self._gather_children(b, up)
                if b is self.root:
                    up[id(b)] = (u, None, None)
                elif self.compressed(b):
                    us, ur = self._split(b, u)
                    xs, xr = self.apply_finv(b, us, ur)
                    T_U, T_V = b.T_lr
                    t = xs + T_U @ (T_V.T @ xr)             # R phi = phi_s + T phi_r
                    g = b.E_hss.matvec(t)                   # u^up = E R phi (E_ids = S order)
                    up[id(b)] = (u, g, None)
                else:
                    g = b.Rt @ u                            # in b.act[b.sk] order
                    if hasattr(b, "E_ids") and not np.array_equal(b.E_ids, b.act[b.sk]):
                        pos = {int(gg): i for i, gg in enumerate(b.act[b.sk])}
                        g = g[[pos[int(x)] for x in b.E_ids]]
                    up[id(b)] = (u, g, None)
        out = np.zeros_like(F2)
        phi = {id(self.root): self.root.Ft @ up[id(self.root)][0]}
        for depth in range(len(self.levels)):
            for b in self.levels[depth]:
                u, g, _ = up[id(b)]
                ph = phi[id(b)]                              # on E_ids order (root: act order)
                if b is self.root:
                    sol = ph
                elif self.compressed(b):
                    # sigma = F^-1 (u - L u^up + L E phi) = F^-1 (u + L (E phi - u^up))
                    w = b.E_hss.matvec(ph) - g
                    T_U, T_V = b.T_lr
                    us, ur = self._split(b, u)
                    xs, xr = self.apply_finv(b, us + w, ur + T_V @ (T_U.T @ w))
                    sol = self._join(b, xs, xr)
                else:
                    if not np.array_equal(b.E_ids, b.act[b.sk]):
                        pos = {int(gg): i for i, gg in enumerate(b.E_ids)}
                        ph = ph[[pos[int(x)] for x in b.act[b.sk]]]
                    sol = b.Dt @ u + b.Lt @ ph
                if not b.children:
                    out[b.act] = sol
                else:
                    for c in b.children:
                        idx = {int(gg): i for i, gg in enumerate(b.act)}
                        phi[id(c)] = sol[[idx[int(x)] for x in c.E_ids]]
        return out[:, 0] if f.ndim == 1 else out

    def _gather_children(self, b, up):
        """u on b.act from the children's up-vectors (each on its E_ids order)."""
        idx = {int(g): i for i, g in enumerate(b.act)}
        u = None
        for c in b.children:
            gv = up[id(c)][1]
            if u is None:
                u = np.zeros((len(b.act), gv.shape[1]), dtype=gv.dtype)
            u[[idx[int(x)] for x in c.E_ids]] = gv
        return u

    def _split(self, b, u):
        idx = {int(g): i for i, g in enumerate(b.act)}
        k = b.blocks
        return u[[idx[int(x)] for x in k["S_ids"]]], u[[idx[int(x)] for x in k["R_ids"]]]

    def _join(self, b, xs, xr):
        idx = {int(g): i for i, g in enumerate(b.act)}
        k = b.blocks
        out = np.zeros((len(b.act), xs.shape[1]), dtype=np.result_type(xs.dtype, xr.dtype))
        out[[idx[int(x)] for x in k["S_ids"]]] = xs
        out[[idx[int(x)] for x in k["R_ids"]]] = xr
        return out
