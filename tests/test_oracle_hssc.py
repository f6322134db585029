"""Pins of the compressed-block (HSS-C) arithmetic of the CPU reference
(oracle/hssc.py, Sec. 3.3), each against its dense definition, and the whole
compressed inverse against the dense solve.  Planted mistakes (a wrong sign,
a dropped term, a transposed operand) in copies of the routines must fail
the same checks."""
import numpy as np
import pytest

from oracle import dense, hssc, nystrom, rskel
from paper_1303_5466_amd import workloads as W


def _ring(n_side=24, m=2, h=1 / 64):
    """A two-layer box boundary (skeleton-like ring), ordered by angle, and
    its dense Laplace matrix a + h^2 K (a = 1 on the diagonal)."""
    ii, jj = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    d = np.minimum.reduce([ii, n_side - 1 - ii, jj, n_side - 1 - jj])
    P = np.stack([ii[d < m], jj[d < m]], 1) * h
    c = P.mean(0)
    order = np.lexsort((np.hypot(*(P - c).T), np.arctan2(P[:, 1] - c[1], P[:, 0] - c[0])))
    P = P[order]
    r = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1))
    np.fill_diagonal(r, 1.0)
    A = h * h * nystrom.laplace_kernel(r)
    np.fill_diagonal(A, 1.0 + nystrom.self_cell_laplace(h))
    return P, A


def test_recompress_keeps_the_eps_rank():
    rng = np.random.default_rng(0)
    U0, V0 = rng.standard_normal((60, 5)), rng.standard_normal((40, 5))
    # the same rank-5 product written with redundant generators, plus noise
    U = np.hstack([U0, U0 @ rng.standard_normal((5, 7))])
    V = np.hstack([V0, np.zeros((40, 7))])
    U2, V2 = hssc.recompress(U, V, 1e-9)
    assert U2.shape[1] == 5
    assert np.linalg.norm(U2 @ V2.T - U0 @ V0.T, 2) <= 1e-9
    # exact zero -> rank 0
    U3, V3 = hssc.recompress(np.zeros((10, 3)), np.ones((8, 3)), 1e-12)
    assert U3.shape[1] == 0


def test_rand_id_reproduces_the_operator():
    rng = np.random.default_rng(1)
    m, n, q = 80, 120, 9
    A = rng.standard_normal((m, q)) @ rng.standard_normal((q, n)) + 1e-13 * rng.standard_normal((m, n))
    J, T, rest = hssc.rand_id(lambda X: A @ X, lambda Y: A.T @ Y, m, n, 1e-10, rng)
    assert len(J) == q
    approx = np.zeros_like(A)
    approx[:, J] = A[:, J]
    approx[:, rest] = A[:, J] @ T
    assert np.linalg.norm(A - approx, 2) <= 1e-9 * np.linalg.norm(A, 2)
    assert sorted(np.concatenate([J, rest]).tolist()) == list(range(n))


@pytest.mark.parametrize("n_side", [16, 40])
def test_hss1d_compress_matvec_and_ranks(n_side):
    P, A = _ring(n_side)
    H = hssc.hss1d_compress(np.arange(len(P)), lambda I, J: A[np.ix_(I, J)], 32, 1e-12)
    assert np.linalg.norm(H.dense() - A, 2) <= 1e-10
    x = np.random.default_rng(2).standard_normal((len(P), 3))
    assert np.allclose(H.matvec(x), A @ x, rtol=0, atol=1e-11)
    assert np.allclose(H.rmatvec(x), A.T @ x, rtol=0, atol=1e-11)
    # off-diagonal ranks of a boundary-curve kernel matrix stay small
    assert H.max_rank() <= 40


def test_hss1d_ranks_grow_slowly_with_the_curve():
    r = []
    for n_side in (32, 64, 128):
        P, A = _ring(n_side, h=1 / 256)
        H = hssc.hss1d_compress(np.arange(len(P)), lambda I, J: A[np.ix_(I, J)], 32, 1e-11)
        r.append(H.max_rank())
    # 4x the points, far less than 4x the rank (logarithmic growth)
    assert r[2] <= 1.6 * r[0] + 8, r


def test_hss1d_invert_sum_split_lowrank():
    P, A = _ring(40)
    n = len(P)
    ids = np.arange(n)
    eps = 1e-12
    H = hssc.hss1d_compress(ids, lambda I, J: A[np.ix_(I, J)], 32, eps)
    Hi = hssc.hss1d_invert(H)
    Ai = np.linalg.inv(A)
    assert np.linalg.norm(Hi.dense() - Ai, 2) <= 1e-10 * np.linalg.norm(Ai, 2)
    rng = np.random.default_rng(3)
    U, V = rng.standard_normal((n, 4)) * 1e-3, rng.standard_normal((n, 4))
    L = hssc.lr_to_hss1d(ids, U, V, 32, eps)
    assert np.linalg.norm(L.dense() - U @ V.T, 2) <= 1e-10
    S = hssc.hss1d_sum(H, L)
    assert np.linalg.norm(S.dense() - (A + U @ V.T), 2) <= 1e-10
    pos = np.arange(10, n - 7)
    Sp = hssc.hss1d_split(H, pos)
    assert np.linalg.norm(Sp.dense() - A[np.ix_(pos, pos)], 2) <= 1e-10


def test_planted_woodbury_mistake_is_caught():
    # a dropped low-rank update of the diagonal blocks in the inverse
    P, A = _ring(24)
    H = hssc.hss1d_compress(np.arange(len(P)), lambda I, J: A[np.ix_(I, J)], 16, 1e-12)
    orig = hssc.add_lowrank
    try:
        hssc.add_lowrank = lambda Hh, U, V: Hh
        bad = hssc.hss1d_invert(H).dense()
    finally:
        hssc.add_lowrank = orig
    Ai = np.linalg.inv(A)
    assert np.linalg.norm(bad - Ai, 2) > 1e-8 * np.linalg.norm(Ai, 2)


def test_inter_lowrank_interpolates_exterior_sources():
    # T = U V^T of Algorithm 3 interpolates the field of every exterior
    # source (not only the proxy ring) as well as the dense-block T
    pts = W.grid_points(64)
    H = hssc.HSSC(pts, None, 1e-10, k_cut=60, hss_leaf=32)
    b = next(bb for lev in H.levels for bb in lev if H.compressed(bb) and len(bb.sk) > 200)
    S_ids = H._ring_order(b, b.act[b.sk])
    R_ids = H._line_order(b, b.act[b.rs])
    U, V = b.T_lr
    assert U.shape[1] < min(len(S_ids), len(R_ids)) // 2      # low rank
    ext = np.setdiff1d(np.arange(H.N), np.concatenate([b.act, np.arange(H.N)[
        (H.ix >= b.x0) & (H.ix < b.x1) & (H.iy >= b.y0) & (H.iy < b.y1)]]))
    Kx_s = H.K(H.points[ext], H.points[S_ids])
    Kx_r = H.K(H.points[ext], H.points[R_ids])
    err = np.linalg.norm(Kx_s @ (U @ V.T) - Kx_r) / np.linalg.norm(Kx_r)
    assert err < 1e-8


@pytest.mark.parametrize("nx,ny,k_cut,kind", [(32, 32, 40, "laplace"), (40, 24, 30, "laplace"),
                                               (48, 48, 50, "laplace"), (32, 32, 40, "helmholtz")])
def test_compressed_inverse_matches_dense_solve(nx, ny, k_cut, kind):
    pts = W.grid_points(nx, ny)
    if kind == "laplace":
        a, b, k = W.coef_sine(pts), None, 0.0
        f = W.rhs_normal(len(pts), 2, nx)
    else:
        a, b, k = None, W.contrast_bump(pts), 20.0
        f = W.rhs_complex_normal(len(pts), 2, nx)
    H = hssc.HSSC(pts, a, 1e-10, k_cut=k_cut, hss_leaf=16, kind=kind, k=k, bvec=b)
    assert H.stats["compressed_boxes"] > 0
    x = H.solve(f)
    ref = dense.solve(pts, f, a, kind, k, b)
    assert dense.rel_error(x, ref) < 1e-10


def test_compressed_E_matches_algorithm1_E():
    # BUILD_Finv + BUILD_E (block elimination, the E^-1 formula of Sec. 3.2 in
    # its dimensionally consistent reading, HSS1D sums and inverses) against
    # Algorithm 1's definition E = (R F^-1 R^T)^-1 for the same box, the same
    # F (children's E and sibling kernel blocks) and the same T = U V^T
    pts = W.grid_points(32)
    a = W.coef_sine(pts)
    H = hssc.HSSC(pts, a, 1e-10, k_cut=40, hss_leaf=16)
    boxes = [b for lev in H.levels for b in lev if H.compressed(b)]
    assert boxes
    for b in boxes[:4]:
        S, R = b.blocks["S_ids"], b.blocks["R_ids"]
        F = H._F_entries(b)(np.concatenate([S, R]), np.concatenate([S, R]))
        T_U, T_V = b.T_lr
        Rm = np.hstack([np.eye(len(S)), T_U @ T_V.T])
        E = np.linalg.inv(Rm @ np.linalg.inv(F) @ Rm.T)
        assert np.linalg.norm(b.E_hss.dense() - E, 2) <= 1e-9 * np.linalg.norm(E, 2)
        # APPLY_Finv against the dense F^-1
        u = np.random.default_rng(5).standard_normal((len(S) + len(R), 2))
        xs, xr = H.apply_finv(b, u[:len(S)], u[len(S):])
        ref = np.linalg.solve(F, u)
        assert np.linalg.norm(np.vstack([xs, xr]) - ref) <= 1e-9 * np.linalg.norm(ref)


def test_planted_build_e_sign_mistake_is_caught():
    # E^-1 = S^-1 + T phi_rs + ...: flipping the sign of the cross terms
    # must break the solve
    pts = W.grid_points(32)
    f = W.rhs_normal(len(pts), 1, 4)
    src = hssc.HSSC._compressed_box

    def bad_box(self, b):
        T_U, T_V = b.T_lr
        b.T_lr = (-T_U, T_V)        # wrong sign of T inside BUILD_E only
        src(self, b)
        b.T_lr = (T_U, T_V)

    hssc.HSSC._compressed_box = bad_box
    try:
        H = hssc.HSSC(pts, None, 1e-10, k_cut=40, hss_leaf=16)
        x = H.solve(f)
    finally:
        hssc.HSSC._compressed_box = src
    assert dense.rel_error(x, dense.solve(pts, f)) > 1e-6
