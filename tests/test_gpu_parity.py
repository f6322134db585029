"""Parity of the HIP path with the CPU reference.  Every call goes through
the C interface (librsd.so via the ctypes binding).  Marked gpu."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, krylov, nystrom, rskel
from paper_1303_5466_amd import rsd, workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rsd.load()


# --- dense building blocks ---------------------------------------------------
@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-13), (np.float32, 2e-5)])
@pytest.mark.parametrize("M,N,K,tA,tB", [(64, 64, 16, 0, 0), (1, 1, 1, 0, 0), (77, 130, 45, 0, 0),
                                         (150, 33, 70, 1, 0), (65, 97, 129, 0, 1), (40, 50, 60, 1, 1),
                                         (300, 17, 3, 0, 0),
                                         # 128-wide tiles (2048 x 2048, K > 128), ragged edges
                                         (2048, 2048, 200, 0, 0), (2050, 2047, 137, 1, 1),
                                         # short K on 64-wide tiles with C loaded up front, every
                                         # transpose, ragged tiles and k panels
                                         (2048, 2048, 64, 0, 0), (2050, 2047, 64, 1, 1), (33, 65, 64, 1, 0),
                                         (97, 31, 50, 0, 1), (5, 300, 17, 1, 0),
                                         # split K: two splits, sixteen splits, one tile of sixteen
                                         (1024, 1024, 1024, 0, 1), (130, 70, 3000, 1, 0),
                                         (16, 16, 5000, 0, 0)])
def test_gemm_matches_numpy(dt, tol, M, N, K, tA, tB):
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.standard_normal((K, M) if tA else (M, K)).astype(dt)
    B = rng.standard_normal((N, K) if tB else (K, N)).astype(dt)
    C0 = rng.standard_normal((M, N)).astype(dt)
    C = rsd.gemm(A, B, C0, alpha=-0.5, beta=2.0, tA=bool(tA), tB=bool(tB))
    ref = -0.5 * ((A.T if tA else A).astype(np.float64) @ (B.T if tB else B).astype(np.float64)) + 2.0 * C0
    assert np.abs(C - ref).max() <= tol * (np.abs(ref).max() + 1) * max(1, K) ** 0.5


def _real_form(Z):
    """Real form of a complex matrix with each entry's two dofs adjacent:
    entry (i, j) becomes the 2 x 2 block [[re, im], [im, -re]]."""
    n = Z.shape[0]
    X = np.zeros((2 * n, 2 * n))
    X[0::2, 0::2] = Z.real
    X[0::2, 1::2] = Z.imag
    X[1::2, 0::2] = Z.imag
    X[1::2, 1::2] = -Z.real
    return X


@pytest.mark.parametrize("n", [1, 7, 32, 33, 100, 130])
def test_gj_paired_pivots_invert_complex_real_forms(n):
    # complex symmetric matrices with an imaginary diagonal: the real part of
    # the first pivot is zero, the complex pivots are not.  The paired
    # elimination inverts the real form; the scalar one does not.
    rng = np.random.default_rng(n)
    d = 1j * (1.0 + rng.random(n))
    B = 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    B = B + B.T
    np.fill_diagonal(B, 0.0)
    Z = np.diag(d) + B
    X = _real_form(Z)
    inv = np.linalg.inv(X)
    P = rsd.gj_invert(X, paired=True)
    assert np.abs(P - inv).max() <= 1e-12 * np.abs(inv).max()
    if n >= 7:
        try:
            S = rsd.gj_invert(X, paired=False)
            assert np.abs(S - inv).max() > 1e-6 * np.abs(inv).max()
        except rsd.RsdError:
            pass


def test_gemm_and_gj_beyond_2gib():
    # operands larger than 2 GiB (the buffer descriptors are based at each
    # tile's first row / column): a 17000 x 17000 float64 C (2.3 GB) updated
    # by a K = 64 product, and the Gauss-Jordan inverse of such a matrix;
    # checked on sampled rows and columns
    n, K = 17000, 64
    rng = np.random.default_rng(11)
    A = rng.standard_normal((n, K))
    B = rng.standard_normal((K, n))
    C0 = np.asfortranarray(rng.standard_normal((n, n)))
    C = rsd.gemm(A, B, C0, alpha=-0.5, beta=2.0)
    rows = rng.integers(0, n, 40)
    cols = np.concatenate([rng.integers(0, n, 40), [0, n - 1]])
    ref = -0.5 * (A[rows] @ B[:, cols]) + 2.0 * C0[np.ix_(rows, cols)]
    assert np.abs(C[np.ix_(rows, cols)] - ref).max() <= 1e-12 * np.abs(ref).max()
    ref_last = -0.5 * (A[-1] @ B) + 2.0 * C0[-1]
    assert np.abs(C[-1] - ref_last).max() <= 1e-12 * np.abs(ref_last).max()
    del C, C0
    M = np.asfortranarray(rng.standard_normal((n, n)) * (0.5 / np.sqrt(n)))
    M[np.diag_indices(n)] += 2.0
    X = rsd.gj_invert(M)
    for c in (0, 1234, n - 1):
        e = np.zeros(n)
        e[c] = 1.0
        assert np.abs(M @ X[:, c] - e).max() <= 1e-12


def test_split_k_gemm_is_repeatable():
    # the partial tiles are summed in split order whichever work-group is last
    rng = np.random.default_rng(4)
    A = rng.standard_normal((90, 4000))
    B = rng.standard_normal((4000, 70))
    C1 = rsd.gemm(A, B)
    for _ in range(3):
        assert np.array_equal(rsd.gemm(A, B), C1)


@pytest.mark.parametrize("n", [1, 5, 32, 33, 100, 257])
def test_gj_inverse_matches_numpy(n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    X = rsd.gj_invert(A)
    assert np.abs(X - np.linalg.inv(A)).max() <= 1e-12 * np.abs(np.linalg.inv(A)).max()


@pytest.mark.parametrize("n", [65, 150, 320])
def test_gj_inverse_float32_several_steps(n):
    # after the first step every pivot block is inverted by the update tile
    # that produces it; float32 blocks take the same route
    rng = np.random.default_rng(100 + n)
    B = rng.standard_normal((n, n))
    A = (B @ B.T / n + 2.0 * np.eye(n)).astype(np.float32)
    X = rsd.gj_invert(A)
    inv = np.linalg.inv(A.astype(np.float64))
    assert X.dtype == np.float32
    assert np.abs(X - inv).max() <= 2e-5 * np.abs(inv).max()


@pytest.mark.parametrize("paired", [False, True])
@pytest.mark.parametrize("where", [0, 64, 130])
def test_gj_reports_zero_pivot_at_any_step(where, paired):
    # block diagonal [I, Z] with Z's first entry zero: the pivot of step
    # where / 64 is exactly zero (no rounding reaches it), whether the pivot
    # kernel inverts the block (first step) or the previous update's tile does
    n = 200
    A = np.eye(n)
    A[where, where] = 0.0
    if paired:
        A[where + 1, where + 1] = 0.0   # the 2 x 2 block [[0, 0], [0, 0]]
    with pytest.raises(rsd.RsdError):
        rsd.gj_invert(A, paired=paired)
    A[where, where] = 3.0
    if paired:
        A[where + 1, where + 1] = -3.0
    X = rsd.gj_invert(A, paired=paired)
    assert np.abs(X - np.linalg.inv(A)).max() <= 1e-15


# --- interpolation matrices (Sec. 3.1 proxy least squares) ----------------
def test_interpolation_matches_reference_qr():
    pts = W.grid_points(64)
    fac = rsd.Factor(pts, None, 1e-10)
    st = fac.stats()
    h = 1 / 64
    seen = set()
    for b in range(st["n_boxes"] - 1):
        info = fac.box_info(b)
        key = (info["level"], info["ax"], info["ay"])
        if key in seen or info["r"] == 0:
            continue
        seen.add(key)
        ids = fac.block(b, 2)
        k = info["k"]
        T = fac.block(b, 0)
        Xsk, Xrs = pts[ids[:k]], pts[ids[k:]]
        m = 2
        zi, zj = np.meshgrid(np.arange(info["x0"] - m, info["x0"] + info["ax"] + m),
                             np.arange(info["y0"] - m, info["y0"] + info["ay"] + m), indexing="ij")
        zi, zj = zi.ravel(), zj.ravel()
        out = ~((zi >= info["x0"]) & (zi < info["x0"] + info["ax"]) &
                (zj >= info["y0"]) & (zj < info["y0"] + info["ay"]))
        Z = np.stack([(zi[out] + .5) * h, (zj[out] + .5) * h], 1)
        Ks = nystrom.laplace_kernel(np.sqrt(((Z[:, None] - Xsk[None]) ** 2).sum(-1)))
        Kr = nystrom.laplace_kernel(np.sqrt(((Z[:, None] - Xrs[None]) ** 2).sum(-1)))
        Tref = rskel.truncated_qrcp_lstsq(Ks, Kr, 1e-10)
        # least-squares solutions agree to the conditioning of the proxy system
        cond = np.linalg.cond(Ks)
        assert np.linalg.norm(T - Tref) <= 50 * cond * 1e-16 * np.linalg.norm(Tref) + 1e-14, key
        res = np.linalg.norm(Ks @ T - Kr) / np.linalg.norm(Kr)
        res_ref = np.linalg.norm(Ks @ Tref - Kr) / np.linalg.norm(Kr)
        assert res <= 1.01 * res_ref + 1e-13, key
    assert len(seen) >= 5


# --- per-box elimination against Algorithm 1 replayed on the CPU -----------
@pytest.mark.parametrize("n,coef", [(32, "const"), (40, "sine")])
def test_E_blocks_match_algorithm1(n, coef):
    from gpu_util import replay_alg1_E
    pts = W.grid_points(n)
    a = W.coef_const(pts) if coef == "const" else W.coef_sine(pts)
    fac = rsd.Factor(pts, a, 1e-10, flags=rsd.RSD_FLAG_KEEP_E)
    E_ref = replay_alg1_E(pts, a, fac, None)
    worst = 0.0
    for b, Er in E_ref.items():
        Eg = fac.block(b, 1)
        rel = np.abs(Eg - Er).max() / np.abs(Er).max()
        worst = max(worst, rel)
    assert worst < 1e-9, worst


# --- end-to-end solves ------------------------------------------------------
def test_laplace64_matches_dense():
    pts, a, f, tol = W.make_workload("laplace64")
    fac = rsd.Factor(pts, a, tol)
    x, _ = fac.solve(_dev(f))
    x = x.cpu().numpy()
    assert dense.rel_error(x, dense.solve(pts, f, a)) < 1e-10


@pytest.mark.parametrize("nx,ny,coef,nrhs", [(37, 37, "sine", 3), (40, 24, "sine", 2),
                                             (64, 48, "const", 1), (8, 8, "sine", 2),
                                             (9, 30, "sine", 1)])
def test_ragged_grids_match_dense(nx, ny, coef, nrhs):
    pts = W.grid_points(nx, ny)
    a = W.coef_const(pts) if coef == "const" else W.coef_sine(pts)
    f = W.rhs_normal(len(pts), nrhs, 4)
    fac = rsd.Factor(pts, a, 1e-10)
    x, _ = fac.solve(f)
    assert dense.rel_error(x, dense.solve(pts, f, a)) < 1e-10


def test_shuffled_points_and_host_pointers():
    pts = W.grid_points(48)
    a = W.coef_sine(pts)
    sp, perm = W.shuffled(pts, 7)
    f = W.rhs_normal(len(pts), 2, 8)
    fac = rsd.Factor(sp, a[perm], 1e-10)
    x, _ = fac.solve(f[perm])
    ref = dense.solve(pts, f, a)
    assert dense.rel_error(x, ref[perm]) < 1e-10


def test_repeated_grid_in_another_order():
    # builds alternate between two orders of one point set, so the grid
    # detection of the previous build is reused (same points) or redone
    # (another order); the grid-ordered factor is the same either way, so the
    # solutions agree bitwise once mapped through the permutation
    pts = W.grid_points(40)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 9)
    sp, perm = W.shuffled(pts, 3)
    xs = []
    for use_shuffled in (False, False, True, False, True, True):
        if use_shuffled:
            x, _ = rsd.Factor(sp, a[perm], 1e-10).solve(f[perm])
            back = np.empty_like(x)
            back[perm] = x
            xs.append(back)
        else:
            x, _ = rsd.Factor(pts, a, 1e-10).solve(f)
            xs.append(x)
    for x in xs[1:]:
        assert np.array_equal(x, xs[0])
    assert dense.rel_error(xs[0], dense.solve(pts, f, a)) < 1e-10


def test_device_pointers_for_every_input():
    pts = W.grid_points(40)
    a = W.coef_sine(pts)
    f = W.rhs_uniform(len(pts), 4, 3)
    fac = rsd.Factor(_dev(pts), _dev(a), 1e-10)
    x, _ = fac.solve(_dev(f))
    assert dense.rel_error(x.cpu().numpy(), dense.solve(pts, f, a)) < 1e-10


def test_repeat_solves_are_bitwise_identical():
    pts = W.grid_points(48)
    f = W.rhs_normal(len(pts), 3, 9)
    fac = rsd.Factor(pts, None, 1e-10)
    x1, _ = fac.solve(f)
    x2, _ = fac.solve(f)
    fac2 = rsd.Factor(pts, None, 1e-10)
    x3, _ = fac2.solve(f)
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)


def test_cached_device_blocks_are_reused_safely():
    # a freed factor's blocks go to the per-device cache and back to the next
    # build; results stay bitwise equal, concurrent factors keep distinct
    # memory, and trimming empties the cache
    pts = W.grid_points(64, 40)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 12)
    fac = rsd.Factor(pts, a, 1e-10)
    x1, _ = fac.solve(f)
    fac.close()
    assert rsd.pool_cached_bytes() > 0
    held = rsd.Factor(pts, a, 1e-10)          # takes the cached blocks
    other = rsd.Factor(W.grid_points(48), None, 1e-10)
    x2, _ = held.solve(f)
    x3, _ = other.solve(W.rhs_normal(48 * 48, 1, 2))
    assert np.array_equal(x1, x2)
    assert dense.rel_error(x3, dense.solve(W.grid_points(48), W.rhs_normal(48 * 48, 1, 2))) < 1e-10
    held.close()
    other.close()
    rsd.pool_set_limit(0)                     # nothing may stay cached
    assert rsd.pool_cached_bytes() == 0
    rsd.pool_set_limit(-1)
    fac = rsd.Factor(pts, a, 1e-10)
    x4, _ = fac.solve(f)
    fac.close()
    assert np.array_equal(x1, x4)
    rsd.pool_trim()
    assert rsd.pool_cached_bytes() == 0


def test_matvec_matches_reference():
    pts = W.grid_points(33, 21)
    a = W.coef_sine(pts)
    s = W.rhs_normal(len(pts), 3, 5)
    fac = rsd.Factor(pts, a, 1e-10)
    y = fac.matvec(s)
    y_ref = nystrom.matvec_direct(pts, s, a)
    assert np.abs(y - y_ref).max() <= 1e-13 * np.abs(y_ref).max()


@pytest.mark.parametrize("nx,ny", [(33, 21), (600, 7), (1500, 3), (2050, 3)])
def test_fft_product_sizes(nx, ny):
    # circulant FFT product: 128x64, 2048x16 (4-line workgroups), 4096x8 (one
    # line per workgroup) and, past 4096, the direct-sum fallback
    pts = W.grid_points(nx, ny)
    a = W.coef_sine(pts)
    s = W.rhs_normal(len(pts), 3, 11)
    fac = rsd.Factor(pts, a, 1e-10)
    y = fac.matvec(s)
    y_ref = nystrom.matvec_direct(pts, s, a)
    assert np.abs(y - y_ref).max() <= 1e-13 * np.abs(y_ref).max()


def test_contrast_form_needs_a_positive_contrast():
    # the contrast form is factored as S (diag(1/b) + K) S, so b must be > 0
    pts = W.grid_points(16)
    b = W.contrast_bump(pts)
    b[7] = 0.0
    with pytest.raises(rsd.RsdError) as ei:
        rsd.Factor(pts, None, 1e-10, contrast=b)
    assert ei.value.status == rsd.RSD_EINVAL


@pytest.mark.parametrize("flags", [0, rsd.RSD_FLAG_FP32_INTERP])
def test_fp32_refined_matches_dense(flags):
    # default: float64 interpolation rounded into the float32 levels;
    # FP32_INTERP: the interpolation problems solved in float32 as well
    pts = W.grid_points(64)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 6)
    fac = rsd.Factor(pts, a, 1e-10, precision=rsd.RSD_PREC_FP32_REFINE, flags=flags)
    x, info = fac.solve(f)
    assert info.rel_residual <= 1e-10
    assert dense.rel_error(x, dense.solve(pts, f, a)) < 1e-10


def test_fp64_with_refinement_steps():
    pts = W.grid_points(40)
    f = W.rhs_normal(len(pts), 1, 6)
    fac = rsd.Factor(pts, None, 1e-10, max_refine=2, refine_tol=1e-13)
    x, info = fac.solve(f)
    assert info.rel_residual <= 1e-13
    assert dense.rel_error(x, dense.solve(pts, f)) < 1e-12


# --- error paths ------------------------------------------------------------------
def test_errors_are_reported():
    pts = W.grid_points(16)
    with pytest.raises(rsd.RsdError) as e:
        rsd.Factor(pts[:-1], None, 1e-10)
    assert e.value.status == rsd.RSD_ENOTGRID
    with pytest.raises(rsd.RsdError) as e:
        rsd.Factor(pts, None, -1.0)
    assert e.value.status == rsd.RSD_EINVAL
    a = np.ones(len(pts))
    a[3] = np.nan
    with pytest.raises(rsd.RsdError) as e:
        rsd.Factor(pts, a, 1e-10)
    assert e.value.status == rsd.RSD_EINVAL
    fac = rsd.Factor(pts, None, 1e-10)
    f = np.ones(len(pts))
    f[0] = np.inf
    with pytest.raises(rsd.RsdError) as e:
        fac.solve(f)
    assert e.value.status == rsd.RSD_EINVAL


def test_singular_pivot_is_detected():
    """a_i = -(self-cell integral) zeroes the diagonal; a 2 x 2 grid is a single
    box inverted directly, whose first pivot is then exactly zero."""
    pts = W.grid_points(2)
    a = np.full(len(pts), -nystrom.self_cell_laplace(1 / 2))
    with pytest.raises(rsd.RsdError) as e:
        rsd.Factor(pts, a, 1e-10, leaf_side=2)
    assert e.value.status == rsd.RSD_ESINGULAR


@pytest.mark.parametrize("n", [2, 4, 8])
def test_single_box_grids(n):
    pts = W.grid_points(n)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 1)
    fac = rsd.Factor(pts, a, 1e-10, leaf_side=8)
    x, _ = fac.solve(f)
    assert dense.rel_error(x, dense.solve(pts, f, a)) < 1e-12


def test_empty_rhs_is_a_no_op():
    pts = W.grid_points(16)
    fac = rsd.Factor(pts, None, 1e-10)
    x = np.zeros((len(pts), 0), order="F")
    st, info = fac.solve_raw(x.ctypes.data, 0, x.ctypes.data)
    assert st == rsd.RSD_OK


# --- full-size workload (the benchmark's configuration) ------------------------
def test_laplace256_full_size_residual_and_sampled_columns():
    pts, a, f, tol = W.make_workload("laplace256")
    fac = rsd.Factor(pts, a, tol)
    x, _ = fac.solve(_dev(f))
    x = x.cpu().numpy()
    # property at any size: small exact residual (cond(A) <= 3 bounds the error)
    r = f - nystrom.matvec_fft(pts, x, a)
    rel = np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)
    assert rel.max() < 1e-10, rel.max()
    # sampled columns against the reference's iterative exact solve
    for c in (0, 9):
        ref, info = krylov.solve(pts, f[:, c], a, tol=1e-13)
        assert dense.rel_error(x[:, c], ref) < 1e-10


def test_laplace512_fp32_refine_full_size():
    """The 512^2 workload as the benchmark runs it: float32 levels on MFMA,
    float64 root, float64 exact residual and refinement to 1e-10, 4 columns."""
    pts, a, f, tol = W.make_workload("laplace512")
    fac = rsd.Factor(_dev(pts), _dev(a), tol, precision=rsd.RSD_PREC_FP32_REFINE)
    x, info = fac.solve(_dev(f))
    x = x.cpu().numpy()
    assert info.rel_residual <= tol
    # the library's residual claim checked by the reference's own exact product
    r = f - nystrom.matvec_fft(pts, x, a)
    rel = np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)
    assert rel.max() < 1e-10, rel.max()
    ref, _ = krylov.solve(pts, f[:, 0], a, tol=1e-13)
    assert dense.rel_error(x[:, 0], ref) < 1e-10
    fac.close()


def test_refinement_reports_enoconv():
    # a target below float64 rounding cannot be met: ENOCONV after the
    # allowed steps, with the last iterate and its residual handed back
    pts = W.grid_points(40)
    a = W.coef_sine(pts)
    f = np.asfortranarray(W.rhs_normal(len(pts), 2, 3))
    fac = rsd.Factor(pts, a, 1e-10, precision=rsd.RSD_PREC_FP32_REFINE, max_refine=1,
                     refine_tol=1e-18)
    x = np.zeros_like(f)
    st, info = fac.solve_raw(f.ctypes.data, 2, x.ctypes.data)
    assert st == rsd.RSD_ENOCONV
    assert info.refine_iters == 1
    assert 0 < info.rel_residual < 1e-6
    ref = dense.solve(pts, f, a)
    assert dense.rel_error(x, ref) < 1e-6         # the iterate is still a solution to fp32 level
    with pytest.raises(rsd.RsdError) as e:
        fac.solve(f)
    assert e.value.status == rsd.RSD_ENOCONV
    fac.close()


# --- batched builds (many independent grids) -----------------------------------
def test_batched_build_equals_single_builds():
    shapes = [(16, 16), (37, 37), (24, 40), (64, 64), (9, 30), (48, 33)]
    rng = np.random.default_rng(21)
    pts = [W.grid_points(nx, ny) for nx, ny in shapes]
    coefs = [W.coef_bumps(p, rng) for p in pts]
    rhs = [rng.standard_normal((p.shape[0], 2)) for p in pts]
    facs = rsd.build_batched(pts, coefs, tol=1e-10, max_inflight=3)
    assert len(facs) == len(shapes)
    for p, a, f, fac in zip(pts, coefs, rhs, facs):
        x_b, _ = fac.solve(np.asfortranarray(f))
        single = rsd.Factor(p, a, 1e-10)
        x_s, _ = single.solve(np.asfortranarray(f))
        # the interpolation matrices are solved by the same launches' arithmetic
        # whichever problems share a chain: bitwise equal
        for box in range(single.stats()["n_boxes"]):
            info = single.box_info(box)
            if info["r"] > 0 and info["parent"] >= 0:
                assert np.array_equal(fac.block(box, 0), single.block(box, 0)), box
        # the merged level products may split K differently: rounding only
        assert np.max(np.abs(x_b - x_s)) <= 1e-12 * np.max(np.abs(x_s))
        assert dense.rel_error(x_b, dense.solve(p, f, a)) < 1e-10
        single.close()
        fac.close()


def test_batched_build_fp32_refine_and_host_device_mix():
    pts, coefs, rhs, tol = W.make_batch(n_inst=5, seed=5, side_lo=20, side_hi=60)
    dev_pts = [_dev(p) if i % 2 else p for i, p in enumerate(pts)]
    facs = rsd.build_batched(dev_pts, coefs, tol=tol, precision=rsd.RSD_PREC_FP32_REFINE)
    for p, a, f, fac in zip(pts, coefs, rhs, facs):
        x, info = fac.solve(f)
        assert info.rel_residual <= tol
        assert dense.rel_error(x, dense.solve(p, f, a)) < 1e-8     # the batch's tolerance
        fac.close()


def test_batched_solve_equals_single_solves():
    pts, coefs, rhs, tol = W.make_batch(n_inst=6, seed=7, side_lo=16, side_hi=70)
    facs = rsd.build_batched(pts, coefs, tol=tol, precision=rsd.RSD_PREC_FP32_REFINE)
    F = [np.asfortranarray(np.stack([f, 2 * f], axis=1)) for f in rhs]
    X = [np.zeros_like(f) for f in F]
    st, infos = rsd.solve_batched_raw(facs, [f.ctypes.data for f in F], 2, [x.ctypes.data for x in X])
    assert st == rsd.RSD_OK
    for fac, f, x, info in zip(facs, F, X, infos):
        x1, info1 = fac.solve(f)
        assert np.array_equal(x, x1)          # same solve, same bits
        assert info.refine_iters == info1.refine_iters and info.rel_residual <= tol
    # a repeated factor is refused before any solve
    st, _ = rsd.solve_batched_raw([facs[0], facs[0]], [F[0].ctypes.data] * 2, 2, [X[0].ctypes.data] * 2)
    assert st == rsd.RSD_EINVAL
    for fac in facs:
        fac.close()


def test_batched_build_reports_singular_instance():
    # the merged Gauss-Jordan launches flag the failing block's own factor
    good16, good8 = W.grid_points(16), W.grid_points(8)
    bad = W.grid_points(2)
    a_bad = np.full(len(bad), -nystrom.self_cell_laplace(1 / 2))
    with pytest.raises(rsd.RsdError) as ei:
        rsd.build_batched([good16, bad, good8], [W.coef_sine(good16), a_bad, W.coef_sine(good8)],
                          tol=1e-10, leaf_side=2)
    assert ei.value.status == rsd.RSD_ESINGULAR
    assert "instance 1" in str(ei.value)


def test_plan_reuse_keeps_factors_independent():
    # a cached plan is copied into each factor: a build without the symmetry
    # split in between must not change a later build of the same shape
    pts = W.grid_points(48)
    a = W.coef_sine(pts)
    f1 = rsd.Factor(pts, a, 1e-10)
    f2 = rsd.Factor(pts, a, 1e-10, flags=rsd.RSD_FLAG_NO_SYMMETRY)
    f3 = rsd.Factor(pts, a, 1e-10)
    for b in range(f1.stats()["n_boxes"]):
        info = f1.box_info(b)
        if info["r"] > 0 and info["parent"] >= 0:
            assert np.array_equal(f1.block(b, 0), f3.block(b, 0)), b
    f = W.rhs_normal(len(pts), 1, 5)
    x1, _ = f1.solve(f)
    x3, _ = f3.solve(f)
    assert np.array_equal(x1, x3)
    for fac in (f1, f2, f3):
        fac.close()


def test_batched_build_reports_failing_instance():
    good = W.grid_points(16)
    bad = W.grid_points(16)[:-3]          # not a complete grid
    with pytest.raises(rsd.RsdError) as ei:
        rsd.build_batched([good, bad, good], None, tol=1e-10)
    assert ei.value.status == rsd.RSD_ENOTGRID
    assert "instance 1" in str(ei.value)


# --- serving: resident factors, queued and coalesced solves ------------------------
def test_server_coalesced_solves_match_dense():
    srv = rsd.Server(n_workers=1, max_coalesce=16)
    grids = [W.grid_points(24), W.grid_points(32, 40), W.grid_points(48)]
    rng = np.random.default_rng(31)
    coefs = [W.coef_bumps(p, rng) for p in grids]
    fids = [srv.submit_factor(p, a, tol=1e-10) for p, a in zip(grids, coefs)]
    reqs = []
    for i in range(30):
        g, nr = i % 3, 1 + (i % 4) // 2
        f = np.asfortranarray(rng.standard_normal((grids[g].shape[0], nr)))
        if i % 5 == 0:      # device buffers: (nrhs, N) contiguous = N x nrhs column-major
            fd = _dev(f.T)
            xd = torch.empty_like(fd)
            reqs.append((g, f, xd, srv.submit_solve(fids[g], fd, xd)))
        else:
            x = np.zeros_like(f, order="F")
            reqs.append((g, f, x, srv.submit_solve(fids[g], f, x)))
    for g, f, x, tk in reqs:
        st, info = srv.wait(tk)
        assert st == rsd.RSD_OK
        xs = x if isinstance(x, np.ndarray) else x.cpu().numpy().T
        assert dense.rel_error(xs, dense.solve(grids[g], f, coefs[g])) < 1e-10
    s = srv.stats()
    assert s["n_done"] == 30 and s["n_requests"] == 30
    assert s["n_batches"] < 30          # requests waiting together were coalesced
    assert 0 < s["p50_ms"] <= s["p99_ms"]
    assert s["n_factors"] == 3
    srv.close()


def test_server_admission_and_errors():
    srv = rsd.Server(max_slots=2, evict_idle=True)
    p16, p20, p24 = W.grid_points(16), W.grid_points(20), W.grid_points(24)
    fa = srv.submit_factor(p16)
    fb = srv.submit_factor(p20)
    fc = srv.submit_factor(p24)            # evicts the least recently used idle factor (fa)
    s = srv.stats()
    assert s["n_factors"] == 2 and s["n_evicted"] == 1
    f = np.ones((p16.shape[0], 1), order="F")
    x = np.zeros_like(f)
    with pytest.raises(rsd.RsdError) as ei:
        srv.submit_solve(fa, f, x)
    assert ei.value.status == rsd.RSD_EINVAL
    st, _ = srv.wait(123456)
    assert st == rsd.RSD_EINVAL
    f20 = np.ones((p20.shape[0], 1), order="F")
    x20 = np.zeros_like(f20)
    tk = srv.submit_solve(fb, f20, x20)
    st, info = srv.wait(tk, timeout_ms=60000)
    assert st == rsd.RSD_OK
    # a served factor is the one rsd_build_factor builds: same solution bits
    direct = rsd.Factor(p20, None, 1e-10)
    xd, _ = direct.solve(f20)
    assert np.array_equal(x20, xd)
    direct.close()
    srv.release_factor(fc)
    assert srv.stats()["n_factors"] == 1
    srv.close()


def test_server_memory_budget_admission():
    # the server sizes a factor before building it: the estimate equals the
    # built factor's bytes; a request larger than the budget fails at once
    p32 = W.grid_points(32)
    a32 = W.coef_sine(p32)
    probe = rsd.Factor(p32, a32, 1e-10)
    fb = probe.stats()["factor_bytes"]
    probe.close()
    assert rsd.estimate_factor_bytes(32, 32, 1e-10) == fb
    srv = rsd.Server(mem_budget=fb // 2)
    with pytest.raises(rsd.RsdError) as ei:
        srv.submit_factor(p32, a32)
    assert ei.value.status == rsd.RSD_ENOMEM
    assert srv.stats()["n_factors"] == 0 and srv.stats()["resident_bytes"] == 0
    srv.close()
    # admission size = factor + coalescing/solve vectors of a full batch
    slot = fb + 6 * len(p32) * 8 * 8
    srv = rsd.Server(mem_budget=int(slot * 1.5), max_coalesce=8, evict_idle=True)
    f1 = srv.submit_factor(p32, a32)
    assert srv.stats()["resident_bytes"] == slot
    f2 = srv.submit_factor(p32, W.coef_sine(p32))
    s = srv.stats()
    assert s["n_factors"] == 1 and s["n_evicted"] == 1 and s["resident_bytes"] <= slot * 1.5
    f = np.asfortranarray(W.rhs_normal(len(p32), 1, 2))
    x = np.zeros_like(f)
    st, _ = srv.wait(srv.submit_solve(f2, f, x))
    assert st == rsd.RSD_OK
    assert dense.rel_error(x, dense.solve(p32, f, W.coef_sine(p32))) < 1e-10
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(f1, f, np.zeros_like(f))     # evicted
    srv.close()


def test_server_queues_factor_requests_until_memory_frees():
    # without eviction a second factor waits in the queue until the first is
    # released; solves submitted for it meanwhile run once it is resident
    p32 = W.grid_points(32)
    slot = rsd.estimate_factor_bytes(32, 32, 1e-10) + 6 * len(p32) * 8 * 8
    srv = rsd.Server(mem_budget=int(slot * 1.5), max_coalesce=8)
    f1 = srv.submit_factor(p32)
    a2 = W.coef_sine(p32)
    f2 = srv.submit_factor(p32, a2, wait=False)
    assert srv.wait_factor(f2, timeout_ms=300) == rsd.RSD_EAGAIN
    s = srv.stats()
    assert s["n_factors"] == 1 and s["n_queued_factors"] == 1 and s["n_evicted"] == 0
    f = np.asfortranarray(W.rhs_normal(len(p32), 2, 5))
    x2 = np.zeros_like(f)
    tk2 = srv.submit_solve(f2, f, x2)             # queued behind the admission
    assert srv.poll(tk2) == 0
    x1 = np.zeros_like(f)
    st, _ = srv.wait(srv.submit_solve(f1, f, x1))
    assert st == rsd.RSD_OK
    srv.release_factor(f1)                         # frees the memory: f2 is admitted and built
    st, _ = srv.wait(tk2, timeout_ms=60000)
    assert st == rsd.RSD_OK
    assert srv.wait_factor(f2) == rsd.RSD_OK
    assert dense.rel_error(x1, dense.solve(p32, f)) < 1e-10
    assert dense.rel_error(x2, dense.solve(p32, f, a2)) < 1e-10
    s = srv.stats()
    assert s["n_factors"] == 1 and s["n_queued_factors"] == 0 and s["n_built"] == 2
    # a request that fails to build reports its status to its waiters
    bad = np.array([[0.0, 0.0], [0.3, 0.0], [0.0, 1.0]])
    with pytest.raises(rsd.RsdError) as ei:
        srv.submit_factor(bad)
    assert ei.value.status == rsd.RSD_ENOTGRID
    srv.close()


def test_server_results_alone_and_in_the_mix():
    # continuous serving: factor requests of different sizes arrive while
    # solves of resident factors run (Poisson arrivals from two client
    # threads, right-hand-side counts 1..5); every result is compared with the
    # same right-hand side solved alone on a directly built factor
    import threading
    import time
    rng = np.random.default_rng(77)
    grids = [W.grid_points(48), W.grid_points(32, 40), W.grid_points(64), W.grid_points(24)]
    coefs = [W.coef_bumps(p, rng) for p in grids]
    alone = []
    for p, a in zip(grids, coefs):
        fac = rsd.Factor(p, a, 1e-10)
        alone.append(fac)
    srv = rsd.Server(n_workers=2, max_coalesce=16)
    fids = [srv.submit_factor(grids[0], coefs[0]), srv.submit_factor(grids[1], coefs[1])]
    work = []
    lock = threading.Lock()

    def client(seed, which):
        r = np.random.default_rng(seed)
        for i in range(24):
            time.sleep(r.exponential(1.0 / 400.0))
            with lock:
                g = which[i % len(which)]
                fid = fids[g] if g < len(fids) else None
            if fid is None:
                continue
            nr = int(r.integers(1, 6))
            f = np.asfortranarray(r.standard_normal((grids[g].shape[0], nr)))
            x = np.zeros_like(f)
            tk = srv.submit_solve(fid, f, x)
            with lock:
                work.append((g, f, x, tk))

    th = [threading.Thread(target=client, args=(1, [0, 1, 2, 3])),
          threading.Thread(target=client, args=(2, [1, 0, 3, 2]))]
    for t in th:
        t.start()
    time.sleep(0.01)
    # two more factor requests arrive while the clients are solving
    f3 = srv.submit_factor(grids[2], coefs[2], wait=False)
    f4 = srv.submit_factor(grids[3], coefs[3], wait=False)
    with lock:
        fids.extend([f3, f4])
    for t in th:
        t.join()
    assert srv.wait_factor(f3) == rsd.RSD_OK and srv.wait_factor(f4) == rsd.RSD_OK
    assert len(work) > 20
    for g, f, x, tk in work:
        st, _ = srv.wait(tk, timeout_ms=120000)
        assert st == rsd.RSD_OK
        xa, _ = alone[g].solve(f)
        assert np.linalg.norm(x - xa) <= 1e-12 * np.linalg.norm(xa)
        assert dense.rel_error(x, dense.solve(grids[g], f, coefs[g])) < 1e-10
    s = srv.stats()
    assert s["n_built"] == 4 and s["n_done"] == len(work)
    srv.close()
    for fac in alone:
        fac.close()


def test_server_binding_checks_buffers():
    srv = rsd.Server()
    p = W.grid_points(16)
    fid = srv.submit_factor(p)
    n = len(p)
    good = np.ones((n, 2))
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(fid, np.ones((n + 1, 2)), np.zeros((n + 1, 2)))   # wrong N
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(fid, good, np.zeros((n, 2), dtype=np.float32))    # wrong out dtype
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(fid, good, np.zeros((n, 1)))                      # short out
    # C-ordered buffers are accepted and filled in the caller's layout
    f = np.ascontiguousarray(W.rhs_normal(n, 2, 9))
    x = np.zeros((n, 2))
    st, _ = srv.wait(srv.submit_solve(fid, f, x))
    assert st == rsd.RSD_OK
    assert dense.rel_error(x, dense.solve(p, f)) < 1e-10
    td = _dev(np.ones((2, n)))
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(fid, td, torch.empty((2, n), dtype=torch.float32, device="cuda:0"))
    with pytest.raises(rsd.RsdError):
        srv.submit_solve(fid, td.t(), torch.empty((n, 2), dtype=torch.float64, device="cuda:0"))
    srv.close()


# --- solve sweeps replayed as a HIP graph -------------------------------------
@pytest.mark.parametrize("precision", [rsd.RSD_PREC_FP64, rsd.RSD_PREC_FP32_REFINE])
def test_solve_sweeps_as_graph_match_launches_one_by_one(precision):
    # the up sweep, root and down sweep of each solve width are captured once
    # and replayed; every replay, with the program's own eager work and
    # synchronisations in between (products, host and device inputs, other
    # widths), gives the bits of a factor that launches them one by one
    pts = W.grid_points(96, 80)
    a = W.coef_sine(pts)
    fg = rsd.Factor(pts, a, 1e-10, precision=precision, flags=rsd.RSD_FLAG_SOLVE_GRAPH)
    fe = rsd.Factor(pts, a, 1e-10, precision=precision)
    for rep in range(5):
        nrhs = 3 if rep % 2 == 0 else 1
        f = W.rhs_normal(len(pts), nrhs, 60 + rep)
        if rep == 3:
            xg, ig = fg.solve(_dev(f))
            xg = xg.cpu().numpy()
        else:
            xg, ig = fg.solve(f)
        xe, ie = fe.solve(f)
        assert np.array_equal(xg, xe), rep
        assert ig.refine_iters == ie.refine_iters
        y = fg.matvec(xg)
        assert np.linalg.norm(y - f) <= 1e-9 * np.linalg.norm(f), rep
    assert fg.stats()["solve_graphs"] == 2 and fe.stats()["solve_graphs"] == 0
    fg.close()
    fe.close()


def test_complex_solve_sweeps_as_graph():
    pts = W.grid_points(48)
    b = 1.0 + 0.3 * np.sin(3 * pts[:, 0]) ** 2
    kw = dict(kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=W.SCATTER_K, contrast=b)
    fg = rsd.Factor(pts, None, 1e-10, flags=rsd.RSD_FLAG_SOLVE_GRAPH, **kw)
    fe = rsd.Factor(pts, None, 1e-10, **kw)
    for rep in range(3):
        f = W.rhs_complex_normal(len(pts), 2, 70 + rep)
        xg, _ = fg.solve(f)
        xe, _ = fe.solve(f)
        assert np.array_equal(xg, xe), rep
    fg.close()
    fe.close()


# --- compressed forward product (Sec. 2.3) ---------------------------------------
@pytest.mark.parametrize("nx,ny,tol,precision", [(64, 64, 1e-10, rsd.RSD_PREC_FP64),
                                                 (50, 40, 1e-10, rsd.RSD_PREC_FP64),
                                                 (37, 37, 1e-6, rsd.RSD_PREC_FP64),
                                                 (256, 256, 1e-10, rsd.RSD_PREC_FP64),
                                                 (128, 128, 1e-10, rsd.RSD_PREC_FP32_REFINE),
                                                 (8, 8, 1e-10, rsd.RSD_PREC_FP64)])
def test_compressed_product_matches_exact(nx, ny, tol, precision):
    # the factor's own recursive-skeleton product against the exact product
    # (FFT, float64) and, at sizes the reference finishes, against the
    # reference's compressed product (same skeletons, same T up to rounding
    # where the interpolation problems are full rank)
    pts = W.grid_points(nx, ny)
    a = W.coef_sine(pts)
    fac = rsd.Factor(pts, a, tol, precision=precision)
    x = W.rhs_normal(len(pts), 3, nx + ny)
    yc = fac.matvec_compressed(x)
    ye = fac.matvec(x)
    rel = np.linalg.norm(yc - ye) / np.linalg.norm(ye)
    bound = 1e-6 if precision == rsd.RSD_PREC_FP32_REFINE else (1e-14 if nx * ny <= 64 else 10 * tol)
    print(f"{nx}x{ny} tol {tol:g}: compressed vs exact {rel:.2e}")
    assert rel <= bound
    if len(pts) <= 4096 and precision == rsd.RSD_PREC_FP64:
        R = rskel.RSkel(pts, a, tol)
        yo = R.forward_matvec(x)
        dr = np.linalg.norm(yc - yo) / np.linalg.norm(yo)
        print(f"  vs the reference's compressed product {dr:.2e}")
        assert dr <= (1e-12 if tol <= 1e-10 else 1e-6)
    fac.close()


def test_compressed_product_arguments():
    pts = W.grid_points(32)
    b = W.contrast_bump(pts)
    fh = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=W.SCATTER_K, contrast=b)
    with pytest.raises(rsd.RsdError) as e:
        fh.matvec_compressed(np.ones(len(pts)))
    assert e.value.status == rsd.RSD_EINVAL
    fh.close()
    fl = rsd.Factor(pts, None, 1e-10)
    assert np.array_equal(fl.matvec_compressed(np.zeros((len(pts), 0))), np.zeros((len(pts), 0)))
    fl.close()


# --- symmetry split of the interpolation problems ------------------------------------
def test_symmetry_split_matches_whole_problems():
    pts = W.grid_points(64)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 41)
    fs = rsd.Factor(pts, a, 1e-10)
    fw = rsd.Factor(pts, a, 1e-10, flags=rsd.RSD_FLAG_NO_SYMMETRY)
    xs, _ = fs.solve(f)
    xw, _ = fw.solve(f)
    xd = dense.solve(pts, f, a)
    assert dense.rel_error(xs, xd) < 1e-10 and dense.rel_error(xw, xd) < 1e-10
    assert np.linalg.norm(xs - xw) <= 1e-11 * np.linalg.norm(xw)
    # every level's T: the four sector solutions recombine to the whole problem's
    seen = set()
    for b in range(fs.stats()["n_boxes"]):
        info = fs.box_info(b)
        if info["level"] in seen or info["r"] == 0:
            continue
        seen.add(info["level"])
        try:
            Ts, Tw = fs.block(b, 0), fw.block(b, 0)
        except rsd.RsdError:
            continue
        assert np.abs(Ts - Tw).max() <= 1e-6 * np.abs(Tw).max(), info["level"]
    fs.close()
    fw.close()


def test_two_layer_interpolation_truncates_at_1e10():
    # with two skeleton layers the float64 interpolation keeps every column
    # (truncation at min(tol, 1e-10)): a looser tolerance gives the same T
    pts = W.grid_points(40, 24)
    a = W.coef_sine(pts)
    f8 = rsd.Factor(pts, a, 1e-8)
    f10 = rsd.Factor(pts, a, 1e-10)
    assert f8.stats()["layers"] == f10.stats()["layers"] == 2
    for b in range(f10.stats()["n_boxes"]):
        info = f10.box_info(b)
        if info["r"] > 0 and info["parent"] >= 0:
            assert np.array_equal(f8.block(b, 0), f10.block(b, 0)), b
    f8.close()
    f10.close()


@pytest.mark.parametrize("n", [50, 75])
def test_one_reflection_split_matches_whole_problems(n):
    # odd halves: many box types are mirror-symmetric along one axis only
    # (two sectors); compare every box's T and the solutions with the whole
    # problems
    pts = W.grid_points(n)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 47)
    fs = rsd.Factor(pts, a, 1e-10)
    fw = rsd.Factor(pts, a, 1e-10, flags=rsd.RSD_FLAG_NO_SYMMETRY)
    xs, _ = fs.solve(f)
    xw, _ = fw.solve(f)
    xd = dense.solve(pts, f, a)
    assert dense.rel_error(xs, xd) < 1e-10 and dense.rel_error(xw, xd) < 1e-10
    assert np.linalg.norm(xs - xw) <= 1e-11 * np.linalg.norm(xw)
    for b in range(fs.stats()["n_boxes"]):
        info = fs.box_info(b)
        if info["r"] == 0 or info["parent"] < 0:
            continue
        Ts, Tw = fs.block(b, 0), fw.block(b, 0)
        assert np.abs(Ts - Tw).max() <= 1e-6 * np.abs(Tw).max(), (b, info["ax"], info["ay"])
    fs.close()
    fw.close()


def _proxy_columns(info, idx, ny, m, h, cols):
    """Proxy matrix K(Z, X) of a box (Sec. 2.2): Z the grid nodes of the ring of
    m layers around it, X the box points idx[cols] (grid indices ix * ny + iy);
    with box-relative coordinates of X."""
    ax, ay = info["ax"], info["ay"]
    zu, zv = np.meshgrid(np.arange(-m, ax + m), np.arange(-m, ay + m), indexing="ij")
    zu, zv = zu.ravel(), zv.ravel()
    ring = ~((zu >= 0) & (zu < ax) & (zv >= 0) & (zv < ay))
    zu, zv = zu[ring], zv[ring]
    xu = idx[cols] // ny - info["x0"]
    xv = idx[cols] % ny - info["y0"]
    return zu, zv, xu, xv


def _kernel_uv(zu, zv, xu, xv, h):
    r = h * np.hypot(zu[:, None] - xu[None, :], zv[:, None] - xv[None, :])
    return nystrom.kernel(r)


def _sector_scale(info, zu, zv, xu, xv, h, ns):
    """|R_11| reference of a split problem: the largest column norm of the
    proxy matrix in the symmetry-adapted basis, (1/sqrt ns) |sum_g chi(g)
    K(Z, g x)| over the skeleton points x and the characters chi of the
    reflection group (u -> ax-1-u, v -> ay-1-v).  With two sectors the group
    is the reflection that maps the skeleton onto itself."""
    ax, ay = info["ax"], info["ay"]
    pts = set(zip(xu.tolist(), xv.tolist()))
    closed_u = ax % 2 == 0 and all((ax - 1 - u, v) in pts for u, v in pts)
    closed_v = ay % 2 == 0 and all((u, ay - 1 - v) in pts for u, v in pts)
    if ns == 4:
        gens = [(1, 1)]
    else:
        gens = ([(1, 0)] if closed_u else []) + ([(0, 1)] if closed_v else [])
    best = []
    for gu, gv in gens:
        elems = [(0, 0), (1, 0)] if (gu, gv) == (1, 0) else [(0, 0), (0, 1)] if (gu, gv) == (0, 1) \
            else [(0, 0), (1, 0), (0, 1), (1, 1)]
        chars = elems   # characters labelled like the elements: chi_c(g) = (-1)^(c . g)
        m = 0.0
        for c in chars:
            col = 0.0
            for g in elems:
                sgn = (-1.0) ** (c[0] * g[0] + c[1] * g[1])
                gxu = ax - 1 - xu if g[0] else xu
                gxv = ay - 1 - xv if g[1] else xv
                col = col + sgn * _kernel_uv(zu, zv, gxu, gxv, h)
            m = max(m, np.linalg.norm(col, axis=0).max() / np.sqrt(ns))
        best.append(m)
    return best


@pytest.mark.parametrize("nx,ny", [(64, 64), (50, 50), (40, 24)])
def test_interpolation_truncation_record(nx, ny):
    # the truncation of Sec. 2.1 keeps the columns with |R_jj| > tol |R_11|:
    # read back every box type's kept rank and |R_11| reference.  The whole
    # problem's reference is its largest skeleton column norm; the sectors of
    # a split type share one reference, the largest column norm in the
    # symmetry-adapted basis (between the whole one and sqrt(ns) times it),
    # and keep together as many columns as the whole problem (the split is
    # used where nothing is truncated)
    pts = W.grid_points(nx, ny)
    a = W.coef_sine(pts)
    h = 1.0 / max(nx, ny)
    fs = rsd.Factor(pts, a, 1e-10)
    fw = rsd.Factor(pts, a, 1e-10, flags=rsd.RSD_FLAG_NO_SYMMETRY)
    m = fs.stats()["layers"]
    seen, n_split = set(), 0
    for b in range(fs.stats()["n_boxes"]):
        info = fs.box_info(b)
        rs, rw = fs.interp_info(b), fw.interp_info(b)
        if info["r"] == 0 or info["parent"] < 0:
            assert rs == [] and rw == []
            continue
        key = (info["level"], info["ax"], info["ay"], info["k"], info["r"])
        if key in seen:
            continue
        seen.add(key)
        k = info["k"]
        idx = fs.block(b, 2)
        zu, zv, xu, xv = _proxy_columns(info, idx, ny, m, h, np.arange(k))
        s_ref = np.linalg.norm(_kernel_uv(zu, zv, xu, xv, h), axis=0).max()
        assert len(rw) == 1
        rank_w, s_w = rw[0]
        assert abs(s_w - s_ref) <= 1e-12 * s_ref, (key, s_w, s_ref)
        assert 0 < rank_w <= k
        if len(rs) > 1:
            n_split += 1
            ns = len(rs)
            scales = {sc for _, sc in rs}
            assert len(scales) == 1, (key, rs)
            s_s = rs[0][1]
            assert s_w * (1 - 1e-12) <= s_s <= np.sqrt(ns) * s_w * (1 + 1e-12), (key, s_s, s_w)
            cands = _sector_scale(info, zu, zv, xu, xv, h, ns)
            assert any(abs(s_s - c) <= 1e-12 * c for c in cands), (key, s_s, cands)
            assert sum(r for r, _ in rs) == rank_w, (key, rs, rank_w)
        else:
            assert rs[0] == rw[0], (key, rs, rw)
    assert n_split > 0
    fs.close()
    fw.close()


@pytest.mark.parametrize("n,tol,layers,precision,flags,mode", [
    (128, 1e-6, 0, rsd.RSD_PREC_FP64, 0, "full"), (64, 1e-8, 0, rsd.RSD_PREC_FP64, 0, "full"),
    (128, 1e-10, 3, rsd.RSD_PREC_FP64, rsd.RSD_FLAG_NO_SYMMETRY, "damped"),
    (128, 1e-10, 3, rsd.RSD_PREC_FP64, 0, "damped"),
    (128, 1e-10, 3, rsd.RSD_PREC_FP64, rsd.RSD_FLAG_NO_DAMPING, "truncated"),
    (128, 1e-6, 2, rsd.RSD_PREC_FP32_REFINE, rsd.RSD_FLAG_FP32_INTERP, "damped")])
def test_interpolation_rank_matches_lapack_pivoting(n, tol, layers, precision, flags, mode):
    # against LAPACK's column-pivoted QR (geqp3) on the same proxy matrices:
    # the default two-layer and one-layer configurations keep every column in
    # both; where truncation would be active (three layers, float32
    # interpolation) the damped least squares keeps every column and its T
    # interpolates the proxy field as well as LAPACK's solution truncated at
    # the damping level; truncation alone (RSD_FLAG_NO_DAMPING, threshold
    # 1e-12 with three layers) keeps within a few columns of LAPACK's rank
    pts = W.grid_points(n)
    a = W.coef_sine(pts)
    h = 1.0 / n
    f = rsd.Factor(pts, a, tol, layers=layers, precision=precision, flags=flags,
                   max_refine=10 if precision != rsd.RSD_PREC_FP64 else 0)
    m = f.stats()["layers"]
    if flags & rsd.RSD_FLAG_FP32_INTERP:
        qtol = max(tol, 1e-6)
    elif mode == "damped":
        qtol = tol
    else:
        qtol = min(tol, 1e-12) if m >= 3 else min(tol, 1e-10) if m == 2 else tol
    seen = set()
    for b in range(f.stats()["n_boxes"]):
        info = f.box_info(b)
        if info["r"] == 0 or info["parent"] < 0:
            continue
        key = (info["level"], info["ax"], info["ay"], info["k"], info["r"])
        if key in seen:
            continue
        seen.add(key)
        k = info["k"]
        idx = f.block(b, 2)
        zu, zv, xu, xv = _proxy_columns(info, idx, n, m, h, np.arange(k))
        Ks = _kernel_uv(zu, zv, xu, xv, h)
        Kr = _kernel_uv(zu, zv, *_proxy_columns(info, idx, n, m, h, np.arange(k, k + info["r"]))[2:], h)
        d = np.abs(np.diag(sla.qr(Ks, mode="r", pivoting=True)[0]))
        rho = int(np.sum(d > qtol * d[0]))
        rec = f.interp_info(b)
        ranks = sum(r for r, _ in rec)
        T = f.block(b, 0)
        res = np.linalg.norm(Ks @ T - Kr) / np.linalg.norm(Kr)
        Tref = rskel.truncated_qrcp_lstsq(Ks, Kr, qtol)
        res_ref = np.linalg.norm(Ks @ Tref - Kr) / np.linalg.norm(Kr)
        print(key, "rank", ranks, "geqp3", rho, "of", k, "residual %.2e (geqp3 %.2e)" % (res, res_ref))
        assert f.interp_damped(b) == (mode == "damped"), key
        if mode == "truncated":
            assert abs(ranks - rho) <= max(2, k // 100), (key, ranks, rho)
        elif mode == "damped":
            assert ranks == k, (key, ranks)
        else:
            assert ranks == rho == k, (key, ranks, rho)
        assert res <= 2 * res_ref + 5 * qtol, (key, res, res_ref)
        if mode == "damped":
            # the damping bounds T like the truncation does
            assert np.abs(T).max() <= 10 * np.abs(Tref).max() + 1, (key, np.abs(T).max(), np.abs(Tref).max())
    f.close()


@pytest.mark.parametrize("flags", [0, rsd.RSD_FLAG_NO_SYMMETRY, rsd.RSD_FLAG_NO_DAMPING])
def test_three_layers_at_a_loose_tolerance(flags):
    # three skeleton layers asked for at tol 1e-10: the interpolation
    # problems are rank deficient at 1e-10; damped at 1e-10 (default) or
    # truncated at 1e-12 (no damping) the solve meets the tolerance (truncated
    # at 1e-10, the window pivoting stopped far too early and the solve was
    # wrong)
    pts = W.grid_points(64)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 2, 53)
    fac = rsd.Factor(pts, a, 1e-10, layers=3, flags=flags)
    assert fac.stats()["layers"] == 3
    x, _ = fac.solve(f)
    err = dense.rel_error(x, dense.solve(pts, f, a))
    print("three layers at 1e-10, flags", flags, "error vs dense %.2e" % err)
    assert err < 1e-10
    fac.close()


@pytest.mark.parametrize("precision,flags", [(rsd.RSD_PREC_FP64, 0), (rsd.RSD_PREC_FP32_REFINE, 0),
                                             (rsd.RSD_PREC_FP32_REFINE, rsd.RSD_FLAG_FP32_INTERP)])
def test_low_accuracy_tolerance(precision, flags):
    # tol 1e-6: one layer, truncation active in the interpolation problems
    pts = W.grid_points(128)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 1, 43)
    fac = rsd.Factor(pts, a, 1e-6, precision=precision, flags=flags)
    x, info = fac.solve(f)
    r = f - nystrom.matvec_fft(pts, x, a)
    assert np.linalg.norm(r) <= 1e-5 * np.linalg.norm(f)


# --- translation-invariant deduplication (constant a) ------------------------
def test_shared_blocks_for_constant_coefficient():
    # with a constant a every box of one type on one level has the same F, E,
    # G and W (Sec. 5.1.2): one block per (level, type), same solution as the
    # factor that builds every box, and far fewer bytes
    pts = W.grid_points(64)
    f = W.rhs_normal(len(pts), 3, 61)
    fd = rsd.Factor(pts, None, 1e-10)
    ff = rsd.Factor(pts, None, 1e-10, flags=rsd.RSD_FLAG_NO_DEDUP)
    xd, _ = fd.solve(f)
    xf, _ = ff.solve(f)
    ref = dense.solve(pts, f)
    assert dense.rel_error(xd, ref) < 1e-10 and dense.rel_error(xf, ref) < 1e-10
    assert np.linalg.norm(xd - xf) <= 1e-12 * np.linalg.norm(xf)
    bd, bf = fd.stats()["factor_bytes"], ff.stats()["factor_bytes"]
    assert bd < 0.5 * bf
    # a constant a other than 1, and a ragged grid whose levels hold several types
    for p, a in ((W.grid_points(40, 24), 1.7 * np.ones(40 * 24)), (W.grid_points(37), None)):
        g = W.rhs_normal(len(p), 1, 7)
        fc = rsd.Factor(p, a, 1e-10)
        x, _ = fc.solve(g)
        assert dense.rel_error(x, dense.solve(p, g, a)) < 1e-10
        fc.close()
    fd.close()
    ff.close()


# --- tile autotuner ------------------------------------------------------------
def test_autotuned_tiles_give_the_same_solution(tmp_path):
    # the tuned table changes tile widths and split-K only: solutions agree
    # with the built-in rule's to rounding; the table survives a save/load
    grids = [W.grid_points(n) for n in (96, 80, 64)]
    rng = np.random.default_rng(12)
    coefs = [W.coef_bumps(p, rng) for p in grids]
    rhs = [W.rhs_normal(len(p), 1, 3) for p in grids]
    rsd.tune_clear()

    def solve_all():
        facs = rsd.build_batched(grids, coefs, tol=1e-10)
        xs = [f.solve(r)[0] for f, r in zip(facs, rhs)]
        for f in facs:
            f.close()
        return xs

    x0 = solve_all()
    n = rsd.autotune(grids, coefs, tol=1e-10, precision=rsd.RSD_PREC_FP64, reps=1)
    assert n > 0
    path = tmp_path / "tune.txt"
    rsd.tune_save(path)
    assert rsd.tune_clear() == n
    rsd.tune_load(path)
    x1 = solve_all()
    for a, b, p, c, r in zip(x0, x1, grids, coefs, rhs):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
    assert dense.rel_error(x1[2], dense.solve(grids[2], rhs[2], coefs[2])) < 1e-10
    rsd.tune_clear()


def test_profiler_pause_keeps_records_and_skips_paused_launches():
    # the roofline figure samples some timed steps: launches made while the
    # profiler is paused are not bracketed, the records of the others stay
    pts = W.grid_points(64)
    a = W.coef_sine(pts)
    f = W.rhs_normal(len(pts), 1, 5)

    def build():
        fac = rsd.Factor(pts, a, 1e-10)
        x, _ = fac.solve(f)
        fac.close()
        return x

    try:
        rsd.profile_enable(True, classes=["factor_gemm_f64"])
        x1 = build()
        one = rsd.profile_query()["factor_gemm_f64"]
        assert one["launches"] > 0 and one["ms"] > 0
        rsd.profile_enable(True, classes=["factor_gemm_f64"])
        rsd.profile_pause(True)
        x2 = build()
        assert rsd.profile_query()["factor_gemm_f64"]["launches"] == 0
        rsd.profile_pause(False)
        x3 = build()
        rsd.profile_pause(True)
        build()
        rsd.profile_pause(False)
        q = rsd.profile_query()["factor_gemm_f64"]
        assert q["launches"] == one["launches"] and q["flops"] == one["flops"]
    finally:
        rsd.profile_enable(False)
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)
