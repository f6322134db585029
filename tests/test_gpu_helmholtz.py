"""The Helmholtz (Lippmann-Schwinger) and contrast-form paths on the device,
through the C interface, against the CPU reference: the scattering operator
A = I + S G S of Sec. 5.4 (S = diag sqrt b, G = (i/4) H0^(1)(k r) of
Sec. 5.3) on Gaussian-bump contrasts, and the Laplace kernel in the same
contrast form."""
import numpy as np
import pytest
import torch

from oracle import dense, krylov, nystrom
from paper_1303_5466_amd import rsd, workloads as W

pytestmark = pytest.mark.gpu

K = W.SCATTER_K


def _incident(pts, b, k=K, src=(-0.5, 0.5)):
    """Right-hand side -sqrt(b) u_in for a point source outside the domain."""
    r = np.sqrt(((pts - np.asarray(src)) ** 2).sum(axis=1))
    return -np.sqrt(b) * nystrom.kernel(r, "helmholtz", k)


def test_exact_complex_product_matches_direct_sum():
    # the device's FFT product of the scattering operator (Hankel function on
    # the device) against the reference's dense rows
    pts = W.grid_points(40, 32)
    b = W.contrast_bump(pts)
    fac = rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b)
    x = W.rhs_complex_normal(len(pts), 3, 11)
    y = fac.matvec(x)
    rows = np.random.default_rng(3).choice(len(pts), 60, replace=False)
    ref = nystrom.assemble(pts, None, "helmholtz", K, b, rows=rows) @ x
    assert np.abs(y[rows] - ref).max() <= 1e-12 * np.abs(ref).max()
    fac.close()


@pytest.mark.parametrize("nx,ny", [(32, 32), (48, 40), (64, 64)])
def test_scattering_fp64_matches_dense(nx, ny):
    pts = W.grid_points(nx, ny)
    b = W.contrast_bump(pts)
    f = np.stack([_incident(pts, b), W.rhs_complex_normal(len(pts), 1, nx)[:, 0]], axis=1)
    fac = rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b)
    assert fac.stats()["complex_values"] == 1
    x, _ = fac.solve(f)
    ref = dense.solve(pts, f, None, "helmholtz", K, b)
    err = dense.rel_error(x, ref)
    print(f"{nx}x{ny}: relative error vs dense {err:.2e}")
    assert err < 1e-9
    # device tensors, one column
    xd, _ = fac.solve(torch.from_numpy(f[:, 0].copy()).to("cuda:0"))
    assert dense.rel_error(xd.cpu().numpy(), ref[:, 0]) < 1e-9
    fac.close()


def test_scattering_fp32_refine_to_1e8():
    # float32 J blocks + float64 complex residual and refinement to 1e-8 on a
    # grid where the float32 factor is a contraction (two skeleton layers);
    # where it is not, the solve reports ENOCONV instead of a wrong answer
    pts = W.grid_points(64)
    b = W.contrast_bump(pts)
    f = np.stack([_incident(pts, b), W.rhs_complex_normal(len(pts), 1, 7)[:, 0]], axis=1)
    fac = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b,
                     precision=rsd.RSD_PREC_FP32_REFINE, layers=2)
    x, info = fac.solve(f)
    assert info.rel_residual <= 1e-8 and info.refine_iters >= 1
    ref = dense.solve(pts, f, None, "helmholtz", K, b)
    err = dense.rel_error(x, ref)
    print(f"float32 + refinement: {info.refine_iters} steps, residual {info.rel_residual:.1e}, error {err:.1e}")
    assert err < 1e-8
    fac.close()
    bad = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b,
                     precision=rsd.RSD_PREC_FP32_REFINE, max_refine=3)
    F = np.asfortranarray(f)
    X = np.zeros_like(F)
    st, info = bad.solve_raw(F.ctypes.data, 2, X.ctypes.data)
    assert st in (rsd.RSD_OK, rsd.RSD_ENOCONV)
    if st == rsd.RSD_OK:
        assert info.rel_residual <= 1e-8
    else:
        assert info.rel_residual > 1e-8
    bad.close()


def test_scattering_128_256_refined_against_reference():
    # the served configuration: float64 (complex128) factor at tol 1e-8 (three
    # layers) plus complex128 refinement; exact residuals of every column and
    # one column against the reference's GMRES
    for n in (128, 256):
        pts = W.grid_points(n)
        b = W.contrast_bump(pts)
        f = np.stack([_incident(pts, b), W.rhs_complex_normal(len(pts), 1, 5)[:, 0]], axis=1)
        fac = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b,
                         max_refine=2)
        assert fac.stats()["layers"] == 3
        x, info = fac.solve(f)
        r = f - nystrom.matvec_fft(pts, x, None, "helmholtz", K, b)
        res = np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)
        assert res.max() <= 1e-8
        if n == 128:
            ref, _ = krylov.solve(pts, f[:, 0], None, "helmholtz", K, b, tol=1e-13)
            assert np.linalg.norm(x[:, 0] - ref) <= 1e-8 * np.linalg.norm(ref)
        fac.close()


def test_laplace_contrast_form_matches_dense():
    pts = W.grid_points(40, 36)
    b = W.contrast_bump(pts, amp=0.8, width=0.2)
    f = W.rhs_normal(len(pts), 2, 19)
    fac = rsd.Factor(pts, None, 1e-10, contrast=b)
    x, _ = fac.solve(f)
    assert dense.rel_error(x, dense.solve(pts, f, None, "laplace", 0.0, b)) < 1e-10
    fac.close()


def test_complex_and_contrast_argument_errors():
    pts = W.grid_points(16)
    b = W.contrast_bump(pts)
    with pytest.raises(rsd.RsdError) as e:        # the contrast must be positive
        rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b * 0)
    assert e.value.status == rsd.RSD_EINVAL
    with pytest.raises(rsd.RsdError):             # a and the contrast together
        rsd.Factor(pts, np.ones(len(pts)), 1e-10, contrast=b)
    with pytest.raises(rsd.RsdError):             # wavenumber must be positive
        rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=0.0, contrast=b)
    with pytest.raises(rsd.RsdError):             # batched builds are Laplace-only
        rsd.build_batched([pts], None, tol=1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ)


def test_served_scattering_factors():
    # Helmholtz factors resident in the server beside a Laplace one; complex
    # requests coalesced per factor equal the direct solves
    srv = rsd.Server(n_workers=2, max_coalesce=8)
    grids = [W.grid_points(48), W.grid_points(32, 40)]
    bs = [W.contrast_bump(p) for p in grids]
    fids = [srv.submit_factor(p, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b)
            for p, b in zip(grids, bs)]
    lap = srv.submit_factor(W.grid_points(24))
    direct = [rsd.Factor(p, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b)
              for p, b in zip(grids, bs)]
    reqs = []
    for i in range(12):
        g = i % 2
        f = np.asfortranarray(W.rhs_complex_normal(len(grids[g]), 1 + i % 3, 100 + i))
        x = np.zeros_like(f)
        reqs.append((g, f, x, srv.submit_solve(fids[g], f, x)))
    fl = np.asfortranarray(W.rhs_normal(24 * 24, 1, 3))
    xl = np.zeros_like(fl)
    tl = srv.submit_solve(lap, fl, xl)
    for g, f, x, tk in reqs:
        st, _ = srv.wait(tk)
        assert st == rsd.RSD_OK
        xa, _ = direct[g].solve(f)
        assert np.linalg.norm(x - xa) <= 1e-12 * np.linalg.norm(xa)
    assert srv.wait(tl)[0] == rsd.RSD_OK
    assert dense.rel_error(xl, dense.solve(W.grid_points(24), fl)) < 1e-10
    srv.close()
    for d in direct:
        d.close()


# --- interface skeleton points and higher wavenumbers (Sec. 5.3) --------------
def test_interface_points_scattering_matches_dense():
    # a few points per wavelength kept on the cut between the children of
    # every box: larger skeletons, same solution as the dense solve
    pts = W.grid_points(64)
    b = W.contrast_bump(pts)
    k = 60.0
    f = W.rhs_complex_normal(len(pts), 2, 81)
    fi = rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=k, contrast=b,
                    interface_ppw=2.0)
    f0 = rsd.Factor(pts, None, 1e-10, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=k, contrast=b)
    grown = 0
    for bx in range(fi.stats()["n_boxes"]):
        a, c = fi.box_info(bx), f0.box_info(bx)
        assert a["k"] >= c["k"]
        grown += a["k"] > c["k"]
    assert grown > 0
    x, _ = fi.solve(f)
    ref = dense.solve(pts, f, None, "helmholtz", k, b)
    err = dense.rel_error(x, ref)
    print("interface points (step 3): error vs dense %.2e" % err)
    assert err < 1e-10
    fi.close()
    f0.close()


@pytest.mark.parametrize("k,ppw,precision", [(100.0, 0.0, rsd.RSD_PREC_FP64), (100.0, 4.0, rsd.RSD_PREC_FP64),
                                             (100.0, 0.0, rsd.RSD_PREC_FP32_REFINE),
                                             (200.0, 0.0, rsd.RSD_PREC_FP64)])
def test_higher_wavenumber_scattering(k, ppw, precision):
    # wavelengths of 8 and 4 grid cells (a leaf box or half of one) on 128^2:
    # with the damped interpolation the three-layer factor stays at the
    # tolerance, with and without interface points, and a complex64 factor
    # refines to it
    pts = W.grid_points(128)
    b = W.contrast_bump(pts)
    f = W.rhs_complex_normal(len(pts), 1, 83)
    fac = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=k, contrast=b,
                     interface_ppw=ppw, precision=precision,
                     max_refine=10 if precision == rsd.RSD_PREC_FP32_REFINE else 0, refine_tol=1e-10)
    x, info = fac.solve(f)
    r = fac.matvec(x) - f
    res = np.linalg.norm(r) / np.linalg.norm(f)
    print(f"k={k:g} ppw={ppw:g}: residual {res:.2e}, {info.refine_iters} refinement steps")
    assert res <= 1e-10
    fac.close()


def test_largest_damped_problems_use_single_column_sub_panels():
    # interface points every grid cell at k = 300 on 256^2 make the 128 x 256
    # box type's damped problem about 10000 rows tall: solved with
    # single-column sub-panels (the panel kernel's local memory), damped, and
    # the factor meets the tolerance
    pts = W.grid_points(256)
    b = W.contrast_bump(pts)
    fac = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=300.0, contrast=b,
                     interface_ppw=4.0)
    for bx in range(fac.stats()["n_boxes"]):
        info = fac.box_info(bx)
        if info["r"] > 0 and info["parent"] >= 0:
            assert fac.interp_damped(bx), info
    f = W.rhs_complex_normal(len(pts), 1, 85)
    x, _ = fac.solve(f)
    assert np.linalg.norm(fac.matvec(x) - f) <= 1e-10 * np.linalg.norm(f)
    fac.close()


def test_scattering_512_complex128():
    # the scattering workload on 512^2: the complex root block (18288^2 in the
    # float64 real form, 2.7 GB) exceeds 2 GiB (descriptors based per tile),
    # the damped problems of the two largest types need single-column
    # sub-panels and float sort keys; complex128 factor, 26 GB
    pts = W.grid_points(512)
    b = W.contrast_bump(pts)
    fac = rsd.Factor(pts, None, 1e-8, kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=K, contrast=b,
                     max_refine=2, refine_tol=1e-8)
    f = W.rhs_complex_normal(len(pts), 1, 87)
    x, info = fac.solve(f)
    res = np.linalg.norm(fac.matvec(x) - f) / np.linalg.norm(f)
    print(f"512^2 complex128: {info.refine_iters} refinement steps, residual {res:.2e}, "
          f"{fac.stats()['factor_bytes'] / 1e9:.1f} GB")
    assert res <= 1e-10
    fac.close()
