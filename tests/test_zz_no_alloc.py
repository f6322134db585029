"""The allocation-free exact product (rsd_matvec_noalloc) against rsd_matvec,
through the C interface: two calls in a row, the second on a smaller input,
then the error paths that are decided on the host."""
import numpy as np
import pytest
import torch

from oracle import nystrom
from paper_1303_5466_amd import rsd, workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(fac, x):
    """x: (N, nrhs) host array -> rsd_matvec_noalloc(x) on device buffers."""
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda:0")   # (nrhs, N) = N x nrhs col-major
    yd = torch.full_like(xd, np.nan)
    st = fac.matvec_noalloc_raw(xd.data_ptr(), x.shape[1], yd.data_ptr())
    assert st == rsd.RSD_OK, rsd.load().rsd_last_error().decode()
    torch.cuda.synchronize()
    return yd.cpu().numpy().T


def test_noalloc_matvec_matches_matvec_twice_then_smaller():
    rng = np.random.default_rng(17)
    big = W.grid_points(96, 80)
    small = W.grid_points(40, 24)
    fb = rsd.Factor(big, W.coef_sine(big), 1e-10)
    a_small = W.coef_bumps(small, rng)
    fs = rsd.Factor(small, a_small, 1e-10)
    xb = rng.standard_normal((big.shape[0], 5))
    xs = rng.standard_normal((small.shape[0], 2))
    y1 = _noalloc(fb, xb)
    assert np.array_equal(y1, fb.matvec(xb))              # same kernels, same work
    y2 = _noalloc(fs, xs)                                  # second call, smaller input
    assert np.array_equal(y2, fs.matvec(xs))
    # and against the exact product on sampled rows (the oracle's direct sum)
    rows = rng.choice(small.shape[0], 40, replace=False)
    ref = nystrom.assemble(small, a_small, rows=rows) @ xs
    assert np.abs(y2[rows] - ref).max() <= 1e-12 * np.abs(ref).max()
    y3 = _noalloc(fb, xb[:, :1])                           # the big one again, one column
    assert np.array_equal(y3, fb.matvec(xb[:, :1]))
    # columns travel through the FFT in pairs, so a lone column rounds differently
    assert np.abs(y3 - y1[:, :1]).max() <= 1e-13 * np.abs(y1[:, :1]).max()
    fb.close()
    fs.close()


def test_noalloc_matvec_rejects_host_buffers_and_oversize():
    p = W.grid_points(32)
    fac = rsd.Factor(p, None, 1e-10)
    x = np.ones((p.shape[0], 1), order="F")
    y = np.zeros_like(x)
    assert fac.matvec_noalloc_raw(x.ctypes.data, 1, y.ctypes.data) == rsd.RSD_EINVAL
    # 2 N nrhs + 3 Mx My doubles beyond the 64 MiB work space
    xd = torch.ones((4096, p.shape[0]), dtype=torch.float64, device="cuda:0")
    yd = torch.zeros_like(xd)
    assert fac.matvec_noalloc_raw(xd.data_ptr(), 4096, yd.data_ptr()) == rsd.RSD_EINVAL
    assert "exceed" in rsd.load().rsd_last_error().decode()
    assert fac.matvec_noalloc_raw(xd.data_ptr(), 0, yd.data_ptr()) == rsd.RSD_OK
    fac.close()
