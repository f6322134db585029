"""ctypes binding of librsd.so (include/rsd.h).  Argument marshalling only:
every step of the factorisation and the solve runs in the native library.

Functions with the C names (rsd_build_factor, rsd_solve, ...) are exposed
as attributes of the loaded library object `lib`; `Factor` and `Plan` are thin
owners around the opaque handles.  Arrays may be NumPy arrays (host memory)
or torch tensors on the GPU (device memory); right-hand sides are N x nrhs
column-major, which is a (N, nrhs) array in Fortran order, or the transpose
of a C-contiguous (nrhs, N) tensor.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsd.so")

RSD_OK, RSD_EINVAL, RSD_ENOTGRID, RSD_ENOMEM, RSD_ESINGULAR, RSD_ENOCONV, RSD_EDEVICE, RSD_EAGAIN = range(8)
STATUS_NAMES = ["OK", "EINVAL", "ENOTGRID", "ENOMEM", "ESINGULAR", "ENOCONV", "EDEVICE", "EAGAIN"]
RSD_KERNEL_LAPLACE, RSD_KERNEL_HELMHOLTZ = 0, 1
RSD_PREC_FP64, RSD_PREC_FP32_REFINE = 0, 1
RSD_FLAG_KEEP_E = 1
RSD_FLAG_NO_SYMMETRY = 2
RSD_FLAG_FP32_INTERP = 4
RSD_FLAG_NO_DEDUP = 8
RSD_FLAG_SOLVE_GRAPH = 16
RSD_FLAG_NO_DAMPING = 32


class rsd_kernel(C.Structure):
    _fields_ = [("type", C.c_int32), ("wavenumber", C.c_double), ("contrast_b", C.c_void_p)]


class rsd_options(C.Structure):
    _fields_ = [("leaf_side", C.c_int32), ("layers", C.c_int32), ("precision", C.c_int32),
                ("max_refine", C.c_int32), ("refine_tol", C.c_double), ("hip_stream", C.c_void_p),
                ("device", C.c_int32), ("flags", C.c_int32), ("interface_ppw", C.c_double)]


class rsd_solve_info(C.Structure):
    _fields_ = [("refine_iters", C.c_int32), ("rel_residual", C.c_double)]


class rsd_factor_stats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("nx", C.c_int64), ("ny", C.c_int64),
                ("n_levels", C.c_int32), ("n_boxes", C.c_int32), ("layers", C.c_int32),
                ("precision", C.c_int32), ("factor_bytes", C.c_int64),
                ("factor_flops", C.c_double), ("solve_bytes", C.c_double),
                ("build_ms", C.c_double), ("complex_values", C.c_int32), ("solve_graphs", C.c_int32)]


class rsd_box_info(C.Structure):
    _fields_ = [("level", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32), ("ax", C.c_int32),
                ("ay", C.c_int32), ("k", C.c_int32), ("r", C.c_int32), ("parent", C.c_int32)]


class rsd_interp_info(C.Structure):
    _fields_ = [("n_problems", C.c_int32), ("rank", C.c_int32 * 4), ("scale", C.c_double * 4),
                ("damped", C.c_int32)]


class rsd_server_options(C.Structure):
    _fields_ = [("mem_budget", C.c_int64), ("max_slots", C.c_int32), ("n_workers", C.c_int32),
                ("max_coalesce", C.c_int32), ("device", C.c_int32), ("evict_idle", C.c_int32)]


class rsd_server_stats(C.Structure):
    _fields_ = [("n_requests", C.c_int64), ("n_done", C.c_int64), ("n_batches", C.c_int64),
                ("n_factors", C.c_int64), ("n_evicted", C.c_int64), ("resident_bytes", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_batch_rhs", C.c_double),
                ("rhs_per_s", C.c_double), ("n_queued_factors", C.c_int64), ("n_built", C.c_int64)]


EXPORTS = {
    "rsd_server_create": (C.c_int, [C.POINTER(rsd_server_options), C.POINTER(C.c_void_p)]),
    "rsd_server_submit_factor": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(rsd_kernel),
                                           C.c_void_p, C.c_double, C.POINTER(rsd_options),
                                           C.POINTER(C.c_int64)]),
    "rsd_server_release_factor": (C.c_int, [C.c_void_p, C.c_int64]),
    "rsd_server_wait_factor": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32]),
    "rsd_autotune": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(rsd_kernel), C.c_void_p,
                               C.c_double, C.POINTER(rsd_options), C.c_int32, C.POINTER(C.c_int32)]),
    "rsd_tune_save": (C.c_int, [C.c_char_p]),
    "rsd_tune_load": (C.c_int, [C.c_char_p]),
    "rsd_tune_clear": (C.c_int, [C.POINTER(C.c_int64)]),
    "rsd_self_cell_integral": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]),
    "rsd_estimate_factor_bytes": (C.c_int, [C.c_int64, C.c_int64, C.POINTER(rsd_kernel), C.c_double,
                                            C.POINTER(rsd_options), C.POINTER(C.c_int64)]),
    "rsd_server_submit_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                          C.POINTER(C.c_int64)]),
    "rsd_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.POINTER(rsd_solve_info)]),
    "rsd_server_poll": (C.c_int32, [C.c_void_p, C.c_int64]),
    "rsd_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(rsd_server_stats)]),
    "rsd_server_destroy": (None, [C.c_void_p]),
    "rsd_build_factor": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(rsd_kernel), C.c_void_p,
                                   C.c_double, C.POINTER(rsd_options), C.POINTER(C.c_void_p)]),
    "rsd_build_factor_batched": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                           C.POINTER(rsd_kernel), C.POINTER(C.c_void_p), C.c_double,
                                           C.POINTER(rsd_options), C.c_int32, C.POINTER(C.c_void_p)]),
    "rsd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                            C.POINTER(rsd_solve_info)]),
    "rsd_solve_batched": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int64,
                                    C.POINTER(C.c_void_p), C.POINTER(rsd_solve_info)]),
    "rsd_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "rsd_matvec_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "rsd_free": (None, [C.c_void_p]),
    "rsd_gemm": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                           C.c_double, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                           C.c_void_p, C.c_int32]),
    "rsd_gj_invert": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int32]),
    "rsd_last_error": (C.c_char_p, []),
    "rsd_profile_enable": (C.c_int, [C.c_int32]),
    "rsd_profile_enable_mask": (C.c_int, [C.c_uint32]),
    "rsd_profile_pause": (C.c_int, [C.c_int32]),
    "rsd_profile_record_count": (C.c_int, [C.POINTER(C.c_int64)]),
    "rsd_profile_record": (C.c_int, [C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "rsd_pool_trim": (C.c_int, [C.c_int32]),
    "rsd_pool_set_limit": (C.c_int, [C.c_int64]),
    "rsd_pool_cached_bytes": (C.c_int, [C.c_int32, C.POINTER(C.c_int64)]),
    "rsd_profile_query": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rsd_factor_get_stats": (C.c_int, [C.c_void_p, C.POINTER(rsd_factor_stats)]),
    "rsd_factor_box_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(rsd_box_info)]),
    "rsd_matvec_compressed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "rsd_factor_interp_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(rsd_interp_info)]),
    "rsd_factor_get_block": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "rsd_plan_create": (C.c_int, [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(C.c_void_p)]),
    "rsd_plan_n_boxes": (C.c_int32, [C.c_void_p]),
    "rsd_plan_n_levels": (C.c_int32, [C.c_void_p]),
    "rsd_plan_box_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(rsd_box_info)]),
    "rsd_plan_box_points": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "rsd_plan_box_symmetry": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "rsd_plan_interp_groups": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    "rsd_check_interp_groups": (C.c_int, [C.c_int32, C.c_void_p]),
    "rsd_plan_free": (None, [C.c_void_p]),
    "rsd_detect_grid": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_void_p]),
}

_lib = None


def load():
    """Load librsd.so; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library missing: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RsdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


def _check(status):
    if status != RSD_OK:
        raise RsdError(status, load().rsd_last_error().decode())


def _ptr(x):
    """(pointer, keepalive) for a NumPy array or torch tensor."""
    if x is None:
        return None, None
    if isinstance(x, np.ndarray):
        return x.ctypes.data, x
    return x.data_ptr(), x          # torch tensor


def _is_torch(x):
    return not isinstance(x, np.ndarray) and hasattr(x, "data_ptr")


class Factor:
    """Owner of an rsd_factor handle."""

    def __init__(self, points, a=None, tol=1e-10, kernel=RSD_KERNEL_LAPLACE, wavenumber=0.0,
                 contrast=None, leaf_side=0, layers=0, precision=RSD_PREC_FP64, max_refine=0,
                 refine_tol=0.0, stream=None, device=-1, flags=0, interface_ppw=0.0):
        lib = load()
        if isinstance(points, np.ndarray):
            points = np.ascontiguousarray(points, dtype=np.float64)
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, dtype=np.float64)
        if isinstance(contrast, np.ndarray):
            contrast = np.ascontiguousarray(contrast, dtype=np.float64)
        n = points.shape[0]
        pp, _k1 = _ptr(points)
        ap, _k2 = _ptr(a)
        bp, _k3 = _ptr(contrast)
        kd = rsd_kernel(kernel, wavenumber, bp)
        opt = rsd_options(leaf_side, layers, precision, max_refine, refine_tol,
                          stream if stream is not None else None, device, flags, interface_ppw)
        h = C.c_void_p()
        self._h = None
        _check(lib.rsd_build_factor(pp, n, C.byref(kd), ap, tol, C.byref(opt), C.byref(h)))
        self._h = h
        self.n = n
        self.complex = kernel == RSD_KERNEL_HELMHOLTZ

    @classmethod
    def _adopt(cls, handle, n, complex_=False):
        obj = cls.__new__(cls)
        obj._h = handle
        obj.n = n
        obj.complex = complex_
        return obj

    def close(self):
        if self._h is not None:
            load().rsd_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def stats(self):
        s = rsd_factor_stats()
        _check(load().rsd_factor_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in rsd_factor_stats._fields_}

    def box_info(self, box):
        b = rsd_box_info()
        _check(load().rsd_factor_box_info(self._h, box, C.byref(b)))
        return {f: getattr(b, f) for f, _ in rsd_box_info._fields_}

    def interp_info(self, box):
        """Truncation record of the box type's interpolation: a list with one
        (kept rank, |R_11| reference) pair per problem it was solved as (empty
        for the root, one pair when solved whole, 2 or 4 for symmetry sectors)."""
        b = rsd_interp_info()
        _check(load().rsd_factor_interp_info(self._h, box, C.byref(b)))
        return [(int(b.rank[i]), float(b.scale[i])) for i in range(b.n_problems)]

    def interp_damped(self, box):
        """Whether the box type's interpolation was solved as damped least squares."""
        b = rsd_interp_info()
        _check(load().rsd_factor_interp_info(self._h, box, C.byref(b)))
        return bool(b.damped)

    def block(self, box, which):
        info = self.box_info(box)
        k, r = info["k"], info["r"]
        if which == 2:
            out = np.zeros(k + r, dtype=np.int64)
            _check(load().rsd_factor_get_block(self._h, box, which, out.ctypes.data))
            return out
        rows, cols = (k, r) if which == 0 else (k, k)
        out = np.zeros((cols, rows), dtype=np.float64)
        _check(load().rsd_factor_get_block(self._h, box, which, out.ctypes.data))
        return out.T.copy()

    def solve_raw(self, rhs_ptr, nrhs, x_ptr):
        info = rsd_solve_info()
        st = load().rsd_solve(self._h, rhs_ptr, nrhs, x_ptr, C.byref(info))
        return st, info

    def solve(self, f):
        """x = A^{-1} f for a NumPy (N,) / (N, nrhs) array or a CUDA tensor of
        the same shape; returns the same kind of object and the solve info.
        Helmholtz factors take and return complex128 values."""
        vec = f.ndim == 1
        if _is_torch(f):
            import torch
            F = f.reshape(self.n, -1)
            nrhs = F.shape[1]
            Ft = F.t().contiguous()
            if self.complex and not Ft.is_complex():
                Ft = Ft.to(torch.complex128)
            Xt = torch.empty_like(Ft)
            st, info = self.solve_raw(Ft.data_ptr(), nrhs, Xt.data_ptr())
            _check(st)
            X = Xt.t()
            return (X[:, 0] if vec else X), info
        dt = np.complex128 if self.complex else np.float64
        F = np.asfortranarray(np.asarray(f, dtype=dt).reshape(self.n, -1))
        X = np.zeros_like(F, order="F")
        st, info = self.solve_raw(F.ctypes.data, F.shape[1], X.ctypes.data)
        _check(st)
        return (X[:, 0] if vec else X), info

    def matvec_compressed(self, x):
        """y ~ A x through the factor's skeletonization (O(N), at the factor's
        tolerance); NumPy (N,) / (N, nrhs) in and out, Laplace factors."""
        vec = x.ndim == 1
        X = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(self.n, -1))
        Y = np.zeros_like(X, order="F")
        _check(load().rsd_matvec_compressed(self._h, X.ctypes.data, X.shape[1], Y.ctypes.data))
        return Y[:, 0] if vec else Y

    def matvec(self, x):
        vec = x.ndim == 1
        dt = np.complex128 if self.complex else np.float64
        X = np.asfortranarray(np.asarray(x, dtype=dt).reshape(self.n, -1))
        Y = np.zeros_like(X, order="F")
        _check(load().rsd_matvec(self._h, X.ctypes.data, X.shape[1], Y.ctypes.data))
        return Y[:, 0] if vec else Y

    def matvec_raw(self, x_ptr, nrhs, y_ptr):
        """rsd_matvec on device (or host) pointers; returns the status."""
        return load().rsd_matvec(self._h, x_ptr, nrhs, y_ptr)

    def matvec_compressed_raw(self, x_ptr, nrhs, y_ptr):
        """rsd_matvec_compressed on device (or host) pointers; returns the status."""
        return load().rsd_matvec_compressed(self._h, x_ptr, nrhs, y_ptr)

    def matvec_noalloc_raw(self, x_ptr, nrhs, y_ptr):
        """rsd_matvec_noalloc on device pointers (N x nrhs column-major);
        returns the status."""
        return load().rsd_matvec_noalloc(self._h, x_ptr, nrhs, y_ptr)


def build_batched(points_list, a_list=None, tol=1e-10, precision=RSD_PREC_FP64, leaf_side=0,
                  layers=0, max_refine=0, refine_tol=0.0, max_inflight=0, flags=0,
                  kernel=RSD_KERNEL_LAPLACE, wavenumber=0.0):
    """rsd_build_factor_batched: one Factor per (points, a) instance."""
    lib = load()
    n_inst = len(points_list)
    keep = []
    pts_p = (C.c_void_p * n_inst)()
    a_p = (C.c_void_p * n_inst)()
    npts = (C.c_int64 * n_inst)()
    for i, pts in enumerate(points_list):
        if isinstance(pts, np.ndarray):
            pts = np.ascontiguousarray(pts, dtype=np.float64)
        p, k = _ptr(pts)
        keep += [pts, k]
        pts_p[i] = p
        npts[i] = pts.shape[0]
        a = a_list[i] if a_list is not None else None
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, dtype=np.float64)
        ap, k2 = _ptr(a)
        keep += [a, k2]
        a_p[i] = ap
    kd = rsd_kernel(kernel, wavenumber, None)
    opt = rsd_options(leaf_side, layers, precision, max_refine, refine_tol, None, -1, flags)
    out = (C.c_void_p * n_inst)()
    _check(lib.rsd_build_factor_batched(n_inst, pts_p, npts, C.byref(kd), a_p, tol, C.byref(opt),
                                        max_inflight, out))
    return [Factor._adopt(C.c_void_p(out[i]), int(npts[i])) for i in range(n_inst)]


def solve_batched_raw(factors, rhs_ptrs, nrhs, x_ptrs):
    """rsd_solve_batched over raw pointers (host or device), one per factor;
    returns (status, list of rsd_solve_info)."""
    n = len(factors)
    fs = (C.c_void_p * n)(*[f.handle.value for f in factors])
    rp = (C.c_void_p * n)(*rhs_ptrs)
    xp = (C.c_void_p * n)(*x_ptrs)
    infos = (rsd_solve_info * n)()
    st = load().rsd_solve_batched(n, fs, rp, nrhs, xp, infos)
    return st, list(infos)


class Server:
    """Resident factors + queued, coalesced solves (rsd_server_*).  Buffers
    passed to submit_solve are kept alive here until their ticket is waited."""

    def __init__(self, mem_budget=0, max_slots=0, n_workers=0, max_coalesce=0, device=-1,
                 evict_idle=False):
        lib = load()
        h = C.c_void_p()
        opt = rsd_server_options(mem_budget, max_slots, n_workers, max_coalesce, device,
                                 1 if evict_idle else 0)
        _check(lib.rsd_server_create(C.byref(opt), C.byref(h)))
        self._h = h
        self._live = {}
        self._n = {}          # factor id -> number of points

    def submit_factor(self, points, a=None, tol=1e-10, precision=RSD_PREC_FP64, leaf_side=0,
                      layers=0, max_refine=0, refine_tol=0.0, wait=True, kernel=RSD_KERNEL_LAPLACE,
                      wavenumber=0.0, contrast=None):
        """Queue a factor request; with wait=True return once it is resident
        (raises the build's error), else at once (see wait_factor)."""
        if isinstance(points, np.ndarray):
            points = np.ascontiguousarray(points, dtype=np.float64)
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, dtype=np.float64)
        if isinstance(contrast, np.ndarray):
            contrast = np.ascontiguousarray(contrast, dtype=np.float64)
        pp, _k1 = _ptr(points)
        ap, _k2 = _ptr(a)
        bp, _k3 = _ptr(contrast)
        kd = rsd_kernel(kernel, wavenumber, bp)
        opt = rsd_options(leaf_side, layers, precision, max_refine, refine_tol, None, -1, 0)
        fid = C.c_int64()
        _check(load().rsd_server_submit_factor(self._h, pp, points.shape[0], C.byref(kd), ap, tol,
                                               C.byref(opt), C.byref(fid)))
        self._n[fid.value] = (int(points.shape[0]), kernel == RSD_KERNEL_HELMHOLTZ)
        if wait:
            self.wait_factor(fid.value)
        return fid.value

    def wait_factor(self, fid, timeout_ms=-1):
        """RSD_OK once resident, RSD_EAGAIN on timeout; raises on a failed build."""
        st = load().rsd_server_wait_factor(self._h, fid, timeout_ms)
        if st not in (RSD_OK, RSD_EAGAIN):
            self._n.pop(fid, None)
            _check(st)
        return st

    def release_factor(self, fid):
        _check(load().rsd_server_release_factor(self._h, fid))
        self._n.pop(fid, None)

    def submit_solve(self, fid, rhs, out):
        """Queue out = A^{-1} rhs.  rhs, out: NumPy arrays of shape (N,) or
        (N, nrhs) (any layout or float dtype for rhs; out must be float64 of
        the same shape, and is filled when the ticket is waited), or contiguous
        float64 torch tensors on the device of shape (N,) or (nrhs, N) (= N x
        nrhs column-major).  Shapes are checked against the factor's N."""
        entry = self._n.get(fid)
        if entry is None:
            raise RsdError(RSD_EINVAL, f"unknown factor {fid}")
        n, cplx = entry
        ndt = np.complex128 if cplx else np.float64
        copy_back = None
        if isinstance(rhs, np.ndarray):
            if rhs.ndim not in (1, 2) or rhs.shape[0] != n:
                raise RsdError(RSD_EINVAL, f"rhs shape {rhs.shape} does not match N = {n}")
            nrhs = 1 if rhs.ndim == 1 else rhs.shape[1]
            if not isinstance(out, np.ndarray) or out.shape != rhs.shape or out.dtype != ndt:
                raise RsdError(RSD_EINVAL, f"out must be a {np.dtype(ndt).name} NumPy array of the rhs shape")
            rhs = np.asfortranarray(rhs, dtype=ndt)
            if not out.flags.f_contiguous:
                copy_back = out
                out = np.zeros(out.shape, dtype=ndt, order="F")
        else:
            import torch
            if not (isinstance(rhs, torch.Tensor) and isinstance(out, torch.Tensor)):
                raise RsdError(RSD_EINVAL, "rhs and out must both be NumPy arrays or torch tensors")
            if rhs.dim() == 1:
                nrhs = 1
                ok = rhs.shape[0] == n
            else:
                nrhs = rhs.shape[0]
                ok = rhs.dim() == 2 and rhs.shape[1] == n
            if not ok:
                raise RsdError(RSD_EINVAL, f"rhs shape {tuple(rhs.shape)} is not (N,) or (nrhs, N), N = {n}")
            tdt = torch.complex128 if cplx else torch.float64
            for name, t in (("rhs", rhs), ("out", out)):
                if t.dtype != tdt or not t.is_contiguous():
                    raise RsdError(RSD_EINVAL, f"{name} must be a contiguous {tdt} tensor")
            if out.shape != rhs.shape or out.device != rhs.device:
                raise RsdError(RSD_EINVAL, "out must have the shape and device of rhs")
        tk = C.c_int64()
        _check(load().rsd_server_submit_solve(self._h, fid, _ptr(rhs)[0], nrhs, _ptr(out)[0],
                                              C.byref(tk)))
        self._live[tk.value] = (rhs, out, copy_back)
        return tk.value

    def wait(self, ticket, timeout_ms=-1):
        """(status, rsd_solve_info); status EAGAIN on timeout."""
        info = rsd_solve_info()
        st = load().rsd_server_wait(self._h, ticket, timeout_ms, C.byref(info))
        if st != RSD_EAGAIN:
            live = self._live.pop(ticket, None)
            if live is not None and live[2] is not None:
                live[2][...] = live[1]
        return st, info

    def poll(self, ticket):
        return load().rsd_server_poll(self._h, ticket)

    def stats(self):
        s = rsd_server_stats()
        _check(load().rsd_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in rsd_server_stats._fields_}

    def close(self):
        if self._h is not None:
            load().rsd_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Host-only tree / skeleton plan (no device needed)."""

    def __init__(self, nx, ny, leaf_side=8, layers=2, interface_step=0):
        lib = load()
        h = C.c_void_p()
        _check(lib.rsd_plan_create(nx, ny, leaf_side, layers, interface_step, C.byref(h)))
        self._h = h

    def __del__(self):
        try:
            if self._h is not None:
                load().rsd_plan_free(self._h)
        except Exception:
            pass

    @property
    def n_boxes(self):
        return load().rsd_plan_n_boxes(self._h)

    @property
    def n_levels(self):
        return load().rsd_plan_n_levels(self._h)

    def box_info(self, box):
        b = rsd_box_info()
        _check(load().rsd_plan_box_info(self._h, box, C.byref(b)))
        return {f: getattr(b, f) for f, _ in rsd_box_info._fields_}

    def box_symmetry(self, box):
        """Reflection group of the box type (bit 0: u, bit 1: v)."""
        g = C.c_int32()
        _check(load().rsd_plan_box_symmetry(self._h, box, C.byref(g)))
        return g.value

    def interp_groups(self, split=True):
        """Sector problems of the plan's interpolation (rsd_plan_interp_groups):
        an (n, 7) int32 array of (owner, sec, g0, gn, p, k, r) rows."""
        lib = load()
        n = C.c_int32()
        _check(lib.rsd_plan_interp_groups(self._h, int(bool(split)), C.byref(n), None))
        out = np.zeros((n.value, 7), dtype=np.int32)
        _check(lib.rsd_plan_interp_groups(self._h, int(bool(split)), C.byref(n), out.ctypes.data))
        return out

    def box_points(self, box):
        info = self.box_info(box)
        out = np.zeros(info["k"] + info["r"], dtype=np.int64)
        _check(load().rsd_plan_box_points(self._h, box, out.ctypes.data))
        return out


def check_interp_groups(table):
    """Run the library's sector-group check on an (n, 7) int32 table; raises
    RsdError (EINVAL) when a group is not one problem's consecutive sectors."""
    t = np.ascontiguousarray(table, dtype=np.int32).reshape(-1, 7)
    _check(load().rsd_check_interp_groups(t.shape[0], t.ctypes.data if t.size else None))


PROF_CLASSES = ["factor_gemm_f64", "factor_gemm_f32", "interp", "gj_pivot", "assembly",
                "solve_gemm", "solve_move", "matvec"]


def pool_trim(device=-1):
    """Hand the cached device blocks back to HIP (device < 0: every device)."""
    _check(load().rsd_pool_trim(device))


def pool_set_limit(nbytes):
    """Per-device limit of cached bytes (< 0: the default)."""
    _check(load().rsd_pool_set_limit(int(nbytes)))


def pool_cached_bytes(device=-1):
    out = C.c_int64()
    _check(load().rsd_pool_cached_bytes(device, C.byref(out)))
    return out.value


def profile_enable(on=True, classes=None):
    """Start (clearing earlier records) or stop the profiler; `classes` limits
    the bracketed launches to those class names."""
    if classes is None:
        _check(load().rsd_profile_enable(1 if on else 0))
    else:
        mask = 0
        for c in classes:
            mask |= 1 << PROF_CLASSES.index(c)
        _check(load().rsd_profile_enable_mask(mask if on else 0))


def profile_pause(paused=True):
    """Stop (or resume) bracketing launches without clearing the records."""
    _check(load().rsd_profile_pause(1 if paused else 0))


def profile_records():
    """Every recorded launch since the last enable, in enqueue order:
    list of dict(cls, ms, flops, bytes, groups)."""
    lib = load()
    n = C.c_int64()
    _check(lib.rsd_profile_record_count(C.byref(n)))
    out = []
    for i in range(n.value):
        c, ms, fl, by, g = C.c_int32(), C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        _check(lib.rsd_profile_record(i, C.byref(c), C.byref(ms), C.byref(fl), C.byref(by), C.byref(g)))
        out.append(dict(cls=PROF_CLASSES[c.value], ms=ms.value, flops=fl.value, bytes=by.value,
                        groups=g.value))
    return out


def profile_query():
    """{class name: dict(ms, launches, flops, bytes)} since the last enable."""
    out = {}
    for i, name in enumerate(PROF_CLASSES):
        ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        _check(load().rsd_profile_query(i, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
        out[name] = dict(ms=ms.value, launches=n.value, flops=fl.value, bytes=by.value)
    return out


def gemm(A, B, C=None, alpha=1.0, beta=0.0, tA=False, tB=False):
    """C = alpha op(A) op(B) + beta C on the device (NumPy in and out)."""
    dt = A.dtype
    code = 0 if dt == np.float64 else 1
    A = np.asfortranarray(A)
    B = np.asfortranarray(B.astype(dt))
    M = A.shape[1] if tA else A.shape[0]
    K = A.shape[0] if tA else A.shape[1]
    N = B.shape[0] if tB else B.shape[1]
    C = np.zeros((M, N), dtype=dt, order="F") if C is None else np.asfortranarray(C.astype(dt))
    _check(load().rsd_gemm(code, M, N, K, int(tA), int(tB), alpha, A.ctypes.data, A.shape[0],
                           B.ctypes.data, B.shape[0], beta, C.ctypes.data, C.shape[0]))
    return C


def gj_invert(A, paired=False):
    """Inverse by the library's blocked Gauss-Jordan (NumPy in and out);
    paired: eliminate pivots two at a time (complex entries in real form)."""
    code = (0 if A.dtype == np.float64 else 1) | (2 if paired else 0)
    X = np.asfortranarray(A.copy())
    _check(load().rsd_gj_invert(code, X.shape[0], X.ctypes.data, X.shape[0]))
    return X


def detect_grid(points):
    pts = np.ascontiguousarray(points, dtype=np.float64)
    nx, ny, h = C.c_int64(), C.c_int64(), C.c_double()
    perm = np.zeros(pts.shape[0], dtype=np.int64)
    _check(load().rsd_detect_grid(pts.ctypes.data, pts.shape[0], C.byref(nx), C.byref(ny),
                                  C.byref(h), perm.ctypes.data))
    return nx.value, ny.value, h.value, perm


def estimate_factor_bytes(nx, ny, tol=1e-10, precision=RSD_PREC_FP64, leaf_side=0, layers=0,
                          kernel=None):
    """Device bytes of the factor of an nx x ny grid (host only)."""
    opt = rsd_options(leaf_side, layers, precision, 0, 0.0, None, -1, 0)
    kd = rsd_kernel(RSD_KERNEL_LAPLACE if kernel is None else kernel, 1.0, None)
    out = C.c_int64()
    _check(load().rsd_estimate_factor_bytes(nx, ny, C.byref(kd), tol, C.byref(opt), C.byref(out)))
    return out.value


def self_cell_integral(h, kernel=RSD_KERNEL_LAPLACE, k=0.0):
    """The library's diagonal term: integral of the kernel over the cell of side h."""
    re, im = C.c_double(), C.c_double()
    _check(load().rsd_self_cell_integral(kernel, h, k, C.byref(re), C.byref(im)))
    return complex(re.value, im.value) if kernel == RSD_KERNEL_HELMHOLTZ else re.value


def autotune(points_list, a_list=None, tol=1e-8, precision=RSD_PREC_FP32_REFINE, reps=2, leaf_side=0, layers=0):
    """rsd_autotune on one grid or a batch (host or device arrays); returns
    the number of shape buckets set."""
    n_inst = len(points_list)
    keep = []
    pts_p = (C.c_void_p * n_inst)()
    a_p = (C.c_void_p * n_inst)()
    npts = (C.c_int64 * n_inst)()
    for i, pts in enumerate(points_list):
        if isinstance(pts, np.ndarray):
            pts = np.ascontiguousarray(pts, dtype=np.float64)
        p, k = _ptr(pts)
        keep += [pts, k]
        pts_p[i] = p
        npts[i] = pts.shape[0]
        a = a_list[i] if a_list is not None else None
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, dtype=np.float64)
        ap, k2 = _ptr(a)
        keep += [a, k2]
        a_p[i] = ap
    kd = rsd_kernel(RSD_KERNEL_LAPLACE, 0.0, None)
    opt = rsd_options(leaf_side, layers, precision, 0, 0.0, None, -1, 0)
    n = C.c_int32()
    _check(load().rsd_autotune(n_inst, pts_p, npts, C.byref(kd), a_p, tol, C.byref(opt), reps, C.byref(n)))
    return n.value


def tune_save(path):
    _check(load().rsd_tune_save(str(path).encode()))


def tune_load(path):
    _check(load().rsd_tune_load(str(path).encode()))


def tune_clear():
    n = C.c_int64()
    _check(load().rsd_tune_clear(C.byref(n)))
    return n.value
