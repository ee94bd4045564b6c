"""Python binding of the H^2 library (include/h2.h) -- argument marshalling only.

Every step of the construction and of the apply runs in the library's HIP
kernels; PyTorch only provides device memory and the current stream.  The
shared library is built in-tree by ``build_lib.py``; if it is missing the
import of this module fails (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # imported first so that the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2.so")

H2_OK, H2_EINVAL, H2_ENOMEM, H2_EDEVICE, H2_EUNSUPPORTED, H2_EINTERNAL = 0, -1, -2, -3, -4, -5
DATAREDUCT = {"volume": 0, "fps": 1, "surface": 2}
KERNELS = {"coulomb": 0, "gaussian": 1, "exponential": 2, "matern32": 3, "bump": 4, "cosine": 5,
           "advection": 6}

EXPORTS = {"perm": (0, np.int32), "parent": (1, np.int32), "first_child": (2, np.int32),
           "nchild": (3, np.int32), "start": (4, np.int32), "count": (5, np.int32),
           "depth": (6, np.int32), "center": (7, np.float64), "side": (8, np.float64),
           "il_ptr": (9, np.int32), "il_col": (10, np.int32), "near_ptr": (11, np.int32),
           "near_col": (12, np.int32), "xstar": (13, np.int32), "ystar": (14, np.int32),
           "rank": (15, np.int32), "mbar": (16, np.int32), "piv": (17, np.int32),
           "skel": (18, np.int32), "T": (19, np.float64), "points": (20, np.float64),
           "B": (21, np.float64), "calib_r": (22, np.int32),
           "rank_v": (23, np.int32), "mbar_v": (24, np.int32), "piv_v": (25, np.int32),
           "skel_v": (26, np.int32), "T_v": (27, np.float64)}


class H2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"h2 status {status}: {msg}")
        self.status = status


class h2_options(C.Structure):
    _fields_ = [("tau", C.c_double), ("r1", C.c_int), ("r2", C.c_int), ("precision", C.c_int),
                ("store_coupling", C.c_int), ("calib_seed", C.c_uint64), ("profile", C.c_int),
                ("r_min", C.c_int), ("datareduct", C.c_int), ("srrqr_f", C.c_double)]


class h2_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int), ("kernel_id", C.c_int), ("nnode", C.c_int),
                ("maxdepth", C.c_int), ("nleaf", C.c_int), ("r1", C.c_int), ("r2", C.c_int),
                ("nnz_il", C.c_int64), ("nnz_near", C.c_int64), ("max_rank", C.c_int),
                ("sum_rank", C.c_int64), ("bytes_U", C.c_int64), ("bytes_B", C.c_int64),
                ("bytes_D", C.c_int64), ("precision", C.c_int), ("t_tree", C.c_double), ("t_lists", C.c_double),
                ("t_calib", C.c_double), ("t_hidr", C.c_double), ("t_basis", C.c_double),
                ("t_blocks", C.c_double), ("mv_gather", C.c_double), ("mv_upward", C.c_double),
                ("mv_coupling", C.c_double), ("mv_downward", C.c_double), ("mv_leaves", C.c_double),
                ("mv_scatter", C.c_double), ("mv_nrhs", C.c_int), ("id_ms", C.c_double),
                ("id_wide_ms", C.c_double), ("id_flops", C.c_double), ("id_wide_flops", C.c_double),
                ("hidr_down_ms", C.c_double), ("hidr_down_bytes", C.c_double),
                ("nonsymmetric", C.c_int), ("max_rank_v", C.c_int), ("sum_rank_v", C.c_int64),
                ("bytes_V", C.c_int64), ("hidr_down_evals", C.c_double)]


SYMBOLS = ["h2_options_default", "h2_build", "h2_build_ex", "h2_build_batched", "h2_rebuild", "h2_matvec",
           "h2_matvec_ex", "h2_matvec_noalloc", "h2_query", "h2_export", "h2_destroy", "h2_last_error"]

_lib = None


def lib():
    """Load libh2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run build_lib.py (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.h2_options_default.argtypes = [C.POINTER(h2_options)]
        L.h2_build.restype = C.c_int
        L.h2_build.argtypes = [vp, C.c_int64, C.c_int, C.c_int, dp, C.c_double, C.c_int, C.POINTER(vp)]
        L.h2_build_ex.restype = C.c_int
        L.h2_build_ex.argtypes = [vp, C.c_int64, C.c_int, C.c_int, dp, C.c_double, C.c_int,
                                  C.POINTER(h2_options), vp, C.POINTER(vp)]
        ip = C.POINTER(C.c_int)
        L.h2_build_batched.restype = C.c_int
        L.h2_build_batched.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(C.c_int64), ip, ip, dp, dp, ip,
                                       C.POINTER(h2_options), vp, C.POINTER(vp)]
        L.h2_rebuild.restype = C.c_int
        L.h2_rebuild.argtypes = [vp, C.c_int, dp, C.c_double]
        L.h2_matvec.restype = C.c_int
        L.h2_matvec.argtypes = [vp, vp, vp, C.c_int]
        L.h2_matvec_ex.restype = C.c_int
        L.h2_matvec_ex.argtypes = [vp, vp, vp, C.c_int, vp]
        L.h2_matvec_noalloc.restype = C.c_int
        L.h2_matvec_noalloc.argtypes = [vp, vp, vp, C.c_int, vp]
        L.h2_query.restype = C.c_int
        L.h2_query.argtypes = [vp, C.POINTER(h2_info)]
        L.h2_export.restype = C.c_int
        L.h2_export.argtypes = [vp, C.c_int, C.c_int, vp, C.c_size_t, C.POINTER(C.c_int64)]
        L.h2_destroy.restype = C.c_int
        L.h2_destroy.argtypes = [vp]
        L.h2_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st):
    if st != H2_OK:
        raise H2Error(st, lib().h2_last_error().decode())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def h2_options_default() -> h2_options:
    o = h2_options()
    lib().h2_options_default(C.byref(o))
    return o


def h2_build(points_soa: torch.Tensor, kernel_id, params, tol, leaf_size, options=None, stream=None):
    """C ABI h2_build_ex: points_soa is a contiguous float64 CUDA tensor [dim, n]."""
    assert points_soa.is_cuda and points_soa.dtype == torch.float64 and points_soa.is_contiguous()
    dim, n = points_soa.shape
    kid = KERNELS[kernel_id] if isinstance(kernel_id, str) else int(kernel_id)
    prm = (C.c_double * 1)(float(params))
    opt = options if options is not None else h2_options_default()
    out = C.c_void_p()
    _check(lib().h2_build_ex(C.c_void_p(points_soa.data_ptr()), n, dim, kid, prm, float(tol), int(leaf_size),
                             C.byref(opt), _stream_ptr(stream), C.byref(out)))
    return out


def h2_build_batched(points_list, kernels, params, tols, leaf_sizes, options=None, stream=None):
    """C ABI h2_build_batched: one contiguous float64 CUDA tensor [dim, n] per
    problem; kernels, params, tols, leaf_sizes are per-problem sequences.
    Returns the list of handles."""
    k = len(points_list)
    for P in points_list:
        assert P.is_cuda and P.dtype == torch.float64 and P.is_contiguous()
    ptrs = (C.c_void_p * k)(*[P.data_ptr() for P in points_list])
    ns = (C.c_int64 * k)(*[P.shape[1] for P in points_list])
    dims = (C.c_int * k)(*[P.shape[0] for P in points_list])
    kids = (C.c_int * k)(*[KERNELS[x] if isinstance(x, str) else int(x) for x in kernels])
    prms = (C.c_double * k)(*[float(x) for x in params])
    tl = (C.c_double * k)(*[float(x) for x in tols])
    lf = (C.c_int * k)(*[int(x) for x in leaf_sizes])
    opt = options if options is not None else h2_options_default()
    out = (C.c_void_p * k)()
    _check(lib().h2_build_batched(k, ptrs, ns, dims, kids, prms, tl, lf, C.byref(opt), _stream_ptr(stream), out))
    return [C.c_void_p(out[i]) for i in range(k)]


def h2_rebuild(handle, kernel_id, params, tol):
    """C ABI h2_rebuild: another kernel / parameter / tolerance on the same
    representor sets (tree, lists, r1, r2, X*, Y* kept)."""
    kid = KERNELS[kernel_id] if isinstance(kernel_id, str) else int(kernel_id)
    prm = (C.c_double * 1)(float(params))
    _check(lib().h2_rebuild(handle, kid, prm, float(tol)))


def h2_matvec(handle, x: torch.Tensor, y: torch.Tensor, nrhs: int, stream=None):
    """C ABI h2_matvec_ex: x, y contiguous CUDA tensors [nrhs, n], float64
    (precision 64) or float32 (precision 32)."""
    _check(lib().h2_matvec_ex(handle, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(nrhs),
                              _stream_ptr(stream)))


def h2_matvec_noalloc(handle, x: torch.Tensor, y: torch.Tensor, nrhs: int, stream=None):
    """C ABI h2_matvec_noalloc: as h2_matvec, on the library's per-device
    scratch array (no allocation)."""
    _check(lib().h2_matvec_noalloc(handle, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(nrhs),
                                   _stream_ptr(stream)))


def h2_query(handle) -> dict:
    info = h2_info()
    _check(lib().h2_query(handle, C.byref(info)))
    return {f: getattr(info, f) for f, _ in h2_info._fields_}


def h2_export(handle, what: str, node: int = -1) -> np.ndarray:
    wid, dt = EXPORTS[what]
    cnt = C.c_int64(0)
    _check(lib().h2_export(handle, wid, int(node), None, 0, C.byref(cnt)))
    buf = np.empty(max(cnt.value, 1), dtype=dt)
    _check(lib().h2_export(handle, wid, int(node), C.c_void_p(buf.ctypes.data), buf.nbytes, C.byref(cnt)))
    return buf[: cnt.value].copy()


def h2_destroy(handle):
    if handle:
        _check(lib().h2_destroy(handle))


class H2Matrix:
    """Owning wrapper: builds on construction, applies with matvec()."""

    def __init__(self, points, kernel="coulomb", prm=1.0, tol=1e-6, leaf=64, tau=0.7, r1=0, r2=0,
                 seed=0x5EED, stream=None, precision=64, r_min=0, datareduct="volume", srrqr_f=0.0,
                 store_coupling=1):
        pts = torch.as_tensor(points, dtype=torch.float64)
        if not pts.is_cuda:
            pts = pts.cuda()
        if pts.dim() == 1:
            pts = pts[:, None]
        self.n, self.d = pts.shape
        soa = pts.t().contiguous()  # [dim, n] layout expected by the C ABI
        opt = h2_options_default()
        opt.tau, opt.r1, opt.r2, opt.calib_seed = tau, r1, r2, seed
        opt.precision, opt.r_min = precision, r_min
        opt.store_coupling = store_coupling
        opt.datareduct = DATAREDUCT[datareduct]
        opt.srrqr_f = srrqr_f
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.stream = stream
        self.handle = h2_build(soa, kernel, prm, tol, leaf, opt, stream)

    def matvec(self, x) -> torch.Tensor:
        x = torch.as_tensor(x, dtype=self.dtype)
        if not x.is_cuda:
            x = x.cuda()
        squeeze = x.dim() == 1
        x2 = (x[None, :] if squeeze else x).contiguous()
        y = torch.empty_like(x2)
        h2_matvec(self.handle, x2, y, x2.shape[0], self.stream)
        return y[0] if squeeze else y

    def info(self) -> dict:
        return h2_query(self.handle)

    def export(self, what, node=-1):
        return h2_export(self.handle, what, node)

    def close(self):
        if getattr(self, "handle", None):
            h2_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
