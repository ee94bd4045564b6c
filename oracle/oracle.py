"""ctypes front end of the plain FP64 CPU oracle (``oracle/h2o.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark use it to check the GPU library.  Nothing in the
product package imports it.

Arrays cross the boundary as NumPy float64 / int32 buffers.  Points are
``[n, d]`` row-major in original order; right-hand sides and results are
``[nrhs, n]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h2o.c")
_LIB = os.path.join(_HERE, "libh2o.so")

KERNELS = {"coulomb": 0, "gaussian": 1, "exponential": 2, "matern32": 3, "bump": 4, "cosine": 5,
           "advection": 6}


def build_library(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.h2o_kappa.restype = C.c_double
        L.h2o_kappa.argtypes = [C.c_int, dp, dp, dp, C.c_int]
        L.h2o_kernel_matrix.argtypes = [C.c_int, dp, C.c_int, dp, C.c_int, dp, C.c_int, dp]
        L.h2o_datareduct.restype = C.c_int
        L.h2o_datareduct.argtypes = [C.c_int, dp, ip, C.c_int, C.c_int, ip]
        L.h2o_datareduct_seg.restype = C.c_int
        L.h2o_datareduct_seg.argtypes = [C.c_int, dp, ip, C.c_int, ip, C.c_int, C.c_int, ip]
        L.h2o_cpqr_id.restype = C.c_int
        L.h2o_cpqr_id.argtypes = [dp, C.c_int, C.c_int, C.c_double, ip, dp, dp]
        L.h2o_splitmix_u01.restype = C.c_double
        L.h2o_splitmix_u01.argtypes = [C.c_uint64, C.c_uint64]
        L.h2o_calibrate_one.restype = C.c_int
        L.h2o_calibrate_one.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                        C.c_uint64, C.c_int, dp]
        L.h2o_calib_shell.restype = C.c_int
        L.h2o_calib_shell.argtypes = [C.c_int, C.c_double, ip]
        L.h2o_calib_points.argtypes = [C.c_int, C.c_double, C.c_double, C.c_uint64, dp, dp]
        L.h2o_build.restype = C.c_void_p
        L.h2o_build.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, C.c_double, C.c_int, C.c_double,
                                C.c_int, C.c_int, C.c_uint64, C.c_int]
        L.h2o_build_ex.restype = C.c_void_p
        L.h2o_build_ex.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, C.c_double, C.c_int, C.c_double,
                                   C.c_int, C.c_int, C.c_uint64, C.c_int, C.c_int, C.c_double]
        L.h2o_srrqr_swaps.restype = C.c_int
        L.h2o_srrqr_swaps.argtypes = [C.c_int, C.c_int, C.c_double, ip, dp]
        L.h2o_datareduct_method.restype = C.c_int
        L.h2o_datareduct_method.argtypes = [C.c_int, C.c_int, dp, ip, C.c_int, ip, C.c_int, C.c_int, ip]
        L.h2o_build_tree_lists.restype = C.c_void_p
        L.h2o_build_tree_lists.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_double]
        L.h2o_free.argtypes = [C.c_void_p]
        L.h2o_info.restype = C.c_longlong
        L.h2o_info.argtypes = [C.c_void_p, C.c_int]
        L.h2o_export_int.restype = C.c_longlong
        L.h2o_export_int.argtypes = [C.c_void_p, C.c_int, ip]
        L.h2o_export_double.restype = C.c_longlong
        L.h2o_export_double.argtypes = [C.c_void_p, C.c_int, dp]
        L.h2o_node_list.restype = C.c_longlong
        L.h2o_node_list.argtypes = [C.c_void_p, C.c_int, C.c_int, ip]
        L.h2o_node_T.restype = C.c_longlong
        L.h2o_node_T.argtypes = [C.c_void_p, C.c_int, dp]
        L.h2o_node_T_side.restype = C.c_longlong
        L.h2o_node_T_side.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        L.h2o_matvec.argtypes = [C.c_void_p, dp, dp, C.c_int]
        L.h2o_matvec_rows.argtypes = [C.c_void_p, dp, C.c_int, ip, C.c_int, dp]
        L.h2o_dense_rows.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, ip, C.c_int, dp,
                                     C.c_int]
        L.h2o_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def kernel_id(k) -> int:
    return KERNELS[k] if isinstance(k, str) else int(k)


def kappa(kid, prm, x, y) -> float:
    x = _f64(x)
    y = _f64(y)
    p = _f64([prm])
    return lib().h2o_kappa(kernel_id(kid), _d(p), _d(x), _d(y), x.size)


def kernel_matrix(kid, prm, X, Y) -> np.ndarray:
    X = _f64(X)
    Y = _f64(Y)
    m, d = X.shape
    s = Y.shape[0]
    A = np.empty((m, s))
    p = _f64([prm])
    lib().h2o_kernel_matrix(kernel_id(kid), _d(p), d, _d(X), m, _d(Y), s, _d(A))
    return A


def datareduct(pts, idx, k) -> np.ndarray:
    pts = _f64(pts)
    idx = _i32(idx)
    out = np.empty(max(1, min(len(idx), k)), dtype=np.int32)
    cnt = lib().h2o_datareduct(pts.shape[1], _d(pts), _i(idx), len(idx), int(k), _i(out))
    return out[:cnt].copy()


def datareduct_seg(pts, idx, seg, k) -> np.ndarray:
    """DataReduct with one reference grid per segment [seg[s], seg[s+1])."""
    pts = _f64(pts)
    idx = _i32(idx)
    seg = _i32(seg)
    out = np.empty(max(1, min(len(idx), k * (len(seg) - 1))), dtype=np.int32)
    cnt = lib().h2o_datareduct_seg(pts.shape[1], _d(pts), _i(idx), len(idx), _i(seg), len(seg) - 1, int(k),
                                   _i(out))
    return out[:cnt].copy()


DATAREDUCT = {"volume": 0, "fps": 1, "surface": 2}


def datareduct_method(method, pts, idx, k, seg=None) -> np.ndarray:
    """DataReduct by method ("volume", "fps" or "surface"); seg as for
    datareduct_seg (None: one segment)."""
    pts = _f64(pts)
    idx = _i32(idx)
    seg = _i32([0, len(idx)] if seg is None else seg)
    out = np.empty(max(1, len(idx)), dtype=np.int32)
    cnt = lib().h2o_datareduct_method(DATAREDUCT[method], pts.shape[1], _d(pts), _i(idx), len(idx), _i(seg),
                                      len(seg) - 1, int(k), _i(out))
    return out[:cnt].copy()


def srrqr_swaps(k, piv, T, f):
    """Strong rank-revealing swaps on an ID (k, piv, T) of cpqr_id: returns
    (number of swaps, piv, T) with max |T| <= f."""
    piv = _i32(piv).copy()
    m = len(piv)
    T = _f64(T).reshape(k, m - k).copy()
    n = lib().h2o_srrqr_swaps(int(k), m, float(f), _i(piv), _d(T))
    return n, piv, T


def cpqr_id(A, tol):
    """Interpolative decomposition of the rows of A (m x s).

    Returns (k, piv, T, absRdiag) with A[piv[k:]] ~ T.T @ A[piv[:k]]."""
    A = _f64(A)
    m, s = A.shape
    piv = np.empty(max(m, 1), dtype=np.int32)
    kk = min(m, s)
    T = np.empty(max(1, kk * m))
    rd = np.empty(max(1, kk))
    k = lib().h2o_cpqr_id(_d(A), m, s, float(tol), _i(piv), _d(T), _d(rd))
    return k, piv[:m].copy(), T[: k * (m - k)].reshape(k, m - k).copy(), rd[:k].copy()


def splitmix_u01(seed, i) -> float:
    return lib().h2o_splitmix_u01(int(seed) & (2**64 - 1), int(i))


def calib_shell(d, tau) -> np.ndarray:
    """Cell offsets [nb, d] of the interaction list of the box [0, 1)^d in
    the uniform tree of unit boxes (the calibration's Z2 boxes)."""
    nb = lib().h2o_calib_shell(d, tau, None)
    out = np.empty((max(nb, 1), d), dtype=np.int32)
    lib().h2o_calib_shell(d, tau, _i(out))
    return out[:nb].copy()


def calib_points(d, side, tau, seed):
    """The calibration's point sets (Z1 [512, d], Z2 [4096, d])."""
    Z1 = np.empty((512, d))
    Z2 = np.empty((4096, d))
    lib().h2o_calib_points(d, side, tau, int(seed) & (2**64 - 1), _d(Z1), _d(Z2))
    return Z1, Z2


def calibrate_one(kid, prm, d, side, tau, eps, seed, r_cap):
    p = _f64([prm])
    e = np.zeros(1)
    r = lib().h2o_calibrate_one(kernel_id(kid), _d(p), d, side, tau, eps, seed, r_cap, _d(e))
    return r, float(e[0])


def dense_rows(pts, kid, prm, x, rows=None, nthreads=0) -> np.ndarray:
    """Rows of K x (K as defined in Section 2); x [nrhs, n] -> [nrhs, len(rows)]."""
    pts = _f64(pts)
    n, d = pts.shape
    x = _f64(np.atleast_2d(x))
    nrhs = x.shape[0]
    p = _f64([prm])
    if rows is None:
        out = np.empty((nrhs, n))
        lib().h2o_dense_rows(_d(pts), n, d, kernel_id(kid), _d(p), _d(x), nrhs, None, n, _d(out),
                             nthreads)
    else:
        rows = _i32(rows)
        out = np.empty((nrhs, len(rows)))
        lib().h2o_dense_rows(_d(pts), n, d, kernel_id(kid), _d(p), _d(x), nrhs, _i(rows), len(rows),
                             _d(out), nthreads)
    return out


def max_threads() -> int:
    return lib().h2o_max_threads()


_INT_FIELDS = {"perm": 0, "parent": 1, "first_child": 2, "nchild": 3, "start": 4, "count": 5,
               "depth": 6, "lvl_ptr": 7, "il_ptr": 8, "il_col": 9, "near_ptr": 10, "near_col": 11,
               "rank": 12, "mbar": 13, "rank_v": 14, "mbar_v": 15}
_DBL_FIELDS = {"center": 0, "side": 1, "points": 2, "calib_err": 3}
# *_v: the column basis V, W (the row basis U, R for a symmetric kernel)
_LISTS = {"xstar": 0, "ystar": 1, "xbar": 2, "piv": 3, "skel": 4, "xbar_v": 5, "piv_v": 6, "skel_v": 7}


class H2Oracle:
    """An oracle H^2 representation (Algorithm 2) built on the CPU."""

    def __init__(self, pts, kernel="coulomb", prm=1.0, tol=1e-6, leaf=64, tau=0.7, r1=0, r2=0,
                 seed=0x5EED, nthreads=0, structure_only=False, datareduct="volume", srrqr_f=0.0):
        pts = _f64(pts)
        self.n, self.d = pts.shape
        self.kid = kernel_id(kernel)
        self.prm = float(prm)
        p = _f64([prm])
        if structure_only:
            h = lib().h2o_build_tree_lists(_d(pts), self.n, self.d, leaf, tau)
        else:
            h = lib().h2o_build_ex(_d(pts), self.n, self.d, self.kid, _d(p), tol, leaf, tau, r1, r2,
                                   seed, nthreads, DATAREDUCT[datareduct], float(srrqr_f))
        if not h:
            raise ValueError("oracle rejected the input")
        self._h = C.c_void_p(h)

    def close(self):
        if self._h:
            lib().h2o_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        g = lambda w: int(lib().h2o_info(self._h, w))  # noqa: E731
        return {"nnode": g(0), "maxdepth": g(1), "r1": g(2), "r2": g(3), "nnz_il": g(4),
                "nnz_near": g(5), "n": g(6), "d": g(7)}

    def get(self, name):
        if name in _INT_FIELDS:
            w = _INT_FIELDS[name]
            cnt = lib().h2o_export_int(self._h, w, None)
            buf = np.empty(max(cnt, 1), dtype=np.int32)
            lib().h2o_export_int(self._h, w, _i(buf))
            return buf[:cnt].copy()
        w = _DBL_FIELDS[name]
        cnt = lib().h2o_export_double(self._h, w, None)
        buf = np.empty(max(cnt, 1))
        lib().h2o_export_double(self._h, w, _d(buf))
        out = buf[:cnt].copy()
        if name == "center":
            out = out.reshape(-1, self.d)
        elif name == "points":
            out = out.reshape(self.n, self.d)
        return out

    def node_list(self, name, i):
        w = _LISTS[name]
        cnt = lib().h2o_node_list(self._h, w, int(i), None)
        buf = np.empty(max(cnt, 1), dtype=np.int32)
        lib().h2o_node_list(self._h, w, int(i), _i(buf))
        return buf[:cnt].copy()

    def node_T(self, i, side=0):
        """T_i of the row basis (side 0) or of the column basis (side 1)."""
        cnt = lib().h2o_node_T_side(self._h, side, int(i), None)
        buf = np.empty(max(cnt, 1))
        lib().h2o_node_T_side(self._h, side, int(i), _d(buf))
        k = int(self.get("rank_v" if side else "rank")[i])
        m = int(self.get("mbar_v" if side else "mbar")[i])
        return buf[:cnt].reshape(k, m - k).copy()

    def matvec(self, x) -> np.ndarray:
        x = _f64(np.atleast_2d(x))
        y = np.empty_like(x)
        lib().h2o_matvec(self._h, _d(x), _d(y), x.shape[0])
        return y

    def matvec_rows(self, x, rows) -> np.ndarray:
        x = _f64(np.atleast_2d(x))
        rows = _i32(rows)
        out = np.empty((x.shape[0], len(rows)))
        lib().h2o_matvec_rows(self._h, _d(x), x.shape[0], _i(rows), len(rows), _d(out))
        return out
