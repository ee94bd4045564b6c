"""The C-ABI library builds, loads and exports every symbol of include/h2.h;
argument validation rejects bad input before any device work.  No GPU needed."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h2.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("h2_build", "h2_build_ex", "h2_matvec", "h2_matvec_ex", "h2_query", "h2_export",
                 "h2_destroy", "h2_last_error", "h2_options_default"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2206_01885_amd import h2
    L = h2.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(h2.SYMBOLS) == declared_functions()


def test_validation_without_device_work():
    from paper_2206_01885_amd import h2
    L = h2.lib()
    out = C.c_void_p(123)
    dummy = C.c_void_p(8)  # never dereferenced: validation fails first
    prm = (C.c_double * 1)(0.1)
    cases = [
        (dummy, 0, 3, 0, prm, 1e-6, 64),      # n < 1
        (dummy, 10, 4, 0, prm, 1e-6, 64),     # dim
        (dummy, 10, 3, 7, prm, 1e-6, 64),     # kernel id
        (dummy, 10, 3, 0, prm, 0.0, 64),      # tol
        (dummy, 10, 3, 0, prm, 1.5, 64),      # tol
        (dummy, 10, 3, 0, prm, 1e-6, 0),      # leaf
        (None, 10, 3, 0, prm, 1e-6, 64),      # NULL points
        (dummy, 10, 3, 1, None, 1e-6, 64),    # Gaussian without params
        (dummy, 10, 3, 5, prm, 1e-6, 64),     # cosine without r1, r2 (no calibration)
    ]
    for args in cases:
        st = L.h2_build(*args, C.byref(out))
        assert st == h2.H2_EINVAL, args
        assert out.value is None
        assert len(L.h2_last_error()) > 0
    bad = (C.c_double * 1)(float("nan"))
    assert L.h2_build(dummy, 10, 3, 1, bad, 1e-6, 64, C.byref(out)) == h2.H2_EINVAL
    opt = h2.h2_options_default()
    assert opt.tau == 0.7 and opt.precision == 64 and opt.r1 == 0
    opt.tau = 1.0
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    opt.tau, opt.precision = 0.7, 16
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    opt.precision, opt.r_min = 32, -1
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    opt = h2.h2_options_default()
    assert opt.store_coupling == 1
    opt.store_coupling = 2
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    opt.store_coupling, opt.precision = 0, 32  # the apply's own coupling evaluation is FP64 only
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EUNSUPPORTED
    assert L.h2_matvec(None, dummy, dummy, 1) == h2.H2_EINVAL
    assert L.h2_matvec_noalloc(None, dummy, dummy, 1, None) == h2.H2_EINVAL
    # r2 is the maximum size of Y_i^*: 1 cannot hold the two parts' grids
    opt = h2.h2_options_default()
    opt.r1, opt.r2 = 8, 1
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    opt.r1, opt.r2 = 8, 4097
    assert L.h2_build_ex(dummy, 10, 3, 0, prm, 1e-6, 64, C.byref(opt), None, C.byref(out)) == h2.H2_EINVAL
    assert L.h2_destroy(None) == h2.H2_OK


def test_batched_validation_without_device_work():
    from paper_2206_01885_amd import h2
    L = h2.lib()
    k = 3
    dummy = C.c_void_p(8)  # never dereferenced: validation fails first
    pts = (C.c_void_p * k)(8, 16, 24)
    ns = (C.c_int64 * k)(10, 20, 30)
    dims = (C.c_int * k)(3, 3, 3)
    kids = (C.c_int * k)(0, 1, 2)
    prms = (C.c_double * k)(1.0, 0.1, 0.2)
    tols = (C.c_double * k)(1e-6, 1e-6, 1e-6)
    leaf = (C.c_int * k)(64, 64, 64)
    out = (C.c_void_p * k)(1, 2, 3)
    assert L.h2_build_batched(0, pts, ns, dims, kids, prms, tols, leaf, None, None, out) == h2.H2_EINVAL
    tols[1] = 2.0  # problem 1 invalid
    assert L.h2_build_batched(k, pts, ns, dims, kids, prms, tols, leaf, None, None, out) == h2.H2_EINVAL
    assert all(v is None for v in out)
    assert b"problem 1" in L.h2_last_error()
    tols[1] = 1e-6
    prms[2] = float("nan")
    assert L.h2_build_batched(k, pts, ns, dims, kids, prms, tols, leaf, None, None, out) == h2.H2_EINVAL
    assert b"problem 2" in L.h2_last_error()
    assert L.h2_build_batched(k, None, ns, dims, kids, prms, tols, leaf, None, None, out) == h2.H2_EINVAL


def test_rebuild_validation_without_device_work():
    from paper_2206_01885_amd import h2
    L = h2.lib()
    dummy = C.c_void_p(8)  # never dereferenced: validation fails first
    prm = (C.c_double * 1)(0.1)
    assert L.h2_rebuild(None, 1, prm, 1e-6) == h2.H2_EINVAL
    assert L.h2_rebuild(dummy, 99, prm, 1e-6) == h2.H2_EINVAL
    assert L.h2_rebuild(dummy, 1, prm, 2.0) == h2.H2_EINVAL
    assert L.h2_rebuild(dummy, 1, None, 1e-6) == h2.H2_EINVAL
    prm[0] = float("nan")
    assert L.h2_rebuild(dummy, 1, prm, 1e-6) == h2.H2_EINVAL


def test_autotune_plan_and_tuning_file():
    """The autotuner's one-at-a-time plan covers every candidate value once
    around the base setting, and the committed tuning.json names only the
    parameters that csrc/tuning.h defines."""
    from paper_2206_01885_amd import autotune, build_lib
    base = autotune.current()
    plan = autotune.variants(base)
    assert plan[0] == ("base", base)
    names = [n for n, _ in plan[1:]]
    assert len(names) == len(set(names))
    for k, vals in autotune.CANDIDATES.items():
        assert base[k] in vals
        got = sorted(p[k] for n, p in plan[1:] if n.startswith(k + "="))
        assert got == sorted(v for v in vals if v != base[k])
        for n, p in plan[1:]:
            if not n.startswith(k + "="):
                assert p[k] == base[k]
    header = open(os.path.join(os.path.dirname(build_lib.HERE), "paper_2206_01885_amd", "csrc", "tuning.h")).read()
    for k, v in build_lib.tuning_params().items():
        assert f"#define {k} " in header, k
        assert v in autotune.CANDIDATES[k]
