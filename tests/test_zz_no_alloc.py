"""h2_matvec_noalloc, the apply that allocates nothing (its work vectors live
in the library's per-device scratch array), against h2_matvec_ex through the
C ABI: bit for bit on two calls in a row, the second with a smaller problem
and fewer right-hand sides (the array keeps the first call's contents), in
FP64 and in the precision mode; a problem too large for the array is
rejected with H2_EUNSUPPORTED."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_01885_amd import h2
    h2.lib()
    return h2


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_equals_matvec(H, precision):
    import torch
    rng = np.random.default_rng(77 + precision)
    dt = torch.float64 if precision == 64 else torch.float32
    cases = [(6000, 3, "coulomb", 1.0, 40, 9), (2500, 2, "gaussian", 0.1, 30, 3)]
    for n, d, kern, prm, leaf, nrhs in cases:
        _say(f"precision {precision} {kern} d{d} n{n} nrhs {nrhs}")
        P = rng.random((n, d))
        g = H.H2Matrix(P, kern, prm, 1e-6, leaf, precision=precision)
        x = torch.tensor(rng.standard_normal((nrhs, n)), device="cuda", dtype=dt)
        y_ref = torch.empty_like(x)
        y_na = torch.full_like(x, float("nan"))
        H.h2_matvec(g.handle, x, y_ref, nrhs, g.stream)
        H.h2_matvec_noalloc(g.handle, x, y_na, nrhs, g.stream)
        torch.cuda.synchronize()
        assert torch.equal(y_na, y_ref), (kern, n)
        g.close()


def test_noalloc_rejects_too_large(H):
    import torch
    n = 1 << 16
    P = np.random.default_rng(5).random((n, 3))
    g = H.H2Matrix(P, "coulomb", 1.0, 1e-6, 64, r1=27, r2=54)
    nrhs = 256  # (2 n + ranks) * 256 doubles > 256 MiB
    x = torch.zeros((nrhs, n), device="cuda", dtype=torch.float64)
    y = torch.empty_like(x)
    with pytest.raises(H.H2Error) as e:
        H.h2_matvec_noalloc(g.handle, x, y, nrhs, g.stream)
    assert e.value.status == H.H2_EUNSUPPORTED
    # the handle still applies with the allocating entry point
    H.h2_matvec(g.handle, x[:1], y[:1], 1, g.stream)
    torch.cuda.synchronize()
    g.close()
