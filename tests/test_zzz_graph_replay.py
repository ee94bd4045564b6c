"""h2_matvec_noalloc captured in a HIP graph and replayed, the use it exists
for (a caller that cannot allocate, e.g. a serving loop under graph
capture): the apply records kernel launches and its completion event (no
memory set or copy nodes), and each of several replays, with new inputs and eager work on the
device between them, equals the eager h2_matvec of the same input bit for
bit."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[graph] {msg}", flush=True)
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
def test_noalloc_apply_replays_in_graph(H, precision):
    import torch
    rng = np.random.default_rng(311 + precision)
    dt = torch.float64 if precision == 64 else torch.float32
    n, nrhs = 6000, 4
    _say(f"precision {precision} coulomb n{n} nrhs {nrhs}")
    g = H.H2Matrix(rng.random((n, 3)), "coulomb", 1.0, 1e-6, 40, precision=precision)
    s = torch.cuda.Stream()
    X = torch.tensor(rng.standard_normal((nrhs, n)), device="cuda", dtype=dt)
    Y = torch.empty_like(X)
    # a first call on the capture stream sets up the scratch array's address
    H.h2_matvec_noalloc(g.handle, X, Y, nrhs, s)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        H.h2_matvec_noalloc(g.handle, X, Y, nrhs, s)
    torch.cuda.synchronize()
    for k in range(3):
        xin = torch.tensor(rng.standard_normal((nrhs, n)), device="cuda", dtype=dt)
        X.copy_(xin)
        Y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        y_ref = torch.empty_like(xin)
        H.h2_matvec(g.handle, xin, y_ref, nrhs)
        torch.cuda.synchronize()
        _say(f"replay {k}: max |diff| {float((Y - y_ref).abs().max()):.1e}")
        assert torch.equal(Y, y_ref), k
    # launch cost: replays against eager applies of the same (small) problem
    reps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        H.h2_matvec_noalloc(g.handle, X, Y, nrhs, s)
    s.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _say(f"eager {1e3 * (t1 - t0) / reps:.3f} ms, replay {1e3 * (t2 - t1) / reps:.3f} ms per apply")
    del graph
    g.close()
