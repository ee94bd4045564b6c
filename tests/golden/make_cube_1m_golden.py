"""Writes tests/golden/cube_1m_oracle.txt: the CPU oracle's H^2 construction
of the headline workload (n = 2^20 points uniform in [0,1]^3, seed 1004,
Coulomb, leaf 128, tol 1e-6, r1 and r2 from the tolerance) reduced to what a
GPU test can compare against without rebuilding it: r1, r2, the node count,
per tree depth the SHA-256 of every node's X_i^*, Y_i^*, rank, row count,
pivots and skeleton (int32 little-endian, nodes in id order, each list
prefixed by its length), and the oracle's H^2 product and the dense product
K x on the workload's 4096 sampled rows for the first two right-hand sides.

Calls only the oracle (oracle/) and the seeded input generator; run from the
repository root:  python tests/golden/make_cube_1m_golden.py
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402
from paper_2206_01885_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_1m_oracle.txt")
LISTS = ("xstar", "ystar", "piv", "skel")


def level_hashes(get_list, rank, mbar, depth):
    """Per depth L >= 1: SHA-256 over the nodes of depth L (id order) of
    [rank, mbar, then each list of LISTS prefixed by its length]."""
    out = {}
    for L in range(1, int(depth.max()) + 1):
        hs = hashlib.sha256()
        for i in np.flatnonzero(depth == L):
            hs.update(np.array([rank[i], mbar[i]], dtype="<i4").tobytes())
            for name in LISTS:
                v = np.asarray(get_list(name, int(i)), dtype="<i4")
                hs.update(np.array([len(v)], dtype="<i4").tobytes())
                hs.update(v.tobytes())
        out[L] = hs.hexdigest()
    return out


def main():
    c = W.config_cube_1m()
    t0 = time.time()
    h = O.H2Oracle(c["points"], c["kernel"], c["prm"], tol=c["tol"], leaf=c["leaf"])
    t1 = time.time()
    info = h.info()
    print(f"oracle build {t1 - t0:.1f} s, {info}", flush=True)
    depth, rank, mbar = h.get("depth"), h.get("rank"), h.get("mbar")
    hashes = level_hashes(h.node_list, rank, mbar, depth)
    rows = np.asarray(c["rows"], dtype=np.int64)
    x = c["x"][:2]
    y = h.matvec_rows(x, rows)
    t2 = time.time()
    print(f"oracle product rows {t2 - t1:.1f} s", flush=True)
    ref = O.dense_rows(c["points"], c["kernel"], c["prm"], x, rows=rows)
    print(f"dense rows {time.time() - t2:.1f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle H^2 construction of n = 2^20 uniform points in [0,1]^3 (seed 1004),\n")
        f.write("# Coulomb, leaf 128, tol 1e-6 (Section 6's cube workload); written by\n")
        f.write("# tests/golden/make_cube_1m_golden.py from the oracle alone.\n")
        f.write(f"r1 {info['r1']}\nr2 {info['r2']}\nnnode {info['nnode']}\nmaxdepth {info['maxdepth']}\n")
        for L, v in hashes.items():
            f.write(f"level {L} {v}\n")
        f.write(f"rows {len(rows)} rhs 2\n")
        for t in range(len(rows)):
            f.write(f"{rows[t]} {y[0, t]:.17e} {y[1, t]:.17e} {ref[0, t]:.17e} {ref[1, t]:.17e}\n")
    e = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"wrote {OUT}; oracle vs dense on the rows {e:.3e}", flush=True)


if __name__ == "__main__":
    main()
