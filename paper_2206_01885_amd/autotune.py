"""Measure the launch parameters of csrc/tuning.h and record the fastest.

One-at-a-time sweeps around the current setting (tuning.json, else the
defaults of csrc/tuning.h): every candidate value of one parameter, the
others held, on the n = 2^20 cube (Coulomb, leaf 128, tol 1e-6, r1 and r2
from the tolerance, 32 right-hand sides; a step is h2_build + h2_matvec +
h2_destroy, as in bench.py).  None of the parameters changes a result.

    python -m paper_2206_01885_amd.autotune build --dir D   # compile the variants (CPU)
    python -m paper_2206_01885_amd.autotune time --dir D --out R.json   # time them (GPU)
    python -m paper_2206_01885_amd.autotune apply R.json    # write tuning.json

then build the library again (it reads tuning.json).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2206_01885_amd import build_lib  # noqa: E402

# defaults of csrc/tuning.h and the values tried for each
DEFAULTS = {"H2_TUNE_SWEEP_T_P": 3, "H2_TUNE_BIN_MIN": 256, "H2_TUNE_SPLIT_MIN": 64, "H2_TUNE_DOWN_WIDE": 2048}
CANDIDATES = {
    "H2_TUNE_SWEEP_T_P": [2, 3, 4],
    "H2_TUNE_BIN_MIN": [0, 256, 1024],
    "H2_TUNE_SPLIT_MIN": [32, 64, 128],
    "H2_TUNE_DOWN_WIDE": [0, 2048, 8192],
}


def current() -> dict:
    p = dict(DEFAULTS)
    p.update(build_lib.tuning_params())
    return p


def variants(base: dict) -> list[tuple[str, dict]]:
    """(name, params): the base setting, then each parameter's other values."""
    out = [("base", dict(base))]
    for k, vals in CANDIDATES.items():
        for v in vals:
            if v != base[k]:
                p = dict(base)
                p[k] = v
                out.append((f"{k}={v}", p))
    return out


def cmd_build(a):
    os.makedirs(a.dir, exist_ok=True)
    plan = []
    for i, (name, p) in enumerate(variants(current())):
        lib = os.path.join(os.path.abspath(a.dir), f"libh2_tune{i}.so")
        print(f"[autotune] building {name}", flush=True)
        build_lib.build(out=lib, params=p)
        plan.append({"name": name, "params": p, "lib": os.path.basename(lib)})
    with open(os.path.join(a.dir, "plan.json"), "w") as f:
        json.dump(plan, f, indent=1)


def time_one(lib: str, steps: int) -> list[float]:
    """Step times (ms) of the workload with the library at `lib`."""
    import time
    import torch
    from paper_2206_01885_amd import h2, workloads
    h2.LIB_PATH = lib
    torch.cuda.set_device(0)
    c = workloads.config_cube_1m()
    P = torch.tensor(c["points"], device="cuda").t().contiguous()
    X = torch.tensor(c["x"][:32], device="cuda")
    Y = torch.empty_like(X)
    out = []
    for k in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hd = h2.h2_build(P, "coulomb", 1.0, 1e-6, 128)
        h2.h2_matvec(hd, X, Y, 32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h2.h2_destroy(hd)
        if k > 0:
            out.append(1e3 * (t1 - t0))
    return out


def cmd_time(a):
    plan = json.load(open(os.path.join(a.dir, "plan.json")))
    res = []
    for v in plan:
        lib = os.path.join(os.path.abspath(a.dir), v["lib"])
        # a process per variant: the library is loaded once per process
        r = subprocess.run([sys.executable, "-m", "paper_2206_01885_amd.autotune", "_one", lib, str(a.steps)],
                           capture_output=True, text=True, cwd=os.path.dirname(HERE), timeout=300)
        if r.returncode != 0:
            sys.stderr.write(r.stderr[-2000:])
            raise SystemExit(f"timing failed for {v['name']}")
        ms = json.loads(r.stdout.strip().splitlines()[-1])
        res.append({"name": v["name"], "params": v["params"], "ms": ms, "median_ms": statistics.median(ms)})
        print(f"[autotune] {v['name']}: {statistics.median(ms):.1f} ms", flush=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)


def cmd_apply(a):
    res = json.load(open(a.results))
    base = next(r for r in res if r["name"] == "base")
    best = dict(base["params"])
    for k in CANDIDATES:
        # the fastest value of k among the base run and k's own variants
        cand = [r for r in res if r["name"] == "base" or r["name"].startswith(k + "=")]
        best[k] = min(cand, key=lambda r: r["median_ms"])["params"][k]
    with open(build_lib.TUNING, "w") as f:
        json.dump({"params": best, "workload": "cube3d-coulomb-n1048576-leaf128-tol1e-6-nrhs32, build + apply",
                   "measurements": [{"name": r["name"], "median_ms": round(r["median_ms"], 2)} for r in res]},
                  f, indent=1)
    print(json.dumps(best))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--dir", required=True)
    t = sub.add_parser("time")
    t.add_argument("--dir", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--steps", type=int, default=3)
    p = sub.add_parser("apply")
    p.add_argument("results")
    o = sub.add_parser("_one")
    o.add_argument("lib")
    o.add_argument("steps", type=int)
    a = ap.parse_args()
    if a.cmd == "build":
        cmd_build(a)
    elif a.cmd == "time":
        cmd_time(a)
    elif a.cmd == "apply":
        cmd_apply(a)
    else:
        print(json.dumps(time_one(a.lib, a.steps)))


if __name__ == "__main__":
    main()
