"""Benchmark of the data-driven H^2 hot path on one MI355X.

Workload: n = 2^20 points uniform in [0,1]^3 (the paper's "cube" dataset),
Coulomb kernel, leaf size 128, tolerance 1e-6, 32 right-hand sides N(0,1).
One step = one pass of the whole hot path: h2_build (tree, lists, r1/r2,
HiDR, batched kernel-block evaluation + CPQR interpolative decomposition,
coupling and nearfield blocks) followed by one h2_matvec with 32 RHS, then
h2_destroy.  Inputs are resident in HBM before the timed region starts.

Printed: one JSON line with the whole-step throughput (Mpts/s), the build and
apply figures, the roofline of the dominant kernel of the step (the top-down
DataReduct of HiDR, k_datareduct_down: its candidate coordinates against the
HBM bandwidth; HIP events on the build's stream), the same for the wide-node
interpolative decompositions (FP64 ALU bound) and the apply's coupling sweep
(k_sweep, HBM bound; HIP events on the apply's stream), the sampled accuracy
against the dense K x, and the CPU oracle timed on a bounded sample of the
same workload.  --copy-calibration instead runs a plain device copy of 1 GiB
(the reference for scaling the HBM counters of a profile).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 78.6


def recorded_traffic(profile, source):
    """HBM bytes per launch recorded in a counter summary under profiles/ (the
    FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy), or None when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        rec = {ln.split(":")[0].strip(): ln.split(":")[1].split()[0] for ln in text.splitlines()
               if ln.startswith(("traffic_bytes_per_launch:", "source_sha256_prefix:"))}
        digest = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
        if rec.get("source_sha256_prefix") != digest:
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, IndexError, ValueError):
        return None


def id_roofline(flops, ms, kernel):
    """Algorithmic FP64 flops of the pivoted-QR IDs over the event-timed
    duration of their launches."""
    achieved = flops / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": None,
            "flops_per_step": flops, "ms_per_step": ms}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--r", type=int, default=0, help="r1 = r, r2 = 2 r override (0: chosen from the tolerance)")
    ap.add_argument("--r-min", type=int, default=0, help="floor on the r chosen from the tolerance (0: none)")
    ap.add_argument("--no-f32", action="store_true", help="skip the precision-mode (FP32 apply) measurement")
    ap.add_argument("--rows", type=int, default=4096, help="sampled rows for the accuracy checks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=1 << 17, help="points of the oracle's bounded sample")
    ap.add_argument("--workload", choices=["cube1m", "batched", "serving", "sphere3", "variants", "large"],
                    default="cube1m",
                    help="cube1m: the headline n=2^20 Coulomb step; batched: 256 independent problems; "
                         "serving: Poisson request stream")
    ap.add_argument("--nreq", type=int, default=64, help="requests of the serving workload")
    ap.add_argument("--load", type=float, default=0.5, help="serving: offered load as a fraction of saturation")
    ap.add_argument("--nprob", type=int, default=256, help="problems of the batched workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device (5 times), the reference for HBM counters")
    return ap.parse_args()


def bench_batched(args):
    """256 independent problems (n log-uniform in [2048, 32768], cube or
    sphere, Coulomb / exponential 0.2 / Matern-3/2 0.2, leaf 64, tol 1e-6,
    FP64): h2_build_batched against a loop of h2_build over the same
    problems; inputs resident in HBM; build throughput = sum of n / wall."""
    import torch
    from paper_2206_01885_amd import h2, workloads
    torch.cuda.set_device(0)
    probs = workloads.config_batched(nprob=args.nprob)
    soa = [torch.tensor(p["points"].T.copy(), device="cuda") for p in probs]
    ks = [p["kernel"] for p in probs]
    prms = [p["prm"] for p in probs]
    tols = [p["tol"] for p in probs]
    leaves = [p["leaf"] for p in probs]
    ntot = sum(int(p["points"].shape[0]) for p in probs)
    opt = h2.h2_options_default()
    opt.profile = 1
    print(f"[bench] batched: {len(probs)} problems, {ntot} points", file=sys.stderr, flush=True)
    # warm-up: a few problems each way
    hs = h2.h2_build_batched(soa[:4], ks[:4], prms[:4], tols[:4], leaves[:4], opt)
    for hd in hs:
        h2.h2_destroy(hd)
    hd = h2.h2_build(soa[0], ks[0], prms[0], tols[0], leaves[0], opt)
    h2.h2_destroy(hd)
    torch.cuda.synchronize()
    loop_t, bat_t = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(len(probs)):
            hd = h2.h2_build(soa[i], ks[i], prms[i], tols[i], leaves[i], opt)
            h2.h2_destroy(hd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hs = h2.h2_build_batched(soa, ks, prms, tols, leaves, opt)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        info = [h2.h2_query(hd) for hd in hs]
        for hd in hs:
            h2.h2_destroy(hd)
        loop_t.append(t1 - t0)
        bat_t.append(t2 - t1)
        print(f"[bench] step {k}: loop {t1 - t0:.3f} s batched {t2 - t1:.3f} s", file=sys.stderr, flush=True)
    tb, tl = float(np.mean(bat_t)), float(np.mean(loop_t))
    # per-problem steps run concurrently on worker streams (their sum exceeds
    # the wall time); calibration and nested bases are shared by all problems
    phases = {f: float(np.sum([i[f] for i in info])) for f in ("t_tree", "t_lists", "t_hidr", "t_blocks")}
    phases["t_calib_shared"] = info[0]["t_calib"]
    phases["t_basis_shared"] = info[0]["t_basis"]
    # the ID launches are shared by all problems: their time once, their flops summed
    roof = id_roofline(float(np.sum([i["id_flops"] for i in info])), info[0]["id_ms"],
                       "k_batched_id (all classes, the batched interpolative decompositions)")
    out = {
        "metric": "batched H2 build Mpts/s (256 independent problems in one h2_build_batched call)",
        "value": ntot / tb / 1e6, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * tb, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched-{len(probs)}-problems-n2048-32768-leaf64-tol1e-6", "points": ntot},
        "loop_ms_per_step": 1e3 * tl, "loop_mpts_s": ntot / tl / 1e6, "speedup_vs_loop": tl / tb,
        "phases_s_sum_over_problems": phases,
        "roofline": roof,
    }
    print(json.dumps(out), flush=True)


def dense_rows_gpu(P, X, rows, chunk=64, kernel="coulomb", prm=1.0):
    """Rows of K x on the GPU in FP64 (torch ops, exact distances): Coulomb
    with kappa(x,x)=0, the Gaussian exp(-r^2/h^2), the Table-1 bump
    exp(-1/(1 - a r^2)) or the Table-1 cosine cos(a x.y)."""
    import torch
    out = []
    for a in range(0, len(rows), chunk):
        r = rows[a:a + chunk]
        Pr = P[r]
        D2 = ((Pr[:, None, :] - P[None, :, :]) ** 2).sum(-1)
        if kernel == "coulomb":
            D = D2.sqrt()
            K = torch.where(D > 0, 1.0 / D, torch.zeros_like(D))
        elif kernel == "gaussian":
            K = torch.exp(-D2 / (prm * prm))
        elif kernel == "exponential":
            K = torch.exp(-D2.sqrt() / prm)
        elif kernel == "bump":
            K = torch.exp(-1.0 / (1.0 - prm * D2))
        elif kernel == "cosine":
            K = torch.cos(prm * (Pr @ P.T))
        elif kernel == "advection":
            D = D2.sqrt()
            d0 = Pr[:, None, 0] - P[None, :, 0]
            K = torch.where(D > 0, torch.exp(prm * (d0 - D)) / D, torch.zeros_like(D))
        else:
            raise ValueError(kernel)
        out.append(K @ X.T)  # [chunk, nrhs]
    return torch.cat(out, 0).T  # [nrhs, rows]


def bench_sphere3(args):
    """The paper's kernel-scaling workload: n points on three unit spheres
    (centres on a triangle of side 1), the Table-1 kernels kappa_4 (bump,
    a = 0.1), kappa_2 (Gaussian, h = 1) and kappa_3 (cosine, a = 1; given
    r1 = 128, r2 = 256, as it has no calibration), leaf 128, tol 1e-6, 32 RHS.  A
    step is one build + one apply per kernel; value = points per second over
    the three kernels' steps."""
    import torch
    from paper_2206_01885_amd import h2, workloads
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, nrhs = args.n, args.nrhs
    rng = np.random.default_rng(1006)
    P = torch.tensor(workloads.three_spheres(rng, n), device=dev)
    Psoa = P.t().contiguous()
    X = torch.tensor(rng.standard_normal((nrhs, n)), device=dev)
    Y = torch.empty_like(X)
    rows = torch.tensor(np.sort(rng.choice(n, args.rows, replace=False)), device=dev)
    opt = h2.h2_options_default()
    opt.r_min = args.r_min
    res = {}
    total = 0.0
    kernels = (("bump", 0.1, 0), ("gaussian", 1.0, 0), ("cosine", 1.0, 128))
    for kern, prm, r in kernels:
        opt.r1, opt.r2 = r, 2 * r
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hd = h2.h2_build(Psoa, kern, prm, 1e-6, 128, opt)
            tb = time.perf_counter()
            h2.h2_matvec(hd, X, Y, nrhs)
            torch.cuda.synchronize()
            te = time.perf_counter()
            if k >= args.warmup:
                times.append((tb - t0, te - tb))
            info = h2.h2_query(hd)
            h2.h2_destroy(hd)
            print(f"[bench] sphere3 {kern} step {k}: build {tb - t0:.3f} s matvec {te - tb:.4f} s",
                  file=sys.stderr, flush=True)
        ref = dense_rows_gpu(P, X, rows, kernel=kern, prm=prm)
        e = ((Y[:, rows] - ref).norm(dim=1) / ref.norm(dim=1)).max().item()
        t = np.array(times)
        total += float(t.sum(axis=1).mean())
        res[kern] = {"prm": prm, "build_s": float(t[:, 0].mean()), "matvec_s": float(t[:, 1].mean()),
                     "r1": info["r1"], "r2": info["r2"], "max_rank": info["max_rank"], "bytes_B": info["bytes_B"],
                     "e_dense_sampled_rows_max_rhs": e}
    out = {
        "metric": "3-sphere H2 build + matvec Mpts/s (Table-1 kernels kappa_4, kappa_2, kappa_3)",
        "value": len(kernels) * n / total / 1e6, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / len(kernels), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sphere3-n{n}-bump0.1-gaussian1-cosine1-leaf128-tol1e-6-nrhs{nrhs}", "n": n,
                   "nrhs": nrhs},
        "kernels": res,
    }
    print(json.dumps(out), flush=True)


def bench_variants(args):
    """The options of the build on the headline cube (n = 2^20, leaf 128,
    tol 1e-6, r1 and r2 from the tolerance, 32 RHS): the volume DataReduct
    (reference), farthest point sampling, the surface method, the strong
    rank-revealing swaps (f = 1.05) and the non-symmetric advection kernel
    (a = 2, r1 = 343, r2 = 686).
    Per option one untimed build, then build + one apply timed; accuracy on
    sampled rows against the dense product."""
    import torch
    from paper_2206_01885_amd import h2
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, nrhs = args.n, args.nrhs
    rng = np.random.default_rng(1004)
    P = torch.tensor(rng.random((n, 3)), device=dev)
    Psoa = P.t().contiguous()
    X = torch.tensor(rng.standard_normal((nrhs, n)), device=dev)
    Y = torch.empty_like(X)
    rows = torch.tensor(np.sort(rng.choice(n, args.rows, replace=False)), device=dev)
    cases = [("volume", "coulomb", 1.0, "volume", 0.0, 0), ("fps", "coulomb", 1.0, "fps", 0.0, 0),
             ("surface", "coulomb", 1.0, "surface", 0.0, 0), ("srrqr1.05", "coulomb", 1.0, "volume", 1.05, 0),
             ("advection2", "advection", 2.0, "volume", 0.0, 343)]
    res = {}
    for name, kern, prm, dr, f, r in cases:
        opt = h2.h2_options_default()
        opt.r_min = args.r_min
        opt.r1, opt.r2 = r, 2 * r
        opt.datareduct = h2.DATAREDUCT[dr]
        opt.srrqr_f = f
        for k in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hd = h2.h2_build(Psoa, kern, prm, 1e-6, 128, opt)
            tb = time.perf_counter()
            h2.h2_matvec(hd, X, Y, nrhs)
            torch.cuda.synchronize()
            te = time.perf_counter()
            info = h2.h2_query(hd)
            h2.h2_destroy(hd)
            print(f"[bench] variants {name} build {tb - t0:.3f} s matvec {te - tb:.4f} s", file=sys.stderr,
                  flush=True)
        ref = dense_rows_gpu(P, X, rows, kernel=kern, prm=prm)
        e = ((Y[:, rows] - ref).norm(dim=1) / ref.norm(dim=1)).max().item()
        res[name] = {"build_s": tb - t0, "matvec_s": te - tb, "t_hidr": info["t_hidr"], "t_basis": info["t_basis"],
                     "t_blocks": info["t_blocks"], "r1": info["r1"], "max_rank": info["max_rank"],
                     "max_rank_v": info["max_rank_v"], "e_dense_sampled_rows_max_rhs": e}
    print(json.dumps({"workload": f"cube3d-n{n}-options-nrhs{nrhs}", "cases": res}), flush=True)


def bench_large(args):
    """Beyond the stored-block limit: n = 2^22 uniform points in [0,1]^3
    (--n overrides), Coulomb, leaf 128, tol 1e-6, r1 and r2 from the
    tolerance, 32 RHS, with
    the coupling blocks evaluated in the apply (store_coupling = 0; stored,
    they would take ~760 GB).  One untimed build + apply, then one timed;
    accuracy on sampled rows against the dense product."""
    import torch
    from paper_2206_01885_amd import h2
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n = args.n if args.n != 1 << 20 else 1 << 22
    nrhs = args.nrhs
    rng = np.random.default_rng(1004)
    P = torch.tensor(rng.random((n, 3)), device=dev)
    Psoa = P.t().contiguous()
    X = torch.tensor(rng.standard_normal((nrhs, n)), device=dev)
    Y = torch.empty_like(X)
    rows = torch.tensor(np.sort(rng.choice(n, args.rows, replace=False)), device=dev)
    opt = h2.h2_options_default()
    opt.r_min = args.r_min
    opt.store_coupling = 0
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hd = h2.h2_build(Psoa, "coulomb", 1.0, 1e-6, 128, opt)
        tb = time.perf_counter()
        h2.h2_matvec(hd, X, Y, nrhs)
        torch.cuda.synchronize()
        te = time.perf_counter()
        info = h2.h2_query(hd)
        h2.h2_destroy(hd)
        print(f"[bench] large n={n} step {k}: build {tb - t0:.3f} s matvec {te - tb:.4f} s", file=sys.stderr,
              flush=True)
    ref = dense_rows_gpu(P, X, rows)
    e = ((Y[:, rows] - ref).norm(dim=1) / ref.norm(dim=1)).max().item()
    print(json.dumps({
        "metric": "H2 build + matvec Mpts/s, coupling blocks evaluated in the apply",
        "value": n / (te - t0) / 1e6, "unit": "Mpts/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * (te - t0), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cube3d-coulomb-n{n}-leaf128-tol1e-6-nrhs{nrhs}-store_coupling0", "n": n},
        "build_s": tb - t0, "matvec_s": te - tb, "nnode": info["nnode"], "r1": info["r1"],
        "max_rank": info["max_rank"], "bytes_D": info["bytes_D"], "e_dense_sampled_rows_max_rhs": e}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, nrhs):
    """The oracle as it stands on a bounded sample: n points of the same
    distribution, same kernel/leaf/tolerance, r1 and r2 from the tolerance
    (the Coulomb kernel is scale invariant, so the oracle's calibration picks
    the r of the full-size GPU line); build + one apply with nrhs RHS."""
    from oracle import oracle as O
    rng = np.random.default_rng(4004)
    P = rng.random((n, 3))
    X = rng.standard_normal((nrhs, n))
    t0 = time.perf_counter()
    h = O.H2Oracle(P, "coulomb", 1.0, tol=1e-6, leaf=128)
    t1 = time.perf_counter()
    h.matvec(X)
    t2 = time.perf_counter()
    cores = O.max_threads()
    oi = h.info()
    return {"value": n / (t2 - t0) / 1e6, "unit": "Mpts/s", "cores": cores, "kind": "oracle",
            "sample": f"n={n} uniform [0,1]^3 Coulomb leaf 128 tol 1e-6, r1={oi['r1']} r2={oi['r2']}, "
                      f"{cores} OpenMP threads on {cpu_model()}: build {t1 - t0:.2f} s + "
                      f"matvec {nrhs} RHS {t2 - t1:.2f} s",
            "build_s": t1 - t0, "matvec_s": t2 - t1, "r1": oi["r1"], "r2": oi["r2"], "cpu_model": cpu_model()}


def cube_1m_golden():
    """The oracle's H^2 product and dense product of the headline workload on
    its 4096 sampled rows (right-hand sides 0 and 1), as written by
    tests/golden/make_cube_1m_golden.py; None if the file is absent."""
    path = os.path.join(ROOT, "tests", "golden", "cube_1m_oracle.txt")
    if not os.path.exists(path):
        return None
    rows, vals = [], []
    for line in open(path):
        t = line.split()
        if not t or t[0].startswith("#") or t[0] in ("r1", "r2", "nnode", "maxdepth", "level", "rows"):
            continue
        rows.append(int(t[0]))
        vals.append([float(v) for v in t[1:]])
    v = np.array(vals)
    return {"rows": np.array(rows), "y_h2": v[:, :2].T.copy(), "y_dense": v[:, 2:].T.copy()}


def bench_serving(args):
    """Request stream (n log-uniform in [1024, 2^20], 2-D or 3-D, cube or
    Gaussian mixture, Coulomb / Gaussian 0.1 / exponential 0.2, tol 1e-6,
    8 right-hand sides, FP32 precision mode), served by serving.Server:
    (1) the plain path -- one FP64 h2_build + h2_matvec per request, one after
    the other; (2) saturation -- all requests at t = 0; (3) Poisson arrivals at
    `load` x the saturation rate.  Reports p50/p99 latency and solves/s."""
    import torch
    from paper_2206_01885_amd import h2, serving, workloads
    torch.cuda.set_device(0)
    cfg = workloads.serving_requests(nreq=args.nreq)
    ntot = sum(int(c["points"].shape[0]) for c in cfg)
    print(f"[bench] serving: {len(cfg)} requests, {ntot} points", file=sys.stderr, flush=True)

    def fresh():
        return [serving.Request(i, c["points"], c["kernel"], c["prm"], c["tol"], c["leaf"], c["x"])
                for i, c in enumerate(cfg)]

    # warm-up
    serving.Server(max_batch=4, keep_outputs=False).run(fresh()[:4])
    # (1) plain FP64 path, sequential
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat_plain = []
    for c in cfg:
        ts = time.perf_counter()
        P = torch.tensor(np.ascontiguousarray(c["points"].T), device="cuda")
        X = torch.tensor(c["x"], device="cuda")
        hd = h2.h2_build(P, c["kernel"], c["prm"], c["tol"], c["leaf"])
        Y = torch.empty_like(X)
        h2.h2_matvec(hd, X, Y, X.shape[0])
        torch.cuda.synchronize()
        h2.h2_destroy(hd)
        lat_plain.append(time.perf_counter() - ts)
    wall_plain = time.perf_counter() - t0
    print(f"[bench] plain FP64 loop {wall_plain:.2f} s", file=sys.stderr, flush=True)
    # (2) saturation
    reqs = fresh()
    t0 = time.perf_counter()
    serving.Server(keep_outputs=False).run(reqs)
    wall_sat = time.perf_counter() - t0
    sat = serving.summarize(reqs, wall_sat)
    print(f"[bench] saturation {wall_sat:.2f} s", file=sys.stderr, flush=True)
    # (3) Poisson arrivals at load x saturation
    rate = args.load * sat["requests_per_s"]
    rng = np.random.default_rng(1005)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(cfg))).tolist()
    reqs = fresh()
    t0 = time.perf_counter()
    serving.Server(keep_outputs=False).run(reqs, arrivals)
    wall_p = time.perf_counter() - t0
    poi = serving.summarize(reqs, wall_p)
    print(f"[bench] poisson {wall_p:.2f} s", file=sys.stderr, flush=True)
    # accuracy of every request: an untimed pass that keeps the outputs, 256
    # sampled rows per request against dense rows (torch FP64 on the GPU)
    reqs = fresh()
    serving.Server(keep_outputs=True).run(reqs)
    rng_rows = np.random.default_rng(1006)
    errs = []
    for c, r in zip(cfg, reqs):
        n = int(c["points"].shape[0])
        rows = np.sort(rng_rows.choice(n, min(256, n), replace=False))
        P = torch.tensor(c["points"], device="cuda")
        X = torch.tensor(c["x"], device="cuda")
        ref = dense_rows_gpu(P, X, torch.tensor(rows, device="cuda"), kernel=c["kernel"], prm=c["prm"])
        got = torch.tensor(np.asarray(r.y)[:, rows], device="cuda", dtype=torch.float64)
        errs.append(((got - ref).norm(dim=1) / ref.norm(dim=1)).max().item())
        del P, X, ref, got
    print(f"[bench] serving accuracy: max {max(errs):.2e} over {len(errs)} requests", file=sys.stderr, flush=True)
    nrhs = sum(int(c["x"].shape[0]) for c in cfg)
    out = {
        "metric": "H2 serving: p50/p99 request latency and solves/s (build + 8-RHS apply per request)",
        "value": sat["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * wall_sat, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving-{len(cfg)}-requests-n1024-1048576-d2or3-tol1e-6-8rhs", "points": ntot},
        "plain_fp64_loop": {"wall_s": wall_plain, "solves_per_s": nrhs / wall_plain,
                            "p50_s": float(np.percentile(lat_plain, 50)),
                            "p99_s": float(np.percentile(lat_plain, 99))},
        "saturation": sat,
        "poisson": dict(poi, offered_load=args.load, offered_requests_per_s=rate),
        "accuracy": {"rows_per_request": 256, "dense_reference": "torch FP64 on the GPU, all 8 RHS",
                     "e_dense_max": max(errs), "e_dense_p50": float(np.percentile(errs, 50)),
                     "e_dense_per_request": errs, "tol": 1e-6},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library runs on one GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * src.numel() * 8, "read_bytes": src.numel() * 8,
                          "write_bytes": src.numel() * 8, "launches": 5}), flush=True)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "serving":
        bench_serving(args)
        return
    if args.workload == "sphere3":
        bench_sphere3(args)
        return
    if args.workload == "variants":
        bench_variants(args)
        return
    if args.workload == "large":
        bench_large(args)
        return
    import torch
    from paper_2206_01885_amd import h2

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    from paper_2206_01885_amd import workloads
    n, nrhs = args.n, args.nrhs
    cfg = workloads.config_cube_1m(n=n, nrhs=max(nrhs, 2), nrows=min(args.rows, n))
    rows = np.asarray(cfg["rows"])
    gold = cube_1m_golden() if (n == 1 << 20 and nrhs >= 2 and args.rows == 4096) else None
    if gold is not None and not np.array_equal(gold["rows"], rows):
        gold = None
    P = torch.tensor(cfg["points"], device=dev)
    Psoa = P.t().contiguous()
    X = torch.tensor(cfg["x"][:nrhs], device=dev)
    Y = torch.empty_like(X)
    del cfg
    opt = h2.h2_options_default()
    opt.r1, opt.r2 = args.r, 2 * args.r
    opt.r_min = args.r_min
    opt.profile = 1
    print(f"[bench] inputs resident: n={n} nrhs={nrhs}", file=sys.stderr, flush=True)

    def step():
        hd = h2.h2_build(Psoa, "coulomb", 1.0, 1e-6, 128, opt)
        tb = time.perf_counter()
        h2.h2_matvec(hd, X, Y, nrhs)
        return hd, tb

    for w in range(args.warmup):
        hd, _ = step()
        torch.cuda.synchronize()
        h2.h2_destroy(hd)
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)

    builds, mvs, coup, idw = [], [], [], []
    keep = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        hd, tb = step()
        torch.cuda.synchronize()
        te = time.perf_counter()
        info = h2.h2_query(hd)
        builds.append(tb - ts)
        mvs.append(te - tb)
        coup.append(info["mv_coupling"] / 1e3)
        idw.append((info["id_wide_flops"], info["id_wide_ms"], info["id_flops"], info["id_ms"],
                    info["hidr_down_bytes"], info["hidr_down_ms"], info["hidr_down_evals"]))
        if k == args.steps - 1:
            keep = (hd, info)
        else:
            h2.h2_destroy(hd)
        print(f"[bench] step {k}: build {tb - ts:.3f} s matvec {te - tb:.4f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    hd, info = keep
    ms_per_step = 1e3 * t_total / args.steps

    # accuracy on sampled rows (outside the timed region)
    ridx = torch.tensor(rows, device=dev)
    ref = dense_rows_gpu(P, X, ridx)
    got = Y[:, ridx]
    e_per_rhs = (got - ref).norm(dim=1) / ref.norm(dim=1)
    e_rows = e_per_rhs.max().item()
    e_rows_mean = e_per_rhs.mean().item()

    def vs_golden(Yrows):
        """Per right-hand side 0, 1: error against the oracle's FP64 H^2
        product and against the oracle's dense product on the 4096 rows."""
        if gold is None:
            return None
        y = Yrows[:2].double().cpu().numpy()
        return {"e_vs_fp64_oracle_h2": [float(np.linalg.norm(y[r] - gold["y_h2"][r]) /
                                              np.linalg.norm(gold["y_h2"][r])) for r in range(2)],
                "e_vs_oracle_dense": [float(np.linalg.norm(y[r] - gold["y_dense"][r]) /
                                            np.linalg.norm(gold["y_dense"][r])) for r in range(2)],
                "rows": int(len(gold["rows"])), "rhs": [0, 1]}

    acc_oracle = vs_golden(got)

    # coupling-sweep roofline: bytes the sweeps must stream = the coupling
    # blocks + xhat reads + yhat writes.  A symmetric kernel stores one block
    # per unordered pair and the apply streams it twice (B_ij x_j for row i,
    # B_ij^T x_i for row j: the right-hand-side panels are as large as the
    # blocks at 32 RHS, so reading the block once and scattering to both rows
    # would move more bytes), with yhat read back and written by the second
    # sweep.
    sym_B = not info["nonsymmetric"]
    coupling_bytes = ((2 if sym_B else 1) * info["bytes_B"] +
                      (4 if sym_B else 2) * 8 * info["sum_rank"] * nrhs)
    t_coup = float(np.mean(coup))
    achieved = coupling_bytes / t_coup / 1e9
    idw = np.array(idw)
    roof_id = id_roofline(float(idw[:, 0].mean()), float(idw[:, 1].mean()),
                          "k_id_fold + k_batched_id<512> (interpolative decompositions of the nodes with "
                          "more than 64 columns)")
    roof_id_all = id_roofline(float(idw[:, 2].mean()), float(idw[:, 3].mean()), "k_batched_id (all classes)")
    # dominant kernel: the top-down DataReduct, one launch per tree level;
    # algorithmic bytes = every candidate coordinate of T_i read once.  The
    # definition's brute-force search (every reference point against every
    # candidate, 3d - 1 flops per squared distance) is reported beside it as
    # the rate at which the box-pruned search completes that work: the
    # kernel evaluates far fewer distances, so this is no roofline.
    dr_bytes, dr_ms, dr_evals = float(idw[:, 4].mean()), float(idw[:, 5].mean()), float(idw[:, 6].mean())
    dr_launches = info["maxdepth"]
    dr_achieved = dr_bytes / (dr_ms / 1e3) / 1e9 if dr_ms > 0 else 0.0
    roof_dr = {"kernel": "k_datareduct_down<3,1024> (HiDR top-down DataReduct)", "bound": "hbm",
               "achieved": dr_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dr_achieved / HBM_PEAK_GBS,
               "traffic": recorded_traffic("k_datareduct_down_cube3d-coulomb-n1048576_hbm-counters.md",
                                           "paper_2206_01885_amd/csrc/hidr.hip"),
               "launches_per_step": dr_launches, "ms_per_launch": dr_ms / dr_launches,
               "bytes_per_launch": dr_bytes / dr_launches,
               "brute_force_equivalent": {
                   "distance_evals_per_launch": dr_evals / dr_launches,
                   "equivalent_tflops": dr_evals * (3 * 3 - 1) / (dr_ms / 1e3) / 1e12 if dr_ms > 0 else 0.0,
                   "note": "rate of completing the definition's all-pairs search; the pruned search "
                           "evaluates far fewer distances"}}
    mv_bytes = (info["bytes_B"] + info["bytes_D"] + info["bytes_U"] + 8 * nrhs * n * 4)
    build_s = float(np.mean(builds))
    mv_s = float(np.mean(mvs))
    # HiDR once for all (outside the timed steps): the same representor sets
    # rebuilt at another tolerance (1e-5)
    Ysave = Y[:, ridx].clone()
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    h2.h2_rebuild(hd, "coulomb", 1.0, 1e-5)
    torch.cuda.synchronize()
    rebuild_s = time.perf_counter() - tr0
    h2.h2_destroy(hd)
    Y64 = Ysave
    del Y

    # coupling blocks evaluated by the apply (store_coupling = 0): no B in
    # memory, same representation otherwise
    otf = None
    if not args.no_f32:
        opt0 = h2.h2_options_default()
        opt0.r1, opt0.r2 = args.r, 2 * args.r
        opt0.r_min = args.r_min
        opt0.store_coupling = 0
        opt0.profile = 1
        Y0 = torch.empty_like(X)
        b0, m0 = [], []
        for k in range(1 + args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            hd0 = h2.h2_build(Psoa, "coulomb", 1.0, 1e-6, 128, opt0)
            tb = time.perf_counter()
            h2.h2_matvec(hd0, X, Y0, nrhs)
            torch.cuda.synchronize()
            te = time.perf_counter()
            if k > 0:
                b0.append(tb - ts)
                m0.append(te - tb)
            i0 = h2.h2_query(hd0)
            h2.h2_destroy(hd0)
            print(f"[bench] store_coupling 0 step {k}: build {tb - ts:.3f} s matvec {te - tb:.4f} s",
                  file=sys.stderr, flush=True)
        e0 = ((Y0[:, ridx] - ref).norm(dim=1) / ref.norm(dim=1)).max().item()
        e0_64 = ((Y0[:, ridx] - Y64).norm(dim=1) / Y64.norm(dim=1)).max().item()
        otf = {"ms_per_step": 1e3 * (float(np.mean(b0)) + float(np.mean(m0))), "build_s": float(np.mean(b0)),
               "matvec_s": float(np.mean(m0)), "mpts_per_s": n / (float(np.mean(b0)) + float(np.mean(m0))) / 1e6,
               "mv_coupling_ms": i0["mv_coupling"], "bytes_B": i0["bytes_B"], "bytes_D": i0["bytes_D"],
               "e_dense_sampled_rows_max_rhs": e0, "e_vs_stored_path_max_rhs": e0_64}
        del Y0

    # precision mode: FP32 blocks and apply (compensated nearfield), same build otherwise
    f32 = None
    if not args.no_f32:
        opt32 = h2.h2_options_default()
        opt32.r1, opt32.r2 = args.r, 2 * args.r
        opt32.r_min = args.r_min
        opt32.precision = 32
        opt32.profile = 1
        X32 = X.float()
        Y32 = torch.empty_like(X32)
        torch.cuda.synchronize()
        hd32 = h2.h2_build(Psoa, "coulomb", 1.0, 1e-6, 128, opt32)
        h2.h2_matvec(hd32, X32, Y32, nrhs)
        torch.cuda.synchronize()
        h2.h2_destroy(hd32)
        b32, m32 = [], []
        for k in range(args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            hd32 = h2.h2_build(Psoa, "coulomb", 1.0, 1e-6, 128, opt32)
            tb = time.perf_counter()
            h2.h2_matvec(hd32, X32, Y32, nrhs)
            torch.cuda.synchronize()
            te = time.perf_counter()
            b32.append(tb - ts)
            m32.append(te - tb)
            i32 = h2.h2_query(hd32)
            h2.h2_destroy(hd32)
        got32 = Y32[:, ridx].double()
        e32 = ((got32 - ref).norm(dim=1) / ref.norm(dim=1)).max().item()
        e32_64 = ((got32 - Y64).norm(dim=1) / Y64.norm(dim=1)).max().item()
        acc32_oracle = vs_golden(got32)
        f32 = {"ms_per_step": 1e3 * (np.mean(b32) + np.mean(m32)), "build_s": float(np.mean(b32)),
               "matvec_s": float(np.mean(m32)), "matvec_phases_ms": {k: i32[k] for k in (
                   "mv_gather", "mv_upward", "mv_coupling", "mv_downward", "mv_leaves", "mv_scatter")},
               "bytes_B": i32["bytes_B"], "bytes_D": i32["bytes_D"],
               "e_dense_sampled_rows_max_rhs": e32, "e_vs_fp64_path_max_rhs": e32_64,
               "vs_oracle": acc32_oracle}
        del Y32, X32

    # precision mode where its decompositions run in FP32 too (tol >= 1e-5):
    # FP64 and FP32 paths side by side at tol 1e-5
    f32_1e5 = None
    if not args.no_f32:
        f32_1e5 = {}
        for prec in (64, 32):
            o5 = h2.h2_options_default()
            o5.r1, o5.r2 = args.r, 2 * args.r
            o5.r_min = args.r_min
            o5.precision = prec
            o5.profile = 1
            Xp = X if prec == 64 else X.float()
            Yp = torch.empty_like(Xp)
            tb5, tm5 = [], []
            for k in range(1 + args.steps):
                torch.cuda.synchronize()
                ts = time.perf_counter()
                hp = h2.h2_build(Psoa, "coulomb", 1.0, 1e-5, 128, o5)
                tb = time.perf_counter()
                h2.h2_matvec(hp, Xp, Yp, nrhs)
                torch.cuda.synchronize()
                te = time.perf_counter()
                if k > 0:
                    tb5.append(tb - ts)
                    tm5.append(te - tb)
                ip = h2.h2_query(hp)
                h2.h2_destroy(hp)
            got = Yp[:, ridx].double()
            f32_1e5[f"fp{prec}"] = {
                "ms_per_step": 1e3 * (np.mean(tb5) + np.mean(tm5)), "build_s": float(np.mean(tb5)),
                "matvec_s": float(np.mean(tm5)), "t_basis_s": ip["t_basis"], "sum_rank": ip["sum_rank"],
                "bytes_B": ip["bytes_B"],
                "e_dense_sampled_rows_max_rhs": ((got - ref).norm(dim=1) / ref.norm(dim=1)).max().item()}
            print(f"[bench] tol 1e-5 precision {prec}: {f32_1e5[f'fp{prec}']}", file=sys.stderr, flush=True)
            del Xp, Yp

    out = {
        "metric": "H2 build Mpts/s + matvec GB/s, n=1M 3D Coulomb @1e-6; p50/p99 latency",
        "value": n / (ms_per_step / 1e3) / 1e6,
        "unit": "Mpts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cube3d-coulomb-n1048576-leaf128-tol1e-6-nrhs32", "n": n, "nrhs": nrhs,
                   "leaf": 128, "tol": 1e-6, "r1": info["r1"], "r2": info["r2"]},
        "build_s": build_s, "build_mpts_s": n / build_s / 1e6,
        "rebuild_tol1e-5_s": rebuild_s,
        "matvec_s": mv_s, "matvec_gbps": mv_bytes / mv_s / 1e9,
        "latency_p50_s": float(np.percentile(np.array(builds) + np.array(mvs), 50)),
        "latency_p99_s": float(np.percentile(np.array(builds) + np.array(mvs), 99)),
        "phases_s": {k: info[k] for k in ("t_tree", "t_lists", "t_calib", "t_hidr", "t_basis", "t_blocks")},
        "matvec_phases_ms": {k: info[k] for k in ("mv_gather", "mv_upward", "mv_coupling", "mv_downward",
                                                   "mv_leaves", "mv_scatter")},
        "structure": {k: info[k] for k in ("nnode", "maxdepth", "nnz_il", "nnz_near", "max_rank", "sum_rank",
                                            "bytes_U", "bytes_B", "bytes_D")},
        "accuracy": {"e_dense_sampled_rows_max_rhs": e_rows, "e_dense_sampled_rows_mean_rhs": e_rows_mean,
                     "rows": int(len(rows)), "dense_reference": "torch FP64 on the GPU, all RHS",
                     "vs_oracle": acc_oracle},
        "precision_f32": f32,
        "precision_tol1e-5": f32_1e5,
        "store_coupling_0": otf,
        "roofline": roof_dr,
        "roofline_id_wide": roof_id,
        "roofline_id_all_classes": roof_id_all,
        "roofline_matvec": {"kernel": "k_sweep + k_sweep_t (coupling sweeps of the apply)", "bound": "hbm",
                            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS,
                            "traffic": recorded_traffic("k_sweep_coupling_cube3d-coulomb-n1048576-nrhs32_hbm-counters.md",
                                                        "paper_2206_01885_amd/csrc/matvec.hip"),
                            "bytes_per_launch": coupling_bytes, "stored_block_bytes": info["bytes_B"],
                            "blocks_streamed_per_apply": 2 if sym_B else 1, "ms_per_launch": 1e3 * t_coup},
    }
    # the HBM rate a plain device copy reaches here (1 GiB read + 1 GiB
    # written per copy), beside the vendor peak
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (time.perf_counter() - tc) / 1e9
    del src, dst
    out["hbm_copy_gbs"] = copy_gbs
    # the launch parameters the library was built with (autotune.py)
    from paper_2206_01885_amd import autotune
    out["tuning"] = {"params": autotune.current(), "source": "paper_2206_01885_amd/tuning.json"}
    for key in ("roofline", "roofline_matvec"):
        if out[key]["unit"] == "GB/s":
            out[key]["frac_of_measured_copy"] = out[key]["achieved"] / copy_gbs
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, nrhs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
