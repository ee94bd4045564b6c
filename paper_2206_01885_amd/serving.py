"""Serving loop for independent H^2 requests (build + apply) on one GPU.

A request is a point set with its kernel and tolerance plus a block of
right-hand sides; serving it means one build and one apply of all its
right-hand sides (FP32 precision mode by default), then returning y.  The
loop keeps the device busy with continuous batching:

* admission: a request that has arrived is admitted while the device memory
  reserved by admitted requests plus its own estimate stays within the HBM
  budget (the estimate is replaced by the handle's measured size once it is
  built; memory is released when the request completes);
* batching: every round, the builder takes all admitted requests that are
  waiting (up to ``max_batch``) and builds them in one h2_build_batched call,
  so their r1/r2 calibration and their nested-basis levels share launches;
* overlap: applies run on a second stream in another thread while the next
  round builds, and requests that arrive while others are on the GPU join
  the next round as memory frees up.

Built handles stay resident until their apply is done.  Every step of a
request runs in the library's HIP kernels through the C ABI; this module
only schedules.  Latency = completion time - arrival time.
"""
from __future__ import annotations

import collections
import threading
import time

import numpy as np
import torch

from . import h2

# Device bytes per point assumed before a request is built (FP32 blocks at
# leaf 64 and tol 1e-6: about 1e5 in 3-D, 3e4 in 2-D), plus a fixed amount;
# replaced by the measured size after the build.
EST_BYTES_PER_POINT = {1: 8e3, 2: 4e4, 3: 1.2e5}
EST_FIXED = 64 << 20


def estimate_bytes(n, d):
    return int(EST_FIXED + EST_BYTES_PER_POINT[d] * n)


def handle_bytes(info):
    n = info["n"]
    return int(info["bytes_B"] + info["bytes_D"] + info["bytes_U"] + 64 * n + EST_FIXED)


class Request:
    __slots__ = ("idx", "points", "kernel", "prm", "tol", "leaf", "x", "arrival", "t_arrive", "t_admit",
                 "t_built", "t_done", "y", "reserved", "handle", "soa", "xd")

    def __init__(self, idx, points, kernel, prm, tol, leaf, x, arrival=0.0):
        self.idx, self.points, self.kernel, self.prm, self.tol, self.leaf = idx, points, kernel, prm, tol, leaf
        self.x, self.arrival = x, arrival
        self.t_arrive = self.t_admit = self.t_built = self.t_done = None
        self.y = None
        self.reserved = 0
        self.handle = None


class Server:
    def __init__(self, hbm_budget=250e9, max_batch=32, precision=32, options=None, keep_outputs=True):
        self.budget = float(hbm_budget)
        self.max_batch = int(max_batch)
        self.precision = precision
        self.opt = options if options is not None else h2.h2_options_default()
        self.opt.precision = precision
        self.keep = keep_outputs
        self.dtype = torch.float32 if precision == 32 else torch.float64

    def run(self, requests, arrivals=None):
        """Serve `requests` (Request objects); arrivals[i] is the arrival time
        of request i in seconds after the start (None: all at once).  Returns
        the requests with their timestamps and outputs filled in."""
        reqs = list(requests)
        if arrivals is None:
            arrivals = [0.0] * len(reqs)
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        lock = threading.Condition()
        waiting = collections.deque()   # arrived, not yet built
        built = collections.deque()     # built, apply pending
        state = {"reserved": 0.0, "arrived": 0, "done": 0, "err": None}
        total = len(reqs)
        bstream = torch.cuda.Stream()
        astream = torch.cuda.Stream()
        t0 = time.perf_counter()

        def builder():
            try:
                torch.cuda.set_device(torch.cuda.current_device())
                while True:
                    with lock:
                        while not waiting and state["arrived"] < total and state["err"] is None:
                            lock.wait()
                        if state["err"] is not None:
                            return
                        if not waiting and state["arrived"] >= total:
                            return
                        batch = []
                        while waiting and len(batch) < self.max_batch:
                            r = waiting[0]
                            est = estimate_bytes(r.points.shape[0], r.points.shape[1])
                            if batch and state["reserved"] + est > self.budget:
                                break
                            if not batch:
                                # the head of the queue waits for memory
                                while state["reserved"] > 0 and state["reserved"] + est > self.budget:
                                    lock.wait()
                                    if state["err"] is not None:
                                        return
                            waiting.popleft()
                            r.reserved = est
                            state["reserved"] += est
                            r.t_admit = time.perf_counter() - t0
                            batch.append(r)
                    with torch.cuda.stream(bstream):
                        for r in batch:
                            r.soa = torch.tensor(np.ascontiguousarray(r.points.T), device="cuda")
                            r.xd = torch.tensor(r.x, dtype=self.dtype, device="cuda")
                        hs = h2.h2_build_batched([r.soa for r in batch], [r.kernel for r in batch],
                                                 [r.prm for r in batch], [r.tol for r in batch],
                                                 [r.leaf for r in batch], self.opt, bstream)
                    now = time.perf_counter() - t0
                    with lock:
                        for r, hd in zip(batch, hs):
                            r.handle = hd
                            r.t_built = now
                            actual = handle_bytes(h2.h2_query(hd))
                            state["reserved"] += actual - r.reserved
                            r.reserved = actual
                            r.soa = None
                            built.append(r)
                        lock.notify_all()
            except BaseException as e:  # surfaced by run()
                with lock:
                    state["err"] = e
                    lock.notify_all()

        def applier():
            try:
                while True:
                    with lock:
                        while not built and state["done"] < total and state["err"] is None:
                            lock.wait()
                        if state["err"] is not None or state["done"] >= total:
                            return
                        r = built.popleft()
                    with torch.cuda.stream(astream):
                        y = torch.empty_like(r.xd)
                        h2.h2_matvec(r.handle, r.xd, y, r.xd.shape[0], astream)
                        astream.synchronize()
                    r.t_done = time.perf_counter() - t0
                    if self.keep:
                        r.y = y.cpu().numpy()
                    h2.h2_destroy(r.handle)
                    r.handle = None
                    r.xd = None
                    with lock:
                        state["reserved"] -= r.reserved
                        state["done"] += 1
                        lock.notify_all()
            except BaseException as e:
                with lock:
                    state["err"] = e
                    lock.notify_all()

        tb = threading.Thread(target=builder, daemon=True)
        ta = threading.Thread(target=applier, daemon=True)
        tb.start()
        ta.start()
        for i in order:
            dt = arrivals[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            r = reqs[i]
            r.arrival = arrivals[i]
            r.t_arrive = time.perf_counter() - t0
            with lock:
                waiting.append(r)
                state["arrived"] += 1
                lock.notify_all()
        tb.join()
        ta.join()
        if state["err"] is not None:
            raise state["err"]
        return reqs


def summarize(reqs, wall):
    lat = np.array([r.t_done - r.arrival for r in reqs])
    nrhs = sum(int(r.x.shape[0]) for r in reqs)
    pts = sum(int(r.points.shape[0]) for r in reqs)
    return {"requests": len(reqs), "wall_s": wall, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "requests_per_s": len(reqs) / wall, "solves_per_s": nrhs / wall, "mpts_per_s": pts / wall / 1e6}
