"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the method's
arithmetic, so both the GPU library and the CPU oracle can be fed from it.

* ``cube``: i.i.d. uniform points in [0,1]^d -- the "cube" dataset of
  Section 6.1.1 (uniform samples in the unit cube).
* ``sphere``: uniform points on the unit sphere surface (normalised Gaussian
  vectors), a stand-in for the paper's manifold datasets (3-sphere, Dino).
* ``three_spheres``: points on three unit spheres whose centres form an
  equilateral triangle of side 1 (the "3-sphere" dataset of Section 6.1.1).
* ``gauss_mixture``: an 8-component Gaussian mixture (sigma = 0.05).
* Right-hand sides are standard normal (the error metric of Section 6 uses
  z ~ N(0, I)).
"""
from __future__ import annotations

import math

import numpy as np

KERNEL_IDS = {"coulomb": 0, "gaussian": 1, "exponential": 2, "matern32": 3, "bump": 4, "cosine": 5,
              "advection": 6}


def cube(rng, n, d):
    return rng.random((n, d))


def sphere(rng, n, d=3):
    v = rng.standard_normal((n, d))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def three_spheres(rng, n):
    c = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, math.sqrt(3.0) / 2.0, 0.0]])
    which = np.arange(n) % 3
    return sphere(rng, n, 3) + c[which]


def gauss_mixture(rng, n, d, k=8, sigma=0.05):
    centres = rng.random((k, d))
    comp = rng.integers(0, k, size=n)
    return centres[comp] + sigma * rng.standard_normal((n, d))


# ---------------------------------------------------------------- configs
# Each returns a dict with the points [n, d] (float64, original order), the
# kernel, its parameter, the tolerance, the leaf size and the right-hand sides
# [nrhs, n]; "rows" are sampled row indices where the config asks for them.

def config_small_coulomb(seed=1001, n=4096):
    """n = 4096 uniform points in [0,1]^3, Coulomb, leaf 64, tol 1e-6, 1 RHS."""
    rng = np.random.default_rng(seed)
    P = cube(rng, n, 3)
    x = rng.standard_normal((1, n))
    return dict(name="cube3d-coulomb-n4096", points=P, kernel="coulomb", prm=1.0, tol=1e-6,
                leaf=64, x=x, rows=None)


def config_gaussian_2d(seed=1002, n=65536, nrhs=16, nrows=1000):
    """n = 65536 uniform points in [0,1]^2, Gaussian h = 0.1, leaf 128, tol 1e-8,
    16 RHS, 1000 sampled rows."""
    rng = np.random.default_rng(seed)
    P = cube(rng, n, 2)
    x = rng.standard_normal((nrhs, n))
    rows = rng.choice(n, nrows, replace=False)
    return dict(name="square2d-gaussian-n65536", points=P, kernel="gaussian", prm=0.1, tol=1e-8,
                leaf=128, x=x, rows=rows)


def config_batched(seed=1003, nprob=256, nmin=2048, nmax=32768):
    """Independent problems: n log-uniform in [2048, 32768], cube or sphere
    (1/2 each), kernel uniform over Coulomb / exponential(0.2) / Matern-3/2(0.2),
    leaf 64, tol 1e-6."""
    rng = np.random.default_rng(seed)
    out = []
    kernels = [("coulomb", 1.0), ("exponential", 0.2), ("matern32", 0.2)]
    for _ in range(nprob):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        geo = "cube" if rng.random() < 0.5 else "sphere"
        P = cube(rng, n, 3) if geo == "cube" else sphere(rng, n, 3)
        kname, prm = kernels[int(rng.integers(0, 3))]
        x = rng.standard_normal((1, n))
        out.append(dict(name=f"{geo}-{kname}-n{n}", points=P, kernel=kname, prm=prm, tol=1e-6,
                        leaf=64, x=x, rows=None))
    return out


def config_cube_1m(seed=1004, n=1 << 20, nrhs=32, nrows=4096):
    """n = 2^20 uniform points in [0,1]^3, Coulomb, leaf 128, tol 1e-6, 32 RHS,
    4096 sampled rows."""
    rng = np.random.default_rng(seed)
    P = cube(rng, n, 3)
    x = rng.standard_normal((nrhs, n))
    rows = rng.choice(n, nrows, replace=False)
    return dict(name="cube3d-coulomb-n1048576", points=P, kernel="coulomb", prm=1.0, tol=1e-6,
                leaf=128, x=x, rows=rows)


def serving_requests(seed=1005, nreq=64, nmin=1024, nmax=1 << 20):
    """Request stream: n log-uniform in [1024, 2^20], d in {2, 3}, cube or
    8-component Gaussian mixture, kernel in {Coulomb, Gaussian 0.1,
    exponential 0.2}, tol 1e-6, 8 RHS each."""
    rng = np.random.default_rng(seed)
    kernels = [("coulomb", 1.0), ("gaussian", 0.1), ("exponential", 0.2)]
    out = []
    for _ in range(nreq):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        d = int(rng.integers(2, 4))
        P = cube(rng, n, d) if rng.random() < 0.5 else gauss_mixture(rng, n, d)
        kname, prm = kernels[int(rng.integers(0, 3))]
        x = rng.standard_normal((8, n))
        out.append(dict(name=f"req-{kname}-d{d}-n{n}", points=P, kernel=kname, prm=prm, tol=1e-6,
                        leaf=64, x=x, rows=None))
    return out
