"""Seeded synthetic inputs for the 3-D heat-diffusion workloads.

This module only draws fields; it holds none of the step's arithmetic and is
shared by the tests, the smoke check and the benchmark, which pass the same
arrays to the HIP library and to the oracle.

Fields are numpy float64 arrays of shape (nz, ny, nx), C order (x fastest).
Random draws are ``numpy.random.default_rng(seed).random(nx*ny*nz)`` reshaped
to that shape; reduced-precision runs round these FP64 draws.

Workloads (grid points are vertex-centred, x_i = i/(n-1) on [0, 1]):

* ``uniform_const``: T0 ~ U[0,1] (seed 0), Ci = 0.5 everywhere.  The 64^3
  forward case, the 256^3 and 32^3 gradient cases and the 1024^3 large case.
* ``bump``: T0 = exp(-((x-.5)^2 + (y-.5)^2 + (z-.5)^2)/0.01) + 0.01*U[0,1]
  (seed 0), Ci = 0.5*(1 + 0.5*u) with u ~ U[0,1] (seed 1).  The 512^3 forward
  case (the grid of the paper's Fig. 1 listing) and the 256^3 precision case.
* ``target``: T_target ~ U[0,1] (seed 2) for the gradient cases.
* ``direction``: a unit-scale U[-1,1] direction (seed 3) for finite differences.
"""
from __future__ import annotations

import numpy as np

SEED_T0 = 0
SEED_CI = 1
SEED_TARGET = 2
SEED_DIRECTION = 3

LAM = 1.0
LX = LY = LZ = 1.0

# (name, grid, nt) of the workloads; dtype variants are chosen by the caller.
WORKLOADS = {
    "uniform64": dict(kind="uniform_const", n=(64, 64, 64), nt=100),
    "bump512": dict(kind="bump", n=(512, 512, 512), nt=100),
    "bump256": dict(kind="bump", n=(256, 256, 256), nt=100),
    "grad256": dict(kind="uniform_const", n=(256, 256, 256), nt=200, ckpt_every=14),
    "grad32": dict(kind="uniform_const", n=(32, 32, 32), nt=200, ckpt_every=14),
    "grad1024": dict(kind="uniform_const", n=(1024, 1024, 1024), nt=500, ckpt_every=32),
}


def uniform(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(nx * ny * nz).reshape(nz, ny, nx)


def uniform_const(nx: int, ny: int, nz: int):
    """(T0, Ci): T0 ~ U[0,1] from seed 0; Ci = 0.5 everywhere."""
    T0 = uniform(nx, ny, nz, SEED_T0)
    Ci = np.full((nz, ny, nx), 0.5)
    return T0, Ci


def bump(nx: int, ny: int, nz: int):
    """(T0, Ci): Gaussian bump plus 0.01*U[0,1] noise (seed 0);
    Ci = 0.5*(1 + 0.5*u), u ~ U[0,1] from seed 1."""
    x = np.arange(nx) / (nx - 1) - 0.5
    y = np.arange(ny) / (ny - 1) - 0.5
    z = np.arange(nz) / (nz - 1) - 0.5
    T0 = uniform(nx, ny, nz, SEED_T0)
    T0 *= 0.01
    # accumulate plane by plane to keep the temporaries small at 512^3 and up
    r2xy = (y[:, None] ** 2) + (x[None, :] ** 2)
    for iz in range(nz):
        T0[iz] += np.exp(-(r2xy + z[iz] ** 2) / 0.01)
    Ci = uniform(nx, ny, nz, SEED_CI)
    Ci *= 0.25
    Ci += 0.5
    return T0, Ci


def target(nx: int, ny: int, nz: int) -> np.ndarray:
    return uniform(nx, ny, nz, SEED_TARGET)


def direction(nx: int, ny: int, nz: int, seed: int = SEED_DIRECTION) -> np.ndarray:
    return 2.0 * uniform(nx, ny, nz, seed) - 1.0


def make(kind: str, nx: int, ny: int, nz: int):
    if kind == "uniform_const":
        return uniform_const(nx, ny, nz)
    if kind == "bump":
        return bump(nx, ny, nz)
    raise ValueError("unknown workload kind %r" % kind)
