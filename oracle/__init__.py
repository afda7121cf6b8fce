"""Oracle for the explicit 3-D heat-diffusion step (plain FP64 CPU code).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
loads or calls anything here, and this package shares no code with it.

The arithmetic lives in ``diff3d_oracle.c`` (plain triple loops, FP64, no
fused multiply-add); this module only compiles it with gcc on first use and
marshals numpy arrays.  ``brute`` holds an exact rational evaluator and a
dense-matrix evaluator for tiny grids, used to pin the C loops.

Source: Omlin & Raess, "High-performance xPU Stencil Computations in Julia"
(JuliaCon 2019 proceedings), Fig. 1: the ``step!`` kernel and the
``diffusion3D`` driver.  Arrays are numpy float64 of shape (nz, ny, nx),
C-contiguous, so x is the fastest index as in the paper's column-major
Julia arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diff3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
               "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i, d = ctypes.c_int, ctypes.c_double
            lib.oracle_scalars.argtypes = [i, i, i, d, d, d, d, dp, dp]
            lib.oracle_scalars.restype = None
            lib.oracle_forward.argtypes = [dp, dp, dp, i, i, i, d, d, d, d, d, i, i]
            lib.oracle_forward.restype = i
            lib.oracle_reverse.argtypes = [dp, dp, dp, dp, dp, i, i, i, d, d, d, d, d, i, i, i]
            lib.oracle_forward2d.argtypes = [dp, dp, dp, i, i, d, d, d, d, i, i]
            lib.oracle_reverse.restype = i
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = i
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("fields are 3-D arrays of shape (nz, ny, nx)")
    if shape is not None and a.shape != shape:
        raise ValueError("field shape %s != %s" % (a.shape, shape))
    return a


def max_threads() -> int:
    return _load().oracle_max_threads()


def scalars(nx: int, ny: int, nz: int, Ci, lam: float = 1.0, lx: float = 1.0, ly: float = 1.0,
            lz: float = 1.0) -> dict:
    """Driver scalars of Fig. 1: dx=lx/(nx-1) (and y, z), inverse spacings,
    dt = min(dx^2,dy^2,dz^2)/lam/max(Ci)/6.1 with the maximum over all of Ci."""
    Ci = _field(Ci, (nz, ny, nx))
    out = np.zeros(7)
    _load().oracle_scalars(nx, ny, nz, lx, ly, lz, lam, _ptr(Ci), _ptr(out))
    keys = ("dx", "dy", "dz", "rdx", "rdy", "rdz", "dt")
    res = {k: float(v) for k, v in zip(keys, out)}
    res["lam"] = float(lam)
    return res


def forward(T0, Ci, lam: float, dt: float, rdx: float, rdy: float, rdz: float, nt: int,
            threads: int = 0) -> np.ndarray:
    """T_nt after nt steps of the Fig. 1 kernel with the buffer swap.  Boundary
    values stay those of T0.  ``threads`` = 0 uses the OpenMP default."""
    T0 = _field(T0)
    Ci = _field(Ci, T0.shape)
    nz, ny, nx = T0.shape
    T = np.empty_like(T0)
    rc = _load().oracle_forward(_ptr(T), _ptr(T0), _ptr(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz,
                                int(nt), int(threads))
    if rc != 0:
        raise ValueError("oracle_forward failed (%d)" % rc)
    return T


def forward2d(T0, Ci, lam: float, dt: float, rdx: float, rdy: float, nt: int, threads: int = 0) -> np.ndarray:
    """T_nt after nt steps of the 2-D form of the step (the Fig. 1 expression
    without the z term) on an (ny, nx) array, boundary fixed."""
    T0 = np.ascontiguousarray(T0, dtype=np.float64)
    Ci = np.ascontiguousarray(Ci, dtype=np.float64)
    if T0.ndim != 2 or Ci.shape != T0.shape:
        raise ValueError("forward2d expects two (ny, nx) arrays")
    ny, nx = T0.shape
    T = np.empty_like(T0)
    rc = _load().oracle_forward2d(_ptr(T), _ptr(T0), _ptr(Ci), nx, ny, lam, dt, rdx, rdy, int(nt), int(threads))
    if rc != 0:
        raise ValueError("oracle_forward2d failed (%d)" % rc)
    return T


def scalars2d(nx: int, ny: int, Ci, lam: float = 1.0, lx: float = 1.0, ly: float = 1.0) -> dict:
    """Driver scalars of the 2-D form: dx = lx/(nx-1), 1/dx, and
    dt = min(dx^2, dy^2)/lam/max(Ci)/4.1 (the 3-D rule's divisor 6.1 = 2*3 +
    0.1 becomes 2*2 + 0.1 in two dimensions)."""
    dx, dy = lx / (nx - 1), ly / (ny - 1)
    cmax = float(np.max(Ci))
    dt = min(dx * dx, dy * dy) / lam / cmax / 4.1
    return {"lam": lam, "dt": dt, "dx": dx, "dy": dy, "rdx": 1.0 / dx, "rdy": 1.0 / dy}


def reverse(T0, Ci, g_nt, lam: float, dt: float, rdx: float, rdy: float, rdz: float, nt: int,
            keep: int = 1, threads: int = 0):
    """Reverse sweep: given g_nt = dLoss/dT_nt, return (dLoss/dT0, dLoss/dCi).
    States are kept every ``keep`` steps and recomputed in between."""
    T0 = _field(T0)
    Ci = _field(Ci, T0.shape)
    g_nt = _field(g_nt, T0.shape)
    nz, ny, nx = T0.shape
    gT0 = np.empty_like(T0)
    gCi = np.empty_like(T0)
    rc = _load().oracle_reverse(_ptr(T0), _ptr(Ci), _ptr(g_nt), _ptr(gT0), _ptr(gCi), nx, ny, nz,
                                lam, dt, rdx, rdy, rdz, int(nt), int(keep), int(threads))
    if rc != 0:
        raise ValueError("oracle_reverse failed (%d)" % rc)
    return gT0, gCi


def loss_and_seed(T_nt, T_target):
    """L = 0.5*||T_nt - T_target||^2 over the whole grid and its gradient
    dL/dT_nt = T_nt - T_target (FP64)."""
    r = _field(T_nt) - _field(T_target)
    return 0.5 * float(np.sum(r * r)), r
