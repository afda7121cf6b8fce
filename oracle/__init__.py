"""Oracle for the explicit 3-D heat-diffusion step (plain FP64 CPU code).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
loads or calls anything here, and this package shares no code with it.

The arithmetic lives in ``diff3d_oracle.c`` (plain triple loops, FP64, no
fused multiply-add) and ``emulate32.c`` (the same loops in FP32 arithmetic
with FP32 or BF16 storage, and the Philox4x32-10 generator behind
stochastic rounding); this module only compiles them with gcc on first use
and marshals numpy arrays.  ``brute`` holds an exact rational evaluator and a
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
_SRC32 = os.path.join(_HERE, "emulate32.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, -ffp-contract=off)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC32))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, _SRC32, "-lm"]
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
            vp, sz, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64
            lib.emul_philox4x32_10.argtypes = [vp, vp, vp]
            lib.emul_philox4x32_10.restype = None
            lib.emul_sr_bits.argtypes = [u64, u64, vp, vp, sz]
            lib.emul_sr_bits.restype = None
            lib.emul_bf16_nearest.argtypes = [vp, vp, sz]
            lib.emul_bf16_nearest.restype = None
            lib.emul_bf16_stochastic.argtypes = [vp, vp, vp, sz]
            lib.emul_bf16_stochastic.restype = None
            lib.emul_forward.argtypes = [vp, vp, vp, i, i, i, d, d, d, d, d, vp, i, i, u64, u64, i]
            lib.emul_forward.restype = i
            lib.emul_reverse32.argtypes = [vp, vp, vp, vp, vp, i, i, i, d, d, d, d, d, i, i, i]
            lib.emul_reverse32.restype = i
            lib.oracle_apply.argtypes = [i, dp, dp, i, i, i, d, d, d]
            lib.oracle_apply.restype = i
            lib.emul_apply32.argtypes = [i, vp, vp, i, i, i, d, d, d, i]
            lib.emul_apply32.restype = i
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


# ---------------------------------------------------------------- FP32 / BF16
# Storage codes of the emulator: FP32, BF16 with stochastic rounding, BF16
# rounded to nearest even.  BF16 fields are numpy uint16 arrays of raw bits.
ST_F32, ST_BF16_SR, ST_BF16_RNE = 1, 2, 3


def _vp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11): four 32-bit output words."""
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _load().emul_philox4x32_10(_vp(c), _vp(k), _vp(o))
    return tuple(int(v) for v in o)


def sr_bits(seed: int, step: int, idx) -> np.ndarray:
    """The 16 random bits of the given linear point indices for the state
    stored after global step index ``step``."""
    i = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.zeros(i.shape, dtype=np.uint16)
    _load().emul_sr_bits(seed & (2 ** 64 - 1), step & (2 ** 64 - 1), _vp(i), _vp(out), i.size)
    return out


def bf16_nearest(x) -> np.ndarray:
    """FP32 values -> BF16 bits, round to nearest even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.uint16)
    _load().emul_bf16_nearest(_vp(x), _vp(out), x.size)
    return out


def bf16_stochastic(x, r) -> np.ndarray:
    """FP32 values -> BF16 bits, stochastic rounding with the 16-bit values r."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    r = np.ascontiguousarray(r, dtype=np.uint16)
    if r.shape != x.shape:
        raise ValueError("one random value per element")
    out = np.zeros(x.shape, dtype=np.uint16)
    _load().emul_bf16_stochastic(_vp(x), _vp(r), _vp(out), x.size)
    return out


def bf16_widen(h) -> np.ndarray:
    """BF16 bits -> FP32 values (exact)."""
    h = np.ascontiguousarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def emulate_forward(T0, Ci, lam: float, dt: float, rdx: float, rdy: float, rdz: float, passes, storage: int,
                    seed: int = 0, step0: int = 0, threads: int = 0) -> np.ndarray:
    """The time loop in FP32 arithmetic with the given storage: T0 and Ci are
    stored values (float32, or uint16 BF16 bits), ``passes`` the pass
    lengths (states inside a pass stay in FP32; the state at the end of each
    pass is stored).  (ny, nx) arrays select the 2-D form (rdz unused).
    Returns the stored final state."""
    dtype = np.float32 if storage == ST_F32 else np.uint16
    T0 = np.ascontiguousarray(T0, dtype=dtype)
    Ci = np.ascontiguousarray(Ci, dtype=dtype)
    if T0.ndim not in (2, 3) or Ci.shape != T0.shape:
        raise ValueError("fields are two (nz, ny, nx) arrays, or two (ny, nx) arrays for the 2-D form")
    if T0.ndim == 2:
        (ny, nx), nz = T0.shape, 1
    else:
        nz, ny, nx = T0.shape
    p = np.ascontiguousarray(passes, dtype=np.int32)
    T = np.empty_like(T0)
    rc = _load().emul_forward(_vp(T), _vp(T0), _vp(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz, _vp(p), p.size,
                              int(storage), seed & (2 ** 64 - 1), step0 & (2 ** 64 - 1), int(threads))
    if rc != 0:
        raise ValueError("emul_forward failed (%d)" % rc)
    return T


def emulate_reverse32(T0, Ci, g_nt, lam: float, dt: float, rdx: float, rdy: float, rdz: float, nt: int,
                      keep: int = 1, threads: int = 0):
    """The reverse sweep in FP32 arithmetic and storage: (dLoss/dT0, dLoss/dCi)."""
    T0 = np.ascontiguousarray(T0, dtype=np.float32)
    Ci = np.ascontiguousarray(Ci, dtype=np.float32)
    g = np.ascontiguousarray(g_nt, dtype=np.float32)
    if T0.ndim != 3 or Ci.shape != T0.shape or g.shape != T0.shape:
        raise ValueError("fields are three (nz, ny, nx) arrays")
    nz, ny, nx = T0.shape
    gT0 = np.empty_like(T0)
    gCi = np.empty_like(T0)
    rc = _load().emul_reverse32(_vp(T0), _vp(Ci), _vp(g), _vp(gT0), _vp(gCi), nx, ny, nz, lam, dt, rdx, rdy, rdz,
                                int(nt), int(keep), int(threads))
    if rc != 0:
        raise ValueError("emul_reverse32 failed (%d)" % rc)
    return gT0, gCi


# Operators of the kernel notation (Fig. 1): interior selection, second
# differences along x, y, z, and the weighted Laplacian of the step.
OP_INN, OP_D2_XI, OP_D2_YI, OP_D2_ZI, OP_LAP = 0, 1, 2, 3, 4


def _interior_shape(shape):
    return tuple(n - 2 for n in shape)


def apply(op: int, A, rdx: float = 1.0, rdy: float = 1.0, rdz: float = 1.0) -> np.ndarray:
    """One operator applied to the FP64 field A, shape (nz, ny, nx) or, for a
    2-D field, (ny, nx); returns its interior values (each dimension shorter
    by two)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    if A.ndim == 3:
        nz, ny, nx = A.shape
    elif A.ndim == 2:
        (ny, nx), nz = A.shape, 1
    else:
        raise ValueError("apply expects a (nz, ny, nx) or (ny, nx) array")
    out = np.empty(_interior_shape(A.shape), dtype=np.float64)
    rc = _load().oracle_apply(int(op), _ptr(out), _ptr(A), nx, ny, nz, rdx, rdy, rdz)
    if rc != 0:
        raise ValueError("oracle_apply failed (%d)" % rc)
    return out


def emulate_apply32(op: int, A, storage: int, rdx: float = 1.0, rdy: float = 1.0, rdz: float = 1.0) -> np.ndarray:
    """One operator in FP32 arithmetic on stored values A (float32, or uint16
    BF16 bits for the BF16 storage codes), 3-D or 2-D as ``apply``."""
    A = np.ascontiguousarray(A, dtype=np.float32 if storage == ST_F32 else np.uint16)
    if A.ndim == 3:
        nz, ny, nx = A.shape
    elif A.ndim == 2:
        (ny, nx), nz = A.shape, 1
    else:
        raise ValueError("emulate_apply32 expects a (nz, ny, nx) or (ny, nx) array")
    out = np.empty(_interior_shape(A.shape), dtype=np.float32)
    rc = _load().emul_apply32(int(op), _vp(out), _vp(A), nx, ny, nz, rdx, rdy, rdz, int(storage))
    if rc != 0:
        raise ValueError("emul_apply32 failed (%d)" % rc)
    return out
