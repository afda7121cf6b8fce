"""Python binding of libdiff3d, the MI355X (gfx950) 3-D heat-diffusion library.

Argument marshalling only: every step runs in the HIP kernels of
``libdiff3d.so`` (built by ``paper_2211_15634_amd/build.py``).  PyTorch supplies
device memory and the current stream.  If the library is missing this module
raises ImportError: there is no fallback path.

Method: the explicit time step of Omlin & Raess, "High-performance xPU
Stencil Computations in Julia", Fig. 1 (``step!`` and the ``diffusion3D``
driver), plus reduced-precision storage and a checkpointed adjoint.

Fields are torch tensors of shape (nz, ny, nx), contiguous, on the GPU, of
dtype float64, float32 or bfloat16 (x is the contiguous axis, as in the
paper's column-major Julia arrays); the 2-D form (step2d, stepn2d, run2d)
takes (ny, nx) tensors of the same dtypes.  bfloat16 fields round
stochastically (``rounding="sr"``, keyed by ``Config.sr_seed`` and
``Config.sr_step``) or to nearest (``rounding="rne"``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiff3d.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libdiff3d.so is not built; run `python paper_2211_15634_amd/build.py` "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

F64, F32, BF16, BF16_RNE = 0, 1, 2, 3
OK, EINVAL, EDTYPE, EWORKSPACE, EHIP = 0, -1, -2, -3, -4
KERNEL_AUTO, KERNEL_NAIVE, KERNEL_ZMARCH, KERNEL_TB2, KERNEL_TBS = 0, 1, 2, 3, 4
MAX_PASS_STEPS = 4
REDUCE_DOUBLES = 1025

_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_ip = ctypes.POINTER(ctypes.c_int)


class _CTile(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("p", ctypes.c_int * 4), ("zlen", ctypes.c_int)]


class _CConfig(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("pass_steps", ctypes.c_int), ("narrow", ctypes.c_int),
                ("reserved", ctypes.c_int), ("sr_seed", ctypes.c_uint64), ("sr_step", ctypes.c_uint64),
                ("zmarch", _CTile), ("tb2", _CTile), ("tbs", _CTile), ("adj", _CTile), ("adj2", _CTile),
                ("rev", _CTile)]


_cfgp = ctypes.POINTER(_CConfig)

_SIGS = {
    "diff3d_strerror": ([_i], ctypes.c_char_p),
    "diff3d_dtype_size": ([_i], _sz),
    "diff3d_version": ([], ctypes.c_char_p),
    "diff3d_scalars": ([_i, _i, _i, _d, _d, _d, _d, _d, _dp], _i),
    "diff3d_max": ([_vp, _sz, _i, _vp, _vp], _i),
    "diff3d_step": ([_vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _d, _i, _vp, _cfgp], _i),
    "diff3d_step2": ([_vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _d, _i, _vp, _cfgp], _i),
    "diff3d_stepn": ([_vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _d, _i, _i, _vp, _cfgp], _i),
    "diff3d_pass_plan": ([_i, _i, _i, _i, _i, _i, _cfgp, _ip, _i], _i),
    "diff3d_run": ([_vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _d, _i, _i, _vp, _vp, _i, _cfgp], _i),
    "diff3d_adjoint_workspace_bytes": ([_i, _i, _i, _i, _i, _i, _cfgp], _sz),
    "diff3d_adjoint_run": ([_vp, _vp, _vp, _vp, _vp, _vp, _sz, _i, _i, _i, _i, _d, _d, _d, _d, _d, _i, _i, _i,
                            _vp, _cfgp], _i),
    "diff3d_loss": ([_vp, _vp, _vp, _sz, _i, _vp, _vp], _i),
    "diff3d_loss_noalloc": ([_vp, _vp, _vp, _sz, _i, _vp, _vp], _i),
    "diff3d_norm2": ([_vp, _sz, _i, _vp, _vp], _i),
    "diff3d_copy": ([_vp, _vp, _sz, _vp], _i),
    "diff3d_philox4x32_10": ([_u32p, _u32p, _u32p], None),
    "diff2d_step": ([_vp, _vp, _vp, _i, _i, _d, _d, _d, _d, _i, _vp, _vp], _i),
    "diff2d_run": ([_vp, _vp, _vp, _i, _i, _d, _d, _d, _d, _i, _i, _vp, _vp], _i),
    "diff2d_stepn": ([_vp, _vp, _vp, _i, _i, _d, _d, _d, _d, _i, _i, _vp, _vp], _i),
    "diff3d_apply": ([_i, _vp, _vp, _i, _i, _i, _d, _d, _d, _i, _vp], _i),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTS = tuple(_SIGS)


@dataclasses.dataclass(frozen=True)
class Tile:
    """Tile override of one kernel family (diff3d_tile): ``p`` holds
    (V, R, NW, NT) for the z-march and two-step kernels, (V, R, NW, 0) for
    the adjoint kernels, (W0, H0, NTH, NT) for the S-step kernel and
    (W0, H0, NTH, 0) for fused reverse passes; ``steps`` is the pass length
    an S-step or reverse override applies to; ``zlen`` the planes per
    z-chunk (0 = automatic).  All zero = the tuned default."""
    steps: int = 0
    p: tuple = (0, 0, 0, 0)
    zlen: int = 0


@dataclasses.dataclass(frozen=True)
class Config:
    """Per-call configuration (diff3d_config): kernel choice, pass length,
    stochastic-rounding seed and first step index, tile overrides.  The
    library keeps no state between calls; the default is a zero-filled
    struct."""
    kernel: int = 0
    pass_steps: int = 0
    narrow: bool = False
    sr_seed: int = 0
    sr_step: int = 0
    zmarch: Tile = Tile()
    tb2: Tile = Tile()
    tbs: Tile = Tile()
    adj: Tile = Tile()
    adj2: Tile = Tile()
    rev: Tile = Tile()

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


def _ctile(t: Tile) -> _CTile:
    p = tuple(int(v) for v in t.p) + (0,) * (4 - len(t.p))
    return _CTile(int(t.steps), (ctypes.c_int * 4)(*p[:4]), int(t.zlen))


def _ccfg(cfg: Config | None):
    if cfg is None:
        return None
    c = _CConfig()
    c.kernel = int(cfg.kernel)
    c.pass_steps = int(cfg.pass_steps)
    c.narrow = int(bool(cfg.narrow))
    c.reserved = 0
    c.sr_seed = int(cfg.sr_seed) & (2 ** 64 - 1)
    c.sr_step = int(cfg.sr_step) & (2 ** 64 - 1)
    for name in ("zmarch", "tb2", "tbs", "adj", "adj2", "rev"):
        setattr(c, name, _ctile(getattr(cfg, name)))
    return ctypes.byref(c)


class Diff3dError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (%d)" % (where, _lib.diff3d_strerror(status).decode(), status))
        self.status = status


def _check(rc: int, where: str):
    if rc != OK:
        raise Diff3dError(rc, where)


def _on(t: torch.Tensor):
    """Make the tensor's device current for a library call (the kernels are
    launched on the current device, into the tensor's current stream)."""
    return torch.cuda.device(t.device)


def _code(t: torch.Tensor, rounding: str = "sr") -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16 if rounding == "sr" else BF16_RNE
    raise TypeError("unsupported dtype %s" % t.dtype)


def _field(t: torch.Tensor, name: str, like: torch.Tensor | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA/HIP tensor" % name)
    if t.dim() != 3 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous (nz, ny, nx) tensor" % name)
    if like is not None and (t.shape != like.shape or t.dtype != like.dtype or t.device != like.device):
        raise ValueError("%s must match shape/dtype/device of the other fields" % name)
    return t


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def version() -> str:
    return _lib.diff3d_version().decode()


def strerror(status: int) -> str:
    return _lib.diff3d_strerror(status).decode()


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    _lib.diff3d_philox4x32_10(c, k, o)
    return tuple(o)


def scalars(nx: int, ny: int, nz: int, cimax: float, lam: float = 1.0, lx: float = 1.0, ly: float = 1.0,
            lz: float = 1.0) -> dict:
    """Driver scalars of Fig. 1 (host arithmetic in the library)."""
    out = (ctypes.c_double * 7)()
    _check(_lib.diff3d_scalars(nx, ny, nz, lx, ly, lz, lam, cimax, out), "scalars")
    keys = ("dx", "dy", "dz", "rdx", "rdy", "rdz", "dt")
    res = {k: float(v) for k, v in zip(keys, out)}
    res["lam"] = float(lam)
    return res


def _acc(device) -> torch.Tensor:
    return torch.empty(REDUCE_DOUBLES, dtype=torch.float64, device=device)


def field_max(x: torch.Tensor) -> torch.Tensor:
    """max(x) as a 0-d float64 device tensor (deterministic reduction)."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    acc = _acc(x.device)
    with _on(x):
        _check(_lib.diff3d_max(_p(x), x.numel(), _code(x), _p(acc), _stream(x)), "max")
    return acc[0]


def problem_scalars(Ci: torch.Tensor, lam: float = 1.0, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0) -> dict:
    """dx, dy, dz, their inverses and dt for the grid of Ci, with max(Ci)
    reduced on the GPU (one device-to-host read)."""
    nz, ny, nx = Ci.shape
    cimax = float(field_max(Ci).item())
    return scalars(nx, ny, nz, cimax, lam=lam, lx=lx, ly=ly, lz=lz)


def _field2d(t: torch.Tensor, name: str, like: torch.Tensor | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA/HIP tensor" % name)
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous (ny, nx) tensor" % name)
    if like is not None and (t.shape != like.shape or t.dtype != like.dtype or t.device != like.device):
        raise ValueError("%s must match shape/dtype/device of the other fields" % name)
    return t


def step2d(T2: torch.Tensor, T: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float,
           rdy: float, rounding: str = "sr", cfg: Config | None = None) -> None:
    """One step of the 2-D form: interior of T2 from T and Ci, (ny, nx) fields
    (float64, float32 or bfloat16; ``rounding`` and ``cfg`` as for step)."""
    _field2d(T, "T")
    _field2d(T2, "T2", T)
    _field2d(Ci, "Ci", T)
    ny, nx = T.shape
    with _on(T):
        _check(_lib.diff2d_step(_p(T2), _p(T), _p(Ci), nx, ny, lam, dt, rdx, rdy, _code(T, rounding), _stream(T),
                                _ccfg(cfg)), "step2d")


def stepn2d(T2: torch.Tensor, T: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
            nsteps: int, rounding: str = "sr", cfg: Config | None = None) -> None:
    """nsteps steps of the 2-D form in one pass: interior of T2 = the state
    nsteps steps after T (T2's boundary untouched)."""
    _field2d(T, "T")
    _field2d(T2, "T2", T)
    _field2d(Ci, "Ci", T)
    ny, nx = T.shape
    with _on(T):
        _check(_lib.diff2d_stepn(_p(T2), _p(T), _p(Ci), nx, ny, lam, dt, rdx, rdy, int(nsteps), _code(T, rounding),
                                 _stream(T), _ccfg(cfg)), "stepn2d")


def run2d(T: torch.Tensor, T2: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
          nt: int, rounding: str = "sr", cfg: Config | None = None) -> None:
    """nt steps of the 2-D form with the swap; the result is left in T."""
    _field2d(T, "T")
    _field2d(T2, "T2", T)
    _field2d(Ci, "Ci", T)
    ny, nx = T.shape
    with _on(T):
        _check(_lib.diff2d_run(_p(T), _p(T2), _p(Ci), nx, ny, lam, dt, rdx, rdy, int(nt), _code(T, rounding),
                               _stream(T), _ccfg(cfg)), "run2d")


# Operators of the kernel notation (diff3d_op): interior selection, second
# differences along x, y, z, and the weighted Laplacian of the step.
OP_INN, OP_D2_XI, OP_D2_YI, OP_D2_ZI, OP_LAP = 0, 1, 2, 3, 4


def apply(op: int, A: torch.Tensor, rdx: float = 1.0, rdy: float = 1.0, rdz: float = 1.0,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """One finite-difference operator of Fig. 1's notation applied to the
    field A, shape (nz, ny, nx) or (ny, nx) for a 2-D field: the values at
    the interior points, each dimension two shorter, in the arithmetic type
    (float64 for float64 fields, float32 for float32 and bfloat16 fields).
    rdx, rdy, rdz (inverse spacings) enter OP_LAP only."""
    if not isinstance(A, torch.Tensor) or not A.is_cuda or not A.is_contiguous():
        raise ValueError("A must be a contiguous CUDA/HIP tensor")
    if A.dim() == 3:
        nz, ny, nx = A.shape
    elif A.dim() == 2:
        (ny, nx), nz = A.shape, 1
    else:
        raise ValueError("A must be a (nz, ny, nx) or (ny, nx) tensor")
    odt = torch.float64 if A.dtype == torch.float64 else torch.float32
    shape = tuple(n - 2 for n in A.shape)
    if out is None:
        out = torch.empty(shape, dtype=odt, device=A.device)
    elif (not out.is_cuda or out.device != A.device or out.dtype != odt or tuple(out.shape) != shape
          or not out.is_contiguous()):
        raise ValueError("out must be a contiguous %s tensor of shape %s on A's device" % (odt, shape))
    with _on(A):
        _check(_lib.diff3d_apply(int(op), _p(out), _p(A), nx, ny, nz, rdx, rdy, rdz, _code(A), _stream(A)), "apply")
    return out


def inn(A: torch.Tensor) -> torch.Tensor:
    """@inn(A): the interior values of A."""
    return apply(OP_INN, A)


def d2_xi(A: torch.Tensor) -> torch.Tensor:
    """@d2_xi(A): second difference along x at the interior points."""
    return apply(OP_D2_XI, A)


def d2_yi(A: torch.Tensor) -> torch.Tensor:
    """@d2_yi(A): second difference along y at the interior points."""
    return apply(OP_D2_YI, A)


def d2_zi(A: torch.Tensor) -> torch.Tensor:
    """@d2_zi(A): second difference along z at the interior points (3-D only)."""
    return apply(OP_D2_ZI, A)


def laplacian(A: torch.Tensor, rdx: float, rdy: float, rdz: float = 1.0) -> torch.Tensor:
    """(d2x*rdx^2 + d2y*rdy^2) + d2z*rdz^2 at the interior points (2-D: no z term)."""
    return apply(OP_LAP, A, rdx, rdy, rdz)


def step(T2: torch.Tensor, T: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
         rdz: float, rounding: str = "sr", cfg: Config | None = None) -> None:
    """One step: interior of T2 from T and Ci (T2's boundary untouched)."""
    _field(T, "T")
    _field(T2, "T2", T)
    _field(Ci, "Ci", T)
    nz, ny, nx = T.shape
    with _on(T):
        _check(_lib.diff3d_step(_p(T2), _p(T), _p(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz, _code(T, rounding),
                                _stream(T), _ccfg(cfg)), "step")


def step2(T2: torch.Tensor, T: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
          rdz: float, rounding: str = "sr", cfg: Config | None = None) -> None:
    """Two steps in one pass: interior of T2 = state two steps after T."""
    _field(T, "T")
    _field(T2, "T2", T)
    _field(Ci, "Ci", T)
    nz, ny, nx = T.shape
    with _on(T):
        _check(_lib.diff3d_step2(_p(T2), _p(T), _p(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz, _code(T, rounding),
                                 _stream(T), _ccfg(cfg)), "step2")


def stepn(T2: torch.Tensor, T: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
          rdz: float, nsteps: int, rounding: str = "sr", cfg: Config | None = None) -> None:
    """nsteps steps in one pass: interior of T2 = state nsteps steps after T."""
    _field(T, "T")
    _field(T2, "T2", T)
    _field(Ci, "Ci", T)
    nz, ny, nx = T.shape
    with _on(T):
        _check(_lib.diff3d_stepn(_p(T2), _p(T), _p(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz, int(nsteps),
                                 _code(T, rounding), _stream(T), _ccfg(cfg)), "stepn")


def pass_plan(shape, nt: int, dtype: torch.dtype, ckpt_every: int = 0, rounding: str = "sr",
              cfg: Config | None = None) -> list:
    """The pass lengths run() takes for these arguments (host logic of the
    library, no GPU work)."""
    nz, ny, nx = shape
    code = {torch.float64: F64, torch.float32: F32}.get(dtype, BF16 if rounding == "sr" else BF16_RNE)
    n = _lib.diff3d_pass_plan(nx, ny, nz, int(nt), int(ckpt_every), code, _ccfg(cfg), None, 0)
    if n < 0:
        raise Diff3dError(n, "pass_plan")
    out = (ctypes.c_int * max(n, 1))()
    _lib.diff3d_pass_plan(nx, ny, nz, int(nt), int(ckpt_every), code, _ccfg(cfg), out, n)
    return list(out[:n])


def run(T: torch.Tensor, T2: torch.Tensor, Ci: torch.Tensor, lam: float, dt: float, rdx: float, rdy: float,
        rdz: float, nt: int, rounding: str = "sr", ckpt: torch.Tensor | None = None, ckpt_every: int = 0,
        cfg: Config | None = None) -> None:
    """nt steps with the swap; the result is left in T (T2 is scratch).
    ``ckpt`` (a uint8 device buffer, e.g. an adjoint workspace) receives
    T_{j*ckpt_every} for j >= 1."""
    _field(T, "T")
    _field(T2, "T2", T)
    _field(Ci, "Ci", T)
    nz, ny, nx = T.shape
    if ckpt is not None:
        if not isinstance(ckpt, torch.Tensor) or not ckpt.is_cuda or not ckpt.is_contiguous() or \
                ckpt.device != T.device:
            raise ValueError("ckpt must be a contiguous GPU buffer on T's device")
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1 with a checkpoint buffer")
        nck = (nt + ckpt_every - 1) // ckpt_every if nt > 0 else 0
        stride = (T.numel() * T.element_size() + 255) // 256 * 256
        if ckpt.numel() * ckpt.element_size() < max(nck - 1, 0) * stride:
            raise ValueError("ckpt buffer too small for %d checkpoints" % max(nck - 1, 0))
    with _on(T):
        _check(_lib.diff3d_run(_p(T), _p(T2), _p(Ci), nx, ny, nz, lam, dt, rdx, rdy, rdz, int(nt), _code(T, rounding),
                               _stream(T), _p(ckpt), int(ckpt_every), _ccfg(cfg)), "run")


def adjoint_workspace_bytes(shape, nt: int, ckpt_every: int, dtype: torch.dtype, cfg: Config | None = None) -> int:
    nz, ny, nx = shape
    code = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[dtype]
    return int(_lib.diff3d_adjoint_workspace_bytes(nx, ny, nz, int(nt), int(ckpt_every), code, _ccfg(cfg)))


def adjoint_run(T0, Ci, gTnt, gT0, gCi, workspace, ckpt_ready: bool, lam, dt, rdx, rdy, rdz, nt: int,
                ckpt_every: int, cfg: Config | None = None) -> None:
    """Reverse sweep: gT0 = dL/dT0 and gCi = dL/dCi from gTnt = dL/dT_nt.
    ``workspace`` is a contiguous device buffer on T0's device of at least
    adjoint_workspace_bytes(..., cfg) bytes."""
    _field(T0, "T0")
    for name, t in (("Ci", Ci), ("gTnt", gTnt), ("gT0", gT0), ("gCi", gCi)):
        _field(t, name, T0)
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or not workspace.is_contiguous() or \
            workspace.device != T0.device:
        raise ValueError("workspace must be a contiguous GPU buffer on T0's device")
    nz, ny, nx = T0.shape
    with _on(T0):
        _check(_lib.diff3d_adjoint_run(_p(T0), _p(Ci), _p(gTnt), _p(gT0), _p(gCi), _p(workspace),
                                       workspace.numel() * workspace.element_size(),
                                       int(bool(ckpt_ready)), nx, ny, nz, lam, dt, rdx, rdy, rdz, int(nt),
                                       int(ckpt_every), _code(T0), _stream(T0), _ccfg(cfg)), "adjoint_run")


def loss(T: torch.Tensor, Tt: torch.Tensor, seed: torch.Tensor | None = None) -> torch.Tensor:
    """0.5*||T - Tt||^2 accumulated in FP64 on the GPU (0-d float64 tensor);
    writes T - Tt into ``seed`` when given."""
    _field(T, "T")
    _field(Tt, "Tt", T)
    if seed is not None:
        _field(seed, "seed", T)
    acc = _acc(T.device)
    with _on(T):
        _check(_lib.diff3d_loss(_p(T), _p(Tt), _p(seed), T.numel(), _code(T), _p(acc), _stream(T)), "loss")
    return acc[0]


def loss_into(out: torch.Tensor, T: torch.Tensor, Tt: torch.Tensor, seed: torch.Tensor | None = None) -> None:
    """The loss of loss() written into ``out`` (a float64 device tensor of at
    least one element), without caller scratch: the library's fixed per-GPU
    array holds the partial sums, so calls that overlap on one GPU race."""
    _field(T, "T")
    _field(Tt, "Tt", T)
    if seed is not None:
        _field(seed, "seed", T)
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64 or out.numel() < 1 or \
            not out.is_contiguous() or out.device != T.device:
        raise ValueError("out must be a contiguous float64 tensor on T's device")
    with _on(T):
        _check(_lib.diff3d_loss_noalloc(_p(T), _p(Tt), _p(seed), T.numel(), _code(T), _p(out), _stream(T)),
               "loss_noalloc")


def norm2(x: torch.Tensor) -> torch.Tensor:
    """||x||^2 accumulated in FP64 on the GPU (0-d float64 tensor)."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    acc = _acc(x.device)
    with _on(x):
        _check(_lib.diff3d_norm2(_p(x), x.numel(), _code(x), _p(acc), _stream(x)), "norm2")
    return acc[0]


def copy_(dst: torch.Tensor, src: torch.Tensor) -> None:
    """Device copy through the library's streaming copy kernel (contiguous
    GPU tensors on one device)."""
    for name, t in (("dst", dst), ("src", src)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous GPU tensor" % name)
    if dst.device != src.device:
        raise ValueError("dst and src must be on one device")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    with _on(src):
        _check(_lib.diff3d_copy(_p(dst), _p(src), nbytes, _stream(src)), "copy")


class Diffuse3D(torch.autograd.Function):
    """T_nt = nt steps of the Fig. 1 scheme from T0 with Ci; differentiable in
    T0 and Ci through the library's checkpointed reverse sweep (a checkpoint
    every ``ckpt_every`` steps, recomputation in between)."""

    @staticmethod
    def forward(ctx, T0, Ci, lam, dt, rdx, rdy, rdz, nt, ckpt_every, cfg=None):
        if T0.dtype not in (torch.float64, torch.float32):
            raise TypeError("gradients are supported for float64 and float32 fields")
        T0 = T0.contiguous()
        Ci = Ci.contiguous()
        T = T0.clone()
        T2 = torch.empty_like(T0)
        ws_bytes = adjoint_workspace_bytes(T0.shape, nt, ckpt_every, T0.dtype, cfg)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=T0.device)
        run(T, T2, Ci, lam, dt, rdx, rdy, rdz, nt, ckpt=ws, ckpt_every=ckpt_every, cfg=cfg)
        ctx.save_for_backward(T0, Ci)
        ctx.ws = ws
        ctx.cfg = cfg
        ctx.args = (lam, dt, rdx, rdy, rdz, int(nt), int(ckpt_every))
        return T

    @staticmethod
    def backward(ctx, gT):
        T0, Ci = ctx.saved_tensors
        lam, dt, rdx, rdy, rdz, nt, ce = ctx.args
        gT = gT.contiguous()
        gT0 = torch.empty_like(T0)
        gCi = torch.empty_like(Ci)
        adjoint_run(T0, Ci, gT, gT0, gCi, ctx.ws, True, lam, dt, rdx, rdy, rdz, nt, ce, cfg=ctx.cfg)
        ctx.ws = None
        return gT0, gCi, None, None, None, None, None, None, None, None


def diffuse(T0, Ci, lam, dt, rdx, rdy, rdz, nt, ckpt_every=None, cfg: Config | None = None):
    """Differentiable nt-step diffusion; ckpt_every defaults to about sqrt(nt)."""
    if ckpt_every is None:
        ckpt_every = max(1, int(round(nt ** 0.5)))
    return Diffuse3D.apply(T0, Ci, lam, dt, rdx, rdy, rdz, nt, ckpt_every, cfg)
