"""Shared test helpers: moving seeded numpy fields to the GPU, the stored
(FP32/BF16) form of a field for the emulator, sub-box oracle evaluation at
sampled points, and error measures."""
from __future__ import annotations

import numpy as np

import oracle


def to_dev(a: np.ndarray, dtype):
    """A numpy FP64 field on the GPU in `dtype`, rounded on the CPU (so the
    emulator can be given the very same stored values, see stored())."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype).contiguous().to("cuda")


def stored(a: np.ndarray, dtype) -> np.ndarray:
    """The stored values to_dev puts on the GPU, as the emulator takes them:
    float32, or BF16 bits as uint16."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype).contiguous()
    if dtype == torch.bfloat16:
        return t.view(torch.int16).numpy().view(np.uint16).copy()
    if dtype == torch.float32:
        return t.numpy().copy()
    raise ValueError("stored() is for the reduced-precision forms")


def bits(t) -> np.ndarray:
    """A GPU tensor's stored values for comparison with the emulator."""
    import torch
    h = t.detach().cpu().contiguous()
    if h.dtype == torch.bfloat16:
        return h.view(torch.int16).numpy().view(np.uint16)
    return h.numpy()


def storage_code(dtype, rounding="sr") -> int:
    import torch
    if dtype == torch.float32:
        return oracle.ST_F32
    if dtype == torch.bfloat16:
        return oracle.ST_BF16_SR if rounding == "sr" else oracle.ST_BF16_RNE
    raise ValueError(dtype)


def emulate_run(lib, T0, Ci, s, nt, dtype, rounding="sr", cfg=None, ckpt_every=0, T0s=None):
    """The emulator's result for lib.run with the same arguments: the pass
    lengths the library's host logic takes for them (lib.pass_plan), each
    pass in FP32 and its final state stored (and rounded).  T0s: stored
    initial values if they are not those of to_dev(T0)."""
    passes = lib.pass_plan(T0.shape, nt, dtype, ckpt_every=ckpt_every, rounding=rounding, cfg=cfg)
    seed = cfg.sr_seed if cfg is not None else 0
    step0 = cfg.sr_step if cfg is not None else 0
    a = stored(T0, dtype) if T0s is None else T0s
    return oracle.emulate_forward(a, stored(Ci, dtype), s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], passes,
                                  storage_code(dtype, rounding), seed=seed, step0=step0)


def to_host(t) -> np.ndarray:
    import torch
    return t.detach().to(dtype=torch.float64).cpu().numpy()


def interior_mask(shape):
    m = np.zeros(shape, bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def max_rel(a: np.ndarray, b: np.ndarray) -> float:
    """max_i |a_i - b_i| / |b_i| (b is the reference; floor 1e-300)."""
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def norm_rel(a: np.ndarray, b: np.ndarray) -> float:
    """max|a - b| / max|b|."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def box(point, radius, shape):
    """Index slices of the box of the given radius around point, clipped to
    the grid, and the point's position inside it."""
    sl, pos = [], []
    for p, n in zip(point, shape):
        lo, hi = max(0, p - radius), min(n, p + radius + 1)
        sl.append(slice(lo, hi))
        pos.append(p - lo)
    return tuple(sl), tuple(pos)


def oracle_forward_at(T0, Ci, s, nt, points):
    """T_nt at the given (iz, iy, ix) points from the oracle run on the box of
    radius nt around each point.  The box faces that are not domain faces are
    held at T0, which is wrong from step 1 on; the error travels one cell per
    step, so the centre, nt cells from those faces, is exact after nt steps
    (the same floating-point operations on the same values as a full run)."""
    out = []
    for p in points:
        sl, pos = box(p, max(nt, 2), T0.shape)
        T = oracle.forward(T0[sl], Ci[sl], s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
        out.append(T[pos])
    return np.array(out)


def oracle_reverse_at(T0, Ci, g, s, nt, points, keep=1):
    """(gT0, gCi) at the given points from the oracle reverse sweep on the box
    of radius nt+1 around each point: within nt steps the adjoint at the
    centre only sees points at distance <= nt, and the forward states it uses
    (centre and neighbours) are exact for the same reason as above."""
    a, b = [], []
    for p in points:
        sl, pos = box(p, max(nt + 1, 2), T0.shape)
        gT0, gCi = oracle.reverse(T0[sl], Ci[sl], g[sl], s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt,
                                  keep=keep)
        a.append(gT0[pos])
        b.append(gCi[pos])
    return np.array(a), np.array(b)


def sample_points(shape, rng, k, include_edges=True):
    nz, ny, nx = shape
    pts = []
    if include_edges:
        pts += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (1, 1, 1), (nz - 2, ny - 2, nx - 2), (0, ny // 2, nx // 2),
                (nz // 2, ny - 1, nx // 3), (nz // 3, 1, nx - 1)]
    for _ in range(k):
        pts.append((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    return pts


def csrc_text() -> str:
    """All host and kernel sources of the library, concatenated."""
    import os
    d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2211_15634_amd", "csrc")
    return "".join(open(os.path.join(d, f)).read() for f in sorted(os.listdir(d)) if f.endswith((".hip", ".hpp")))


def instantiated_configs(kind: str, size: int):
    """The tile configurations the library instantiates (read from its
    source): kind "FWD" -> [(V, R, NW, NT)], kind "ADJ" -> [(V, R, NW)]."""
    import os
    import re
    text = csrc_text().replace("\\\n", " ")
    m = re.search(r"#define DIFF3D_%s_CFGS_%d\(X\)(.*)" % (kind, size), text)
    assert m, (kind, size)
    return [tuple(int(v) for v in t.split(",")) for t in re.findall(r"X\(([\d ,]+)\)", m.group(1))]
