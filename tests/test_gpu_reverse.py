"""Fused reverse passes (S adjoint steps per pass, forward states recomputed
on chip) on the GPU.  Same operation order as the single reverse step, so
FP64 must be bit-identical to the oracle's reverse sweep and FP32 to the
oracle's FP32 emulation of it."""
import numpy as np
import pytest

import oracle
from helpers import instantiated_configs, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(shape, seed=0):
    nz, ny, nx = shape
    rng = np.random.default_rng(400 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    g = rng.standard_normal(shape)
    s = oracle.scalars(nx, ny, nz, Ci, lx=0.9, ly=1.2, lz=1.0)
    return T0, Ci, g, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def _adjoint(lib, T0, Ci, g, s, nt, C, dtype=torch.float64, ready=False, cfg=None):
    T0d, Cid, gd = to_dev(T0, dtype), to_dev(Ci, dtype), to_dev(g, dtype)
    ws = torch.empty(lib.adjoint_workspace_bytes(T0.shape, nt, C, dtype, cfg), dtype=torch.uint8, device="cuda")
    if ready:
        T = T0d.clone()
        lib.run(T, torch.empty_like(T), Cid, *_sc(s), nt, ckpt=ws, ckpt_every=C, cfg=cfg)
    gT0 = torch.full_like(T0d, float("nan"))
    gCi = torch.full_like(T0d, float("nan"))
    lib.adjoint_run(T0d, Cid, gd, gT0, gCi, ws, ready, *_sc(s), nt, C, cfg=cfg)
    torch.cuda.synchronize()
    return to_host(gT0), to_host(gCi)


def _reference(T0, Ci, g, s, nt, dtype):
    if dtype == torch.float64:
        return oracle.reverse(T0, Ci, g, *_sc(s), nt)
    f32 = lambda a: stored(a, torch.float32)
    a, b = oracle.emulate_reverse32(f32(T0), f32(Ci), f32(g), *_sc(s), nt)
    return a.astype(np.float64), b.astype(np.float64)


def _cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4)):
        for cfg in instantiated_configs("REV", size):
            for zlen in (0, 1, 2, 3, 4):
                out.append((name, cfg, zlen))
    return out


@pytest.mark.parametrize("dtype,cfg,zlen", _cases())
def test_rev_configs(lib, dtype, cfg, zlen):
    """Every instantiated fused-pass configuration and several z-chunk
    lengths, with segments whose first pass is shorter (one or two steps).
    A chunk of zlen planes takes zlen + 2S plane iterations, so zlen = 1..4
    ends the four-way unrolled plane loop after each of its four copies."""
    S, W0, H0, NTH = cfg
    tdt = torch.float64 if dtype == "f64" else torch.float32
    T0, Ci, g, s = _inputs((13, 45, 150), seed=sum(cfg) + zlen)
    nt, C = 11, 7
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=S, rev=lib.Tile(steps=S, p=(W0, H0, NTH, 0), zlen=zlen))
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C, dtype=tdt, cfg=c)
    rT0, rCi = _reference(T0, Ci, g, s, nt, tdt)
    np.testing.assert_array_equal(gT0, rT0)
    np.testing.assert_array_equal(gCi, rCi)


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (5, 70, 33), (9, 3, 130), (6, 66, 64), (7, 65, 65),
                                   (6, 57, 177), (5, 33, 200)])
def test_rev_small_and_ragged(lib, P, shape):
    """Grids with one or two interior planes, regions wider than the grid or
    ending on its edge, one-plane z-chunks; checkpoints from the time loop
    and from the sweep's own forward pass."""
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=P, rev=lib.Tile(zlen=1))
    T0, Ci, g, s = _inputs(shape, seed=P)
    for nt, C in ((2, 2), (5, 3), (9, 9), (8, 4)):
        rT0, rCi = oracle.reverse(T0, Ci, g, *_sc(s), nt)
        for ready in (False, True):
            gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C, ready=ready, cfg=c)
            np.testing.assert_array_equal(gT0, rT0)
            np.testing.assert_array_equal(gCi, rCi)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rev_default_matches_oracle(lib, dtype):
    """The default (fused) reverse sweep and the single-step sweep both equal
    the oracle (FP64) or its FP32 emulation bit for bit on a grid of several
    tiles and z-chunks, nt = 40, C = 14."""
    tdt = torch.float64 if dtype == "f64" else torch.float32
    T0, Ci, g, s = _inputs((40, 70, 140), seed=21)
    rT0, rCi = _reference(T0, Ci, g, s, 40, tdt)
    for c in (None, lib.Config(kernel=lib.KERNEL_ZMARCH)):
        gT0, gCi = _adjoint(lib, T0, Ci, g, s, 40, 14, dtype=tdt, ready=True, cfg=c)
        np.testing.assert_array_equal(gT0, rT0)
        np.testing.assert_array_equal(gCi, rCi)
