"""The time loops (3-D and 2-D) and the reverse sweep under stream capture.

diff3d_run, diff2d_run and diff3d_adjoint_run enqueue only kernels on the caller's
stream (fills and copies are kernels too: no memset or memcpy nodes, no host
synchronisation, no allocation), so a caller can capture a call once into a
graph and replay it, which removes the per-launch cost on small grids.  Every
replay is checked bit for bit against the eager call, with eager work and
synchronisations between the replays; the captured arguments (the config's
stochastic-rounding seed and step included) are fixed, so each replay draws
the same random bits as the eager call.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

INT_VIEW = {torch.float64: torch.int64, torch.float32: torch.int32, torch.bfloat16: torch.int16}


def _capture(fn):
    """Warm up on a side stream, then capture fn into a graph."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1 + 0.5 * rng.random(shape))
    return T0, Ci


def _same_bits(a, b):
    return torch.equal(a.view(INT_VIEW[a.dtype]), b.view(INT_VIEW[b.dtype]))


@pytest.mark.parametrize("dtype,rounding", [(torch.float64, "sr"), (torch.float32, "sr"),
                                            (torch.bfloat16, "sr"), (torch.bfloat16, "rne")],
                         ids=("f64", "f32", "bf16_sr", "bf16_rne"))
@pytest.mark.parametrize("shape,nt", [((64, 64, 64), 100), ((13, 37, 150), 23)], ids=("64cube", "ragged"))
def test_run_graph_replays(lib, dtype, rounding, shape, nt):
    print("graph run", shape, nt, dtype, rounding, flush=True)
    T0h, Cih = _fields(shape, seed=21)
    nz, ny, nx = shape
    s = oracle.scalars(nx, ny, nz, Cih)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    cfg = lib.Config(sr_seed=77, sr_step=5)
    T0 = torch.from_numpy(T0h).to(dtype).cuda()
    Ci = torch.from_numpy(Cih).to(dtype).cuda()
    ref = T0.clone()
    lib.run(ref, torch.empty_like(ref), Ci, *sc, nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    T, T2 = T0.clone(), torch.empty_like(T0)
    g = _capture(lambda: lib.run(T, T2, Ci, *sc, nt, rounding=rounding, cfg=cfg))
    for rep in range(3):
        T.copy_(T0)
        torch.cuda.synchronize()
        g.replay()
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert _same_bits(T, ref), "replay %d differs from the eager run" % rep
    if dtype == torch.float64:
        assert np.array_equal(ref.cpu().numpy(), oracle.forward(T0h, Cih, *sc, nt))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=("f64", "f32"))
def test_adjoint_graph_replays(lib, dtype):
    shape, nt, C = (19, 24, 70), 40, 14
    print("graph adjoint", shape, nt, C, dtype, flush=True)
    T0h, Cih = _fields(shape, seed=22)
    g0 = np.random.default_rng(23).standard_normal(shape)
    nz, ny, nx = shape
    s = oracle.scalars(nx, ny, nz, Cih)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    dev = lambda a: torch.from_numpy(a).to(dtype).cuda()
    T0, Ci, gT = dev(T0h), dev(Cih), dev(g0)
    ws = torch.empty(lib.adjoint_workspace_bytes(shape, nt, C, dtype), dtype=torch.uint8, device="cuda")
    r0, rc = torch.empty_like(T0), torch.empty_like(T0)
    lib.adjoint_run(T0, Ci, gT, r0, rc, ws, False, *sc, nt, C)
    torch.cuda.synchronize()
    gT0, gCi = torch.empty_like(T0), torch.empty_like(T0)
    g = _capture(lambda: lib.adjoint_run(T0, Ci, gT, gT0, gCi, ws, False, *sc, nt, C))
    for rep in range(3):
        gT0.fill_(float("nan"))
        gCi.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert _same_bits(gT0, r0) and _same_bits(gCi, rc), "replay %d differs from the eager sweep" % rep
    if dtype == torch.float64:
        ra, rb = oracle.reverse(T0h, Cih, g0, *sc, nt)
        assert np.array_equal(r0.cpu().numpy(), ra) and np.array_equal(rc.cpu().numpy(), rb)


@pytest.mark.parametrize("dtype,rounding", [(torch.float64, "sr"), (torch.float32, "sr"),
                                            (torch.bfloat16, "sr"), (torch.bfloat16, "rne")],
                         ids=("f64", "f32", "bf16_sr", "bf16_rne"))
@pytest.mark.parametrize("nt", [16, 23])
def test_run2d_graph_replays(lib, dtype, rounding, nt):
    """The 2-D time loop (an even and an odd number of passes: the loop then
    starts from a boundary copy or from a full copy) captured and replayed."""
    shape = (131, 517)
    print("graph run2d", shape, nt, dtype, rounding, flush=True)
    ny, nx = shape
    rng = np.random.default_rng(24)
    T0h = rng.random(shape)
    Cih = 0.5 * (1 + 0.5 * rng.random(shape))
    s = oracle.scalars2d(nx, ny, Cih)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"])
    cfg = lib.Config(sr_seed=5, sr_step=2)
    T0 = torch.from_numpy(T0h).to(dtype).cuda()
    Ci = torch.from_numpy(Cih).to(dtype).cuda()
    ref = T0.clone()
    lib.run2d(ref, torch.empty_like(ref), Ci, *sc, nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    T, T2 = T0.clone(), torch.empty_like(T0)
    g = _capture(lambda: lib.run2d(T, T2, Ci, *sc, nt, rounding=rounding, cfg=cfg))
    for rep in range(3):
        T.copy_(T0)
        torch.cuda.synchronize()
        g.replay()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert _same_bits(T, ref), "replay %d differs from the eager run" % rep
    if dtype == torch.float64:
        assert np.array_equal(ref.cpu().numpy(), oracle.forward2d(T0h, Cih, *sc, nt))
