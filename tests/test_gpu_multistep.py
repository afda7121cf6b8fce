"""S-step passes (temporal blocking over 2..4 steps) on the GPU.

Inside a pass the intermediate states stay in the compute type, so FP64 and
FP32 passes give the bits of S single steps (FP64: the oracle's) and BF16
passes round once per pass, exactly as the oracle's emulator does with the
same pass lengths and random draws."""
import numpy as np
import pytest

import oracle
from helpers import bits, emulate_run, instantiated_configs, interior_mask, storage_code, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16_rne": torch.bfloat16}


def _rounding(dtype):
    return "rne" if dtype == "bf16_rne" else "sr"


def _inputs(shape, seed=0):
    nz, ny, nx = shape
    rng = np.random.default_rng(300 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(nx, ny, nz, Ci, ly=1.1, lz=0.9)
    return T0, Ci, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def _gpu_run(lib, T0, Ci, s, nt, dtype=torch.float64, rounding="sr", cfg=None):
    T = to_dev(T0, dtype)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, dtype), *_sc(s), nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    return T


def _check(lib, T, T0, Ci, s, nt, dtype, cfg, ckpt_every=0):
    if dtype == "f64":
        np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
    else:
        ref = emulate_run(lib, T0, Ci, s, nt, TDT[dtype], _rounding(dtype), cfg=cfg, ckpt_every=ckpt_every)
        np.testing.assert_array_equal(bits(T), ref)


def _cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4), ("bf16", 2), ("bf16_rne", 2)):
        for cfg in instantiated_configs("TBS", size):
            for zlen in (0, 1, 3):
                out.append((name, cfg, zlen))
    return out


@pytest.mark.parametrize("dtype,cfg,zlen", _cases())
def test_tbs_configs(lib, dtype, cfg, zlen):
    """Every instantiated S-step configuration and several z-chunk lengths
    (shorter and longer than the halo), over whole passes and a remainder."""
    S, W0, H0, NTH, NT = cfg
    shape = (15, 61, 150)
    T0, Ci, s = _inputs(shape, seed=sum(cfg) + zlen)
    nt = 2 * S + 1
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=S, sr_seed=91, sr_step=3,
                   tbs=lib.Tile(steps=S, p=(W0, H0, NTH, NT), zlen=zlen))
    T = _gpu_run(lib, T0, Ci, s, nt, dtype=TDT[dtype], rounding=_rounding(dtype), cfg=c)
    _check(lib, T, T0, Ci, s, nt, dtype, c)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16_rne"])
@pytest.mark.parametrize("nsteps", [1, 2, 3, 4])
@pytest.mark.parametrize("kernel", ["auto", "tbs"])
def test_stepn_semantics(lib, dtype, nsteps, kernel):
    """diff3d_stepn writes the interior of T2 with the state nsteps steps on
    and leaves T2's boundary alone: FP64/FP32 bit-identical to nsteps
    diff3d_step calls, BF16 to the emulator's single pass (drawing with
    index sr_step + nsteps - 1)."""
    tdt, rounding = TDT[dtype], _rounding(dtype)
    shape = (17, 45, 200)
    T0, Ci, s = _inputs(shape, seed=nsteps)
    T, C = to_dev(T0, tdt), to_dev(Ci, tdt)
    c = lib.Config(kernel=lib.KERNEL_TBS if kernel == "tbs" else lib.KERNEL_AUTO, sr_seed=8, sr_step=100)
    Q = torch.full_like(T, float("nan"))
    b = torch.from_numpy(~interior_mask(shape)).cuda()
    Q[b] = -5.0
    lib.stepn(Q, T, C, *_sc(s), nsteps, rounding=rounding, cfg=c)
    torch.cuda.synchronize()
    assert torch.all(Q[b] == -5.0)
    Qf = Q.clone()
    Qf[b] = T[b]
    if tdt in (torch.float64, torch.float32):
        R = T.clone()
        for j in range(nsteps):
            M = R.clone()
            lib.step(M, R, C, *_sc(s), rounding=rounding, cfg=c.replace(sr_step=100 + j))
            R = M
        torch.cuda.synchronize()
        assert torch.equal(Qf, R)
    else:
        ref = oracle.emulate_forward(stored(T0, tdt), stored(Ci, tdt), *_sc(s), [nsteps], storage_code(tdt, rounding),
                                     seed=8, step0=100)
        np.testing.assert_array_equal(bits(Qf), ref)


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (5, 70, 33), (9, 3, 130), (20, 66, 64), (6, 130, 7),
                                   (7, 65, 65), (9, 120, 121), (5, 33, 200), (6, 57, 177)])
def test_tbs_small_and_ragged(lib, S, shape):
    """S-step passes on grids with one or two interior planes, regions
    wider than the grid, a last region ending exactly on or one point past
    the grid's edge, ragged x and y tiles and one-plane z-chunks."""
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=S, tbs=lib.Tile(zlen=1))
    T0, Ci, s = _inputs(shape, seed=S)
    for nt in (S, S + 1, 2 * S + 3):
        ref = oracle.forward(T0, Ci, *_sc(s), nt)
        np.testing.assert_array_equal(to_host(_gpu_run(lib, T0, Ci, s, nt, cfg=c)), ref)
    for dtype in ("f32", "bf16"):
        T = _gpu_run(lib, T0, Ci, s, 2 * S + 3, dtype=TDT[dtype], cfg=c.replace(sr_seed=S))
        _check(lib, T, T0, Ci, s, 2 * S + 3, dtype, c.replace(sr_seed=S))


@pytest.mark.parametrize("S", [2, 3, 4])
def test_tbs_checkpoints_written(lib, S):
    """Passes are shortened so that every checkpointed state is stored."""
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=S)
    shape = (12, 30, 70)
    T0, Ci, s = _inputs(shape, seed=7)
    nt, C = 23, 5
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64, c), dtype=torch.uint8, device="cuda")
    T = to_dev(T0, torch.float64)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, torch.float64), *_sc(s), nt, ckpt=ws, ckpt_every=C, cfg=c)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
    stride = (T.numel() * 8 + 255) // 256 * 256
    for j in range(1, (nt + C - 1) // C):
        field = ws[(j - 1) * stride:(j - 1) * stride + T.numel() * 8].view(torch.float64).reshape(shape)
        np.testing.assert_array_equal(to_host(field), oracle.forward(T0, Ci, *_sc(s), j * C))


def test_tbs_adjoint_bit_exact(lib):
    """The reverse sweep with the S-step kernel selected (checkpoints from
    S-step passes) is bit-identical to the oracle's."""
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=3)
    shape = (14, 20, 72)
    T0, Ci, s = _inputs(shape, seed=11)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(shape)
    nt, C = 17, 4
    gT0_ref, gCi_ref = oracle.reverse(T0, Ci, g, *_sc(s), nt)
    dev = lambda a: to_dev(a, torch.float64)
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64, c), dtype=torch.uint8, device="cuda")
    T, T2 = dev(T0), torch.empty(shape, dtype=torch.float64, device="cuda")
    lib.run(T, T2, dev(Ci), *_sc(s), nt, ckpt=ws, ckpt_every=C, cfg=c)
    gT0, gCi = torch.empty_like(T), torch.empty_like(T)
    lib.adjoint_run(dev(T0), dev(Ci), dev(g), gT0, gCi, ws, True, *_sc(s), nt, C, cfg=c)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(gT0), gT0_ref)
    np.testing.assert_array_equal(to_host(gCi), gCi_ref)


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("shape", [(9, 40, 192), (9, 40, 190), (7, 33, 120), (6, 20, 64), (5, 9, 1000)])
def test_tbs_stochastic_rounding_draws(lib, S, shape):
    """Stochastic rounding in S-step passes draws the Philox bits the
    emulator draws for each stored point, whether or not rows start on a
    multiple of 8 points (a wave's blocks are evaluated together)."""
    T0, Ci, s = _inputs(shape, seed=30 + S)
    c = lib.Config(kernel=lib.KERNEL_TBS, pass_steps=S, sr_seed=0xABCDEF12345, sr_step=(1 << 32) - 2)
    T = _gpu_run(lib, T0, Ci, s, 2 * S + 1, dtype=torch.bfloat16, rounding="sr", cfg=c)
    _check(lib, T, T0, Ci, s, 2 * S + 1, "bf16", c)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16_rne"])
@pytest.mark.parametrize("nt,C", [(31, 7), (30, 14), (9, 4), (12, 6), (5, 1), (8, 8)])
def test_default_passes_checkpoints(lib, dtype, nt, C):
    """With the default pass length the time loop splits each stretch between
    checkpoints into passes of near-equal length and the pass reaching a
    checkpointed state writes it into its slot: every slot (boundary
    included) and the final state equal the oracle (FP64) or the emulator
    run to that state with the same passes."""
    tdt, rounding = TDT[dtype], _rounding(dtype)
    shape = (11, 37, 90)
    T0, Ci, s = _inputs(shape, seed=nt + C)
    nbytes = {torch.float64: 8, torch.float32: 4, torch.bfloat16: 2}[tdt]
    c = lib.Config(sr_seed=5, sr_step=40)
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
    T = to_dev(T0, tdt)
    lib.run(T, torch.empty_like(T), to_dev(Ci, tdt), *_sc(s), nt, ckpt=ws, ckpt_every=C, rounding=rounding, cfg=c)
    torch.cuda.synchronize()
    stride = (T.numel() * nbytes + 255) // 256 * 256
    slots = [ws[(j - 1) * stride:(j - 1) * stride + T.numel() * nbytes].view(tdt).reshape(shape)
             for j in range(1, (nt + C - 1) // C)]
    if dtype == "f64":
        np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
        for j, f in enumerate(slots, start=1):
            np.testing.assert_array_equal(to_host(f), oracle.forward(T0, Ci, *_sc(s), j * C))
    else:
        passes = lib.pass_plan(shape, nt, tdt, ckpt_every=C, rounding=rounding, cfg=c)
        ends = np.cumsum(passes)
        assert all(j * C in ends for j in range(1, len(slots) + 1))
        code = storage_code(tdt, rounding)
        np.testing.assert_array_equal(
            bits(T), oracle.emulate_forward(stored(T0, tdt), stored(Ci, tdt), *_sc(s), passes, code, 5, 40))
        for j, f in enumerate(slots, start=1):
            upto = passes[:int(np.searchsorted(ends, j * C)) + 1]
            assert sum(upto) == j * C
            ref = oracle.emulate_forward(stored(T0, tdt), stored(Ci, tdt), *_sc(s), upto, code, 5, 40)
            np.testing.assert_array_equal(bits(f), ref)
