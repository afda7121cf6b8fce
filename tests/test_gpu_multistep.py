"""S-step passes (temporal blocking over 2..4 steps) on the GPU.

Intermediate states are rounded exactly as storing them would round them, so
an S-step pass must give the bits of S single steps: FP64 against the oracle,
the other storage types against the naive kernel with the same random draws."""
import os

import numpy as np
import pytest

import oracle
from helpers import instantiated_configs, interior_mask, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16_rne": torch.bfloat16}
ENV = ("DIFF3D_SCFG", "DIFF3D_SZLEN", "DIFF3D_ZCFG", "DIFF3D_ZLEN", "DIFF3D_TCFG", "DIFF3D_TZLEN")


@pytest.fixture(autouse=True)
def _reset(lib):
    saved = {k: os.environ.get(k) for k in ENV}
    lib.set_kernel(lib.KERNEL_AUTO)
    lib.set_pass_steps(0)
    yield
    lib.set_kernel(lib.KERNEL_AUTO)
    lib.set_pass_steps(0)
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def _inputs(shape, seed=0):
    nz, ny, nx = shape
    rng = np.random.default_rng(300 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(nx, ny, nz, Ci, ly=1.1, lz=0.9)
    return T0, Ci, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def _gpu_run(lib, T0, Ci, s, nt, dtype=torch.float64, rounding="sr"):
    T = to_dev(T0, dtype)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, dtype), *_sc(s), nt, rounding=rounding)
    torch.cuda.synchronize()
    return T


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
    tdt, rounding = TDT[dtype], ("rne" if dtype == "bf16_rne" else "sr")
    shape = (15, 61, 150)
    T0, Ci, s = _inputs(shape, seed=sum(cfg) + zlen)
    nt = 2 * S + 1
    os.environ["DIFF3D_SZLEN"] = str(zlen)
    os.environ["DIFF3D_SCFG"] = "%d,%d,%d,%d" % (W0, H0, NTH, NT)
    lib.set_kernel(lib.KERNEL_TBS)
    lib.set_pass_steps(S)
    lib.set_sr_seed(91, 3)
    T = _gpu_run(lib, T0, Ci, s, nt, dtype=tdt, rounding=rounding)
    if dtype == "f64":
        ref = oracle.forward(T0, Ci, *_sc(s), nt)
        np.testing.assert_array_equal(to_host(T), ref)
    else:
        lib.set_kernel(lib.KERNEL_NAIVE)
        lib.set_sr_seed(91, 3)
        R = _gpu_run(lib, T0, Ci, s, nt, dtype=tdt, rounding=rounding)
        assert torch.equal(T, R)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16_rne"])
@pytest.mark.parametrize("nsteps", [1, 2, 3, 4])
@pytest.mark.parametrize("kernel", ["auto", "tbs"])
def test_stepn_equals_single_steps(lib, dtype, nsteps, kernel):
    """diff3d_stepn writes the interior of T2 with the state nsteps steps on,
    bit-identical to nsteps diff3d_step calls, leaves T2's boundary alone
    and advances the stochastic-rounding step index by nsteps."""
    tdt, rounding = TDT[dtype], ("rne" if dtype == "bf16_rne" else "sr")
    shape = (17, 45, 200)
    T0, Ci, s = _inputs(shape, seed=nsteps)
    T, C = to_dev(T0, tdt), to_dev(Ci, tdt)
    lib.set_sr_seed(8, 100)
    R = T.clone()
    for _ in range(nsteps):
        M = R.clone()
        lib.step(M, R, C, *_sc(s), rounding=rounding)
        R = M
    after_single = T.clone()
    lib.step(after_single, R, C, *_sc(s), rounding=rounding)     # next index: 100 + nsteps
    lib.set_kernel(lib.KERNEL_TBS if kernel == "tbs" else lib.KERNEL_AUTO)
    lib.set_sr_seed(8, 100)
    Q = torch.full_like(T, float("nan"))
    b = torch.from_numpy(~interior_mask(shape)).cuda()
    Q[b] = -5.0
    lib.stepn(Q, T, C, *_sc(s), nsteps, rounding=rounding)
    after_multi = T.clone()
    Qf = Q.clone()
    Qf[b] = R[b]
    lib.step(after_multi, Qf, C, *_sc(s), rounding=rounding)
    torch.cuda.synchronize()
    m = torch.from_numpy(interior_mask(shape)).cuda()
    assert torch.equal(Q[m], R[m])
    assert torch.all(Q[b] == -5.0)
    assert torch.equal(after_multi, after_single)


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (5, 70, 33), (9, 3, 130), (20, 66, 64), (6, 130, 7),
                                   (7, 65, 65), (9, 120, 121), (5, 33, 200), (6, 57, 177)])
def test_tbs_small_and_ragged(lib, S, shape):
    """S-step passes on grids with one or two interior planes, regions
    wider than the grid, a last region ending exactly on or one point past
    the grid's edge, ragged x and y tiles and one-plane z-chunks."""
    os.environ["DIFF3D_SZLEN"] = "1"
    lib.set_kernel(lib.KERNEL_TBS)
    lib.set_pass_steps(S)
    T0, Ci, s = _inputs(shape, seed=S)
    for nt in (S, S + 1, 2 * S + 3):
        ref = oracle.forward(T0, Ci, *_sc(s), nt)
        np.testing.assert_array_equal(to_host(_gpu_run(lib, T0, Ci, s, nt)), ref)


@pytest.mark.parametrize("S", [2, 3, 4])
def test_tbs_checkpoints_written(lib, S):
    """Passes are shortened so that every checkpointed state is stored."""
    lib.set_kernel(lib.KERNEL_TBS)
    lib.set_pass_steps(S)
    shape = (12, 30, 70)
    T0, Ci, s = _inputs(shape, seed=7)
    nt, C = 23, 5
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
    T = to_dev(T0, torch.float64)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, torch.float64), *_sc(s), nt, ckpt=ws, ckpt_every=C)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
    stride = (T.numel() * 8 + 255) // 256 * 256
    for j in range(1, (nt + C - 1) // C):
        field = ws[(j - 1) * stride:(j - 1) * stride + T.numel() * 8].view(torch.float64).reshape(shape)
        np.testing.assert_array_equal(to_host(field), oracle.forward(T0, Ci, *_sc(s), j * C))


def test_tbs_adjoint_bit_exact(lib):
    """The reverse sweep with the S-step kernel selected (checkpoints from
    S-step passes) is bit-identical to the oracle's."""
    lib.set_kernel(lib.KERNEL_TBS)
    lib.set_pass_steps(3)
    shape = (14, 20, 72)
    T0, Ci, s = _inputs(shape, seed=11)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(shape)
    nt, C = 17, 4
    gT0_ref, gCi_ref = oracle.reverse(T0, Ci, g, *_sc(s), nt)
    dev = lambda a: to_dev(a, torch.float64)
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
    T, T2 = dev(T0), torch.empty(shape, dtype=torch.float64, device="cuda")
    lib.run(T, T2, dev(Ci), *_sc(s), nt, ckpt=ws, ckpt_every=C)
    gT0, gCi = torch.empty_like(T), torch.empty_like(T)
    lib.adjoint_run(dev(T0), dev(Ci), dev(g), gT0, gCi, ws, True, *_sc(s), nt, C)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(gT0), gT0_ref)
    np.testing.assert_array_equal(to_host(gCi), gCi_ref)


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("shape", [(9, 40, 192), (9, 40, 190), (7, 33, 120), (6, 20, 64)])
def test_tbs_stochastic_rounding_draws(lib, S, shape):
    """Stochastic rounding in S-step passes draws the same Philox bits per
    point and step as single steps, whether a wave's blocks are evaluated
    together (rows on multiples of 8 or room for 9 blocks per level) or per
    point."""
    T0, Ci, s = _inputs(shape, seed=30 + S)
    lib.set_kernel(lib.KERNEL_TBS)
    lib.set_pass_steps(S)
    lib.set_sr_seed(0xABCDEF12345, 77)
    T = _gpu_run(lib, T0, Ci, s, 2 * S + 1, dtype=torch.bfloat16, rounding="sr")
    lib.set_kernel(lib.KERNEL_NAIVE)
    lib.set_sr_seed(0xABCDEF12345, 77)
    R = _gpu_run(lib, T0, Ci, s, 2 * S + 1, dtype=torch.bfloat16, rounding="sr")
    assert torch.equal(T, R)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nt,C", [(31, 7), (30, 14), (9, 4), (12, 6), (5, 1), (8, 8)])
def test_default_passes_checkpoints(lib, dtype, nt, C):
    """With the default pass length the time loop splits each stretch between
    checkpoints into passes of near-equal length and the pass reaching a
    checkpointed state writes it into its slot: every slot (boundary
    included) and the final state equal single steps (FP64: the oracle)."""
    tdt, rounding = TDT[dtype], "sr"
    shape = (11, 37, 90)
    T0, Ci, s = _inputs(shape, seed=nt + C)
    nbytes = {"f64": 8, "f32": 4, "bf16": 2}[dtype]

    def fill(kernel):
        lib.set_kernel(kernel)
        lib.set_sr_seed(5, 40)
        ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, tdt), dtype=torch.uint8, device="cuda")
        T = to_dev(T0, tdt)
        lib.run(T, torch.empty_like(T), to_dev(Ci, tdt), *_sc(s), nt, ckpt=ws, ckpt_every=C, rounding=rounding)
        torch.cuda.synchronize()
        stride = (T.numel() * nbytes + 255) // 256 * 256
        slots = [ws[(j - 1) * stride:(j - 1) * stride + T.numel() * nbytes].view(tdt).reshape(shape).clone()
                 for j in range(1, (nt + C - 1) // C)]
        return T, slots

    T, slots = fill(lib.KERNEL_AUTO)
    if dtype == "f64":
        np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
        for j, f in enumerate(slots, start=1):
            np.testing.assert_array_equal(to_host(f), oracle.forward(T0, Ci, *_sc(s), j * C))
    else:
        R, rslots = fill(lib.KERNEL_ZMARCH)
        assert torch.equal(T, R)
        for f, g in zip(slots, rslots):
            assert torch.equal(f, g)
