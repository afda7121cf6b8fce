"""Forward step and time loop on the GPU against the oracle.

The FP64 kernels evaluate the step in the oracle's operation order with no
contraction, so FP64 results must be bit-identical to the oracle's.  The
FP32 and BF16 forms must be bit-identical to the oracle's FP32 emulator
with the same storage, pass lengths and stochastic-rounding draws."""
import numpy as np
import pytest

import oracle
import workloads
from helpers import (bits, emulate_run, instantiated_configs, interior_mask, oracle_forward_at, sample_points,
                     storage_code, stored, to_dev, to_host)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [  # (nz, ny, nx): several tiles, ragged tails, minimal grids
    (7, 9, 131),      # nx odd: narrow (V=1) path
    (21, 37, 128),    # wide vectors, ragged y tile
    (40, 66, 256),
    (3, 3, 3),        # a single interior point
    (5, 3, 64),
    (18, 70, 70),     # nx % 16 != 0 for bf16/fp32 wide vectors
]

TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16_rne": torch.bfloat16}


def _rounding(dtype):
    return "rne" if dtype == "bf16_rne" else "sr"


def _inputs(shape, seed=0):
    nz, ny, nx = shape
    rng = np.random.default_rng(100 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(nx, ny, nz, Ci, ly=1.3, lz=0.8)
    return T0, Ci, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def _gpu_run(lib, T0, Ci, s, nt, dtype=torch.float64, rounding="sr", cfg=None):
    T = to_dev(T0, dtype)
    T2 = torch.empty_like(T)
    C = to_dev(Ci, dtype)
    lib.run(T, T2, C, *_sc(s), nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    return T, T2


def _check(lib, T, T0, Ci, s, nt, dtype, cfg):
    """T (GPU, after run) against the oracle (FP64) or the emulator."""
    if dtype == "f64":
        np.testing.assert_array_equal(to_host(T), oracle.forward(T0, Ci, *_sc(s), nt))
    else:
        ref = emulate_run(lib, T0, Ci, s, nt, TDT[dtype], _rounding(dtype), cfg=cfg)
        np.testing.assert_array_equal(bits(T), ref)


KERNELS = {"naive": 1, "zmarch": 2, "tb2": 3}


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kernel", ["naive", "zmarch", "tb2"])
def test_fp64_bit_exact(lib, shape, kernel):
    cfg = lib.Config(kernel=KERNELS[kernel])
    T0, Ci, s = _inputs(shape)
    for nt in (1, 2, 6, 7):
        ref = oracle.forward(T0, Ci, *_sc(s), nt)
        T, _ = _gpu_run(lib, T0, Ci, s, nt, cfg=cfg)
        np.testing.assert_array_equal(to_host(T), ref)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "bf16_rne"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kernel", ["naive", "zmarch", "tb2", "auto"])
def test_reduced_precision_bit_exact(lib, dtype, shape, kernel):
    """FP32 and BF16 storage: every kernel equals the emulator bit for bit
    (same FP32 operation order; BF16 rounded once per pass, with the same
    Philox draws under stochastic rounding)."""
    cfg = lib.Config(kernel={"auto": 0, **KERNELS}[kernel], sr_seed=0x1234_5678_9ABC, sr_step=17)
    T0, Ci, s = _inputs(shape, seed=4)
    for nt in (1, 2, 7):
        T, _ = _gpu_run(lib, T0, Ci, s, nt, dtype=TDT[dtype], rounding=_rounding(dtype), cfg=cfg)
        _check(lib, T, T0, Ci, s, nt, dtype, cfg)


def _cfg_cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4), ("bf16", 2), ("bf16_rne", 2)):
        for cfg in instantiated_configs("FWD", size):
            for zlen in (0, 1, 3):
                out.append((name, cfg, zlen))
    return out


@pytest.mark.parametrize("dtype,cfg,zlen", _cfg_cases())
def test_zmarch_configs(lib, dtype, cfg, zlen):
    """Every instantiated z-march configuration and several z-chunk lengths,
    bit-identical to the oracle (FP64) or the emulator."""
    shape = (13, 45, 192)
    T0, Ci, s = _inputs(shape, seed=sum(cfg) + zlen)
    c = lib.Config(kernel=lib.KERNEL_ZMARCH, sr_seed=77, zmarch=lib.Tile(p=cfg, zlen=zlen))
    T, _ = _gpu_run(lib, T0, Ci, s, 4, dtype=TDT[dtype], rounding=_rounding(dtype), cfg=c)
    _check(lib, T, T0, Ci, s, 4, dtype, c)


def _tb2_cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4), ("bf16", 2), ("bf16_rne", 2)):
        for cfg in instantiated_configs("TB2", size):
            for zlen in (0, 1, 3):
                out.append((name, cfg, zlen))
    return out


@pytest.mark.parametrize("dtype,cfg,zlen", _tb2_cases())
def test_tb2_configs(lib, dtype, cfg, zlen):
    """Every instantiated two-step configuration and several z-chunk lengths
    (two passes of two steps and a single step), bit-identical to the oracle
    (FP64) or the emulator."""
    shape = (14, 37, 192)
    T0, Ci, s = _inputs(shape, seed=sum(cfg) + zlen + 50)
    c = lib.Config(kernel=lib.KERNEL_TB2, sr_seed=78, tb2=lib.Tile(p=cfg, zlen=zlen))
    T, _ = _gpu_run(lib, T0, Ci, s, 5, dtype=TDT[dtype], rounding=_rounding(dtype), cfg=c)
    _check(lib, T, T0, Ci, s, 5, dtype, c)


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (5, 70, 33), (9, 3, 130), (20, 66, 64)])
def test_tb2_small_and_ragged(lib, shape):
    """Two-step passes on grids with one or two interior planes, ragged x
    and y tiles and z-chunks shorter than the halo."""
    c = lib.Config(kernel=lib.KERNEL_TB2, tb2=lib.Tile(zlen=1))
    T0, Ci, s = _inputs(shape, seed=3)
    for nt in (2, 4, 9):
        ref = oracle.forward(T0, Ci, *_sc(s), nt)
        T, _ = _gpu_run(lib, T0, Ci, s, nt, cfg=c)
        np.testing.assert_array_equal(to_host(T), ref)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16_rne"])
def test_step2_semantics(lib, dtype):
    """diff3d_step2 writes the interior of T2 with the state two steps on and
    leaves T2's boundary alone: FP64/FP32 bit-identical to two diff3d_step
    calls, BF16 to the emulator's one two-step pass (drawing with index
    sr_step + 1)."""
    tdt, rounding = TDT[dtype], _rounding(dtype)
    shape = (19, 34, 256)
    T0, Ci, s = _inputs(shape, seed=9)
    T, C = to_dev(T0, tdt), to_dev(Ci, tdt)
    c = lib.Config(sr_seed=5, sr_step=40)
    Q = torch.full_like(T, float("nan"))
    b = torch.from_numpy(~interior_mask(shape)).cuda()
    Q[b] = -3.0
    lib.step2(Q, T, C, *_sc(s), rounding=rounding, cfg=c)
    torch.cuda.synchronize()
    m = torch.from_numpy(interior_mask(shape)).cuda()
    assert torch.all(Q[b] == -3.0)
    Qf = Q.clone()
    Qf[b] = T[b]
    if tdt in (torch.float64, torch.float32):
        M = T.clone()
        lib.step(M, T, C, *_sc(s), rounding=rounding, cfg=c)
        R = M.clone()
        lib.step(R, M, C, *_sc(s), rounding=rounding, cfg=c.replace(sr_step=41))
        torch.cuda.synchronize()
        assert torch.equal(Q[m], R[m])
    else:
        ref = oracle.emulate_forward(stored(T0, tdt), stored(Ci, tdt), *_sc(s), [2], storage_code(tdt, rounding),
                                     seed=5, step0=40)
        np.testing.assert_array_equal(bits(Qf), ref)


def test_narrow_fallback_ragged_rows(lib):
    """A wide configuration on rows that are not a multiple of its vector
    width falls back to one point per lane, still bit-exact."""
    shape = (9, 21, 190)
    T0, Ci, s = _inputs(shape)
    c = lib.Config(kernel=lib.KERNEL_ZMARCH, zmarch=lib.Tile(p=(2, 4, 4, 0)))
    ref = oracle.forward(T0, Ci, *_sc(s), 3)
    T, _ = _gpu_run(lib, T0, Ci, s, 3, cfg=c)
    np.testing.assert_array_equal(to_host(T), ref)
    # the same with one point per lane requested explicitly
    T, _ = _gpu_run(lib, T0, Ci, s, 3, cfg=c.replace(narrow=True))
    np.testing.assert_array_equal(to_host(T), ref)


def test_uniform64_config_bit_exact(lib):
    """64^3 FP64, T0 ~ U[0,1] (seed 0), Ci = 0.5, dt by the 6.1 rule, nt = 100."""
    T0, Ci = workloads.uniform_const(64, 64, 64)
    s = oracle.scalars(64, 64, 64, Ci)
    ref = oracle.forward(T0, Ci, *_sc(s), 100)
    T, _ = _gpu_run(lib, T0, Ci, s, 100)
    np.testing.assert_array_equal(to_host(T), ref)


def test_scalars_from_device_max(lib):
    T0, Ci = workloads.bump(48, 40, 36)
    a = oracle.scalars(48, 40, 36, Ci)
    b = lib.problem_scalars(to_dev(Ci, torch.float64))
    assert a == b
    # max over the whole array, boundary included
    Ci2 = Ci.copy()
    Ci2[-1, -1, -1] = 3.0
    assert float(lib.field_max(to_dev(Ci2, torch.float64))) == 3.0
    assert float(lib.field_max(to_dev(Ci2, torch.float32))) == 3.0


def test_step_sentinels(lib):
    """One step writes every interior point and no boundary point of T2."""
    for kernel in (lib.KERNEL_NAIVE, lib.KERNEL_ZMARCH):
        c = lib.Config(kernel=kernel)
        for shape in ((9, 17, 130), (12, 20, 128)):
            T0, Ci, s = _inputs(shape)
            for dt_ in (torch.float64, torch.float32, torch.bfloat16):
                T = to_dev(T0, dt_)
                C = to_dev(Ci, dt_)
                T2 = torch.full_like(T, float("nan"))
                m = torch.from_numpy(~interior_mask(shape)).cuda()
                T2[m] = -7.0
                lib.step(T2, T, C, *_sc(s), cfg=c)
                torch.cuda.synchronize()
                h = to_host(T2)
                assert np.all(np.isfinite(h[interior_mask(shape)]))
                assert np.all(h[~interior_mask(shape)] == -7.0)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16_rne"])
def test_constant_field_kept_exactly(lib, dtype):
    tdt = TDT[dtype]
    shape = (20, 33, 256)
    _, Ci, s = _inputs(shape)
    T0 = np.full(shape, 1.7)
    T, _ = _gpu_run(lib, T0, Ci, s, 9, dtype=tdt, rounding=_rounding(dtype))
    c = to_dev(T0, tdt)
    assert torch.equal(T, c)


def test_stateless_and_seeded(lib):
    """Two identical calls give identical bits (no state is kept between
    calls); the seed and the first step index select the random draws."""
    shape = (24, 48, 128)
    T0, Ci, s = _inputs(shape)
    c = lib.Config(sr_seed=99, sr_step=5)
    for tdt in (torch.float64, torch.float32, torch.bfloat16):
        a, _ = _gpu_run(lib, T0, Ci, s, 8, dtype=tdt, cfg=c)
        b, _ = _gpu_run(lib, T0, Ci, s, 8, dtype=tdt, cfg=c)
        assert torch.equal(a, b)
    for other in (c.replace(sr_seed=100), c.replace(sr_step=6)):
        d, _ = _gpu_run(lib, T0, Ci, s, 8, dtype=torch.bfloat16, cfg=other)
        assert not torch.equal(a, d)


def test_run_semantics(lib):
    shape = (10, 12, 64)
    T0, Ci, s = _inputs(shape)
    # nt = 0 leaves T alone
    T, _ = _gpu_run(lib, T0, Ci, s, 0)
    np.testing.assert_array_equal(to_host(T), T0)
    # odd nt: the result is still in T; T2's boundary was set from T
    T, T2 = _gpu_run(lib, T0, Ci, s, 3)
    ref = oracle.forward(T0, Ci, *_sc(s), 3)
    np.testing.assert_array_equal(to_host(T), ref)
    b = ~interior_mask(shape)
    np.testing.assert_array_equal(to_host(T2)[b], T0[b])
    # run(nt=1) equals a single step on a copy
    Td = to_dev(T0, torch.float64)
    T2d = Td.clone()
    lib.step(T2d, Td, to_dev(Ci, torch.float64), *_sc(s))
    T1, _ = _gpu_run(lib, T0, Ci, s, 1)
    assert torch.equal(T1, T2d)


@pytest.mark.parametrize("kernel", ["zmarch", "tb2"])
def test_checkpoints_written(lib, kernel):
    c = lib.Config(kernel=KERNELS[kernel])
    shape = (12, 14, 64)
    T0, Ci, s = _inputs(shape)
    nt, C = 23, 5
    ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64, c), dtype=torch.uint8, device="cuda")
    T = to_dev(T0, torch.float64)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, torch.float64), *_sc(s), nt, ckpt=ws, ckpt_every=C, cfg=c)
    torch.cuda.synchronize()
    stride = (T.numel() * 8 + 255) // 256 * 256
    for j in range(1, (nt + C - 1) // C):
        field = ws[(j - 1) * stride:(j - 1) * stride + T.numel() * 8].view(torch.float64).reshape(shape)
        ref = oracle.forward(T0, Ci, *_sc(s), j * C)
        np.testing.assert_array_equal(to_host(field), ref)


def test_copy_kernel(lib):
    for n in (1, 15, 16, 17, 4096 + 3, 1 << 20):
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        lib.copy_(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)


def test_bump512_sampled_bit_exact(lib):
    """512^3 FP64 bump workload, nt = 100, in the launch configuration the
    benchmark uses; sampled points against the oracle on sub-boxes (cheap:
    the whole-grid comparison is in test_gpu_headline)."""
    n = 512
    T0, Ci = workloads.bump(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    T, _ = _gpu_run(lib, T0, Ci, s, 100)
    got = to_host(T)
    del T
    torch.cuda.empty_cache()
    rng = np.random.default_rng(5)
    pts = sample_points(T0.shape, rng, 3)
    ref = oracle_forward_at(T0, Ci, s, 100, pts)
    np.testing.assert_array_equal(np.array([got[p] for p in pts]), ref)
    # properties at full size: boundary untouched, bounded by the data range
    b = ~interior_mask(T0.shape)
    assert np.array_equal(got[b], T0[b])
    assert got.min() >= T0.min() and got.max() <= T0.max()
