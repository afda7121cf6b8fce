"""The 2-D form of the step (the Fig. 1 expression without the z term) on the
GPU: FP64 bit-identical to the oracle; FP32 and both BF16 forms bit-identical
to the FP32 emulator's 2-D form on the same stored inputs and within their
error bounds against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from helpers import bits, stored

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(shape, seed=0):
    ny, nx = shape
    rng = np.random.default_rng(500 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars2d(nx, ny, Ci, lx=1.0, ly=1.3)
    return T0, Ci, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"])


SHAPES = [(3, 3), (4, 5), (5, 70), (67, 3), (3, 64), (3, 65), (130, 129), (64, 257), (200, 63), (33, 1000)]


@pytest.mark.parametrize("shape", SHAPES)
def test_step_bitwise_and_boundary_untouched(lib, shape):
    T0, Ci, s = _inputs(shape, seed=shape[0] + shape[1])
    T = torch.from_numpy(T0).cuda()
    C = torch.from_numpy(Ci).cuda()
    T2 = torch.full_like(T, float("nan"))
    b = torch.ones(shape, dtype=torch.bool)
    b[1:-1, 1:-1] = False
    b = b.cuda()
    T2[b] = -5.0
    lib.step2d(T2, T, C, *_sc(s))
    torch.cuda.synchronize()
    ref = oracle.forward2d(T0, Ci, *_sc(s), 1)
    got = T2.cpu().numpy()
    inner = ~b.cpu().numpy()
    np.testing.assert_array_equal(got[inner], ref[inner])
    assert np.all(got[~inner] == -5.0)


@pytest.mark.parametrize("shape", [(3, 3), (9, 130), (129, 64), (70, 70), (257, 300)])
@pytest.mark.parametrize("nt", [0, 1, 2, 7, 41])
def test_run_bitwise(lib, shape, nt):
    T0, Ci, s = _inputs(shape, seed=nt)
    T = torch.from_numpy(T0).cuda()
    lib.run2d(T, torch.empty_like(T), torch.from_numpy(Ci).cuda(), *_sc(s), nt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(T.cpu().numpy(), oracle.forward2d(T0, Ci, *_sc(s), nt))


def test_run_4096_bitwise(lib):
    """A grid of many strips and y-chunks (the launch the benchmark uses at
    8192^2), compared whole."""
    shape = (4096, 4096)
    T0, Ci, s = _inputs(shape, seed=3)
    T = torch.from_numpy(T0).cuda()
    lib.run2d(T, torch.empty_like(T), torch.from_numpy(Ci).cuda(), *_sc(s), 10)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(T.cpu().numpy(), oracle.forward2d(T0, Ci, *_sc(s), 10))


def test_fp32_against_fp64_oracle(lib):
    """FP32 storage and arithmetic, 100 steps of a Gaussian bump on 1024^2:
    max relative error against the FP64 oracle within 1e-5."""
    n = 1024
    xs = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(xs, xs)
    rng = np.random.default_rng(9)
    T0 = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.01) + 0.01 * rng.random((n, n))
    Ci = 0.5 * (1.0 + 0.5 * rng.random((n, n)))
    s = oracle.scalars2d(n, n, Ci)
    ref = oracle.forward2d(T0, Ci, *_sc(s), 100)
    T = torch.from_numpy(T0).to("cuda", torch.float32)
    lib.run2d(T, torch.empty_like(T), torch.from_numpy(Ci).to("cuda", torch.float32), *_sc(s), 100)
    torch.cuda.synchronize()
    rel = np.max(np.abs(T.double().cpu().numpy() - ref) / np.abs(ref))
    assert rel <= 1e-5, rel


ROUNDINGS = [("sr", oracle.ST_BF16_SR), ("rne", oracle.ST_BF16_RNE)]
SEED, STEP0 = 0x5EED_0F_2D, 11


def _bf16_case(shape, seed):
    T0, Ci, s = _inputs(shape, seed=seed)
    T0s, Cis = stored(T0, torch.bfloat16), stored(Ci, torch.bfloat16)
    return T0, Ci, T0s, Cis, s


def _plan2d(nt, P=8):
    """The time loop's pass lengths for the BF16 forms: near-equal passes of
    at most eight steps."""
    m = (nt + P - 1) // P
    out, done = [], 0
    for i in range(m):
        n = (nt - done + (m - i) - 1) // (m - i)
        out.append(n)
        done += n
    return out


@pytest.mark.parametrize("rounding,storage", ROUNDINGS, ids=("sr", "rne"))
@pytest.mark.parametrize("shape", [(3, 3), (5, 70), (40, 65), (70, 257)])
@pytest.mark.parametrize("n", range(1, 9))
def test_stepn_bf16_bitwise(lib, shape, n, rounding, storage):
    """n steps in one pass with BF16 storage (FP32 arithmetic, one rounding
    at the end of the pass, stochastic rounding drawn with step index
    sr_step + n - 1): bit-identical to the emulator, boundary untouched."""
    T0, Ci, T0s, Cis, s = _bf16_case(shape, seed=30 + n)
    T = torch.from_numpy(T0).to(torch.bfloat16).cuda()
    C = torch.from_numpy(Ci).to(torch.bfloat16).cuda()
    T2 = T.clone()
    cfg = lib.Config(sr_seed=SEED, sr_step=STEP0)
    if n == 1:
        lib.step2d(T2, T, C, *_sc(s), rounding=rounding, cfg=cfg)
    else:
        lib.stepn2d(T2, T, C, *_sc(s), n, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    want = oracle.emulate_forward(T0s, Cis, s["lam"], s["dt"], s["rdx"], s["rdy"], 0.0, [n], storage,
                                  seed=SEED, step0=STEP0)
    np.testing.assert_array_equal(bits(T2), want)


@pytest.mark.parametrize("rounding,storage", ROUNDINGS, ids=("sr", "rne"))
@pytest.mark.parametrize("nt", [1, 8, 9, 20, 41])
def test_run_bf16_bitwise(lib, nt, rounding, storage):
    """The BF16 time loop (near-equal passes of at most eight steps, e.g. 20
    as 7, 7, 6) bit-identical to the emulator over the same passes."""
    shape = (150, 333)
    T0, Ci, T0s, Cis, s = _bf16_case(shape, seed=9)
    T = torch.from_numpy(T0).to(torch.bfloat16).cuda()
    C = torch.from_numpy(Ci).to(torch.bfloat16).cuda()
    cfg = lib.Config(sr_seed=SEED, sr_step=STEP0)
    lib.run2d(T, torch.empty_like(T), C, *_sc(s), nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    passes = _plan2d(nt)
    assert sum(passes) == nt and max(passes) <= 8
    want = oracle.emulate_forward(T0s, Cis, s["lam"], s["dt"], s["rdx"], s["rdy"], 0.0, passes, storage,
                                  seed=SEED, step0=STEP0)
    np.testing.assert_array_equal(bits(T), want)


def test_bf16_sr_draws_depend_on_seed_and_step(lib):
    """Equal arguments give equal bits; another seed or first step index
    gives other bits (the call keeps no state)."""
    T0, Ci, _, _, s = _bf16_case((64, 200), seed=12)
    C = torch.from_numpy(Ci).to(torch.bfloat16).cuda()
    outs = []
    for seed, step in ((1, 0), (1, 0), (2, 0), (1, 5)):
        T = torch.from_numpy(T0).to(torch.bfloat16).cuda()
        lib.run2d(T, torch.empty_like(T), C, *_sc(s), 12, cfg=lib.Config(sr_seed=seed, sr_step=step))
        outs.append(T)
    torch.cuda.synchronize()
    assert torch.equal(outs[0].view(torch.int16), outs[1].view(torch.int16))
    assert not torch.equal(outs[0].view(torch.int16), outs[2].view(torch.int16))
    assert not torch.equal(outs[0].view(torch.int16), outs[3].view(torch.int16))


def test_bf16_error_against_fp64_oracle(lib):
    """A 2-D Gaussian bump with noise (the 3-D workload's shape in 2-D),
    1024^2, 100 steps: max relative error against the FP64 oracle on the
    whole grid, stochastic rounding gated at 2e-2 like the 3-D form;
    round-to-nearest reported (it stagnates where the per-step change is
    below half a BF16 unit)."""
    n = 1024
    x = np.arange(n) / (n - 1) - 0.5
    rng = np.random.default_rng(0)
    T0 = np.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / 0.01) + 0.01 * rng.random((n, n))
    Ci = 0.5 * (1.0 + 0.5 * np.random.default_rng(1).random((n, n)))
    s = oracle.scalars2d(n, n, Ci)
    ref = oracle.forward2d(T0, Ci, *_sc(s), 100)
    errs = {}
    for rounding in ("sr", "rne"):
        T = torch.from_numpy(T0).to(torch.bfloat16).cuda()
        C = torch.from_numpy(Ci).to(torch.bfloat16).cuda()
        lib.run2d(T, torch.empty_like(T), C, *_sc(s), 100, rounding=rounding)
        torch.cuda.synchronize()
        got = T.double().cpu().numpy()
        errs[rounding] = float(np.max(np.abs(got - ref) / np.abs(ref)))
    print("2-D 1024^2 bump, 100 steps, max relative error vs FP64: BF16-SR %.2e, BF16-RNE %.2e"
          % (errs["sr"], errs["rne"]), flush=True)
    assert errs["sr"] <= 2e-2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(37, 256), (50, 1024), (19, 72)])
def test_alignment_independent(lib, dtype, shape):
    """Fields one element off 16-byte alignment give the same bits as
    aligned ones."""
    T0, Ci, s = _inputs(shape, seed=shape[1])
    n = T0.size

    def run(offset):
        bt = torch.zeros(n + 8, dtype=dtype, device="cuda")
        bc = torch.zeros(n + 8, dtype=dtype, device="cuda")
        T = bt[offset:offset + n].view(shape)
        C = bc[offset:offset + n].view(shape)
        T.copy_(torch.from_numpy(T0).to(dtype))
        C.copy_(torch.from_numpy(Ci).to(dtype))
        S = torch.empty_like(T)
        lib.run2d(T, S, C, *_sc(s), 9)
        torch.cuda.synchronize()
        return T.clone()

    assert torch.equal(run(0), run(1))


def _emulate32_2d(T0, Ci, s, nt):
    """The FP32 emulator of the oracle on the 2-D field embedded in a 3-D one:
    three identical z planes and rdz = 0, so the z term of the 3-D step is
    exactly zero and its middle plane takes the 2-D step."""
    T3 = np.repeat(T0[None].astype(np.float32), 3, axis=0)
    C3 = np.repeat(Ci[None].astype(np.float32), 3, axis=0)
    out = oracle.emulate_forward(T3, C3, s["lam"], s["dt"], s["rdx"], s["rdy"], 0.0, [1] * nt, oracle.ST_F32)
    return out[1]


STEPN_SHAPES = [(3, 3), (5, 70), (67, 3), (9, 64), (40, 65), (130, 129), (70, 257), (19, 1000)]


@pytest.mark.parametrize("shape", STEPN_SHAPES)
@pytest.mark.parametrize("n", range(1, 9))
def test_stepn_bitwise(lib, shape, n):
    """n steps in one pass: FP64 equal to the oracle, FP32 equal to the FP32
    emulator, boundary untouched; ragged grids across several 64-lane
    regions and y-chunks."""
    T0, Ci, s = _inputs(shape, seed=n)
    for tdt in (torch.float64, torch.float32):
        T = torch.from_numpy(T0).to(tdt).cuda()
        C = torch.from_numpy(Ci).to(tdt).cuda()
        T2 = T.clone()
        lib.stepn2d(T2, T, C, *_sc(s), n)
        torch.cuda.synchronize()
        got = T2.cpu().numpy()
        if tdt == torch.float64:
            np.testing.assert_array_equal(got, oracle.forward2d(T0, Ci, *_sc(s), n))
        else:
            np.testing.assert_array_equal(got, _emulate32_2d(T0.astype(np.float32), Ci.astype(np.float32), s, n))


@pytest.mark.parametrize("nt", [1, 7, 8, 9, 23, 41])
def test_run_fp32_bitwise_emulator(lib, nt):
    """The FP32 time loop (passes of up to eight steps) equal to the FP32
    emulator bit for bit."""
    shape = (150, 333)
    T0, Ci, s = _inputs(shape, seed=7)
    T = torch.from_numpy(T0).float().cuda()
    lib.run2d(T, torch.empty_like(T), torch.from_numpy(Ci).float().cuda(), *_sc(s), nt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(T.cpu().numpy(),
                                  _emulate32_2d(T0.astype(np.float32), Ci.astype(np.float32), s, nt))


def test_stepn_rejects(lib):
    T = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    for n in (0, 9):
        with pytest.raises(lib.Diff3dError):
            lib.stepn2d(T.clone(), T, T.clone(), 1.0, 1e-3, 1.0, 1.0, n)
