"""Checkpointed reverse sweep on the GPU: against the oracle's FP64 reverse
sweep (bit for bit: same operation order) and its FP32 emulation, central
finite differences, the dot-product identity and the sine-mode closed form
at full size."""
import math

import numpy as np
import pytest

import oracle
import workloads
from helpers import instantiated_configs, norm_rel, oracle_reverse_at, sample_points, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(shape, seed=0):
    nz, ny, nx = shape
    rng = np.random.default_rng(200 + seed)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    g = rng.standard_normal(shape)
    s = oracle.scalars(nx, ny, nz, Ci, lx=1.1, ly=0.9, lz=1.0)
    return T0, Ci, g, s


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def _adjoint(lib, T0, Ci, g, s, nt, C, dtype=torch.float64, ready=False, cfg=None):
    T0d, Cid, gd = to_dev(T0, dtype), to_dev(Ci, dtype), to_dev(g, dtype)
    ws = torch.empty(lib.adjoint_workspace_bytes(T0.shape, nt, C, dtype, cfg), dtype=torch.uint8, device="cuda")
    if ready:
        T = T0d.clone()
        lib.run(T, torch.empty_like(T), Cid, *_sc(s), nt, ckpt=ws, ckpt_every=C, cfg=cfg)
    gT0 = torch.empty_like(T0d)
    gCi = torch.empty_like(T0d)
    lib.adjoint_run(T0d, Cid, gd, gT0, gCi, ws, ready, *_sc(s), nt, C, cfg=cfg)
    torch.cuda.synchronize()
    return to_host(gT0), to_host(gCi)


def _emulated32(T0, Ci, g, s, nt):
    """The oracle's FP32 reverse sweep on the FP32 inputs the GPU gets."""
    f32 = lambda a: stored(a, torch.float32)
    a, b = oracle.emulate_reverse32(f32(T0), f32(Ci), f32(g), *_sc(s), nt)
    return a.astype(np.float64), b.astype(np.float64)


@pytest.mark.parametrize("shape,nt,C", [((6, 5, 7), 5, 2), ((19, 37, 131), 9, 4), ((21, 20, 128), 13, 5),
                                        ((3, 3, 3), 4, 3), ((8, 70, 64), 7, 1), ((9, 9, 192), 6, 10)])
@pytest.mark.parametrize("kernel", ["naive", "zmarch", "tb2", "auto"])
def test_fp64_matches_oracle_bitwise(lib, shape, nt, C, kernel):
    c = lib.Config(kernel={"naive": lib.KERNEL_NAIVE, "zmarch": lib.KERNEL_ZMARCH, "tb2": lib.KERNEL_TB2,
                           "auto": lib.KERNEL_AUTO}[kernel])
    T0, Ci, g, s = _inputs(shape)
    rT0, rCi = oracle.reverse(T0, Ci, g, *_sc(s), nt)
    for ready in (False, True):
        gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C, ready=ready, cfg=c)
        np.testing.assert_array_equal(gT0, rT0)
        np.testing.assert_array_equal(gCi, rCi)
    # FP32: the oracle's FP32 emulation, bit for bit
    eT0, eCi = _emulated32(T0, Ci, g, s, nt)
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C, dtype=torch.float32, ready=True, cfg=c)
    np.testing.assert_array_equal(gT0, eT0)
    np.testing.assert_array_equal(gCi, eCi)


def _adj_cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4)):
        for cfg in instantiated_configs("ADJ", size):
            for azlen in (0, 1, 5):
                out.append((name, cfg, azlen))
    return out


@pytest.mark.parametrize("dtype,cfg,azlen", _adj_cases())
def test_adjoint_configs(lib, dtype, cfg, azlen):
    """Every instantiated adjoint configuration and several z-chunk lengths:
    FP64 bit-identical to the oracle, FP32 to its FP32 emulation."""
    c = lib.Config(kernel=lib.KERNEL_ZMARCH, adj=lib.Tile(p=tuple(cfg) + (0,), zlen=azlen))
    T0, Ci, g, s = _inputs((11, 23, 128), seed=azlen + sum(cfg))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, 5, 3, dtype=tdt, cfg=c)
    if dtype == "f64":
        rT0, rCi = oracle.reverse(T0, Ci, g, *_sc(s), 5)
    else:
        rT0, rCi = _emulated32(T0, Ci, g, s, 5)
    np.testing.assert_array_equal(gT0, rT0)
    np.testing.assert_array_equal(gCi, rCi)


def _adj2_cases():
    out = []
    for name, size in (("f64", 8), ("f32", 4)):
        for cfg in instantiated_configs("ADJ2", size):
            for zlen in (0, 1, 3):
                out.append((name, cfg, zlen))
    return out


@pytest.mark.parametrize("dtype,cfg,zlen", _adj2_cases())
def test_adjoint_two_step_configs(lib, dtype, cfg, zlen):
    """Every instantiated two-step adjoint configuration and several z-chunk
    lengths: FP64 bit-identical to the oracle, FP32 to its FP32 emulation."""
    c = lib.Config(kernel=lib.KERNEL_TB2, adj2=lib.Tile(p=tuple(cfg) + (0,), zlen=zlen))
    T0, Ci, g, s = _inputs((13, 21, 128), seed=zlen + sum(cfg) + 7)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, 9, 4, dtype=tdt, cfg=c)
    if dtype == "f64":
        rT0, rCi = oracle.reverse(T0, Ci, g, *_sc(s), 9)
    else:
        rT0, rCi = _emulated32(T0, Ci, g, s, 9)
    np.testing.assert_array_equal(gT0, rT0)
    np.testing.assert_array_equal(gCi, rCi)


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (5, 70, 33), (9, 3, 130), (6, 66, 64)])
def test_adjoint_two_step_small_and_ragged(lib, shape):
    c = lib.Config(kernel=lib.KERNEL_TB2, adj2=lib.Tile(zlen=1), tb2=lib.Tile(zlen=1))
    T0, Ci, g, s = _inputs(shape, seed=11)
    for nt, C in ((2, 2), (5, 3), (8, 8)):
        rT0, rCi = oracle.reverse(T0, Ci, g, *_sc(s), nt)
        gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C, cfg=c)
        np.testing.assert_array_equal(gT0, rT0)
        np.testing.assert_array_equal(gCi, rCi)


def test_zero_steps(lib):
    T0, Ci, g, s = _inputs((5, 6, 7))
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, 0, 3)
    np.testing.assert_array_equal(gT0, g)
    assert np.all(gCi == 0)


def _grad32():
    """32^3 instance of the gradient workload: T0 ~ U[0,1] (seed 0), Ci = 0.5,
    T_target ~ U[0,1] (seed 2), nt = 200, a checkpoint every 14 steps."""
    n = 32
    T0, Ci = workloads.uniform_const(n, n, n)
    Tt = workloads.target(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    return T0, Ci, Tt, s


def test_grad32_against_oracle_and_loss(lib):
    T0, Ci, Tt, s = _grad32()
    nt, C = 200, 14
    Tn = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    L_ref, r = oracle.loss_and_seed(Tn, Tt)
    rT0, rCi = oracle.reverse(T0, Ci, r, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    # GPU: forward with checkpoints, FP64 loss and seed on the GPU, reverse sweep
    T0d, Cid, Ttd = to_dev(T0, torch.float64), to_dev(Ci, torch.float64), to_dev(Tt, torch.float64)
    ws = torch.empty(lib.adjoint_workspace_bytes(T0.shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
    T = T0d.clone()
    lib.run(T, torch.empty_like(T), Cid, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, ckpt=ws, ckpt_every=C)
    seed = torch.empty_like(T)
    L = lib.loss(T, Ttd, seed)
    gT0, gCi = torch.empty_like(T), torch.empty_like(T)
    lib.adjoint_run(T0d, Cid, seed, gT0, gCi, ws, True, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, C)
    torch.cuda.synchronize()
    assert float(L) == pytest.approx(L_ref, rel=1e-14)
    np.testing.assert_array_equal(to_host(seed), r)
    np.testing.assert_array_equal(to_host(gT0), rT0)
    np.testing.assert_array_equal(to_host(gCi), rCi)
    assert float(lib.norm2(gT0)) == pytest.approx(float(np.sum(rT0 * rT0)), rel=1e-14)


def test_grad32_finite_differences(lib):
    """Central differences of the GPU loss along seeded directions: T0 (the loss
    is quadratic in T0, so the difference is exact up to rounding) and Ci."""
    T0, Ci, Tt, s = _grad32()
    nt, C = 200, 14
    Ttd = to_dev(Tt, torch.float64)

    def loss(T0_, Ci_):
        T = to_dev(T0_, torch.float64)
        lib.run(T, torch.empty_like(T), to_dev(Ci_, torch.float64), s["lam"], s["dt"], s["rdx"], s["rdy"],
                s["rdz"], nt)
        return float(lib.loss(T, Ttd))

    T = to_dev(T0, torch.float64)
    lib.run(T, torch.empty_like(T), to_dev(Ci, torch.float64), s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    seed = torch.empty_like(T)
    lib.loss(T, Ttd, seed)
    gT0, gCi = _adjoint(lib, T0, Ci, to_host(seed), s, nt, C)
    v = workloads.direction(32, 32, 32)
    for eps in (1e-2, 1e-4):
        fd = (loss(T0 + eps * v, Ci) - loss(T0 - eps * v, Ci)) / (2 * eps)
        assert fd == pytest.approx(float(np.sum(gT0 * v)), rel=1e-6)
    mask = np.zeros(Ci.shape)
    mask[1:-1, 1:-1, 1:-1] = 1.0
    w = v * mask
    eps = 1e-6
    fd = (loss(T0, Ci + eps * w) - loss(T0, Ci - eps * w)) / (2 * eps)
    assert fd == pytest.approx(float(np.sum(gCi * w)), rel=1e-6)
    # a boundary change of Ci does not change the loss at all
    wb = v * (1.0 - mask)
    assert loss(T0, Ci + 1e-3 * wb) == loss(T0, Ci)


def test_autograd_function(lib):
    T0, Ci, Tt, s = _grad32()
    nt, C = 60, 8
    T0d = to_dev(T0, torch.float64).requires_grad_(True)
    Cid = to_dev(Ci, torch.float64).requires_grad_(True)
    Tn = lib.diffuse(T0d, Cid, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, C)
    L = 0.5 * ((Tn - to_dev(Tt, torch.float64)) ** 2).sum()
    L.backward()
    Tn_ref = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    _, r = oracle.loss_and_seed(Tn_ref, Tt)
    rT0, rCi = oracle.reverse(T0, Ci, r, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    np.testing.assert_array_equal(to_host(Tn), Tn_ref)
    np.testing.assert_array_equal(to_host(T0d.grad), rT0)
    np.testing.assert_array_equal(to_host(Cid.grad), rCi)


def test_fp32_against_fp64_oracle(lib):
    T0, Ci, Tt, s = _grad32()
    nt, C = 200, 14
    Tn = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    _, r = oracle.loss_and_seed(Tn, Tt)
    rT0, rCi = oracle.reverse(T0, Ci, r, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    gT0, gCi = _adjoint(lib, T0, Ci, r, s, nt, C, dtype=torch.float32, ready=True)
    e0, e1 = norm_rel(gT0, rT0), norm_rel(gCi, rCi)
    print("fp32 adjoint norm-relative errors: gT0 %.3e gCi %.3e" % (e0, e1), flush=True)
    assert e0 <= 1e-5 and e1 <= 1e-4
    eT0, eCi = _emulated32(T0, Ci, r, s, nt)
    np.testing.assert_array_equal(gT0, eT0)
    np.testing.assert_array_equal(gCi, eCi)


def test_grad256_dot_product(lib):
    """<A^nt x, y> = <x, (A^T)^nt y> at 256^3, nt = 200, checkpoints every 14."""
    n, nt, C = 256, 200, 14
    x, Ci = workloads.uniform_const(n, n, n)
    y = workloads.target(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    xd, Cid, yd = to_dev(x, torch.float64), to_dev(Ci, torch.float64), to_dev(y, torch.float64)
    Ax = xd.clone()
    lib.run(Ax, torch.empty_like(Ax), Cid, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    ws = torch.empty(lib.adjoint_workspace_bytes(x.shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
    ATy, gCi = torch.empty_like(xd), torch.empty_like(xd)
    lib.adjoint_run(xd, Cid, yd, ATy, gCi, ws, False, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, C)
    lhs = float((Ax * yd).sum())
    rhs = float((xd * ATy).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_grad256_sampled_against_oracle(lib):
    """256^3 with the 14-step checkpoint layout (two segments), nt = 20, a
    seeded adjoint seed; sampled points against the oracle on sub-boxes."""
    n, nt, C = 256, 20, 14
    T0, Ci = workloads.uniform_const(n, n, n)
    Ci = Ci * (1.0 + 0.2 * workloads.uniform(n, n, n, 1))
    g = workloads.direction(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    gT0, gCi = _adjoint(lib, T0, Ci, g, s, nt, C)
    rng = np.random.default_rng(9)
    pts = sample_points(T0.shape, rng, 6)
    a, b = oracle_reverse_at(T0, Ci, g, s, nt, pts)
    np.testing.assert_array_equal(np.array([gT0[p] for p in pts]), a)
    np.testing.assert_array_equal(np.array([gCi[p] for p in pts]), b)


def test_sine_mode_closed_form_128(lib):
    """Interior gradient g^(2nt) s, faces from the inward neighbour, edges 0,
    and sum(gCi) = nt g^(2nt-1) (-dt lam kappa) ||s||^2, at 128^3."""
    n, nt, C = 128, 40, 7
    c = 0.5
    Ci = np.full((n, n, n), c)
    s = oracle.scalars(n, n, n, Ci)
    x = np.sin(np.pi * np.arange(n) / (n - 1))
    sm = x[:, None, None] * x[None, :, None] * x[None, None, :]
    sm[0] = sm[-1] = 0
    sm[:, 0] = sm[:, -1] = 0
    sm[:, :, 0] = sm[:, :, -1] = 0
    kap = 3 * 4.0 * math.sin(math.pi / (2 * (n - 1))) ** 2 * s["rdx"] ** 2
    gg = 1.0 - s["dt"] * s["lam"] * c * kap
    Tn = sm * gg ** nt
    gT0, gCi = _adjoint(lib, sm, Ci, Tn, s, nt, C)
    assert np.max(np.abs(gT0[1:-1, 1:-1, 1:-1] - gg ** (2 * nt) * sm[1:-1, 1:-1, 1:-1])) <= 1e-13
    geo = gg ** nt * (1 - gg ** nt) / (1 - gg)
    face = s["dt"] * s["lam"] * c * s["rdx"] ** 2 * geo * sm[1:-1, 1:-1, 1]
    np.testing.assert_allclose(gT0[1:-1, 1:-1, 0], face, rtol=1e-9, atol=1e-15)
    assert np.all(gT0[0, 0, :] == 0) and np.all(gT0[:, -1, -1] == 0)
    expect = nt * gg ** (2 * nt - 1) * (-s["dt"] * s["lam"] * kap) * float(np.sum(sm * sm))
    assert float(np.sum(gCi)) == pytest.approx(expect, rel=1e-6)
