"""The headline configurations compared with the oracle over the whole grid,
in the launch configuration the benchmark times (the library's default
time loop and reverse sweep):

* bump 512^3 FP64, nt = 100: bit-identical to the FP64 oracle;
* bump 512^3 in FP32, BF16 with stochastic rounding and BF16 rounded to
  nearest: max relative error over all points against the FP64 oracle
  (gates FP32 <= 1e-5, BF16 with stochastic rounding <= 2e-2; nearest
  rounding is reported), and bit-identical to the oracle's FP32 emulator;
* gradient 256^3, nt = 200, a checkpoint every 14 steps, FP64: dL/dT0 and
  dL/dCi bit-identical to the oracle's reverse sweep (states kept every 14
  steps); FP32 bit-identical to its FP32 emulation, its error against FP64
  reported and bounded."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from helpers import bits, emulate_run, max_rel, norm_rel, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OUT = os.environ.get("DIFF3D_REPORT_DIR", "")


def _report(name, rec):
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "headline_%s.json" % name), "w") as f:
            json.dump(rec, f, indent=1)
    print(name, rec, flush=True)


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


@pytest.fixture(scope="module")
def bump512():
    n = 512
    T0, Ci = workloads.bump(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    ref = oracle.forward(T0, Ci, *_sc(s), 100)
    return T0, Ci, s, ref


def _gpu_run(lib, T0, Ci, s, nt, dtype, rounding="sr", cfg=None):
    T = to_dev(T0, dtype)
    T2 = torch.empty_like(T)
    C = to_dev(Ci, dtype)
    lib.run(T, T2, C, *_sc(s), nt, rounding=rounding, cfg=cfg)
    torch.cuda.synchronize()
    out = T.cpu()
    del T, T2, C
    torch.cuda.empty_cache()
    return out


def test_bump512_fp64_whole_grid(lib, bump512):
    T0, Ci, s, ref = bump512
    got = _gpu_run(lib, T0, Ci, s, 100, torch.float64).numpy()
    diff = int(np.count_nonzero(got != ref))
    _report("bump512_fp64", {"points": int(ref.size), "points_differing": diff,
                             "max_abs_diff": float(np.max(np.abs(got - ref)))})
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("form", ["fp32", "bf16_sr", "bf16_rne"])
def test_bump512_precision_whole_grid(lib, bump512, form):
    T0, Ci, s, ref = bump512
    tdt = torch.float32 if form == "fp32" else torch.bfloat16
    rounding = "rne" if form == "bf16_rne" else "sr"
    cfg = lib.Config(sr_seed=2024)
    T = _gpu_run(lib, T0, Ci, s, 100, tdt, rounding, cfg=cfg)
    emu = emulate_run(lib, T0, Ci, s, 100, tdt, rounding, cfg=cfg)
    np.testing.assert_array_equal(bits(T), emu)
    got = T.to(torch.float64).numpy()
    rec = {"max_rel": max_rel(got, ref), "norm_rel": norm_rel(got, ref),
           "passes": lib.pass_plan(T0.shape, 100, tdt, rounding=rounding)}
    _report("bump512_" + form, rec)
    if form == "fp32":
        assert rec["max_rel"] <= 1e-5
    elif form == "bf16_sr":
        assert rec["max_rel"] <= 2e-2


@pytest.fixture(scope="module")
def grad256():
    n, nt, C = 256, 200, 14
    T0, Ci = workloads.uniform_const(n, n, n)
    Tt = workloads.target(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    Tn = oracle.forward(T0, Ci, *_sc(s), nt)
    L, r = oracle.loss_and_seed(Tn, Tt)
    rT0, rCi = oracle.reverse(T0, Ci, r, *_sc(s), nt, keep=C)
    return T0, Ci, Tt, s, nt, C, L, r, rT0, rCi


def _gpu_gradient(lib, T0, Ci, Tt, s, nt, C, dtype):
    """Forward with checkpoints, loss and seed on the GPU, reverse sweep."""
    T0d, Cid, Ttd = to_dev(T0, dtype), to_dev(Ci, dtype), to_dev(Tt, dtype)
    ws = torch.empty(lib.adjoint_workspace_bytes(T0.shape, nt, C, dtype), dtype=torch.uint8, device="cuda")
    T = T0d.clone()
    lib.run(T, torch.empty_like(T), Cid, *_sc(s), nt, ckpt=ws, ckpt_every=C)
    seed = torch.empty_like(T)
    L = float(lib.loss(T, Ttd, seed))
    gT0, gCi = torch.empty_like(T), torch.empty_like(T)
    lib.adjoint_run(T0d, Cid, seed, gT0, gCi, ws, True, *_sc(s), nt, C)
    torch.cuda.synchronize()
    out = L, seed.cpu(), gT0.cpu(), gCi.cpu()
    del T0d, Cid, Ttd, ws, T, seed, gT0, gCi
    torch.cuda.empty_cache()
    return out


def test_grad256_fp64_whole_grid(lib, grad256):
    T0, Ci, Tt, s, nt, C, L_ref, r, rT0, rCi = grad256
    L, seed, gT0, gCi = _gpu_gradient(lib, T0, Ci, Tt, s, nt, C, torch.float64)
    _report("grad256_fp64", {"loss": L, "loss_ref": L_ref,
                             "gT0_points_differing": int(np.count_nonzero(gT0.numpy() != rT0)),
                             "gCi_points_differing": int(np.count_nonzero(gCi.numpy() != rCi))})
    assert L == pytest.approx(L_ref, rel=1e-14)
    np.testing.assert_array_equal(seed.numpy(), r)
    np.testing.assert_array_equal(gT0.numpy(), rT0)
    np.testing.assert_array_equal(gCi.numpy(), rCi)


def test_grad256_fp32_whole_grid(lib, grad256):
    T0, Ci, Tt, s, nt, C, L_ref, r, rT0, rCi = grad256
    L, seed, gT0, gCi = _gpu_gradient(lib, T0, Ci, Tt, s, nt, C, torch.float32)
    # the emulator's FP32 reverse sweep from the FP32 seed the GPU formed
    # (T_nt - T_target rounded to FP32: compared with the emulated forward)
    f32 = lambda a: stored(a, torch.float32)
    Tn32 = oracle.emulate_forward(f32(T0), f32(Ci), *_sc(s), [1] * nt, oracle.ST_F32)
    seed32 = (Tn32.astype(np.float64) - f32(Tt).astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(seed.numpy(), seed32)
    eT0, eCi = oracle.emulate_reverse32(f32(T0), f32(Ci), seed32, *_sc(s), nt, keep=C)
    np.testing.assert_array_equal(gT0.numpy(), eT0)
    np.testing.assert_array_equal(gCi.numpy(), eCi)
    g0, gc = gT0.double().numpy(), gCi.double().numpy()
    rec = {"loss": L, "loss_ref": L_ref, "gT0_norm_rel": norm_rel(g0, rT0), "gCi_norm_rel": norm_rel(gc, rCi)}
    _report("grad256_fp32", rec)
    assert rec["gT0_norm_rel"] <= 1e-5 and rec["gCi_norm_rel"] <= 1e-4
