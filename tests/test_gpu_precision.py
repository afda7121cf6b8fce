"""Reduced-precision storage forms against the FP64 oracle.

Gates: FP32 storage with FP32 arithmetic within 1e-5 max relative error
after 100 steps; BF16 storage with FP32 arithmetic and stochastic rounding
within 2e-2.  BF16 with round-to-nearest-even is reported only: near the
bump the change over a pass is below half a BF16 ulp and the field
stagnates.  Each form is also bit-identical to the oracle's FP32 emulator."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from helpers import bits, emulate_run, max_rel, norm_rel, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# measured errors are printed, and also written as JSON when this names a folder
OUT = os.environ.get("DIFF3D_REPORT_DIR", "")


def _run(lib, T0, Ci, s, nt, dtype, rounding="sr", emulate=False):
    cfg = lib.Config(sr_seed=2024)
    T = to_dev(T0, dtype)
    T2 = torch.empty_like(T)
    lib.run(T, T2, to_dev(Ci, dtype), s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, rounding=rounding,
            cfg=cfg)
    torch.cuda.synchronize()
    if emulate and dtype != torch.float64:
        np.testing.assert_array_equal(bits(T), emulate_run(lib, T0, Ci, s, nt, dtype, rounding, cfg=cfg))
    return to_host(T)


def _report(name, rec):
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "precision_%s.json" % name), "w") as f:
            json.dump(rec, f, indent=1)
    print(name, rec, flush=True)


def test_uniform64_fp32(lib):
    T0, Ci = workloads.uniform_const(64, 64, 64)
    s = oracle.scalars(64, 64, 64, Ci)
    ref = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], 100)
    got = _run(lib, T0, Ci, s, 100, torch.float32, emulate=True)
    e = max_rel(got, ref)
    _report("uniform64", {"fp32_max_rel": e, "fp32_norm_rel": norm_rel(got, ref)})
    assert e <= 1e-5


def test_bump256_precision_forms(lib):
    """The 256^3 instance of the bump workload, nt = 100, three storage forms,
    each over the whole grid against the FP64 oracle (gated) and bit for bit
    against the emulator."""
    n = 256
    T0, Ci = workloads.bump(n, n, n)
    s = oracle.scalars(n, n, n, Ci)
    ref = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], 100)
    rec = {"threads": oracle.max_threads()}
    f32 = _run(lib, T0, Ci, s, 100, torch.float32, emulate=True)
    rec["fp32_max_rel"], rec["fp32_norm_rel"] = max_rel(f32, ref), norm_rel(f32, ref)
    sr = _run(lib, T0, Ci, s, 100, torch.bfloat16, "sr", emulate=True)
    rec["bf16_sr_max_rel"], rec["bf16_sr_norm_rel"] = max_rel(sr, ref), norm_rel(sr, ref)
    rne = _run(lib, T0, Ci, s, 100, torch.bfloat16, "rne", emulate=True)
    rec["bf16_rne_max_rel"], rec["bf16_rne_norm_rel"] = max_rel(rne, ref), norm_rel(rne, ref)
    # the error of merely storing the inputs in BF16, for scale
    q = to_host(to_dev(T0, torch.bfloat16))
    rec["bf16_input_quantisation_max_rel"] = max_rel(q, T0)
    _report("bump256", rec)
    assert rec["fp32_max_rel"] <= 1e-5
    assert rec["bf16_sr_max_rel"] <= 2e-2


def test_bf16_sr_unbiased_on_slow_decay(lib):
    """Stochastic rounding keeps the mean decay of a sine mode whose per-step
    change is far below half a BF16 ulp, where RNE stagnates."""
    n = 96
    Ci = np.full((n, n, n), 0.5)
    s = oracle.scalars(n, n, n, Ci)
    x = np.sin(np.pi * np.arange(n) / (n - 1))
    T0 = x[:, None, None] * x[None, :, None] * x[None, None, :]
    T0[0] = T0[-1] = 0
    T0[:, 0] = T0[:, -1] = 0
    T0[:, :, 0] = T0[:, :, -1] = 0
    ref = oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], 100)
    sr = _run(lib, T0, Ci, s, 100, torch.bfloat16, "sr")
    rne = _run(lib, T0, Ci, s, 100, torch.bfloat16, "rne")
    c = (slice(n // 2 - 8, n // 2 + 8),) * 3
    drop_ref = float(np.mean(T0[c] - ref[c]))
    drop_sr = float(np.mean(to_host(to_dev(T0, torch.bfloat16))[c] - sr[c]))
    drop_rne = float(np.mean(to_host(to_dev(T0, torch.bfloat16))[c] - rne[c]))
    _report("sine96", {"drop_ref": drop_ref, "drop_sr": drop_sr, "drop_rne": drop_rne})
    assert abs(drop_sr - drop_ref) <= 0.1 * abs(drop_ref)
