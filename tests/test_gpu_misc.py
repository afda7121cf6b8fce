"""Reductions, loss seeds, the copy reference and extreme grid shapes."""
import numpy as np
import pytest

import oracle
import workloads
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 100003, 3 * 1024 * 256 + 5])
def test_reductions(lib, dtype, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    xd, yd = torch.from_numpy(x).to("cuda", dtype), torch.from_numpy(y).to("cuda", dtype)
    xq, yq = to_host(xd), to_host(yd)          # the values as stored
    assert float(lib.field_max(xd)) == xq.max()
    assert float(lib.norm2(xd)) == pytest.approx(float(np.sum(xq * xq)), rel=1e-13)
    seed = torch.empty_like(xd)
    L = float(lib.loss(xd.view(1, 1, n), yd.view(1, 1, n), seed.view(1, 1, n)))
    r = xq - yq
    assert L == pytest.approx(0.5 * float(np.sum(r * r)), rel=1e-13)
    expect = torch.from_numpy(r).to("cuda", dtype)     # RNE of the FP64 difference
    if dtype == torch.bfloat16:
        # the library rounds the FP64 difference through FP32 to BF16 (nearest even)
        expect = torch.from_numpy(r.astype(np.float32)).to("cuda").to(torch.bfloat16)
    assert torch.equal(seed, expect)
    # deterministic: the same bits on a second call
    assert float(lib.norm2(xd)) == float(lib.norm2(xd))


def test_unaligned_fields(lib):
    """Fields that start 2 bytes past a 16-byte boundary (BF16 views): the
    one-point-per-lane kernels and the 16-bit copy for the final swap."""
    shape = (9, 20, 64)
    n = int(np.prod(shape))
    T0, Ci = workloads.bump(shape[2], shape[1], shape[0])
    s = oracle.scalars(shape[2], shape[1], shape[0], Ci)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    outs = []
    for off in (0, 1):
        bufs = [torch.zeros(n + 8, dtype=torch.bfloat16, device="cuda") for _ in range(3)]
        T, T2, C = (b[off:off + n].view(shape) for b in bufs)
        T.copy_(to_dev(T0, torch.bfloat16))
        C.copy_(to_dev(Ci, torch.bfloat16))
        lib.run(T, T2, C, *sc, 5, cfg=lib.Config(sr_seed=3))       # odd: ends with a copy T2 -> T
        torch.cuda.synchronize()
        outs.append(T.clone())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("shape", [(3, 3, 2000), (3, 700, 3), (900, 3, 4), (5, 130, 257)])
def test_extreme_shapes(lib, shape):
    """Grids far from cubic: one tile row, one z-chunk, long z marches."""
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(nx, ny, nz, Ci)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    ref = oracle.forward(T0, Ci, *sc, 7)
    for kernel in (lib.KERNEL_NAIVE, lib.KERNEL_ZMARCH, lib.KERNEL_TB2, lib.KERNEL_AUTO):
        T = to_dev(T0, torch.float64)
        lib.run(T, torch.empty_like(T), to_dev(Ci, torch.float64), *sc, 7, cfg=lib.Config(kernel=kernel))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_host(T), ref)
    g = rng.standard_normal(shape)
    rT0, rCi = oracle.reverse(T0, Ci, g, *sc, 7)
    T0d, Cid = to_dev(T0, torch.float64), to_dev(Ci, torch.float64)
    ws = torch.empty(lib.adjoint_workspace_bytes(shape, 7, 3, torch.float64), dtype=torch.uint8, device="cuda")
    gT0, gCi = torch.empty_like(T0d), torch.empty_like(T0d)
    lib.adjoint_run(T0d, Cid, to_dev(g, torch.float64), gT0, gCi, ws, False, *sc, 7, 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(gT0), rT0)
    np.testing.assert_array_equal(to_host(gCi), rCi)


def test_python_binding_rejects(lib):
    T = torch.zeros((4, 5, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        lib.step(T[:, :, :5], T, T, 1.0, 1e-3, 1.0, 1.0, 1.0)            # shape mismatch
    with pytest.raises(ValueError):
        lib.step(torch.zeros_like(T).transpose(0, 2), T, T, 1.0, 1e-3, 1.0, 1.0, 1.0)   # not contiguous
    with pytest.raises(lib.Diff3dError):
        lib.step(T, T, torch.zeros_like(T), 1.0, 1e-3, 1.0, 1.0, 1.0)     # T2 aliases T
    with pytest.raises(TypeError):
        lib.step(T.half(), T.half(), T.half(), 1.0, 1e-3, 1.0, 1.0, 1.0)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        lib.run(T, torch.empty_like(T), T.clone(), 1.0, 1e-3, 1.0, 1.0, 1.0, 10, ckpt=ws, ckpt_every=3)
    # host buffers never reach the library (a GPU kernel would fault on them)
    g, gT0, gCi = torch.zeros_like(T), torch.empty_like(T), torch.empty_like(T)
    wsz = lib.adjoint_workspace_bytes(T.shape, 10, 3, torch.float64)
    for bad_ws in (torch.empty(wsz, dtype=torch.uint8), torch.empty(2 * wsz, dtype=torch.uint8, device="cuda")[::2]):
        with pytest.raises(ValueError):
            lib.adjoint_run(T, T, g, gT0, gCi, bad_ws, False, 1.0, 1e-3, 1.0, 1.0, 1.0, 10, 3)
    with pytest.raises(ValueError):
        lib.run(T, torch.empty_like(T), T.clone(), 1.0, 1e-3, 1.0, 1.0, 1.0, 10,
                ckpt=torch.empty(wsz, dtype=torch.uint8), ckpt_every=3)
    src = torch.ones(64, dtype=torch.uint8, device="cuda")
    for dst in (torch.empty(64, dtype=torch.uint8), torch.empty(128, dtype=torch.uint8, device="cuda")[::2]):
        with pytest.raises(ValueError):
            lib.copy_(dst, src)
    with pytest.raises(ValueError):
        lib.copy_(torch.empty(64, dtype=torch.uint8, device="cuda"), torch.ones(64, dtype=torch.uint8))
    # a configuration the library does not instantiate is refused before any launch
    with pytest.raises(lib.Diff3dError):
        lib.run(T, torch.empty_like(T), T.clone(), 1.0, 1e-3, 1.0, 1.0, 1.0, 10,
                cfg=lib.Config(zmarch=lib.Tile(p=(3, 3, 3, 3))))


def test_side_stream(lib):
    """Work is enqueued on the caller's current stream: the time loop and the
    reverse sweep run inside a side stream give the default stream's bits."""
    import oracle
    from helpers import to_dev
    shape = (20, 40, 96)
    rng = np.random.default_rng(77)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    g = rng.standard_normal(shape)
    s = oracle.scalars(shape[2], shape[1], shape[0], Ci)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    nt, C = 30, 6

    def run_all():
        T, Cd, gd = to_dev(T0, torch.float64), to_dev(Ci, torch.float64), to_dev(g, torch.float64)
        ws = torch.zeros(lib.adjoint_workspace_bytes(shape, nt, C, torch.float64), dtype=torch.uint8, device="cuda")
        T2 = torch.empty_like(T)
        Tn = T.clone()
        lib.run(Tn, T2, Cd, *sc, nt, ckpt=ws, ckpt_every=C)
        gT0, gCi = torch.empty_like(T), torch.empty_like(T)
        lib.adjoint_run(T, Cd, gd, gT0, gCi, ws, True, *sc, nt, C)
        return Tn, gT0, gCi

    ref = run_all()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = run_all()
    side.synchronize()
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


def test_bench_json_contract():
    """bench.py prints one JSON line with the keys and units of the contract:
    whole-job T_eff, the roofline of its dominant kernel (measured on the
    stream the kernel runs on) and, for one GPU only, no scaling claims."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--quick", "--steps", "2", "--warmup", "1"],
                       cwd=root, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["unit"] == "GB/s"
    assert d["value"] > 0 and d["higher_is_better"] is True and d["dtype"] == "f64"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert "workload" in d["config"]
    # more than one GPU is refused with a message
    r2 = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                        capture_output=True, text=True, timeout=120)
    assert r2.returncode != 0 and "one GPU" in r2.stderr
