"""The large gradient form: 1024^3 FP32 (4.3 GB per field), a checkpoint
every 32 steps (at nt = 500 a workspace of 26 fields, about 112 GB; here
nt = 40), 64-bit offsets."""
import numpy as np
import pytest

import oracle
import workloads
from helpers import norm_rel, oracle_forward_at, oracle_reverse_at, sample_points, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_grad1024_fp32_sampled(lib):
    """Forward nt=40 (two segments of the 32-step checkpoint layout) and the
    reverse sweep at 1024^3 FP32, sampled points against the FP64 oracle on
    sub-boxes; the FP32 error is reported and bounded."""
    n, nt, C = 1024, 40, 32
    field = n ** 3 * 4
    need = lib.adjoint_workspace_bytes((n, n, n), nt, C, torch.float32) + 7 * field
    free, total = torch.cuda.mem_get_info()
    if free < need + 4e9:
        pytest.skip("needs %.0f GB of free device memory" % (need / 1e9))
    T0h = workloads.uniform(n, n, n, workloads.SEED_T0)
    Cih = np.full((n, n, n), 0.5)
    s = oracle.scalars(n, n, n, Cih)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    T0 = torch.from_numpy(T0h.astype(np.float32)).cuda()
    Ci = torch.full((n, n, n), 0.5, dtype=torch.float32, device="cuda")
    ws = torch.empty(lib.adjoint_workspace_bytes(T0.shape, nt, C, torch.float32), dtype=torch.uint8, device="cuda")
    T = T0.clone()
    lib.run(T, torch.empty_like(T), Ci, *sc, nt, ckpt=ws, ckpt_every=C)
    g = workloads.direction(n, n, n)
    gd = torch.from_numpy(g.astype(np.float32)).cuda()
    gT0, gCi = torch.empty_like(T0), torch.empty_like(T0)
    lib.adjoint_run(T0, Ci, gd, gT0, gCi, ws, True, *sc, nt, C)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pts = sample_points((n, n, n), rng, 4)
    # the FP32 inputs as the oracle sees them
    T0q = T0h.astype(np.float32).astype(np.float64)
    gq = g.astype(np.float32).astype(np.float64)
    idx = tuple(np.array(p) for p in zip(*pts))
    got_T = to_host(T[idx])
    got_g0 = to_host(gT0[idx])
    got_gc = to_host(gCi[idx])
    del T, gT0, gCi, ws, gd, T0, Ci
    torch.cuda.empty_cache()
    ref_T = oracle_forward_at(T0q, Cih, s, nt, pts)
    ref_g0, ref_gc = oracle_reverse_at(T0q, Cih, gq, s, nt, pts)
    e_T, e_g0 = norm_rel(got_T, ref_T), norm_rel(got_g0, ref_g0)
    e_gc = float(np.max(np.abs(got_gc - ref_gc)) / max(np.max(np.abs(ref_gc)), 1e-30))
    print("1024^3 FP32 vs FP64 oracle at sampled points: T %.2e gT0 %.2e gCi %.2e" % (e_T, e_g0, e_gc), flush=True)
    assert e_T <= 1e-5 and e_g0 <= 1e-5 and e_gc <= 1e-4


def _errors(a32, b64):
    """(max |a - b| / max |b|, max_i |a_i - b_i| / |b_i|) over the whole
    grid, in z-slabs to bound the temporaries."""
    num = den = rel = 0.0
    for z in range(0, b64.shape[0], 128):
        a = a32[z:z + 128].double()
        b = b64[z:z + 128]
        d = (a - b).abs()
        num = max(num, float(d.max()))
        den = max(den, float(b.abs().max()))
        rel = max(rel, float((d / b.abs().clamp_min(1e-300)).max()))
    return num / den, rel


def test_c5_forward_whole_grid_against_fp64(lib):
    """The large form's forward as configured (1024^3 FP32, nt = 500, a
    checkpoint every 32 steps) on the whole grid: every checkpoint and the
    final state against the FP64 time loop from the same FP32 initial state
    (the FP64 loop is bit-identical to the oracle on every grid the oracle
    can run), and the maximum principle (constant Ci: values stay within the
    initial range, up to a few FP32 roundings).  Error bound: each step
    rounds a handful of FP32 operations (relative 5u, u = 2^-24) and the
    scheme does not amplify errors, so after nt steps the normwise error is
    at most nt * 5u = 1.5e-4; the maximum relative error is reported."""
    n, nt, C = 1024, 500, 32
    field4, field8 = n ** 3 * 4, n ** 3 * 8
    ws_bytes = lib.adjoint_workspace_bytes((n, n, n), nt, C, torch.float32)
    need = ws_bytes + 3 * field4 + 3 * field8 + 2e9
    free, total = torch.cuda.mem_get_info()
    if free < need + 4e9:
        pytest.skip("needs %.0f GB of free device memory" % (need / 1e9))
    T0f = workloads.uniform(n, n, n, workloads.SEED_T0).astype(np.float32)
    s = oracle.scalars(n, n, n, np.full((n, n, n), 0.5))
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    lo, hi = float(T0f.min()), float(T0f.max())
    T32 = torch.from_numpy(T0f).cuda()
    T64 = T32.double()
    del T0f
    Ci32 = torch.full((n, n, n), 0.5, dtype=torch.float32, device="cuda")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    lib.run(T32, torch.empty_like(T32), Ci32, *sc, nt, ckpt=ws, ckpt_every=C)
    Ci64 = torch.full((n, n, n), 0.5, dtype=torch.float64, device="cuda")
    S64 = torch.empty_like(T64)
    stride = (field4 + 255) // 256 * 256
    tol = 4 * 2.0 ** -24
    worst = (0.0, 0.0)
    done = 0
    for j in range(1, (nt - 1) // C + 1):
        lib.run(T64, S64, Ci64, *sc, j * C - done)
        done = j * C
        slot = ws[(j - 1) * stride:(j - 1) * stride + field4].view(torch.float32).view(n, n, n)
        e = _errors(slot, T64)
        worst = (max(worst[0], e[0]), max(worst[1], e[1]))
        assert float(slot.min()) >= lo - tol and float(slot.max()) <= hi + tol, j
    lib.run(T64, S64, Ci64, *sc, nt - done)
    e = _errors(T32, T64)
    torch.cuda.synchronize()
    print("1024^3 FP32 nt=500 vs the FP64 time loop, whole grid: checkpoints normwise %.2e max rel %.2e, "
          "final normwise %.2e max rel %.2e" % (worst[0], worst[1], e[0], e[1]), flush=True)
    bound = nt * 5 * 2.0 ** -24
    inside = float(T32.min()) >= lo - tol and float(T32.max()) <= hi + tol
    del T32, T64, S64, Ci32, Ci64, ws, slot
    torch.cuda.empty_cache()
    assert worst[0] <= bound and e[0] <= bound
    assert inside


def _normwise(a32, b64):
    """max |a - b| / max |b| over the whole grid, in z-slabs."""
    num = den = 0.0
    for z in range(0, b64.shape[0], 128):
        b = b64[z:z + 128]
        num = max(num, float((a32[z:z + 128].double() - b).abs().max()))
        den = max(den, float(b.abs().max()))
    return num / max(den, 1e-300)


def test_c5_adjoint_whole_grid_against_fp64(lib):
    """The large form's reverse sweep as configured (1024^3 FP32, nt = 500, a
    checkpoint every 32 steps): gT0 and gCi on the whole grid against the
    FP64 reverse sweep of the same FP32 inputs.  The FP64 sweep is the
    library's (bit-identical to the oracle on every grid the oracle can run),
    taken in five parts of 100 steps to fit in memory: part p starts from
    T_{100p} (the FP64 time loop from T0) with the multiplier the later parts
    returned, and the Ci gradient is the sum of the parts' (this changes only
    the FP64 summation order of gCi).  Bounds: gT0 is the transposed time
    loop, so as for the forward at most nt * 5u = 1.5e-4 normwise (u =
    2^-24); gCi sums nt products of such multipliers and Laplacians, gated at
    1e-4 of its largest magnitude."""
    n, nt, C = 1024, 500, 32
    parts, C64 = 5, 17
    lp = nt // parts
    field4, field8 = n ** 3 * 4, n ** 3 * 8
    ws32 = lib.adjoint_workspace_bytes((n, n, n), nt, C, torch.float32)
    ws64 = lib.adjoint_workspace_bytes((n, n, n), lp, C64, torch.float64)
    need = max(ws32 + 5 * field4, ws64 + 8 * field8 + 3 * field4) + 2e9
    free, total = torch.cuda.mem_get_info()
    if free < need + 4e9:
        pytest.skip("needs %.0f GB of free device memory" % (need / 1e9))
    s = oracle.scalars(n, n, n, np.full((n, n, n), 0.5))
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    T0 = torch.from_numpy(workloads.uniform(n, n, n, workloads.SEED_T0).astype(np.float32)).cuda()
    gd = torch.from_numpy(workloads.direction(n, n, n).astype(np.float32)).cuda()
    Ci = torch.full((n, n, n), 0.5, dtype=torch.float32, device="cuda")
    gT0, gCi = torch.empty_like(T0), torch.empty_like(T0)
    ws = torch.empty(ws32, dtype=torch.uint8, device="cuda")
    print("1024^3 FP32 adjoint, nt=500, C=32", flush=True)
    lib.adjoint_run(T0, Ci, gd, gT0, gCi, ws, False, *sc, nt, C)
    torch.cuda.synchronize()
    del ws, Ci
    torch.cuda.empty_cache()
    T64 = T0.double()
    lam = gd.double()
    del T0, gd
    Ci64 = torch.full((n, n, n), 0.5, dtype=torch.float64, device="cuda")
    gtot = torch.zeros_like(T64)
    gpart, out, Ts, S = (torch.empty_like(T64) for _ in range(4))
    ws = torch.empty(ws64, dtype=torch.uint8, device="cuda")
    for p in reversed(range(parts)):
        print("FP64 reference, steps %d..%d" % (p * lp, (p + 1) * lp - 1), flush=True)
        Ts.copy_(T64)
        if p:
            lib.run(Ts, S, Ci64, *sc, p * lp)
        lib.adjoint_run(Ts, Ci64, lam, out, gpart, ws, False, *sc, lp, C64)
        gtot += gpart
        lam, out = out, lam
    torch.cuda.synchronize()
    del ws, gpart, out, Ts, S, Ci64, T64
    torch.cuda.empty_cache()
    e_g0, e_gc = _normwise(gT0, lam), _normwise(gCi, gtot)
    print("1024^3 FP32 nt=500 C=32 reverse vs FP64, whole grid: gT0 normwise %.2e, gCi normwise %.2e"
          % (e_g0, e_gc), flush=True)
    del gT0, gCi, lam, gtot
    torch.cuda.empty_cache()
    assert e_g0 <= nt * 5 * 2.0 ** -24
    assert e_gc <= 1e-4
