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
