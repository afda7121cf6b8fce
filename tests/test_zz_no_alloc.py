"""The allocation-free loss entry point (diff3d_loss_noalloc) against
diff3d_loss through the C ABI: the same kernels with the partial sums in the
library's fixed per-GPU array instead of caller scratch, so the loss, the
seed and every bit must agree; two calls in a row, the second on a smaller
input (the array keeps the first call's partials, which must not leak)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _call_both(lib, T, Tt, code):
    n = T.numel()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    acc = torch.full((lib.REDUCE_DOUBLES,), float("nan"), dtype=torch.float64, device="cuda")
    seed_a = torch.full_like(T, float("nan"))
    rc = lib._lib.diff3d_loss(ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(Tt.data_ptr()),
                              ctypes.c_void_p(seed_a.data_ptr()), n, code, ctypes.c_void_p(acc.data_ptr()), stream)
    assert rc == lib.OK
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    seed_b = torch.full_like(T, float("nan"))
    rc = lib._lib.diff3d_loss_noalloc(ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(Tt.data_ptr()),
                                      ctypes.c_void_p(seed_b.data_ptr()), n, code, ctypes.c_void_p(out.data_ptr()),
                                      stream)
    assert rc == lib.OK
    torch.cuda.synchronize()
    return acc[0].item(), out[0].item(), seed_a, seed_b


@pytest.mark.parametrize("dtype,code", [(torch.float64, 0), (torch.float32, 1), (torch.bfloat16, 2)])
def test_noalloc_loss_matches_scratch_loss(lib, dtype, code):
    rng = np.random.default_rng(7)
    for n in (3 * 1024 * 256 + 77, 1000):          # 1024 partials, then 4
        T = torch.from_numpy(rng.random((1, 1, n))).to(dtype).cuda()
        Tt = torch.from_numpy(rng.random((1, 1, n))).to(dtype).cuda()
        a, b, sa, sb = _call_both(lib, T, Tt, code)
        assert a == b and np.isfinite(a)
        assert torch.equal(sa, sb)
        r = T.double().cpu().numpy() - Tt.double().cpu().numpy()
        assert b == pytest.approx(0.5 * float(np.sum(r * r)), rel=1e-12)


def test_noalloc_loss_python_wrapper_and_rejects(lib):
    T = torch.rand((8, 9, 10), dtype=torch.float64, device="cuda")
    Tt = torch.rand_like(T)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    lib.loss_into(out, T, Tt)
    assert out.item() == lib.loss(T, Tt).item()
    with pytest.raises(ValueError):
        lib.loss_into(torch.empty(1, dtype=torch.float64), T, Tt)       # host output
    assert lib._lib.diff3d_loss_noalloc(None, None, None, 10, 0, None, None) == lib.EINVAL
    p = ctypes.c_void_p(T.data_ptr())
    assert lib._lib.diff3d_loss_noalloc(p, p, None, 1 << 40, 0, ctypes.c_void_p(out.data_ptr()), None) == lib.EINVAL
    assert lib._lib.diff3d_loss_noalloc(p, p, None, 0, 0, ctypes.c_void_p(out.data_ptr()), None) == lib.EINVAL
    assert lib._lib.diff3d_loss_noalloc(p, p, None, 10, 9, ctypes.c_void_p(out.data_ptr()), None) == lib.EDTYPE
