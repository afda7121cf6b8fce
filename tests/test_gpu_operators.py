"""The finite-difference operators on the GPU (diff3d_apply) against the
oracle, bit for bit: FP64 fields against oracle.apply, FP32 and BF16 fields
against the FP32 emulation of the same operators on the same stored values.

The operators are the device functions every stencil of the library is
built of (interior selection, second differences along x, y and z, the
weighted Laplacian of Fig. 1's step), so these tests also pin the operation
order the steps use.  Grids are ragged (no dimension a multiple of the
256-point runs or of any tile) and span several runs along x; one case has
more (row, run) pairs than the launch's grid, so the grid-stride loop wraps.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import stored, to_dev

pytestmark = pytest.mark.gpu

OPS3 = ("INN", "D2_XI", "D2_YI", "D2_ZI", "LAP")
OPS2 = ("INN", "D2_XI", "D2_YI", "LAP")
RD = (63.0, 37.0, 19.0)
DTYPES = (torch.float64, torch.float32, torch.bfloat16)


def _op(mod, name):
    return getattr(mod, "OP_" + name)


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    return 0.25 + rng.random(shape)


def _expect(name, A, dtype, rd):
    if dtype == torch.float64:
        return oracle.apply(_op(oracle, name), A, *rd)
    st = oracle.ST_F32 if dtype == torch.float32 else oracle.ST_BF16_RNE
    return oracle.emulate_apply32(_op(oracle, name), stored(A, dtype), st, *rd)


def _check(lib, name, A, dtype, rd=RD):
    print("apply", name, A.shape, dtype, flush=True)
    dev = to_dev(A, dtype)
    got = lib.apply(_op(lib, name), dev, *rd)
    torch.cuda.synchronize()
    want = _expect(name, A, dtype, rd)
    g = got.cpu().numpy()
    assert g.dtype == want.dtype and g.shape == want.shape
    assert np.array_equal(g.view(np.uint64 if g.itemsize == 8 else np.uint32),
                          want.view(np.uint64 if want.itemsize == 8 else np.uint32)), \
        "%s %s %s: %d of %d differ" % (name, A.shape, dtype, int((g != want).sum()), g.size)


@pytest.mark.parametrize("dtype", DTYPES, ids=("f64", "f32", "bf16"))
@pytest.mark.parametrize("name", OPS3)
def test_apply3d_matches_oracle(lib, name, dtype):
    _check(lib, name, _field((19, 35, 603), seed=3), dtype)


@pytest.mark.parametrize("dtype", DTYPES, ids=("f64", "f32", "bf16"))
@pytest.mark.parametrize("name", OPS2)
def test_apply2d_matches_oracle(lib, name, dtype):
    _check(lib, name, _field((517, 131), seed=4), dtype)


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (4, 3, 258), (5, 7, 257)])
def test_apply_small_and_edge_shapes(lib, shape):
    A = _field(shape, seed=5)
    for name in OPS3:
        _check(lib, name, A, torch.float64)
    A2 = A[0]
    for name in OPS2:
        _check(lib, name, A2, torch.float32)


def test_apply_grid_stride_wraps(lib):
    """(ny-2)*(nz-2) rows of one run each exceed the launch's 2^20 workgroups."""
    A = _field((1030, 1026, 40), seed=6)
    assert (1030 - 2) * (1026 - 2) > (1 << 20)
    for name in ("D2_ZI", "LAP"):
        _check(lib, name, A, torch.float32)


def test_apply_bf16_either_rounding_code(lib):
    """Both BF16 codes widen the stored bits the same way."""
    A = _field((9, 10, 70), seed=7)
    dev = to_dev(A, torch.bfloat16)
    nz, ny, nx = dev.shape
    outs = []
    for code in (lib.BF16, lib.BF16_RNE):
        out = torch.empty((nz - 2, ny - 2, nx - 2), dtype=torch.float32, device="cuda")
        rc = lib._lib.diff3d_apply(lib.OP_LAP, lib._p(out), lib._p(dev), nx, ny, nz, *RD, code, lib._stream(dev))
        assert rc == lib.OK
        outs.append(out)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_apply_out_argument_and_composition(lib):
    """`out=` is filled in place; and one GPU step equals the update formed
    from the GPU Laplacian with the oracle's arithmetic (so the step and the
    operator share their operation order)."""
    A = _field((11, 12, 77), seed=8)
    Ci = 0.5 + 0.25 * _field((11, 12, 77), seed=9)
    T = to_dev(A, torch.float64)
    C = to_dev(Ci, torch.float64)
    out = torch.empty((9, 10, 75), dtype=torch.float64, device="cuda")
    assert lib.apply(lib.OP_LAP, T, *RD, out=out) is out
    lam, dt = 1.0, 2e-5
    T2 = T.clone()
    lib.step(T2, T, C, lam, dt, *RD)
    torch.cuda.synchronize()
    lap = out.cpu().numpy()
    inn = (slice(1, -1),) * 3
    want = A[inn] + dt * ((lam * Ci[inn]) * lap)
    assert np.array_equal(T2.cpu().numpy()[inn], want)


def test_apply_python_validation(lib):
    A = torch.zeros((6, 6, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        lib.apply(lib.OP_INN, A.cpu())
    with pytest.raises(ValueError):
        lib.apply(lib.OP_INN, A, out=torch.empty((4, 4, 4), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        lib.apply(lib.OP_INN, A, out=torch.empty((4, 4, 4), dtype=torch.float64))
    with pytest.raises(lib.Diff3dError):
        lib.apply(lib.OP_D2_ZI, A[0].contiguous())
