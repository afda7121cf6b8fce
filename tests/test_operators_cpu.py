"""Pins for the oracle's finite-difference operators (CPU only).

Fig. 1 writes the step with @inn, @d2_xi, @d2_yi and @d2_zi; the paper does
not print their definitions.  The oracle reads @d2_xi as the difference of
the two one-sided differences.  These tests pin oracle.apply (FP64) and
oracle.emulate_apply32 (FP32 arithmetic) against things other than
themselves:

* exact rational arithmetic on small grids, with the second difference
  written the other way round (A[p] - 2A[c] + A[m]) -- dyadic inputs make
  every FP64 operation exact, so any slip of index, stride, sign or axis
  shows as a mismatch;
* quadratics, whose second differences are constants (2a per axis in index
  units) and linear fields, whose second differences vanish;
* an axis permutation (d2 along y of A is d2 along x of A with x and y
  swapped);
* the sine mode, an eigenvector of the discrete Laplacian with a closed-form
  eigenvalue;
* the step itself: one oracle time step equals the update formed from the
  Laplacian operator (which ties the operators to the pinned step);
* numpy float32 arithmetic for the FP32 emulation.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

OPS3 = (oracle.OP_INN, oracle.OP_D2_XI, oracle.OP_D2_YI, oracle.OP_D2_ZI, oracle.OP_LAP)
OPS2 = (oracle.OP_INN, oracle.OP_D2_XI, oracle.OP_D2_YI, oracle.OP_LAP)


def _dyadic(shape, seed, bits=10):
    """Random values k / 2^bits, k in [-2^bits, 2^bits]: sums and differences
    of a few of them, and products with powers of two, are exact in FP64 and
    in FP32."""
    rng = np.random.default_rng(seed)
    return rng.integers(-2 ** bits, 2 ** bits + 1, size=shape).astype(np.float64) / 2 ** bits


def _exact_op(op, A, cx, cy, cz):
    """The operator in exact rationals over the dictionary of grid values,
    second difference as A[p] - 2*A[c] + A[m]."""
    twod = A.ndim == 2
    B = A[None] if twod else A
    nz, ny, nx = B.shape
    F = {(z, y, x): Fraction(float(B[z, y, x])) for z in range(nz) for y in range(ny) for x in range(nx)}
    zr = range(0, 1) if twod else range(1, nz - 1)
    out = []
    for z in zr:
        for y in range(1, ny - 1):
            for x in range(1, nx - 1):
                c = F[(z, y, x)]
                dx = F[(z, y, x + 1)] - 2 * c + F[(z, y, x - 1)]
                dy = F[(z, y + 1, x)] - 2 * c + F[(z, y - 1, x)]
                dz = 0 if twod else F[(z + 1, y, x)] - 2 * c + F[(z - 1, y, x)]
                out.append({oracle.OP_INN: c, oracle.OP_D2_XI: dx, oracle.OP_D2_YI: dy, oracle.OP_D2_ZI: dz,
                            oracle.OP_LAP: dx * cx + dy * cy + dz * cz}[op])
    shape = tuple(n - 2 for n in A.shape)
    return np.array(out, dtype=object).reshape(shape)


@pytest.mark.parametrize("op", OPS3)
def test_apply3d_exact_rational(op):
    A = _dyadic((5, 4, 6), seed=11 + op)
    rd = (2.0, 0.5, 4.0)          # powers of two: the weights are exact
    got = oracle.apply(op, A, *rd)
    want = _exact_op(op, A, *(Fraction(r) * Fraction(r) for r in rd))
    assert got.shape == (3, 2, 4)
    assert all(Fraction(float(g)) == w for g, w in zip(got.ravel(), want.ravel()))


@pytest.mark.parametrize("op", OPS2)
def test_apply2d_exact_rational(op):
    A = _dyadic((5, 7), seed=23 + op)
    rd = (0.25, 8.0, 3.0)
    got = oracle.apply(op, A, *rd)
    want = _exact_op(op, A, Fraction(rd[0]) ** 2, Fraction(rd[1]) ** 2, 0)
    assert got.shape == (3, 5)
    assert all(Fraction(float(g)) == w for g, w in zip(got.ravel(), want.ravel()))


def test_apply_quadratic_and_linear():
    nz, ny, nx = 6, 7, 9
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c = 3.0, -5.0, 7.0
    A = a * x * x + b * y * y + c * z * z + 2.0 * x - 3.0 * y + 4.0 * z + 1.0
    assert np.all(oracle.apply(oracle.OP_D2_XI, A) == 2 * a)
    assert np.all(oracle.apply(oracle.OP_D2_YI, A) == 2 * b)
    assert np.all(oracle.apply(oracle.OP_D2_ZI, A) == 2 * c)
    rd = (2.0, 4.0, 0.5)
    lap = 2 * a * rd[0] ** 2 + 2 * b * rd[1] ** 2 + 2 * c * rd[2] ** 2
    assert np.all(oracle.apply(oracle.OP_LAP, A, *rd) == lap)
    L = 2.0 * x - 3.0 * y + 4.0 * z + 1.0
    for op in (oracle.OP_D2_XI, oracle.OP_D2_YI, oracle.OP_D2_ZI, oracle.OP_LAP):
        assert np.all(oracle.apply(op, L, *rd) == 0.0)
    # constants are preserved exactly whatever their value
    K = np.full((nz, ny, nx), 0.1)
    assert np.all(oracle.apply(oracle.OP_LAP, K, 3.0, 7.0, 11.0) == 0.0)
    assert np.array_equal(oracle.apply(oracle.OP_INN, A), A[1:-1, 1:-1, 1:-1])


def test_apply_axis_permutation():
    A = np.random.default_rng(5).random((7, 5, 6))
    At = np.ascontiguousarray(A.transpose(0, 2, 1))      # x <-> y
    assert np.array_equal(oracle.apply(oracle.OP_D2_YI, A), oracle.apply(oracle.OP_D2_XI, At).transpose(0, 2, 1))
    Az = np.ascontiguousarray(A.transpose(2, 1, 0))      # x <-> z
    assert np.array_equal(oracle.apply(oracle.OP_D2_ZI, A), oracle.apply(oracle.OP_D2_XI, Az).transpose(2, 1, 0))
    A2 = A[3]
    assert np.array_equal(oracle.apply(oracle.OP_D2_YI, A2),
                          oracle.apply(oracle.OP_D2_XI, np.ascontiguousarray(A2.T)).T)


def test_apply_sine_mode_eigenvalue():
    """sin(p pi i/(n-1)) per axis is an eigenvector of the weighted second
    difference: Lap = -sum_d 4 sin^2(p_d pi/(2(n_d-1))) c_d times the mode."""
    n = (12, 10, 14)                    # (nz, ny, nx)
    p = (3, 2, 5)
    rd = (13.0, 9.0, 11.0)              # rdx, rdy, rdz
    i = [np.arange(m) for m in n]
    mz, my, mx = (np.sin(pp * math.pi * ii / (m - 1)) for pp, ii, m in zip(p, i, n))
    A = mz[:, None, None] * my[None, :, None] * mx[None, None, :]
    kappa = (4 * math.sin(p[2] * math.pi / (2 * (n[2] - 1))) ** 2 * rd[0] ** 2
             + 4 * math.sin(p[1] * math.pi / (2 * (n[1] - 1))) ** 2 * rd[1] ** 2
             + 4 * math.sin(p[0] * math.pi / (2 * (n[0] - 1))) ** 2 * rd[2] ** 2)
    got = oracle.apply(oracle.OP_LAP, A, *rd)
    want = -kappa * A[1:-1, 1:-1, 1:-1]
    assert np.max(np.abs(got - want)) <= 1e-12 * kappa


def test_step_is_update_of_laplacian():
    """One oracle step on the interior equals t + dt*((lam*Ci)*Lap(T)) with
    Lap from the operator, bit for bit (the step's evaluation order)."""
    rng = np.random.default_rng(9)
    T = rng.random((9, 8, 11))
    Ci = 0.5 + 0.5 * rng.random((9, 8, 11))
    lam, dt, rd = 1.0, 1e-3, (10.0, 9.0, 7.0)
    T1 = oracle.forward(T, Ci, lam, dt, *rd, 1)
    lap = oracle.apply(oracle.OP_LAP, T, *rd)
    inn = (slice(1, -1),) * 3
    assert np.array_equal(T1[inn], T[inn] + dt * ((lam * Ci[inn]) * lap))


def test_step2d_is_update_of_laplacian():
    rng = np.random.default_rng(10)
    T = rng.random((13, 17))
    Ci = 0.5 + 0.5 * rng.random((13, 17))
    lam, dt, rd = 1.0, 1e-3, (10.0, 9.0)
    T1 = oracle.forward2d(T, Ci, lam, dt, *rd, 1)
    lap = oracle.apply(oracle.OP_LAP, T, *rd)
    assert np.array_equal(T1[1:-1, 1:-1], T[1:-1, 1:-1] + dt * ((lam * Ci[1:-1, 1:-1]) * lap))


def _np32(op, A, rd):
    """The operators in numpy float32 arithmetic (each numpy float32 operation
    rounds once, as IEEE single precision), by slicing."""
    A = A.astype(np.float32)
    cx, cy, cz = (np.float32(r * r) for r in rd)
    if A.ndim == 2:
        t = A[1:-1, 1:-1]
        dx = (A[1:-1, 2:] - t) - (t - A[1:-1, :-2])
        dy = (A[2:, 1:-1] - t) - (t - A[:-2, 1:-1])
        return {oracle.OP_INN: t, oracle.OP_D2_XI: dx, oracle.OP_D2_YI: dy, oracle.OP_LAP: dx * cx + dy * cy}[op]
    t = A[1:-1, 1:-1, 1:-1]
    dx = (A[1:-1, 1:-1, 2:] - t) - (t - A[1:-1, 1:-1, :-2])
    dy = (A[1:-1, 2:, 1:-1] - t) - (t - A[1:-1, :-2, 1:-1])
    dz = (A[2:, 1:-1, 1:-1] - t) - (t - A[:-2, 1:-1, 1:-1])
    return {oracle.OP_INN: t, oracle.OP_D2_XI: dx, oracle.OP_D2_YI: dy, oracle.OP_D2_ZI: dz,
            oracle.OP_LAP: (dx * cx + dy * cy) + dz * cz}[op]


@pytest.mark.parametrize("op", OPS3)
def test_emulate_apply32_matches_numpy_float32(op):
    A = np.random.default_rng(31 + op).random((7, 6, 9))
    rd = (10.3, 9.7, 7.1)
    got = oracle.emulate_apply32(op, A.astype(np.float32), oracle.ST_F32, *rd)
    assert got.dtype == np.float32
    assert np.array_equal(got, _np32(op, A, rd))


@pytest.mark.parametrize("op", OPS2)
def test_emulate_apply32_2d_matches_numpy_float32(op):
    A = np.random.default_rng(41 + op).random((8, 10))
    rd = (10.3, 9.7, 1.0)
    got = oracle.emulate_apply32(op, A.astype(np.float32), oracle.ST_F32, *rd)
    assert np.array_equal(got, _np32(op, A, rd))


@pytest.mark.parametrize("op", OPS3)
def test_emulate_apply32_bf16_is_f32_of_widened(op):
    """BF16 storage: the operator of the exactly widened values."""
    h = np.random.default_rng(51 + op).integers(0x3C00, 0x3F80, size=(5, 6, 7)).astype(np.uint16)
    w = oracle.bf16_widen(h)
    for st in (oracle.ST_BF16_SR, oracle.ST_BF16_RNE):
        assert np.array_equal(oracle.emulate_apply32(op, h, st, 3.0, 5.0, 7.0),
                              oracle.emulate_apply32(op, w, oracle.ST_F32, 3.0, 5.0, 7.0))


def test_emulate_apply32_exact_on_dyadic():
    A = _dyadic((5, 4, 6), seed=77, bits=8)
    for op in OPS3:
        got = oracle.emulate_apply32(op, A.astype(np.float32), oracle.ST_F32, 2.0, 0.5, 4.0)
        assert np.array_equal(got.astype(np.float64), oracle.apply(op, A, 2.0, 0.5, 4.0))


def test_apply_rejects_bad_arguments():
    A2 = np.zeros((5, 6))
    with pytest.raises(ValueError):
        oracle.apply(oracle.OP_D2_ZI, A2)
    with pytest.raises(ValueError):
        oracle.apply(7, np.zeros((4, 4, 4)))
    with pytest.raises(ValueError):
        oracle.emulate_apply32(oracle.OP_D2_ZI, A2.astype(np.float32), oracle.ST_F32)
