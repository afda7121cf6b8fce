"""Pins for the oracle (CPU only).

Each test checks the oracle against something other than itself: a closed
form, an invariant, exact rational arithmetic, an explicit matrix, a
complex-step derivative, finite differences or the paper's own initial
state.  A plausible slip anywhere in the oracle (a dropped term, a wrong
sign, index or stride, a transposed operand, a missing boundary term in the
reverse sweep) fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from oracle import brute

EPS = np.finfo(np.float64).eps
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scal(nx, ny, nz, Ci, lx=1.0, ly=1.0, lz=1.0, lam=1.0, divisor=None):
    s = oracle.scalars(nx, ny, nz, Ci, lam=lam, lx=lx, ly=ly, lz=lz)
    if divisor is not None:
        s["dt"] = s["dt"] * 6.1 / divisor
    return s


def _fwd(T0, Ci, s, nt):
    return oracle.forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)


def _rev(T0, Ci, g, s, nt, keep=1):
    return oracle.reverse(T0, Ci, g, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt, keep=keep)


def sine_mode(nx, ny, nz, p):
    """prod_d sin(p_d*pi*i_d/(n_d-1)) with the boundary set to exactly 0."""
    sx = np.sin(p[0] * np.pi * np.arange(nx) / (nx - 1))
    sy = np.sin(p[1] * np.pi * np.arange(ny) / (ny - 1))
    sz = np.sin(p[2] * np.pi * np.arange(nz) / (nz - 1))
    s = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    s[0, :, :] = s[-1, :, :] = 0.0
    s[:, 0, :] = s[:, -1, :] = 0.0
    s[:, :, 0] = s[:, :, -1] = 0.0
    return s


def amplification(nx, ny, nz, p, c, s):
    """g = 1 - dt*lam*c*sum_d 4 sin^2(p_d pi/(2(n_d-1))) (1/h_d)^2 for a sine
    mode at constant Ci = c (the mode is an eigenvector of the Dirichlet
    second difference with eigenvalue -4 sin^2(p pi/(2(n-1))))."""
    kap = 0.0
    for pd, nd, r in zip(p, (nx, ny, nz), (s["rdx"], s["rdy"], s["rdz"])):
        kap += 4.0 * math.sin(pd * math.pi / (2 * (nd - 1))) ** 2 * r * r
    return 1.0 - s["dt"] * s["lam"] * c * kap, kap


# ---------------------------------------------------------------- scalars

def test_scalars_closed_form():
    # dx = 1/(n-1) on the unit domain; dt = dx^2 * 2/6.1 for lam=1, max(Ci)=0.5
    Ci = np.full((4, 5, 64), 0.5)
    s = oracle.scalars(64, 5, 4, Ci)
    assert s["dx"] == 1.0 / 63
    assert s["rdx"] == 1.0 / (1.0 / 63)
    assert s["dt"] == pytest.approx(2.0 / (6.1 * 63 * 63), rel=4 * EPS)
    assert s["dt"] == pytest.approx(8.2607e-5, rel=1e-4)


def test_scalars_max_over_whole_array_including_boundary():
    Ci = np.full((5, 5, 5), 0.5)
    Ci[0, 0, 0] = 2.0          # a corner: outside the interior, still counts
    s = oracle.scalars(5, 5, 5, Ci)
    assert s["dt"] == pytest.approx((0.25 ** 2) / 2.0 / 6.1, rel=4 * EPS)
    for where in ((4, 4, 4), (0, 0, 0), (4, 0, 3)):   # first and last element included
        Ci = np.full((5, 5, 5), 0.5)
        Ci[where] = 4.0
        s = oracle.scalars(5, 5, 5, Ci)
        assert s["dt"] == pytest.approx((0.25 ** 2) / 4.0 / 6.1, rel=4 * EPS)


def test_scalars_min_spacing_and_lengths():
    Ci = np.full((11, 6, 9), 0.5)
    s = oracle.scalars(9, 6, 11, Ci, lx=2.0, ly=0.5, lz=3.0, lam=2.0)
    dx, dy, dz = 2.0 / 8, 0.5 / 5, 3.0 / 10
    assert (s["dx"], s["dy"], s["dz"]) == (dx, dy, dz)
    assert s["dt"] == pytest.approx(dy * dy / 2.0 / 0.5 / 6.1, rel=4 * EPS)


def test_paper_driver_constant_state_is_kept():
    """Fig. 1 starts from T = 1.7 everywhere with Ci = 1/c0: a constant field,
    which the scheme keeps bit for bit ((c - c) - (c - c) = 0 exactly)."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_driver.json")))
    n = 24  # the invariant does not depend on the grid size
    Ci = np.full((n, n, n), 1.0 / g["c0"])
    T0 = np.full((n, n, n), g["T_init"])
    s = _scal(n, n, n, Ci, lx=g["lx"], ly=g["ly"], lz=g["lz"], lam=g["lam"])
    T = _fwd(T0, Ci, s, g["nt"])
    assert np.array_equal(T, T0)
    # and the paper's own dt at its 512^3 grid, as a closed form
    big = oracle.scalars(g["nx"], 3, 3, np.full((3, 3, g["nx"]), 1.0 / g["c0"]),
                         lam=g["lam"], lx=g["lx"], ly=0.01, lz=0.01)
    assert big["dt"] == pytest.approx(2.0 / (g["dt_divisor"] * 511 * 511), rel=4 * EPS)


# ---------------------------------------------------------------- forward

def test_constant_field_bit_exact_random_ci():
    rng = np.random.default_rng(7)
    Ci = 0.5 + 0.5 * rng.random((9, 8, 7))
    T0 = np.full((9, 8, 7), 1.7)
    s = _scal(7, 8, 9, Ci)
    assert np.array_equal(_fwd(T0, Ci, s, 13), T0)


@pytest.mark.parametrize("shape,p,nt", [
    ((17, 13, 11), (1, 1, 1), 30),
    ((17, 13, 11), (1, 2, 3), 30),
    ((17, 13, 11), (15, 11, 9), 30),   # p = n - 2: near-checkerboard mode, |g| close to 1
    ((9, 24, 6), (2, 5, 4), 17),
])
def test_sine_mode_amplification(shape, p, nt):
    nx, ny, nz = shape
    c = 0.5
    Ci = np.full((nz, ny, nx), c)
    s = _scal(nx, ny, nz, Ci, lx=1.0, ly=1.3, lz=0.7)
    g, _ = amplification(nx, ny, nz, p, c, s)
    T0 = sine_mode(nx, ny, nz, p)
    T = _fwd(T0, Ci, s, nt)
    expect = g ** nt * T0
    err = np.max(np.abs(T - expect)) / np.max(np.abs(T0))
    assert err <= 20 * nt * EPS, (g, err)


def test_sine_mode_mixed_with_constant_ci_value():
    # the amplification must scale with Ci and lam as dt*lam*Ci
    nx, ny, nz = 12, 10, 14
    for c, lam in ((0.25, 1.0), (0.5, 2.0), (0.125, 3.0)):
        Ci = np.full((nz, ny, nx), c)
        s = _scal(nx, ny, nz, Ci, lam=lam)
        g, _ = amplification(nx, ny, nz, (2, 1, 3), c, s)
        T0 = sine_mode(nx, ny, nz, (2, 1, 3))
        T = _fwd(T0, Ci, s, 10)
        assert np.max(np.abs(T - g ** 10 * T0)) <= 200 * EPS


def test_max_principle_at_paper_bound():
    nx, ny, nz = 16, 12, 10
    T0, _ = workloads.uniform_const(nx, ny, nz)
    Ci = 0.5 * (1.0 + 0.5 * workloads.uniform(nx, ny, nz, 1))
    s = _scal(nx, ny, nz, Ci)
    for nt in (1, 5, 40):
        T = _fwd(T0, Ci, s, nt)
        assert T.min() >= T0.min() - 4 * EPS
        assert T.max() <= T0.max() + 4 * EPS
    # checkerboard: the least damped mode, still bounded at the 6.1 divisor
    ii = np.indices((nz, ny, nx)).sum(axis=0)
    cb = np.where(ii % 2 == 0, 1.0, -1.0)
    Cc = np.full((nz, ny, nx), 0.5)
    sc = _scal(nx, ny, nz, Cc)
    assert np.max(np.abs(_fwd(cb, Cc, sc, 20))) <= 1.0 + 4 * EPS


def test_max_principle_negative_control():
    """With the divisor below 6 the centre weight turns negative and the
    checkerboard grows: the bound test above is not vacuous."""
    nx = ny = nz = 10
    ii = np.indices((nz, ny, nx)).sum(axis=0)
    cb = np.where(ii % 2 == 0, 1.0, -1.0)
    Ci = np.full((nz, ny, nx), 0.5)
    s = _scal(nx, ny, nz, Ci, divisor=5.5)
    T = _fwd(cb, Ci, s, 1)
    # interior checkerboard point: T*(1 - 12*c*dt/h^2) = T*(1 - 12/5.5)
    assert T[4, 4, 4] == pytest.approx(cb[4, 4, 4] * (1 - 12.0 / 5.5), rel=1e-12)
    assert np.max(np.abs(T)) > 1.0


@pytest.mark.parametrize("shape,nt", [((4, 4, 4), 1), ((4, 4, 4), 2), ((5, 4, 6), 1),
                                      ((5, 4, 6), 3), ((6, 5, 4), 2)])
def test_exact_rational_brute_force(shape, nt):
    nx, ny, nz = shape
    rng = np.random.default_rng(11 + nx + 7 * nz)
    T0 = rng.random((nz, ny, nx))
    Ci = 0.4 + 0.2 * rng.random((nz, ny, nx))
    s = _scal(nx, ny, nz, Ci, lx=1.0, ly=1.7, lz=0.6)
    T = _fwd(T0, Ci, s, nt)
    ex = brute.exact_to_array(brute.exact_forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"],
                                                  s["rdz"], nt), T0.shape)
    exf = ex.astype(np.float64)
    scale = np.max(np.abs(exf))
    err = max(abs(float(ex[i] - Fraction(float(T[i]))))
              for i in np.ndindex(T.shape))
    assert err <= 8 * nt * EPS * scale
    # boundary untouched
    mask = np.ones(T.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(T[mask], T0[mask])


def test_axis_permutation_symmetry():
    n = 11
    T0, _ = workloads.uniform_const(n, n, n)
    Ci = 0.5 * (1.0 + 0.5 * workloads.uniform(n, n, n, 1))
    s = _scal(n, n, n, Ci)
    ref = _fwd(T0, Ci, s, 9)
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)):
        Tp = _fwd(T0.transpose(perm), Ci.transpose(perm), s, 9)
        assert np.max(np.abs(Tp - ref.transpose(perm))) <= 64 * EPS


def test_matrix_forward_agrees():
    nx, ny, nz = 5, 6, 7
    rng = np.random.default_rng(3)
    T0 = rng.random((nz, ny, nx))
    Ci = 0.3 + 0.4 * rng.random((nz, ny, nx))
    s = _scal(nx, ny, nz, Ci, ly=2.0)
    T = _fwd(T0, Ci, s, 4)
    M = brute.matrix_forward(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], 4)
    assert np.max(np.abs(T - M)) <= 64 * EPS


def test_zero_steps_is_identity():
    T0, Ci = workloads.uniform_const(5, 4, 3)
    s = _scal(5, 4, 3, Ci)
    assert np.array_equal(_fwd(T0, Ci, s, 0), T0)


# ---------------------------------------------------------------- reverse

def test_reverse_dot_product():
    nx, ny, nz = 9, 8, 10
    rng = np.random.default_rng(5)
    Ci = 0.5 * (1.0 + 0.5 * rng.random((nz, ny, nx)))
    s = _scal(nx, ny, nz, Ci)
    x = rng.standard_normal((nz, ny, nx))
    y = rng.standard_normal((nz, ny, nx))
    for nt in (1, 7):
        Ax = _fwd(x, Ci, s, nt)
        ATy, _ = _rev(x, Ci, y, s, nt)
        lhs, rhs = float(np.sum(Ax * y)), float(np.sum(x * ATy))
        assert abs(lhs - rhs) <= 1e-13 * (np.sum(np.abs(Ax * y)))


@pytest.mark.parametrize("shape,nt", [((4, 4, 4), 2), ((5, 6, 7), 3), ((7, 5, 4), 1)])
def test_reverse_matches_matrix_transpose(shape, nt):
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 100 + nz)
    T0 = rng.random((nz, ny, nx))
    Ci = 0.4 + 0.2 * rng.random((nz, ny, nx))
    g = rng.standard_normal((nz, ny, nx))
    s = _scal(nx, ny, nz, Ci, lz=1.4)
    gT0, _ = _rev(T0, Ci, g, s, nt)
    ref = brute.matrix_grad_T0(Ci, g, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    assert np.max(np.abs(gT0 - ref)) <= 64 * EPS * np.max(np.abs(ref))


@pytest.mark.parametrize("shape,nt", [((4, 4, 4), 2), ((5, 4, 6), 3)])
def test_reverse_ci_gradient_complex_step(shape, nt):
    nx, ny, nz = shape
    rng = np.random.default_rng(17 + nt)
    T0 = rng.random((nz, ny, nx))
    tgt = rng.random((nz, ny, nx))
    Ci = 0.4 + 0.2 * rng.random((nz, ny, nx))
    s = _scal(nx, ny, nz, Ci, lx=0.8)
    Tn = _fwd(T0, Ci, s, nt)
    _, r = oracle.loss_and_seed(Tn, tgt)
    _, gCi = _rev(T0, Ci, r, s, nt)
    ref = brute.complex_step_grad_Ci(T0, Ci, tgt, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], nt)
    assert np.max(np.abs(gCi - ref)) <= 1e-13 * np.max(np.abs(ref))
    mask = np.ones(Ci.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.all(gCi[mask] == 0.0)


def test_reverse_sine_mode_closed_form():
    """T0 = sine mode s at constant Ci, target 0.  Interior gradient is
    g^(2nt) s; a face point b takes c*(1/h_n)^2*s[b+n]*g^nt*(1-g^nt)/(1-g)
    from its inward neighbour b+n; edges and corners get 0.  The sum of the
    Ci gradient is nt*g^(2nt-1)*(-dt*lam*kappa)*||s||^2."""
    nx, ny, nz = 12, 10, 9
    p = (1, 2, 1)
    cval = 0.5
    Ci = np.full((nz, ny, nx), cval)
    s = _scal(nx, ny, nz, Ci, ly=1.2, lz=0.9)
    g, kap = amplification(nx, ny, nz, p, cval, s)
    sm = sine_mode(nx, ny, nz, p)
    nt = 15
    Tn = _fwd(sm, Ci, s, nt)
    gT0, gCi = _rev(sm, Ci, Tn, s, nt)
    c = s["dt"] * s["lam"] * cval
    interior = gT0[1:-1, 1:-1, 1:-1]
    assert np.max(np.abs(interior - g ** (2 * nt) * sm[1:-1, 1:-1, 1:-1])) <= 200 * EPS
    geo = g ** nt * (1 - g ** nt) / (1 - g)
    # x faces (ix = 0 and nx-1) on interior y, z
    fx = c * s["rdx"] ** 2 * geo
    assert np.allclose(gT0[1:-1, 1:-1, 0], fx * sm[1:-1, 1:-1, 1], rtol=1e-12, atol=1e-15)
    assert np.allclose(gT0[1:-1, 1:-1, -1], fx * sm[1:-1, 1:-1, -2], rtol=1e-12, atol=1e-15)
    fy = c * s["rdy"] ** 2 * geo
    assert np.allclose(gT0[1:-1, 0, 1:-1], fy * sm[1:-1, 1, 1:-1], rtol=1e-12, atol=1e-15)
    fz = c * s["rdz"] ** 2 * geo
    assert np.allclose(gT0[-1, 1:-1, 1:-1], fz * sm[-2, 1:-1, 1:-1], rtol=1e-12, atol=1e-15)
    # edges and corners
    for e in (gT0[0, 0, :], gT0[0, :, 0], gT0[:, 0, 0], gT0[-1, -1, :], gT0[:, -1, -1]):
        assert np.all(e == 0.0)
    expect = nt * g ** (2 * nt - 1) * (-s["dt"] * s["lam"] * kap) * float(np.sum(sm * sm))
    assert float(np.sum(gCi)) == pytest.approx(expect, rel=1e-12)


def test_reverse_finite_differences():
    nx, ny, nz = 8, 7, 9
    T0, Ci = workloads.uniform_const(nx, ny, nz)
    Ci = Ci * (1.0 + 0.2 * workloads.uniform(nx, ny, nz, 1))
    tgt = workloads.target(nx, ny, nz)
    s = _scal(nx, ny, nz, Ci)
    nt = 12

    def loss(T0_, Ci_):
        return oracle.loss_and_seed(_fwd(T0_, Ci_, s, nt), tgt)[0]

    _, r = oracle.loss_and_seed(_fwd(T0, Ci, s, nt), tgt)
    gT0, gCi = _rev(T0, Ci, r, s, nt)
    v = workloads.direction(nx, ny, nz)
    # the loss is quadratic in T0: a central difference is exact up to rounding
    e = 1e-3
    fd = (loss(T0 + e * v, Ci) - loss(T0 - e * v, Ci)) / (2 * e)
    assert fd == pytest.approx(float(np.sum(gT0 * v)), rel=1e-9)
    e = 1e-6
    fd = (loss(T0, Ci + e * v) - loss(T0, Ci - e * v)) / (2 * e)
    assert fd == pytest.approx(float(np.sum(gCi * v)), rel=1e-6)


def test_reverse_keep_is_bit_exact():
    nx, ny, nz = 7, 6, 8
    T0, Ci = workloads.uniform_const(nx, ny, nz)
    g = workloads.target(nx, ny, nz)
    s = _scal(nx, ny, nz, Ci)
    a = _rev(T0, Ci, g, s, 23, keep=1)
    for keep in (3, 5, 23, 40):
        b = _rev(T0, Ci, g, s, 23, keep=keep)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reverse_zero_steps():
    T0, Ci = workloads.uniform_const(5, 4, 3)
    g = workloads.target(5, 4, 3)
    s = _scal(5, 4, 3, Ci)
    gT0, gCi = _rev(T0, Ci, g, s, 0)
    assert np.array_equal(gT0, g) and np.all(gCi == 0.0)


def test_oracle_rejects_bad_sizes():
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((2, 4, 4)), np.zeros((2, 4, 4)), 1.0, 1e-3, 1.0, 1.0, 1.0, 1)
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((4, 4, 4)), np.zeros((4, 4, 4)), 1.0, 1e-3, 1.0, 1.0, 1.0, -1)


# ---------------------------------------------------------------- 2-D form
# The same step without the z term on an (ny, nx) grid; pinned the same way.

def _scal2(nx, ny, Ci, lx=1.0, ly=1.0, lam=1.0, divisor=None):
    s = oracle.scalars2d(nx, ny, Ci, lam=lam, lx=lx, ly=ly)
    if divisor is not None:
        s["dt"] = s["dt"] * 4.1 / divisor
    return s


def _fwd2(T0, Ci, s, nt):
    return oracle.forward2d(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], nt)


def test_2d_scalars_closed_form():
    nx, ny = 65, 33
    Ci = np.full((ny, nx), 0.5)
    Ci[3, 7] = 0.8                                 # max(Ci) over the whole array
    s = _scal2(nx, ny, Ci, lx=1.0, ly=1.0)
    assert s["dx"] == 1.0 / 64 and s["dy"] == 1.0 / 32
    assert s["dt"] == (1.0 / 64) ** 2 / 1.0 / 0.8 / 4.1


@pytest.mark.parametrize("shape,nt", [((4, 5), 1), ((4, 5), 3), ((5, 4), 2), ((6, 6), 2), ((3, 7), 2)])
def test_2d_exact_rational_brute_force(shape, nt):
    ny, nx = shape
    rng = np.random.default_rng(31 + nx + 5 * ny)
    T0 = rng.random((ny, nx))
    Ci = 0.4 + 0.2 * rng.random((ny, nx))
    s = _scal2(nx, ny, Ci, lx=1.0, ly=1.6)
    T = _fwd2(T0, Ci, s, nt)
    ex = brute.exact_forward2d(T0, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], nt)
    scale = float(np.max(np.abs(ex.astype(np.float64))))
    err = max(abs(float(ex[i] - Fraction(float(T[i])))) for i in np.ndindex(T.shape))
    assert err <= 8 * nt * EPS * scale
    mask = np.ones(T.shape, bool)
    mask[1:-1, 1:-1] = False
    assert np.array_equal(T[mask], T0[mask])


@pytest.mark.parametrize("p,nt", [((1, 1), 25), ((3, 2), 25), ((31, 19), 25)])   # (31, 19): n - 2, near-checkerboard
def test_2d_sine_mode_amplification(p, nt):
    nx, ny = 33, 21
    c = 0.5
    Ci = np.full((ny, nx), c)
    s = _scal2(nx, ny, Ci, lx=1.0, ly=1.4)
    xs = np.sin(p[0] * np.pi * np.arange(nx) / (nx - 1))
    ys = np.sin(p[1] * np.pi * np.arange(ny) / (ny - 1))
    xs[0] = xs[-1] = 0.0
    ys[0] = ys[-1] = 0.0
    T0 = np.outer(ys, xs)
    kap = (4 * math.sin(p[0] * math.pi / (2 * (nx - 1))) ** 2 * s["rdx"] ** 2
           + 4 * math.sin(p[1] * math.pi / (2 * (ny - 1))) ** 2 * s["rdy"] ** 2)
    g = 1.0 - s["dt"] * s["lam"] * c * kap
    T = _fwd2(T0, Ci, s, nt)
    err = np.max(np.abs(T - g ** nt * T0)) / np.max(np.abs(T0))
    assert err <= 20 * nt * EPS, (g, err)


def test_2d_constant_field_and_transpose():
    rng = np.random.default_rng(8)
    Ci = 0.5 + 0.5 * rng.random((9, 13))
    s = _scal2(13, 9, Ci, lx=1.0, ly=0.7)
    T0 = np.full((9, 13), 1.7)
    assert np.array_equal(_fwd2(T0, Ci, s, 11), T0)
    # swapping the axes (and their spacings) transposes the result bit for bit
    T0 = rng.random((9, 13))
    A = _fwd2(T0, Ci, s, 7)
    B = oracle.forward2d(T0.T, Ci.T, s["lam"], s["dt"], s["rdy"], s["rdx"], 7)
    assert np.array_equal(A, B.T)


def test_2d_max_principle_and_negative_control():
    nx, ny = 24, 17
    rng = np.random.default_rng(5)
    T0 = rng.random((ny, nx))
    Ci = 0.25 + 0.5 * rng.random((ny, nx))
    s = _scal2(nx, ny, Ci)
    for nt in (1, 6, 50):
        T = _fwd2(T0, Ci, s, nt)
        assert T.min() >= T0.min() - 4 * EPS and T.max() <= T0.max() + 4 * EPS
    # checkerboard on a square grid (dx = dy: centre weight 1 - 4/divisor):
    # bounded at the 4.1 divisor, overshooting below 4
    n = 17
    cb = (np.indices((n, n)).sum(axis=0) % 2).astype(np.float64)
    Cc = np.full((n, n), 0.5)
    ok = _fwd2(cb, Cc, _scal2(n, n, Cc), 3)
    assert ok.min() >= -4 * EPS and ok.max() <= 1 + 4 * EPS
    bad = _fwd2(cb, Cc, _scal2(n, n, Cc, divisor=3.5), 3)
    assert bad.min() < -1e-3 or bad.max() > 1 + 1e-3
