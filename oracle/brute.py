"""Brute-force evaluators for tiny grids (TEST INFRASTRUCTURE ONLY).

Two formulations of the Fig. 1 time step that share nothing with the C loops
in ``diff3d_oracle.c`` and are used to pin them:

* ``exact_forward``: the step evaluated in exact rational arithmetic
  (``fractions.Fraction``) over a dictionary of grid points, with the second
  difference written as A[i+1] - 2*A[i] + A[i-1] (equal to the paper's
  difference of differences in exact arithmetic).

* ``step_matrix``: the step written as an explicit N x N matrix:
  row i of an interior point is e_i + c_i*L[i, :], with c_i = dt*lam*Ci[i]
  and L the 7-point operator (weight (1/h_d)^2 on the two neighbours along
  axis d, minus twice their sum on the centre); boundary rows are e_i.
  Powers and transposes of this matrix give the forward result and the
  exact reverse-mode gradient with respect to T0; a complex-step
  derivative of the loss through the same matrix gives dLoss/dCi without
  cancellation.

Source: Omlin & Raess, "High-performance xPU Stencil Computations in
Julia", Fig. 1 (the step kernel and the interior-only update).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _points(nx, ny, nz):
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                yield ix, iy, iz


def _interior(p, nx, ny, nz):
    ix, iy, iz = p
    return 0 < ix < nx - 1 and 0 < iy < ny - 1 and 0 < iz < nz - 1


def exact_forward(T0, Ci, lam, dt, rdx, rdy, rdz, nt):
    """Exact rational value of T_nt.  All float inputs are converted exactly
    to Fractions; returns a dict {(ix, iy, iz): Fraction}."""
    nz, ny, nx = T0.shape
    T = {p: Fraction(float(T0[p[2], p[1], p[0]])) for p in _points(nx, ny, nz)}
    C = {p: Fraction(float(Ci[p[2], p[1], p[0]])) for p in _points(nx, ny, nz)}
    lam, dt = Fraction(lam), Fraction(dt)
    w = (Fraction(rdx) ** 2, Fraction(rdy) ** 2, Fraction(rdz) ** 2)
    for _ in range(nt):
        new = dict(T)  # boundary values carry over unchanged
        for p in T:
            if not _interior(p, nx, ny, nz):
                continue
            lap = Fraction(0)
            for axis in range(3):
                up = list(p); up[axis] += 1
                dn = list(p); dn[axis] -= 1
                lap += w[axis] * (T[tuple(up)] - 2 * T[p] + T[tuple(dn)])
            new[p] = T[p] + dt * lam * C[p] * lap
        T = new
    return T


def exact_to_array(T, shape, dtype=object):
    nz, ny, nx = shape
    out = np.empty(shape, dtype=dtype)
    for (ix, iy, iz), v in T.items():
        out[iz, iy, ix] = v
    return out


def step_matrix(Ci, lam, dt, rdx, rdy, rdz, dtype=np.float64):
    """The one-step matrix A (N x N, N = nx*ny*nz, linear index
    ix + nx*(iy + ny*iz)), so that T_{k+1} = A @ T_k for flattened fields."""
    nz, ny, nx = Ci.shape
    n = nx * ny * nz
    A = np.zeros((n, n), dtype=dtype)
    w = (rdx * rdx, rdy * rdy, rdz * rdz)
    strides = (1, nx, nx * ny)
    for p in _points(nx, ny, nz):
        ix, iy, iz = p
        i = ix + nx * (iy + ny * iz)
        A[i, i] = 1.0
        if not _interior(p, nx, ny, nz):
            continue
        c = dt * lam * Ci[iz, iy, ix]
        for axis in range(3):
            A[i, i] += -2.0 * c * w[axis]
            A[i, i + strides[axis]] += c * w[axis]
            A[i, i - strides[axis]] += c * w[axis]
    return A


def matrix_forward(T0, Ci, lam, dt, rdx, rdy, rdz, nt):
    A = step_matrix(Ci, lam, dt, rdx, rdy, rdz)
    x = T0.reshape(-1).astype(np.float64)
    for _ in range(nt):
        x = A @ x
    return x.reshape(T0.shape)


def matrix_grad_T0(Ci, g_nt, lam, dt, rdx, rdy, rdz, nt):
    """dLoss/dT0 = (A^T)^nt g_nt, from the explicit matrix."""
    A = step_matrix(Ci, lam, dt, rdx, rdy, rdz)
    y = g_nt.reshape(-1).astype(np.float64)
    for _ in range(nt):
        y = A.T @ y
    return y.reshape(g_nt.shape)


def complex_step_grad_Ci(T0, Ci, T_target, lam, dt, rdx, rdy, rdz, nt, h=1e-30):
    """dLoss/dCi for Loss = 0.5*sum((T_nt - T_target)^2), by the complex-step
    derivative Im(Loss(Ci + i*h*e_j))/h through the explicit matrix."""
    flatC = Ci.reshape(-1).astype(np.float64)
    x0 = T0.reshape(-1).astype(np.complex128)
    tgt = T_target.reshape(-1).astype(np.complex128)
    g = np.zeros(flatC.size)
    for j in range(flatC.size):
        Cj = flatC.astype(np.complex128)
        Cj[j] += 1j * h
        A = step_matrix(Cj.reshape(Ci.shape), lam, dt, rdx, rdy, rdz, dtype=np.complex128)
        x = x0
        for _ in range(nt):
            x = A @ x
        r = x - tgt
        g[j] = (0.5 * np.sum(r * r)).imag / h
    return g.reshape(Ci.shape)


def exact_forward2d(T0, Ci, lam, dt, rdx, rdy, nt):
    """Exact rational value of T_nt for the 2-D form on an (ny, nx) array,
    second differences as A[i+1] - 2*A[i] + A[i-1]; returns an object array."""
    ny, nx = T0.shape
    T = [[Fraction(float(T0[y, x])) for x in range(nx)] for y in range(ny)]
    C = [[Fraction(float(Ci[y, x])) for x in range(nx)] for y in range(ny)]
    lam, dt = Fraction(lam), Fraction(dt)
    wx, wy = Fraction(rdx) ** 2, Fraction(rdy) ** 2
    for _ in range(nt):
        new = [row[:] for row in T]
        for y in range(1, ny - 1):
            for x in range(1, nx - 1):
                lap = (wx * (T[y][x + 1] - 2 * T[y][x] + T[y][x - 1])
                       + wy * (T[y + 1][x] - 2 * T[y][x] + T[y - 1][x]))
                new[y][x] = T[y][x] + dt * lam * C[y][x] * lap
        T = new
    out = np.empty((ny, nx), dtype=object)
    for y in range(ny):
        for x in range(nx):
            out[y, x] = T[y][x]
    return out
