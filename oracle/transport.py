"""Spatial discretisation and the streaming operators (Sec. 3.3.2, eq. KLS).

Rows of every n x c matrix are cells, x fastest: row (k*ny + j)*nx + i.
Second-order one-sided differences along axis d with two zero ghost layers on
each side (vacuum boundary):
  backward  (d^b f)_i = ( 3 f_i - 4 f_{i-1} + f_{i-2}) / (2 Delta_d)
  forward   (d^f f)_i = (-3 f_i + 4 f_{i+1} - f_{i+2}) / (2 Delta_d)
The streaming term of eq. streamscattsplit, upwinded per eigen-family:
  F_S(u) = - sum_d [ d^b_d(s o u) A_d^+ + d^f_d(s o u) A_d^- ]
(s = 1/S the inverse stopping power, "s o" scales rows).  Positive eigenvalues
move particles towards +d and take the backward (upwind) difference.

Galerkin forms (eq. KLS with F = F_S):
  K-step  dK/dt = -sum_d [ d^b(sK) B_d^+ + d^f(sK) B_d^- ],  B_d^{+-} = V^T A_d^{+-} V
  L-step  dL/dt = -sum_d [ A_d^+ L C_d^{bT} + A_d^- L C_d^{fT} ], C_d^{b,f} = U^T d^{b,f}(sU)
  S-step  dS/dt = -sum_d [ C_d^b S B_d^+ + C_d^f S B_d^- ]
RK4 is the classic four-stage method (Sec. 3.3.3).
"""
from __future__ import annotations

import numpy as np


def _axis_and_delta(grid, d):
    # array layout (nz, ny, nx, c): x -> axis 2, y -> axis 1, z -> axis 0
    return (2, 1, 0)[d], (grid.dx, grid.dy, grid.dz)[d]


def _as_cube(Y, grid):
    return Y.reshape(grid.nz, grid.ny, grid.nx, -1)


def diff(Y, grid, d, kind):
    """d^b_d Y (kind='b') or d^f_d Y (kind='f') for Y of shape (n, c)."""
    ax, h = _axis_and_delta(grid, d)
    F = _as_cube(Y, grid)
    pad = [(0, 0)] * 4
    pad[ax] = (2, 2)
    P = np.pad(F, pad)
    L = F.shape[ax]

    def sl(off):
        idx = [slice(None)] * 4
        idx[ax] = slice(2 + off, 2 + off + L)
        return P[tuple(idx)]

    if kind == "b":
        out = (3.0 * sl(0) - 4.0 * sl(-1) + sl(-2)) / (2.0 * h)
    elif kind == "f":
        out = (-3.0 * sl(0) + 4.0 * sl(1) - sl(2)) / (2.0 * h)
    else:
        raise ValueError(kind)
    return out.reshape(Y.shape)


def streaming_full(u, s, Apm, grid):
    """F_S(u) for the full moment matrix u (n x m); Apm = [(A_d^+, A_d^-)]."""
    su = s[:, None] * u
    out = np.zeros_like(u)
    for d, (Ap, Am) in enumerate(Apm):
        out -= diff(su, grid, d, "b") @ Ap + diff(su, grid, d, "f") @ Am
    return out


def kstep_rhs(K, s, Bpm, grid):
    sK = s[:, None] * K
    out = np.zeros_like(K)
    for d, (Bp, Bm) in enumerate(Bpm):
        out -= diff(sK, grid, d, "b") @ Bp + diff(sK, grid, d, "f") @ Bm
    return out


def lstep_rhs(L, Apm, Cbf):
    out = np.zeros_like(L)
    for (Ap, Am), (Cb, Cf) in zip(Apm, Cbf):
        out -= Ap @ L @ Cb.T + Am @ L @ Cf.T
    return out


def sstep_rhs(S, Cbf, Bpm):
    out = np.zeros_like(S)
    for (Cb, Cf), (Bp, Bm) in zip(Cbf, Bpm):
        out -= Cb @ S @ Bp + Cf @ S @ Bm
    return out


def projections(X, Y, s, grid, dim):
    """[(X^T d^b_d(sY), X^T d^f_d(sY)) for d < dim]."""
    sY = s[:, None] * Y
    return [(X.T @ diff(sY, grid, d, "b"), X.T @ diff(sY, grid, d, "f")) for d in range(dim)]


def galerkin_angular(V, Apm):
    """[(V^T A_d^+ V, V^T A_d^- V)]."""
    return [(V.T @ Ap @ V, V.T @ Am @ V) for Ap, Am in Apm]


def rk4(f, y, h, nsteps):
    """Classic RK4 with nsteps steps of size h."""
    for _ in range(nsteps):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y
