"""Pins of the spatial operators, the Galerkin forms and RK4 (Sec. 3.3.2, eq. KLS)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import pn
from oracle import transport as tr
from workloads.problem import Grid


def brute_stencil(grid, d, kind):
    """Dense n x n second-order one-sided difference, entries written out per
    cell with the paper's index formula idx(i,j,k) = (k-1) nx ny + (j-1) nx + i
    (1-based), neighbours outside the grid omitted (zero ghosts)."""
    n = grid.n
    D = np.zeros((n, n))
    h = (grid.dx, grid.dy, grid.dz)[d]
    sgn = -1 if kind == "b" else 1          # neighbours at i-1, i-2 (b) or i+1, i+2 (f)
    coef = {0: 3.0, 1: -4.0, 2: 1.0}
    nz = grid.nz
    for k in range(1, nz + 1):
        for j in range(1, grid.ny + 1):
            for i in range(1, grid.nx + 1):
                row = (k - 1) * grid.nx * grid.ny + (j - 1) * grid.nx + i - 1
                for off, cf in coef.items():
                    ii, jj, kk = i, j, k
                    if d == 0:
                        ii += sgn * off
                    elif d == 1:
                        jj += sgn * off
                    else:
                        kk += sgn * off
                    if 1 <= ii <= grid.nx and 1 <= jj <= grid.ny and 1 <= kk <= nz:
                        col = (kk - 1) * grid.nx * grid.ny + (jj - 1) * grid.nx + ii - 1
                        D[row, col] += (cf if kind == "b" else -cf) / (2.0 * h)
    return D


GRIDS = [Grid(7, 5, 1, 0.1, 0.07, 0.1), Grid(5, 4, 6, 0.1, 0.2, 0.05)]


@pytest.mark.parametrize("grid", GRIDS)
def test_stencil_matches_brute_force(grid):
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((grid.n, 3))
    for d in range(grid.dim):
        for kind in "bf":
            D = brute_stencil(grid, d, kind)
            assert np.abs(tr.diff(Y, grid, d, kind) - D @ Y).max() < 1e-12
        # with zero ghosts the backward operator is minus the transpose of the forward one
        assert np.abs(brute_stencil(grid, d, "b").T + brute_stencil(grid, d, "f")).max() < 1e-12


def test_stencil_second_order():
    errs = []
    for nx in (32, 64, 128):
        L = 1.0
        g = Grid(nx, 1, 1, L / nx, 1.0, 1.0)
        x = (np.arange(nx) + 0.5) * g.dx
        f = np.sin(2 * x)[:, None]
        for kind in "bf":
            dfx = tr.diff(f, g, 0, kind)[:, 0]
            interior = slice(4, nx - 4)
            errs.append((kind, np.abs(dfx[interior] - 2 * np.cos(2 * x[interior])).max()))
    eb = [e for k, e in errs if k == "b"]
    assert 3.5 < eb[0] / eb[1] < 4.5 and 3.5 < eb[1] / eb[2] < 4.5


def test_telescoping_boundary_flux():
    # sum_i (d^b f)_i = (3 f_N - f_{N-1}) / (2 h): an exact outflow flux
    rng = np.random.default_rng(2)
    g = Grid(11, 1, 1, 0.3, 1.0, 1.0)
    f = rng.standard_normal((11, 1))
    s = tr.diff(f, g, 0, "b").sum()
    assert abs(s - (3 * f[-1, 0] - f[-2, 0]) / (2 * 0.3)) < 1e-12


def assembled_streaming(grid, s, Apm):
    """vec(D Y B) = (B^T kron D) vec(Y): the full-rank streaming operator as one matrix."""
    n = grid.n
    Sm = np.diag(s)
    L = 0
    for d, (Ap, Am) in enumerate(Apm):
        Db, Df = brute_stencil(grid, d, "b"), brute_stencil(grid, d, "f")
        L = L - np.kron(Ap.T, Db @ Sm) - np.kron(Am.T, Df @ Sm)
    return L


def test_streaming_operator_kronecker():
    grid = Grid(5, 4, 1, 0.1, 0.1, 0.1)
    rng = np.random.default_rng(3)
    N = 3
    Apm = pn.split_streaming(N, 2)
    s = 1.0 + rng.random(grid.n)
    u = rng.standard_normal((grid.n, pn.n_moments(N)))
    L = assembled_streaming(grid, s, Apm)
    vec = lambda X: X.reshape(-1, order="F")
    assert np.abs(L @ vec(u) - vec(tr.streaming_full(u, s, Apm, grid))).max() < 1e-11


def test_rk4_is_fourth_order_taylor_and_converges_to_expm():
    grid = Grid(4, 4, 1, 0.1, 0.1, 0.1)
    rng = np.random.default_rng(4)
    N = 1
    Apm = pn.split_streaming(N, 2)
    s = np.full(grid.n, 0.2)
    L = assembled_streaming(grid, s, Apm)
    m = pn.n_moments(N)
    u = rng.standard_normal((grid.n, m))
    vec = lambda X: X.reshape(-1, order="F")
    f = lambda X: tr.streaming_full(X, s, Apm, grid)
    h = 0.05
    P = np.eye(L.shape[0])
    term = np.eye(L.shape[0])
    for j in range(1, 5):
        term = term @ (h * L) / j
        P = P + term
    assert np.abs(vec(tr.rk4(f, u, h, 1)) - P @ vec(u)).max() < 1e-12
    errs = []
    for hh in (0.04, 0.02):
        exact = scipy.linalg.expm(hh * L) @ vec(u)
        errs.append(np.abs(vec(tr.rk4(f, u, hh, 1)) - exact).max())
    assert 24 < errs[0] / errs[1] < 40          # local error O(h^5)


@pytest.mark.parametrize("dim,nu", [(2, 0.45), (3, 0.35)])
def test_rk4_stable_at_cfl(dim, nu):
    # The RK4 amplification polynomial of the upwind operator stays inside the
    # unit disc at the step rule's CFL number (vacuum boundaries, s = 1).
    grid = Grid(6, 6, 6 if dim == 3 else 1, 0.1, 0.1, 0.1)
    N = 3
    Apm = pn.split_streaming(N, dim)
    L = assembled_streaming(grid, np.ones(grid.n), Apm)
    z = np.linalg.eigvals(nu * 0.1 * L)
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    assert np.abs(R).max() <= 1.0 + 1e-10


def test_literal_stencil_pairing_is_unstable():
    # Pairing the forward-biased difference with positive eigenvalues (the
    # pairing as printed) gives eigenvalues with positive real part.
    grid = Grid(12, 1, 1, 0.1, 0.1, 0.1)
    Ap, Am = pn.split_streaming(1, 1)[0]
    Db, Df = brute_stencil(grid, 0, "b"), brute_stencil(grid, 0, "f")
    upwind = -np.kron(Ap.T, Db) - np.kron(Am.T, Df)
    literal = -np.kron(Ap.T, Df) - np.kron(Am.T, Db)
    assert np.linalg.eigvals(upwind).real.max() < 1e-10
    assert np.linalg.eigvals(literal).real.max() > 1.0


@pytest.mark.parametrize("grid", GRIDS)
def test_galerkin_forms_match_definitions(grid):
    # eq. KLS: K' = F(K V^T) V, L' = F(U L^T)^T U, S' = U^T F(U S V^T) V
    rng = np.random.default_rng(5)
    N = 3
    m = pn.n_moments(N)
    Apm = pn.split_streaming(N, grid.dim)
    s = 0.5 + rng.random(grid.n)
    F = lambda u: tr.streaming_full(u, s, Apm, grid)
    U, _ = np.linalg.qr(rng.standard_normal((grid.n, 4)))
    V, _ = np.linalg.qr(rng.standard_normal((m, 4)))
    K = rng.standard_normal((grid.n, 4))
    Lm = rng.standard_normal((m, 4))
    S = rng.standard_normal((4, 4))
    Bpm = tr.galerkin_angular(V, Apm)
    Cbf = tr.projections(U, U, s, grid, grid.dim)
    assert np.abs(tr.kstep_rhs(K, s, Bpm, grid) - F(K @ V.T) @ V).max() < 1e-11
    assert np.abs(tr.lstep_rhs(Lm, Apm, Cbf) - F(U @ Lm.T).T @ U).max() < 1e-11
    assert np.abs(tr.sstep_rhs(S, Cbf, Bpm) - U.T @ F(U @ S @ V.T) @ V).max() < 1e-11
