"""Pins of the reference's coefficient assembly and of its step as a whole
(Sec. 3.1, Sec. 3.3.1, Sec. 3.3.3, Sec. 2.2), each against a fact fixed
outside the reference's own formulas:

  * the scattering operator assembled on the sphere by quadrature from its
    definition (gain integral of the differential cross section minus the
    total cross section, Sec. 2.1): real spherical harmonics are its
    eigenfunctions with eigenvalue G_l - G_0, and the implicit-Euler
    self-scattering step of the full-rank and low-rank references is the
    resolvent of that operator;
  * particle balance of the full-rank step: the change of the zeroth moment
    summed over the grid equals the boundary outflow (summed differences
    telescope to the two outermost cells of every grid line) plus what the
    uncollided flux loses by removal (Sec. 3.1);
  * the low-rank step at full angular rank r = m < n converges to the
    full-rank step at second order in the energy step;
  * a 90 degree rotation of beam and grid rotates the full-rank dose.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import coeffs, dlra, fullrank, pn, solver
from oracle import transport as tr
from workloads import configs


# ---------------------------------------------------------------- helpers

def sphere_quadrature(N):
    """Gauss-Legendre in mu x uniform in phi, exact for polynomials of degree
    <= 2N + 3 on the sphere; returns directions (q, 3) and weights (q,)."""
    nmu, nphi = N + 3, 2 * N + 6
    x, w = np.polynomial.legendre.leggauss(nmu)
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    MU, PH = np.meshgrid(x, ph, indexing="ij")
    W = np.repeat(w, nphi) * (2.0 * math.pi / nphi)
    mu, phi = MU.ravel(), PH.ravel()
    s = np.sqrt(1.0 - mu**2)
    om = np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)
    return om, mu, phi, W


def table_moments(problem, E, l_max):
    """(G_0(E), G_0(E) - G_l(E) for l <= l_max) of every base material,
    interpolated linearly in the tables (the mixture rule's inputs)."""
    mat = problem.materials
    G0 = np.array([np.interp(E, mat.e, mat.G0[i]) for i in range(mat.n_mat)])
    dG = np.array([[np.interp(E, mat.e, mat.dG[i, :, l]) for l in range(l_max + 1)]
                   for i in range(mat.n_mat)])
    return G0, dG


def scattering_operator_on_sphere(N, G0, dG):
    """Gamma_pq = int int m_p(W) Sig_s(W.W') m_q(W') dW dW' - Sig_t delta_pq for
    one material, with Sig_s given by its Legendre moments
    G_l = 2 pi int P_l Sig_s dmu (so Sig_s(mu) = sum_l (2l+1)/(4 pi) G_l P_l(mu)
    restricted to l <= N, the part that acts on P_N) and Sig_t = G_0.  The
    total cross section is split off as G_0 times the degree-N reproducing
    kernel sum_l (2l+1)/(4 pi) P_l, which acts as the identity on P_N; the
    remaining kernel has the moments G_l - G_0 = -dG_l and no cancellation."""
    om, mu, phi, W = sphere_quadrature(N)
    Y = pn.real_sh(N, mu, phi)                              # (q, m)
    cosang = np.clip(om @ om.T, -1.0, 1.0)
    kern = np.zeros_like(cosang)
    for l in range(N + 1):
        kern += (2 * l + 1) / (4.0 * math.pi) * (-dG[l]) * eval_legendre(l, cosang)
    return (Y * W[:, None]).T @ kern @ (Y * W[:, None])


def line_sums(F, grid, d, kind):
    """Sum over every grid line along axis d of the one-sided difference of F
    (n x c), from the telescoped form only: with zero ghosts,
    sum_i (3 f_i - 4 f_{i-1} + f_{i-2}) = 3 f_last - f_(last-1)  (backward),
    sum_i (-3 f_i + 4 f_{i+1} - f_{i+2}) = -3 f_first + f_second (forward)."""
    cube = F.reshape(grid.nz, grid.ny, grid.nx, -1)
    ax = (2, 1, 0)[d]
    h = (grid.dx, grid.dy, grid.dz)[d]
    L = cube.shape[ax]

    def take(i):
        if not 0 <= i < L:
            return 0.0
        return np.take(cube, i, axis=ax).reshape(-1, cube.shape[-1]).sum(axis=0)

    if kind == "b":
        return (3.0 * take(L - 1) - take(L - 2)) / (2.0 * h)
    return (-3.0 * take(0) + take(1)) / (2.0 * h)


def outflow_rate(Y, s, Apm, grid):
    """Sum over cells of the zeroth moment of the streaming term F_S(Y)."""
    sY = s[:, None] * Y
    tot = 0.0
    for d, (Ap, Am) in enumerate(Apm):
        tot -= line_sums(sY, grid, d, "b") @ Ap[:, 0] + line_sums(sY, grid, d, "f") @ Am[:, 0]
    return float(tot)


# ---------------------------------------------------------------- scattering

@pytest.mark.parametrize("N", [2, 3, 5])
def test_scattering_eigenvalues_on_the_sphere(N):
    # the oracle's self-scattering coefficients a_{il} are the eigenvalues of
    # the scattering operator assembled from its definition: diagonal in the
    # real harmonics, equal within a degree, G_l - G_0 <= 0
    p = configs.small_2d(N=N, mats="slab")
    c = coeffs.step_coeffs(p, p.beams[0], 4)
    G0, dG = table_moments(p, c.e_half, N)
    ell, _ = pn.degree_order(N)
    for i in range(p.materials.n_mat):
        Gam = scattering_operator_on_sphere(N, G0[i], dG[i])
        scale = np.abs(Gam).max()
        off = Gam - np.diag(np.diag(Gam))
        assert np.abs(off).max() <= 1e-12 * scale
        assert np.abs(np.diag(Gam) - c.a[i, ell]).max() <= 1e-12 * scale
        assert np.all(np.diag(Gam)[ell >= 1] < 0.0)
        assert np.abs(np.diag(Gam)[0]) <= 1e-12 * scale


def test_pure_scattering_step_is_the_resolvent():
    # no streaming, no source: one step of the full-rank reference and the
    # low-rank collided step (U = I) apply (I - dt s sum_i w_i Gamma_i)^{-1}
    # cell by cell; the zeroth moment is conserved and every other degree decays
    N = 3
    p = configs.small_2d(nx=5, ny=3, N=N, mats="slab", r=15)
    m, n = p.m, p.grid.n
    c = coeffs.step_coeffs(p, p.beams[0], 2)
    G0, dG = table_moments(p, c.e_half, N)
    Gams = [scattering_operator_on_sphere(N, G0[i], dG[i]) for i in range(p.materials.n_mat)]
    w = p.materials.w
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((n, m))
    ref = np.empty_like(u0)
    for x in range(n):
        A = np.eye(m) - c.dt * c.s[x] * sum(w[i, x] * Gams[i] for i in range(len(Gams)))
        ref[x] = np.linalg.solve(A, u0[x])
    no_stream = [(np.zeros((m, m)), np.zeros((m, m))) for _ in range(p.grid.dim)]
    u1, dose = fullrank.step(u0, np.zeros(n), c, no_stream, p, np.zeros(n))
    assert np.abs(u1 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(u1[:, 0] - u0[:, 0]).max() <= 1e-14 * np.abs(u0[:, 0]).max()
    ell, _ = pn.degree_order(N)
    assert np.all(np.abs(u1[:, ell >= 1]) < np.abs(u0[:, ell >= 1]))
    # low-rank collided step with U = I spanning every cell
    U = np.eye(n)
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    S = u0 @ V
    U2, St, Vt = dlra.collided(U, S[:, :m], V, c, w, N, p.options.with_(r=m))
    assert np.abs(U2 @ St @ Vt.T - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- particle balance

def test_full_rank_particle_balance():
    # per energy step: sum_x du_0 = RK4-weighted boundary outflow
    #                              + dt sum_x sum_i w_i Sig~_i psibar / sqrt(4 pi),
    # Sig~_i = G_0 - G_{N+1} the removal rate of the uncollided flux (the
    # ray tracer's absorption coefficient), to round-off
    p = configs.small_2d(nx=12, ny=10, N=3, mats="slab", n_steps=10)
    beam = p.beams[0]
    psibar, _ = solver.uncollided(p, beam)
    Apm = solver.streaming_split(p)
    N = p.options.pn_degree
    w = p.materials.w
    u = np.zeros((p.grid.n, p.m))
    checked = 0
    for k in range(6):
        c = coeffs.step_coeffs(p, beam, k)
        # boundary outflow of the RK4 substeps, from the stage inputs
        y = u.copy()
        out = 0.0
        F = lambda Y: tr.streaming_full(Y, c.s, Apm, p.grid)
        for _ in range(c.n_sub):
            k1 = F(y)
            k2 = F(y + 0.5 * c.h * k1)
            k3 = F(y + 0.5 * c.h * k2)
            out += c.h / 6.0 * (outflow_rate(y, c.s, Apm, p.grid)
                                + 2.0 * outflow_rate(y + 0.5 * c.h * k1, c.s, Apm, p.grid)
                                + 2.0 * outflow_rate(y + 0.5 * c.h * k2, c.s, Apm, p.grid)
                                + outflow_rate(y + c.h * k3, c.s, Apm, p.grid))
            k4 = F(y + c.h * k3)
            y = y + (c.h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        _, dG = table_moments(p, c.e_half, N + 1)
        removal = dG[:, N + 1]                                   # (n_mat,)
        gain = c.dt * float((removal @ w) @ psibar[k]) / math.sqrt(4.0 * math.pi)
        u_new, _ = fullrank.step(u, np.zeros(p.grid.n), c, Apm, p, psibar[k])
        lhs = u_new[:, 0].sum() - u[:, 0].sum()
        rhs = out + gain
        scale = abs(out) + abs(gain) + np.abs(u[:, 0]).sum()
        assert abs(lhs - rhs) <= 1e-12 * scale, (k, lhs, rhs)
        checked += gain > 0
        u = u_new
    assert checked >= 3


# ---------------------------------------------------------------- DLRA -> full rank

def test_low_rank_at_full_angular_rank_converges_at_second_order():
    # r = m < n in homogeneous water: the low-rank step differs from the
    # full-rank step only by the Galerkin error of the S-step, O(dt^3) per
    # step (with one RK4 substep per energy step), so the dose difference
    # falls by about 4 per halving of dt
    errs = []
    for ns in (64, 128, 256):
        p = configs.small_2d(nx=10, ny=10, N=2, r=9, n_steps=ns, mats="water", E0=20.0, dx=0.1,
                             aug_tol=1e-12, floor_tol=1e-14)
        assert max(coeffs.step_coeffs(p, p.beams[0], k).n_sub for k in range(ns)) == 1
        a = solver.run_beam_dlra(p, p.beams[0])
        b = solver.run_beam_fullrank(p, p.beams[0], psibar=a["psibar"], Du=a["dose_u"])
        errs.append(np.linalg.norm(a["dose_c"] - b["dose_c"]) / np.linalg.norm(b["dose_c"]))
    order = math.log2(errs[0] / errs[2]) / 2.0
    assert 1.6 < order < 2.6, errs
    assert errs[2] < 1e-5


# ---------------------------------------------------------------- symmetry

def test_full_rank_dose_rotates_with_the_beam():
    # beam along +x entering at height y0, and the same beam rotated by 90
    # degrees about the z axis (along +y, entering at x = L - y0) on a square
    # grid: the dose rotates with it, D_y(L - y, x) = D_x(x, y)
    n, dx = 10, 0.05
    p = configs.small_2d(nx=n, ny=n, N=3, n_steps=6, mats="random", dx=dx)
    L = n * dx
    bx = p.beams[0]
    y0 = bx.pos[1]
    by = dataclasses.replace(bx, pos=(L - y0, 0.0, 0.0), dir=(0.0, 1.0, 0.0))
    # the phantom rotates too: w_y(L - y, x) = w_x(x, y)
    wx = p.materials.w.reshape(-1, n, n)                 # [mat][j(y)][i(x)]
    wy = np.empty_like(wx)
    for j in range(n):
        for i in range(n):
            wy[:, i, n - 1 - j] = wx[:, j, i]
    px = p.single_beam(0)
    py = dataclasses.replace(p, beams=[by],
                             materials=dataclasses.replace(p.materials, w=wy.reshape(-1, n * n)))
    Dx = solver.run_beam_fullrank(px, bx)["dose"].reshape(n, n)
    Dy = solver.run_beam_fullrank(py, by)["dose"].reshape(n, n)
    rot = np.empty_like(Dx)
    for j in range(n):
        for i in range(n):
            rot[i, n - 1 - j] = Dx[j, i]
    assert np.abs(Dy - rot).max() <= 1e-11 * np.abs(Dx).max()
    # and the rotation is not a symmetry of the dose itself
    assert np.abs(Dx - rot).max() > 1e-3 * np.abs(Dx).max()
