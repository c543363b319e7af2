"""Pins of the reference's variants of the method:

  * Fokker-Planck collisions (Sec. 2.1, Sec. 3.1, Sec. 3.3.1): the collision
    operator (xi_1/2) L assembled on the sphere by finite differences of the
    Laplace-Beltrami operator; no removal of the uncollided flux;
  * non-uniform energy grids (Sec. 6): grid properties, step integrals that
    partition the same energy integral, energy balance;
  * a joint source of several beams in one collided solve (Sec. 4.3): the
    full-rank joint solve is the weighted sum of the single-beam solves;
  * the twelve-element material decomposition (Sec. 2.1).
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import coeffs, dlra, fullrank, pn, raytrace, solver
from oracle import transport as tr
from workloads import configs


# ---------------------------------------------------------------- Fokker-Planck

def laplace_beltrami_on_sphere(N, h=1e-4):
    """L_pq = int m_p L m_q dOmega with L = d/dmu (1 - mu^2) d/dmu
    + 1/(1 - mu^2) d^2/dphi^2 applied by central differences of the real
    harmonics at the nodes of a product rule exact for degree 2N + 3."""
    nmu, nphi = N + 3, 2 * N + 6
    x, wx = np.polynomial.legendre.leggauss(nmu)
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    MU, PH = np.meshgrid(x, ph, indexing="ij")
    mu, phi = MU.ravel(), PH.ravel()
    W = np.repeat(wx, nphi) * (2.0 * math.pi / nphi)
    Y = lambda a, b: pn.real_sh(N, a, b)
    f0 = Y(mu, phi)
    fp, fm = Y(mu + h, phi), Y(mu - h, phi)
    d1 = (fp - fm) / (2.0 * h)
    d2 = (fp - 2.0 * f0 + fm) / (h * h)
    dphi2 = (Y(mu, phi + h) - 2.0 * f0 + Y(mu, phi - h)) / (h * h)
    Lf = ((1.0 - mu**2)[:, None] * d2 - 2.0 * mu[:, None] * d1
          + dphi2 / (1.0 - mu**2)[:, None])
    return (f0 * W[:, None]).T @ Lf


def test_fokker_planck_pure_scattering_step():
    # no streaming, no source: the Fokker-Planck step is the implicit-Euler
    # resolvent of sum_i w_i (xi_i / 2) L with L assembled on the sphere and
    # xi_i = 2 pi int (1 - mu) Sigma_s dmu = G_0 - G_1 from the tables
    N = 3
    p = configs.small_2d(nx=4, ny=3, N=N, mats="slab", collision="fokker_planck")
    m, n = p.m, p.grid.n
    c = coeffs.step_coeffs(p, p.beams[0], 3)
    Lmat = laplace_beltrami_on_sphere(N)
    ell, _ = pn.degree_order(N)
    assert np.abs(Lmat - np.diag(-(ell * (ell + 1.0)))).max() < 1e-5 * N * (N + 1)
    mat = p.materials
    xi = np.array([np.interp(c.e_half, mat.e, mat.dG[i, :, 1]) for i in range(mat.n_mat)])
    w = mat.w
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal((n, m))
    ref = np.empty_like(u0)
    for x in range(n):
        A = np.eye(m) - c.dt * c.s[x] * sum(w[i, x] * 0.5 * xi[i] * Lmat for i in range(len(xi)))
        ref[x] = np.linalg.solve(A, u0[x])
    no_stream = [(np.zeros((m, m)), np.zeros((m, m))) for _ in range(2)]
    u1, _ = fullrank.step(u0, np.zeros(n), c, no_stream, p, np.zeros(n))
    assert np.abs(u1 - ref).max() <= 1e-6 * np.abs(ref).max()
    # in-scattering: the whole operator acting on the beam direction, no
    # particles moved into the zeroth moment
    TM = pn.beam_moments(N, p.beams[0].dir)
    for i in range(mat.n_mat):
        assert np.abs(c.g[:, i] - 0.5 * xi[i] * (Lmat @ TM)).max() <= 1e-6 * np.abs(c.g).max()
    assert np.all(c.g[0] == 0.0)


def test_fokker_planck_uncollided_flux_is_not_removed():
    # Gamma_out = 0: int psi_u dE is the same in every cell of a row until the
    # spectrum reaches E_cut, while the Boltzmann tracer attenuates it
    p = configs.small_2d(nx=16, ny=4, N=3, mats="slab", E0=40.0)
    for coll, conserved in (("fokker_planck", True), ("boltzmann", False)):
        q = p.with_options(collision=coll)
        edges = coeffs.energy_edges(q, q.beams)
        ps, _ = raytrace.Tracer(q, q.beams[0], edges).trace()
        dt = -np.diff(edges)
        tot = (dt[:, None] * ps).sum(axis=0).reshape(4, 16)
        row = tot[2]
        if conserved:
            assert np.abs(row / row[0] - 1.0).max() < 1e-12
        else:
            assert row[-1] < (1.0 - 1e-4) * row[0]


def test_fokker_planck_particle_balance_and_full_rank():
    # no source in the zeroth moment: the collided zeroth moment changes only
    # by the boundary outflow; the DLRA step at full rank is the full-rank step
    p = configs.small_2d(nx=4, ny=4, N=3, r=16, n_steps=5, mats="slab",
                         collision="fokker_planck", aug_tol=1e-12, floor_tol=1e-14)
    a = solver.run_beam_dlra(p, p.beams[0])
    b = solver.run_beam_fullrank(p, p.beams[0], psibar=a["psibar"], Du=a["dose_u"])
    st = a["state"]
    assert (np.linalg.norm(st.U @ st.S @ st.V.T - b["u"]) / np.linalg.norm(b["u"])) < 1e-11
    q = configs.small_2d(nx=10, ny=8, N=3, mats="slab", n_steps=6, collision="fokker_planck")
    beam = q.beams[0]
    edges = coeffs.energy_edges(q, [beam])
    psibar, _ = solver.uncollided(q, beam, edges=edges)
    Apm = solver.streaming_split(q)
    u = np.zeros((q.grid.n, q.m))
    rng = np.random.default_rng(2)
    u[:, :] = 1e-3 * rng.random((q.grid.n, q.m))
    for k in range(3):
        c = coeffs.step_coeffs(q, beam, k, edges)
        y = u.copy()
        out = 0.0
        F = lambda Y: tr.streaming_full(Y, c.s, Apm, q.grid)
        s0 = lambda Y: float(F(Y)[:, 0].sum())
        for _ in range(c.n_sub):
            k1 = F(y)
            k2 = F(y + 0.5 * c.h * k1)
            k3 = F(y + 0.5 * c.h * k2)
            k4 = F(y + c.h * k3)
            out += c.h / 6.0 * (s0(y) + 2 * s0(y + 0.5 * c.h * k1) + 2 * s0(y + 0.5 * c.h * k2)
                                + s0(y + c.h * k3))
            y = y + (c.h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        u_new, _ = fullrank.step(u, np.zeros(q.grid.n), c, Apm, q, psibar[k])
        lhs = u_new[:, 0].sum() - u[:, 0].sum()
        assert abs(lhs - out) <= 1e-12 * (abs(out) + np.abs(u[:, 0]).sum())
        u = u_new


# ---------------------------------------------------------------- energy grids

@pytest.mark.parametrize("mode", ["uniform", "proportional", "cfl"])
def test_energy_grid_properties(mode):
    p = configs.small_2d(mats="slab", n_steps=16, egrid=mode)
    E = coeffs.energy_edges(p, p.beams)
    o = p.options
    e_max = p.beams[0].E0 + o.e_max_sigmas * p.beams[0].sigma_E
    assert E.shape == (17,) and E[0] == e_max and E[-1] == o.e_cut
    assert np.all(np.diff(E) < 0.0)
    dt = -np.diff(E)
    if mode == "uniform":
        assert np.abs(dt / dt[0] - 1.0).max() < 1e-12
    elif mode == "proportional":
        ratio = E[:-1] / E[1:]
        assert np.abs(ratio / ratio[0] - 1.0).max() < 1e-12
    else:
        # dt_k / S_min(E_{k+1/2}): the same for every step to the accuracy of
        # the midpoint rule over one step
        mid = 0.5 * (E[:-1] + E[1:])
        cfl = dt / np.array([coeffs.min_stopping(p, e) for e in mid])
        assert np.abs(cfl / cfl.mean() - 1.0).max() < 0.02
        assert dt[-1] > 2.0 * dt[0]   # long steps at low energy, where S is large


def test_step_integrals_partition_the_energy_integral():
    # the ray tracer's DG flux does not depend on the step grid; the step
    # averages of any grid times the step lengths sum to the same integral
    base = configs.small_2d(nx=10, ny=4, mats="slab", n_steps=12, E0=30.0)
    tots = []
    for mode in ("uniform", "proportional", "cfl"):
        q = base.with_options(egrid=mode)
        E = coeffs.energy_edges(q, q.beams)
        ps, _ = raytrace.Tracer(q, q.beams[0], E).trace()
        tots.append((-np.diff(E))[:, None] * ps)
    s = [t.sum(axis=0) for t in tots]
    assert np.abs(s[1] - s[0]).max() <= 1e-13 * np.abs(s[0]).max()
    assert np.abs(s[2] - s[0]).max() <= 1e-13 * np.abs(s[0]).max()
    assert np.abs(tots[1] - tots[0]).max() > 1e-3 * np.abs(tots[0]).max()


def test_user_grid_and_energy_balance():
    # a user grid equal to the proportional one gives the same run; on a water
    # box that stops the beam all energy between E0 and E_cut is deposited
    p = configs.small_2d(nx=24, ny=16, N=3, mats="water", n_steps=30, E0=25.0,
                         egrid="proportional", dx=0.05)
    E = coeffs.energy_edges(p, p.beams)
    a = solver.run_beam_dlra(p, p.beams[0])
    q = p.with_options(egrid="user", egrid_points=tuple(E))
    b = solver.run_beam_dlra(q, q.beams[0])
    assert np.array_equal(a["dose"], b["dose"])
    tot = a["dose"].sum() * p.grid.dx * p.grid.dy
    assert abs(tot - (p.beams[0].E0 - p.options.e_cut)) < 0.02 * p.beams[0].E0


def test_nonuniform_grid_dlra_full_rank_equals_full_rank():
    p = configs.small_2d(nx=4, ny=4, N=3, r=16, n_steps=6, mats="slab", egrid="proportional",
                         aug_tol=1e-12, floor_tol=1e-14)
    a = solver.run_beam_dlra(p, p.beams[0])
    b = solver.run_beam_fullrank(p, p.beams[0], psibar=a["psibar"], Du=a["dose_u"])
    assert np.linalg.norm(a["dose_c"] - b["dose_c"]) / np.linalg.norm(b["dose_c"]) < 1e-11


# ---------------------------------------------------------------- joint source

def test_joint_full_rank_is_the_weighted_sum_of_beams():
    p = configs.small_joint_2d(n_steps=6)
    edges = coeffs.energy_edges(p, p.beams)
    joint = solver.run_joint_fullrank(p)
    tot = np.zeros(p.grid.n)
    for b in p.beams:
        tot += b.weight * solver.run_beam_fullrank(p, b, edges=edges)["dose"]
    assert np.abs(joint["dose"] - tot).max() <= 1e-12 * np.abs(tot).max()


def test_joint_dlra_at_full_rank_and_first_step():
    p = configs.small_joint_2d(nx=4, ny=4, N=3, r=16, n_steps=5, aug_tol=1e-12, floor_tol=1e-14)
    a = solver.run_joint_dlra(p)
    b = solver.run_joint_fullrank(p, psibar=a["psibar"], Du=a["dose_u"])
    st = a["state"]
    assert np.linalg.norm(st.U @ st.S @ st.V.T - b["u"]) / np.linalg.norm(b["u"]) < 1e-11
    # from zero, one step reproduces the joint source (n_beams * n_mat <= r)
    q = configs.small_joint_2d(r=8, aug_tol=1e-12, floor_tol=1e-14)
    edges = coeffs.energy_edges(q, q.beams)
    ps, _ = solver.joint_uncollided(q, edges)
    Apm = solver.streaming_split(q)
    cs = [coeffs.step_coeffs(q, b, 0, edges) for b in q.beams]
    Q, G = dlra.source_factors(q.materials.w, [ps[0][0], ps[1][0]], [c.g for c in cs])
    st = dlra.initial_state(q, G)
    st = dlra.step(st, cs[0], Apm, q, None, sources=(Q, G))
    ref = cs[0].dt * Q @ G.T
    assert np.linalg.norm(st.U @ st.S @ st.V.T - ref) / np.linalg.norm(ref) < 1e-12


def test_joint_low_rank_close_to_separate_beams():
    # the joint low-rank solve approximates the sum of the separate ones (the
    # full-rank solves agree exactly), to the truncation tolerance
    p = configs.small_joint_2d(rank_mode="adaptive", r=4, r_min=2, r_max=14, trunc_tol=1e-5)
    edges = coeffs.energy_edges(p, p.beams)
    joint = solver.run_joint_dlra(p)["dose"]
    sep = sum(b.weight * solver.run_beam_dlra(p, b, edges=edges)["dose"] for b in p.beams)
    assert np.linalg.norm(joint - sep) / np.linalg.norm(sep) < 1e-3


# ---------------------------------------------------------------- twelve elements

def test_element_decomposition():
    p = configs.small_2d(nx=8, ny=6, mats="slab")
    q = configs.to_elements(p)
    assert q.materials.n_mat == 12
    assert np.abs(q.materials.w.sum(axis=0) - p.materials.w.sum(axis=0)).max() < 1e-14
    # water: hydrogen and oxygen only, by mass fraction
    names = q.materials.names
    wat = configs.small_2d(nx=8, ny=6, mats="water")
    qw = configs.to_elements(wat)
    nz = [names[i] for i in range(12) if qw.materials.w[i].max() > 0]
    assert nz == ["H", "O"]
    # twelve materials at full rank: DLRA = full rank
    r = configs.to_elements(configs.small_2d(nx=4, ny=4, N=3, r=16, n_steps=4, mats="slab",
                                             aug_tol=1e-12, floor_tol=1e-14))
    a = solver.run_beam_dlra(r, r.beams[0])
    b = solver.run_beam_fullrank(r, r.beams[0], psibar=a["psibar"], Du=a["dose_u"])
    assert np.linalg.norm(a["dose_c"] - b["dose_c"]) / np.linalg.norm(b["dose_c"]) < 1e-11
