"""Pins of the reference ray tracer (Sec. 3.2) against closed forms."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import raytrace
from workloads import configs
from workloads.problem import Beam, Grid, Materials, Options, Problem


def synthetic_problem(S=5.0, T=0.0, sig=0.0, nx=40, dx=0.1, N=3, E0=50.0, sE=0.5, G=128):
    """One row of one material with energy-independent S, T and removal Sigma~."""
    grid = Grid(nx, 1, 1, dx, dx, dx)
    e = np.linspace(0.1, 400.0, 50)
    ne = e.size
    dG = np.zeros((1, ne, N + 2))
    dG[0, :, N + 1] = sig                      # Sigma~ = G_0 - G_{N+1}
    mats = Materials(("x",), np.ones((1, grid.n)), e, np.full((1, ne), S),
                     np.full((1, ne), T), np.full((1, ne), 1e3), dG)
    # E_max 12 sigma above E0: the spectrum vanishes at both ends of the energy
    # range, so boundary terms cannot enter the moment identities
    o = Options(pn_degree=N, n_steps=10, n_groups=G, e_max_sigmas=12.0)
    beam = Beam(E0=E0, sigma_E=sE, spot_sigma=0.3, pos=(0.0, 0.05, 0.0), dir=(1.0, 0.0, 0.0))
    return Problem(grid, mats, [beam], o)


def moments(dg, c):
    """(M0, M1, M2) = int E^j psi dE, exact for the piecewise quadratics."""
    xq, wq = np.polynomial.legendre.leggauss(6)
    E = dg.lo[:, None] + 0.5 * dg.h * (xq[None, :] + 1.0)
    ph = dg._phi(xq)
    vals = c.reshape(dg.G, 3) @ ph
    w = 0.5 * dg.h * wq[None, :]
    return [float(np.sum(w * E**j * vals)) for j in range(3)]


def test_removal_is_the_crank_nicolson_factor():
    sig = 0.7
    p = synthetic_problem(sig=sig)
    tr = raytrace.Tracer(p, p.beams[0])
    c = tr.c0.copy()
    M0 = moments(tr.dg, c)[0]
    n_total = 0
    for cell in range(12):
        P, ns = tr.propagator(cell, 0.1)
        for _ in range(ns):
            c = P @ c
        n_total += ns
    h = 0.1 / 10
    factor = ((1 - 0.5 * h * sig) / (1 + 0.5 * h * sig)) ** n_total
    assert abs(moments(tr.dg, c)[0] / M0 - factor) < 1e-12
    # and exp(-sig z) to O(h^2)
    assert abs(factor - math.exp(-sig * 1.2)) < 1e-5


def test_drift_and_straggling_moments_exact():
    # constant S and T, no removal: mean drifts by -S z and the variance grows
    # by T z exactly (E and E^2 are in the DG space; CN is exact for them)
    S, T = 4.0, 0.35
    p = synthetic_problem(S=S, T=T)
    tr = raytrace.Tracer(p, p.beams[0])
    c = tr.c0.copy()
    m0 = moments(tr.dg, c)
    z = 0.0
    for cell in range(15):
        P, ns = tr.propagator(cell, 0.1)
        for _ in range(ns):
            c = P @ c
        z += 0.1
    m = moments(tr.dg, c)
    assert abs(m[0] - m0[0]) < 1e-12
    mean0, mean = m0[1] / m0[0], m[1] / m[0]
    var0, var = m0[2] / m0[0] - mean0**2, m[2] / m[0] - mean**2
    assert abs((mean - mean0) + S * z) < 1e-9
    assert abs((var - var0) - T * z) < 1e-9


def test_operator_conserves_particles_up_to_cutoff_outflow():
    # with no removal: d/dz int psi = -S*(E_cut) psi(E_cut) exactly
    p = synthetic_problem(S=3.0, T=0.2, G=16)
    dg = raytrace.EnergyDG(1.0, 52.5, 16)
    mat = p.materials
    A = dg.operator(mat.e, mat.S[0], mat.T[0], mat.dG[0, :, -1])
    rows = A[0::3, :].sum(axis=0)
    ref = np.zeros(3 * 16)
    ref[:3] = -3.0 * np.array([1.0, -1.0, 1.0])
    assert np.abs(rows - ref).max() < 1e-12


def test_row_subset_is_the_full_march_on_those_rows():
    # a row subset of the march (the full-size GPU test samples rows) gives
    # exactly the full march's values on its rows and zero elsewhere
    p = configs.small_3d(n=6, N=2, n_steps=5)
    tr = raytrace.Tracer(p, p.beams[0])
    ps, du = tr.trace()
    rows = tr.grid_rows()
    pick = [3, 17, 20]
    ps2, du2 = raytrace.Tracer(p, p.beams[0]).trace(rows=pick)
    cells = rows[pick].ravel()
    assert np.array_equal(ps2[:, cells], ps[:, cells]) and np.array_equal(du2[cells], du[cells])
    rest = np.setdiff1d(np.arange(p.grid.n), cells)
    assert not ps2[:, rest].any() and not du2[rest].any()
    assert np.abs(ps[:, cells]).max() > 0.0


def test_cell_subset_is_the_per_cell_trace_on_those_cells():
    p = configs.small_oblique_2d(angle_deg=60.0)
    tr = raytrace.Tracer(p, p.beams[0])
    ps, du = tr.trace(rowwise=False)
    pick = np.flatnonzero(du)[[0, 5, -1]]
    ps2, du2 = raytrace.Tracer(p, p.beams[0]).trace(rowwise=False, cells=pick)
    assert np.array_equal(ps2[:, pick], ps[:, pick]) and np.array_equal(du2[pick], du[pick])
    rest = np.setdiff1d(np.arange(p.grid.n), pick)
    assert not ps2[:, rest].any() and not du2[rest].any()


def test_row_march_equals_per_cell_rays():
    p = configs.small_2d(nx=10, ny=6, N=2, mats="slab", n_steps=6, E0=20.0)
    tr = raytrace.Tracer(p, p.beams[0])
    a = tr.trace(rowwise=True)
    b = raytrace.Tracer(p, p.beams[0]).trace(rowwise=False)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_oblique_ray_pieces_cover_the_path():
    g = Grid(9, 7, 1, 0.1, 0.1, 0.1)
    om = (math.cos(0.6), math.sin(0.6), 0.0)
    centers = g.centers()
    for cell in (0, 13, 40, 62):
        xc = centers[cell]
        pieces = raytrace.ray_pieces(g, xc, om)
        total = sum(L for _, L in pieces)
        # entry parameter from the slab method
        t_in = max(min((0 - xc[d]) / om[d], (L - xc[d]) / om[d])
                   for d, L in ((0, 0.9), (1, 0.7)))
        assert abs(total + t_in) < 1e-12
        assert pieces[-1][0] == cell
        assert all(L > 0 for _, L in pieces)
