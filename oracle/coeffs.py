"""Energy grid and per-step coefficients (Sec. 3.3, eq. discAngle, Sec. 3.3.3).

Pseudo-time t = E_max - E (Sec. 3.3).  Readings used where the paper is silent:
  * E_max = E0 + e_max_sigmas * sigma_E, E_cut = options.e_cut, uniform steps
    dt = (E_max - E_cut) / n_steps, E_k = E_max - k dt;
  * every energy-dependent coefficient of step k is frozen at E_{k+1/2};
  * tables are interpolated linearly in E (clamped at the table ends);
  * mixtures follow eq. mixXS: S(x,E) = sum_i w_i(x) S_i(E), likewise for the
    Legendre moments;
  * extended transport correction (Sec. 3.3.1): delta_i = G_{i,N+1},
    self-scattering uses G_l - G_0 (delta cancels), in-scattering uses
    G_l - G_{N+1}, uncollided removal uses G_0 - G_{N+1};
  * the K/L/S ODEs of one step take n_sub RK4 substeps,
    n_sub = ceil(dt / (nu * min_x S(x, E_{k+1/2}) * min_d Delta_d)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import pn


def energy_grid(beam, opts):
    e_max = beam.E0 + opts.e_max_sigmas * beam.sigma_E
    e_cut = opts.e_cut
    return e_max, e_cut, (e_max - e_cut) / opts.n_steps


def interp(e_tab, table, E):
    """Linear interpolation of table[..., n_e] at energy E (scalar)."""
    tab = np.asarray(table)
    flat = tab.reshape(-1, tab.shape[-1])
    out = np.array([np.interp(E, e_tab, row) for row in flat])
    return out.reshape(tab.shape[:-1])


@dataclass
class StepCoeffs:
    k: int
    e_half: float
    dt: float
    stop: np.ndarray      # (n,)  S(x, E_{k+1/2}), MeV/cm
    s: np.ndarray         # (n,)  1 / stop
    a: np.ndarray         # (n_mat, N+1)  G_l - G_0
    g: np.ndarray         # (m, n_mat)    (G_l(p) - G_{N+1}) * T_M[p]
    n_sub: int
    h: float


def min_spacing(grid):
    return min(grid.dx, grid.dy) if grid.dim == 2 else min(grid.dx, grid.dy, grid.dz)


def step_coeffs(problem, beam, k):
    o = problem.options
    mat = problem.materials
    N = o.pn_degree
    e_max, e_cut, dt = energy_grid(beam, o)
    E = e_max - (k + 0.5) * dt
    S_i = interp(mat.e, mat.S, E)                       # (n_mat,)
    stop = mat.w.T @ S_i                                # (n,)
    dG = np.stack([interp(mat.e, mat.dG[:, :, l], E) for l in range(N + 2)], axis=1)
    a = -dG[:, : N + 1]                                 # G_l - G_0
    gt = dG[:, N + 1][:, None] - dG[:, : N + 1]         # G_l - G_{N+1}
    ell, _ = pn.degree_order(N)
    TM = pn.beam_moments(N, beam.dir)
    g = (gt[:, ell] * TM[None, :]).T                    # (m, n_mat)
    nu = o.cfl(problem.grid.dim)
    n_sub = max(1, math.ceil(dt / (nu * stop.min() * min_spacing(problem.grid)) - 1e-9))
    return StepCoeffs(k, E, dt, stop, 1.0 / stop, a, g, n_sub, dt / n_sub)
