"""Energy grid and per-step coefficients (Sec. 3.3, eq. discAngle, Sec. 3.3.3).

Pseudo-time t = E_max - E (Sec. 3.3).  Readings used where the paper is silent:
  * E_max = max over the run's beams of E0 + e_max_sigmas * sigma_E,
    E_cut = options.e_cut;
  * energy grid E_0 = E_max > E_1 > ... > E_n = E_cut, step k spanning
    [E_{k+1}, E_k] with dt_k = E_k - E_{k+1}:
      uniform       equal steps (the paper's experiments);
      proportional  steps proportional to the energy, E_k = E_cut (E_max/E_cut)^(1-k/n):
                    short steps at low energy, where protons lose energy fastest
                    (the non-uniform grid the paper's Sec. 6 proposes);
      cfl           equal steps of residual range in the least-stopping voxel,
                    R(E_k) = (1 - k/n) R(E_max) with R(E) = int_{E_cut}^E dE'/S_min(E'),
                    S_min(E) = min_x S(x, E), so that dt_k / S_min is the same for
                    every step and every step takes the same number of RK4
                    substeps; R is the trapezoid rule on 4096 equal intervals and
                    is inverted by linear interpolation;
      user          the energies given in options.egrid_points;
  * every energy-dependent coefficient of step k is frozen at the midpoint
    E_{k+1/2} = (E_k + E_{k+1}) / 2;
  * tables are interpolated linearly in E (clamped at the table ends);
  * mixtures follow eq. mixXS: S(x,E) = sum_i w_i(x) S_i(E), likewise for the
    Legendre moments;
  * Boltzmann collisions with the extended transport correction (Sec. 3.3.1):
    delta_i = G_{i,N+1}; self-scattering uses G_l - G_0 (delta cancels),
    in-scattering uses G_l - G_{N+1}, uncollided removal uses G_0 - G_{N+1};
  * Fokker-Planck collisions (Sec. 2.1, Sec. 3.1): eigenvalues
    -xi_1 l (l+1) / 2 of the scaled Laplace-Beltrami operator, with the
    momentum-transfer coefficient xi_1 = 2 pi int (1 - mu) Sigma_s dmu = G_0 - G_1;
    the uncollided flux is not removed (Gamma_out = 0) and sources the whole
    operator (Gamma_in = Gamma): self- and in-scattering both use
    -xi_1 l (l+1) / 2, removal is zero.  The stabilising moment correction the
    paper cites for this model is not specified there and is not applied;
  * the K/L/S ODEs of one step take n_sub RK4 substeps,
    n_sub = ceil(dt_k / (nu * min_x S(x, E_{k+1/2}) * min_d Delta_d)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import pn

CFL_GRID_INTERVALS = 4096


def interp(e_tab, table, E):
    """Linear interpolation of table[..., n_e] at energy E (scalar)."""
    tab = np.asarray(table)
    flat = tab.reshape(-1, tab.shape[-1])
    out = np.array([np.interp(E, e_tab, row) for row in flat])
    return out.reshape(tab.shape[:-1])


def e_max_of(beams, opts):
    return max(b.E0 + opts.e_max_sigmas * b.sigma_E for b in beams)


def min_stopping(problem, E):
    """S_min(E) = min over voxels of sum_i w_i S_i(E) (MeV/cm)."""
    mat = problem.materials
    return float(np.min(mat.w.T @ interp(mat.e, mat.S, E)))


def energy_edges(problem, beams):
    """E_0 = E_max > ... > E_n = E_cut for a run over `beams`."""
    o = problem.options
    n = o.n_steps
    e_max, e_cut = e_max_of(beams, o), o.e_cut
    mode = getattr(o, "egrid", "uniform")
    k = np.arange(n + 1)
    if mode == "uniform":
        dt = (e_max - e_cut) / n
        E = e_max - k * dt
    elif mode == "proportional":
        E = e_cut * (e_max / e_cut) ** (1.0 - k / n)
    elif mode == "cfl":
        K = CFL_GRID_INTERVALS
        h = (e_max - e_cut) / K
        x = e_cut + h * np.arange(K + 1)
        inv = np.array([1.0 / min_stopping(problem, xi) for xi in x])
        R = np.concatenate([[0.0], np.cumsum(0.5 * h * (inv[:-1] + inv[1:]))])
        target = R[-1] * (1.0 - k / n)
        E = np.interp(target, R, x)
    elif mode == "user":
        E = np.asarray(o.egrid_points, dtype=np.float64)
        if E.shape != (n + 1,) or np.any(np.diff(E) >= 0.0):
            raise ValueError("egrid_points must hold n_steps + 1 descending energies")
    else:
        raise ValueError(mode)
    E = np.array(E, dtype=np.float64)
    if mode != "user":
        E[0], E[-1] = e_max, e_cut
    return E


def energy_grid(beam, opts):
    """(E_max, E_cut, dt) of the uniform grid of one beam."""
    e_max = beam.E0 + opts.e_max_sigmas * beam.sigma_E
    e_cut = opts.e_cut
    return e_max, e_cut, (e_max - e_cut) / opts.n_steps


@dataclass
class StepCoeffs:
    k: int
    e_half: float
    dt: float
    stop: np.ndarray      # (n,)  S(x, E_{k+1/2}), MeV/cm
    s: np.ndarray         # (n,)  1 / stop
    a: np.ndarray         # (n_mat, N+1)  self-scattering eigenvalues
    g: np.ndarray         # (m, n_mat)    in-scattering source directions of the beam
    n_sub: int
    h: float


def min_spacing(grid):
    return min(grid.dx, grid.dy) if grid.dim == 2 else min(grid.dx, grid.dy, grid.dz)


def collision_eigenvalues(problem, dG_half):
    """(a, gt): self-scattering a_{il} and in-scattering factors gt_{il},
    l = 0..N, from the table differences dG_half[i, l] = G_0 - G_l at E_{k+1/2}."""
    N = problem.options.pn_degree
    if getattr(problem.options, "collision", "boltzmann") == "fokker_planck":
        ell = np.arange(N + 1)
        xi1 = dG_half[:, 1]
        a = -0.5 * xi1[:, None] * (ell * (ell + 1))[None, :]
        return a, a.copy()
    a = -dG_half[:, : N + 1]                                      # G_l - G_0
    gt = dG_half[:, N + 1][:, None] - dG_half[:, : N + 1]         # G_l - G_{N+1}
    return a, gt


def removal(problem, dG_half):
    """Removal rate of the uncollided flux per material (cm^2/g)."""
    N = problem.options.pn_degree
    if getattr(problem.options, "collision", "boltzmann") == "fokker_planck":
        return np.zeros(dG_half.shape[0])
    return dG_half[:, N + 1]


def step_coeffs(problem, beam, k, edges=None):
    o = problem.options
    mat = problem.materials
    N = o.pn_degree
    E_edges = energy_edges(problem, [beam]) if edges is None else edges
    dt = float(E_edges[k] - E_edges[k + 1])
    E = 0.5 * (E_edges[k] + E_edges[k + 1])
    S_i = interp(mat.e, mat.S, E)                       # (n_mat,)
    stop = mat.w.T @ S_i                                # (n,)
    dG = np.stack([interp(mat.e, mat.dG[:, :, l], E) for l in range(N + 2)], axis=1)
    a, gt = collision_eigenvalues(problem, dG)
    ell, _ = pn.degree_order(N)
    TM = pn.beam_moments(N, beam.dir)
    g = (gt[:, ell] * TM[None, :]).T                    # (m, n_mat)
    nu = o.cfl(problem.grid.dim)
    n_sub = max(1, math.ceil(dt / (nu * stop.min() * min_spacing(problem.grid)) - 1e-9))
    return StepCoeffs(k, E, dt, stop, 1.0 / stop, a, g, n_sub, dt / n_sub)
