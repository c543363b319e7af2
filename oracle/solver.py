"""Drivers: whole-problem runs of the reference solvers.

Deposited energy = uncollided part (ray tracer) + collided part (DLRA or full
rank), MeV/cm^3 per source proton (per cm in 2D).

  run_beam_*    one beam at unit weight on that beam's own energy grid (or
                the grid given as `edges`)
  run_joint_*   all beams of the problem in one collided solve: a common
                energy grid (E_max the largest of the beams'), each beam's
                uncollided flux scaled by its weight, and the in-scattering
                source sum_b sum_i (w_i o psi_b) g_{i,b}^T (the joint source
                of the paper's two-beam case, Sec. 4.3)
"""
from __future__ import annotations

import numpy as np

from . import coeffs, dlra, fullrank, pn, raytrace


def streaming_split(problem):
    return pn.split_streaming(problem.options.pn_degree, problem.grid.dim)


def uncollided(problem, beam, rowwise=True, edges=None):
    return raytrace.Tracer(problem, beam, edges).trace(rowwise=rowwise)


def run_beam_dlra(problem, beam, n_steps=None, psibar=None, Du=None, state=None,
                  Apm=None, callback=None, edges=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    edges = coeffs.energy_edges(problem, [beam]) if edges is None else edges
    if psibar is None:
        psibar, Du = uncollided(problem, beam, edges=edges)
    Apm = streaming_split(problem) if Apm is None else Apm
    if state is None:
        st = dlra.initial_state(problem, coeffs.step_coeffs(problem, beam, 0, edges).g)
    else:
        st = state
    for k in range(st.k, n_steps):
        c = coeffs.step_coeffs(problem, beam, k, edges)
        st = dlra.step(st, c, Apm, problem, psibar[k])
        if callback is not None:
            callback(k, st)
    return dict(dose_c=st.dose_c, dose_u=Du, dose=st.dose_c + Du, state=st, psibar=psibar)


def run_beam_fullrank(problem, beam, n_steps=None, psibar=None, Du=None, Apm=None,
                      edges=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    edges = coeffs.energy_edges(problem, [beam]) if edges is None else edges
    if psibar is None:
        psibar, Du = uncollided(problem, beam, edges=edges)
    Apm = streaming_split(problem) if Apm is None else Apm
    u = np.zeros((problem.grid.n, problem.m))
    dose_c = np.zeros(problem.grid.n)
    for k in range(n_steps):
        c = coeffs.step_coeffs(problem, beam, k, edges)
        u, dose_c = fullrank.step(u, dose_c, c, Apm, problem, psibar[k])
    return dict(dose_c=dose_c, dose_u=Du, dose=dose_c + Du, u=u, psibar=psibar)


def joint_uncollided(problem, edges):
    """Per-beam uncollided tables on the common grid, scaled by the beam weights:
    (psibar [n_beams][n_steps][n], Du summed over beams)."""
    ps, Du = [], np.zeros(problem.grid.n)
    for b in problem.beams:
        p_b, d_b = uncollided(problem, b, edges=edges)
        ps.append(b.weight * p_b)
        Du += b.weight * d_b
    return np.stack(ps), Du


def _joint_step_data(problem, edges, k, psibar):
    cs = [coeffs.step_coeffs(problem, b, k, edges) for b in problem.beams]
    Q, G = dlra.source_factors(problem.materials.w, [psibar[b][k] for b in range(len(cs))],
                               [c.g for c in cs])
    return cs[0], Q, G


def run_joint_dlra(problem, n_steps=None, psibar=None, Du=None, Apm=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    edges = coeffs.energy_edges(problem, problem.beams)
    if psibar is None:
        psibar, Du = joint_uncollided(problem, edges)
    Apm = streaming_split(problem) if Apm is None else Apm
    _, _, G0 = _joint_step_data(problem, edges, 0, psibar)
    st = dlra.initial_state(problem, G0)
    for k in range(n_steps):
        c, Q, G = _joint_step_data(problem, edges, k, psibar)
        st = dlra.step(st, c, Apm, problem, None, sources=(Q, G))
    return dict(dose_c=st.dose_c, dose_u=Du, dose=st.dose_c + Du, state=st, psibar=psibar)


def run_joint_fullrank(problem, n_steps=None, psibar=None, Du=None, Apm=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    edges = coeffs.energy_edges(problem, problem.beams)
    if psibar is None:
        psibar, Du = joint_uncollided(problem, edges)
    Apm = streaming_split(problem) if Apm is None else Apm
    u = np.zeros((problem.grid.n, problem.m))
    dose_c = np.zeros(problem.grid.n)
    for k in range(n_steps):
        c, Q, G = _joint_step_data(problem, edges, k, psibar)
        u, dose_c = fullrank.step(u, dose_c, c, Apm, problem, None, sources=(Q, G))
    return dict(dose_c=dose_c, dose_u=Du, dose=dose_c + Du, u=u, psibar=psibar)


def run_dlra(problem, **kw):
    total = np.zeros(problem.grid.n)
    per_beam = []
    for b in problem.beams:
        res = run_beam_dlra(problem, b, **kw)
        total += b.weight * res["dose"]
        per_beam.append(res)
    return total, per_beam
