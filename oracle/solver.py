"""Drivers: whole-problem runs of the reference solvers (per beam, summed with
beam weights).  Deposited energy = uncollided part (ray tracer) + collided
part (DLRA or full rank), MeV/cm^3 per source proton (per cm in 2D)."""
from __future__ import annotations

import numpy as np

from . import coeffs, dlra, fullrank, pn, raytrace


def streaming_split(problem):
    return pn.split_streaming(problem.options.pn_degree, problem.grid.dim)


def uncollided(problem, beam, rowwise=True):
    return raytrace.Tracer(problem, beam).trace(rowwise=rowwise)


def run_beam_dlra(problem, beam, n_steps=None, psibar=None, Du=None, state=None,
                  Apm=None, callback=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    if psibar is None:
        psibar, Du = uncollided(problem, beam)
    Apm = streaming_split(problem) if Apm is None else Apm
    if state is None:
        st = dlra.initial_state(problem, coeffs.step_coeffs(problem, beam, 0).g)
    else:
        st = state
    for k in range(st.k, n_steps):
        c = coeffs.step_coeffs(problem, beam, k)
        st = dlra.step(st, c, Apm, problem, psibar[k])
        if callback is not None:
            callback(k, st)
    return dict(dose_c=st.dose_c, dose_u=Du, dose=st.dose_c + Du, state=st, psibar=psibar)


def run_beam_fullrank(problem, beam, n_steps=None, psibar=None, Du=None, Apm=None):
    o = problem.options
    n_steps = o.n_steps if n_steps is None else n_steps
    if psibar is None:
        psibar, Du = uncollided(problem, beam)
    Apm = streaming_split(problem) if Apm is None else Apm
    u = np.zeros((problem.grid.n, problem.m))
    dose_c = np.zeros(problem.grid.n)
    for k in range(n_steps):
        c = coeffs.step_coeffs(problem, beam, k)
        u, dose_c = fullrank.step(u, dose_c, c, Apm, problem, psibar[k])
    return dict(dose_c=dose_c, dose_u=Du, dose=dose_c + Du, u=u, psibar=psibar)


def run_dlra(problem, **kw):
    total = np.zeros(problem.grid.n)
    per_beam = []
    for b in problem.beams:
        res = run_beam_dlra(problem, b, **kw)
        total += b.weight * res["dose"]
        per_beam.append(res)
    return total, per_beam
