"""Full-rank step: the same discretisation on the dense moment matrix u (n x m).

Lie splitting of eq. streamscattsplit (eq. split-streaming, eq. split-scattering):
  1. u <- RK4^{n_sub}(F_S, u, dt)                     (streaming)
  2. u[x, p] <- u[x, p] / (1 - dt s(x) sum_i w_i(x) a_{i,l(p)})
                                                       (implicit Euler, diagonal self-scattering)
  3. u <- u + dt sum_i (w_i o psi_u) g_i^T             (explicit Euler, in-scattering)
  4. D_c += dt sqrt(4 pi) u[:, 0]
This is the low-rank step with U and V spanning everything; it is the plain
definition the DLRA step reduces to at full rank.
"""
from __future__ import annotations

import math

import numpy as np

from . import pn
from . import transport as tr


def step(u, dose_c, c, Apm, problem, psibar_k, sources=None):
    """One step; the source is one beam's (psibar_k with c.g) or the factor pair
    sources = (Q, G) of several beams (Q G^T = sum_b sum_i (w_i o psi_b) g_{i,b}^T)."""
    g, o = problem.grid, problem.options
    w = problem.materials.w
    ell, _ = pn.degree_order(o.pn_degree)
    u = tr.rk4(lambda x: tr.streaming_full(x, c.s, Apm, g), u, c.h, c.n_sub)
    wa = w.T @ c.a                                       # (n, N+1): sum_i w_i a_{i,l}
    u = u / (1.0 - c.dt * c.s[:, None] * wa[:, ell])
    if sources is None:
        u = u + c.dt * (w.T * psibar_k[:, None]) @ c.g.T
    else:
        Q, G = sources
        u = u + c.dt * Q @ G.T
    dose_c = dose_c + c.dt * math.sqrt(4.0 * math.pi) * u[:, 0]
    return u, dose_c
