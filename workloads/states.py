"""Seeded synthetic low-rank states (orthonormal bases, decaying diagonal
coefficients) for injected-state tests.  Data generation only."""
from __future__ import annotations

import numpy as np


def random_low_rank_state(n: int, m: int, r: int, seed: int = 7, decades: float = 6.0):
    """U (n x r) and V (m x r) with orthonormal columns from seeded Gaussian
    matrices, S = diag(10^0 .. 10^-decades) (r x r), all FP64."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((m, r)))
    S = np.diag(np.logspace(0.0, -decades, r))
    return U, S, V


def synthetic_uncollided(grid, beam, depth, width, seed: int = 13):
    """A seeded synthetic step-averaged uncollided flux (n,) with the shape of
    one energy step's table: a lateral Gaussian of the beam's spot around its
    axis times a band around `depth` (cm along the beam) of half-width
    `width`, modulated by seeded noise of 10 %.  Data generation only."""
    rng = np.random.default_rng(seed)
    xc = grid.centers()
    om = np.asarray(beam.dir, dtype=np.float64)
    rel = xc - np.asarray(beam.pos, dtype=np.float64)
    t = rel @ om
    perp = np.linalg.norm(rel - t[:, None] * om[None, :], axis=1)
    s = beam.spot_sigma
    lat = np.exp(-0.5 * (perp / s) ** 2) / (2.0 * np.pi * s * s)
    band = np.exp(-0.5 * ((t - depth) / width) ** 2)
    return lat * band * (1.0 + 0.1 * rng.standard_normal(grid.n))

