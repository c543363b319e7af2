"""Seeded synthetic inputs for the plan objective (per-beam dose maps, beam
weights, a target region).  Data generation only."""
from __future__ import annotations

import numpy as np


def synthetic_plan(n_cells: int, n_beams: int, seed: int = 5, target_frac: float = 0.2):
    """Per-beam doses (non-negative, [n_beams][n_cells], FP64), weights in
    [0.5, 1.5], a target mask (uint8, contiguous run of target_frac of the
    cells), a prescription level and the out-of-target penalty (0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    doses = rng.gamma(2.0, 0.5, size=(n_beams, n_cells))
    w = rng.uniform(0.5, 1.5, size=n_beams)
    target = np.zeros(n_cells, dtype=np.uint8)
    nt = max(1, int(target_frac * n_cells))
    t0 = int(rng.integers(0, n_cells - nt + 1))
    target[t0:t0 + nt] = 1
    dhat = float(rng.uniform(0.5, 2.0))
    return doses, w, target, dhat, 0.1


def centre_target(grid, half_width_cm: float) -> np.ndarray:
    """Target mask (uint8, x-fastest cells) of the square (2D) or cube (3D) of
    the given half width around the grid centre."""
    x = (np.arange(grid.nx) + 0.5) * grid.dx
    y = (np.arange(grid.ny) + 0.5) * grid.dy
    z = (np.arange(grid.nz) + 0.5) * grid.dz
    cx, cy, cz = x.mean(), y.mean(), z.mean()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    inside = (np.abs(X - cx) <= half_width_cm) & (np.abs(Y - cy) <= half_width_cm)
    if grid.nz > 1:
        inside &= np.abs(Z - cz) <= half_width_cm
    return inside.reshape(-1).astype(np.uint8)
