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
