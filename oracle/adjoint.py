"""Gradient of a treatment-plan objective with respect to the beam weights
(test infrastructure; FP64, plain numpy).

The dose of a plan is the weighted sum of the beams' doses at unit weight,
D = sum_b w_b D_b: the transport solve is linear in the incoming flux, so each
beam's dose scales with its weight (the beam source enters linearly, Sec. 3.2,
and the collided equations are linear in the flux, Sec. 3.3).  For the
objective J(w) = sum_{x in T} (D(x) - dhat)^2 + lam sum_{x not in T} D(x)^2
the gradient is therefore the closed form
    dJ/dw_b = sum_x g(x) D_b(x),   g = 2 (D - dhat) on T,  2 lam D off T,
i.e. the adjoint of the (linear) dose map applied to dJ/dD.  The gradient
with respect to voxel densities, which needs the reverse sweep through the
integrator, is not implemented here.
"""
from __future__ import annotations

import numpy as np


def plan_dose(doses: np.ndarray, w: np.ndarray) -> np.ndarray:
    """D = sum_b w_b D_b for doses [n_beams][n_cells]."""
    return np.asarray(w, dtype=np.float64) @ np.asarray(doses, dtype=np.float64)


def objective(doses, w, target, dhat: float, lam: float) -> float:
    D = plan_dose(doses, w)
    t = np.asarray(target) != 0
    return float(np.sum((D[t] - dhat) ** 2) + lam * np.sum(D[~t] ** 2))


def dose_gradient(doses, w, target, dhat: float, lam: float) -> np.ndarray:
    """dJ/dD per cell."""
    D = plan_dose(doses, w)
    t = np.asarray(target) != 0
    return np.where(t, 2.0 * (D - dhat), 2.0 * lam * D)


def weight_gradient(doses, w, target, dhat: float, lam: float) -> np.ndarray:
    """dJ/dw_b = <dJ/dD, D_b> for every beam b."""
    return np.asarray(doses, dtype=np.float64) @ dose_gradient(doses, w, target, dhat, lam)


def unit_weight_level(doses, target) -> float:
    """Mean target dose of the plan at unit weights (the prescription level
    of the objective when none is given)."""
    D = np.asarray(doses, dtype=np.float64).sum(axis=0)
    return float(D[np.asarray(target) != 0].mean())
