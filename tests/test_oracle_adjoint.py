"""Pins of the plan-objective gradient of the reference (oracle/adjoint.py)."""
import numpy as np

from oracle import adjoint
from workloads.plan import synthetic_plan


def test_hand_computed_three_cells():
    # D = 1*[1,2,0] + 2*[0,1,3] = [1,4,6]; target = cells 0, 1; dhat = 2, lam = 0.1
    # J = (1-2)^2 + (4-2)^2 + 0.1*36 = 8.6; dJ/dD = [-2, 4, 1.2]
    # dJ/dw = [1*-2 + 2*4, 1*4 + 3*1.2] = [6, 7.6]
    doses = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0]])
    w = np.array([1.0, 2.0])
    target = np.array([1, 1, 0], dtype=np.uint8)
    assert abs(adjoint.objective(doses, w, target, 2.0, 0.1) - 8.6) < 1e-14
    np.testing.assert_allclose(adjoint.dose_gradient(doses, w, target, 2.0, 0.1),
                               [-2.0, 4.0, 1.2], rtol=0, atol=1e-14)
    np.testing.assert_allclose(adjoint.weight_gradient(doses, w, target, 2.0, 0.1),
                               [6.0, 7.6], rtol=0, atol=1e-13)


def test_central_difference_is_exact_for_the_quadratic():
    # J is quadratic in w, so the central difference equals the derivative up
    # to rounding for any step
    doses, w, target, dhat, lam = synthetic_plan(2000, 5, seed=11)
    g = adjoint.weight_gradient(doses, w, target, dhat, lam)
    for h in (1e-3, 0.25):
        for b in range(len(w)):
            e = np.zeros_like(w)
            e[b] = h
            fd = (adjoint.objective(doses, w + e, target, dhat, lam) -
                  adjoint.objective(doses, w - e, target, dhat, lam)) / (2 * h)
            assert abs(fd - g[b]) <= 1e-9 * max(1.0, abs(g[b]))


def test_minimum_without_penalty_is_least_squares():
    # lam = 0 and a full target: J = |Dw - dhat|^2, whose zero gradient is the
    # least-squares solution of doses^T w = dhat
    doses, _, _, dhat, _ = synthetic_plan(300, 4, seed=3)
    target = np.ones(300, dtype=np.uint8)
    w_ls = np.linalg.lstsq(doses.T, np.full(300, dhat), rcond=None)[0]
    g = adjoint.weight_gradient(doses, w_ls, target, dhat, 0.0)
    assert np.abs(g).max() <= 1e-9 * np.abs(doses).sum()


def test_unit_weight_level():
    doses = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0]])
    assert adjoint.unit_weight_level(doses, np.array([1, 1, 0])) == 2.0
