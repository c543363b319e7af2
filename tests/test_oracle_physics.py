"""Whole-run physics pins of the reference solver on the 2D water workload
(64x64 cells of 1 mm, 70 MeV, P_7, rank 10, 100 steps)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import solver
from workloads import configs


@pytest.fixture(scope="module")
def c1_run():
    p = configs.c1()
    res = solver.run_beam_dlra(p, p.beams[0])
    return p, res


def test_bragg_peak_at_csda_range(c1_run):
    # distal 80% point of the laterally integrated depth dose within
    # max(dx, 1% R) of the CSDA range int_{E_cut}^{E0} dE / S(E)
    p, res = c1_run
    mat = p.materials
    R = quad(lambda E: 1.0 / np.interp(E, mat.e, mat.S[0]), p.options.e_cut, p.beams[0].E0,
             limit=200)[0]
    depth = res["dose"].reshape(64, 64).sum(axis=0)
    dd = depth / depth.max()
    x = (np.arange(64) + 0.5) * p.grid.dx
    i = int(np.argmax(dd))
    j = i + int(np.argmax(dd[i:] < 0.8))
    r80 = x[j - 1] + (x[j] - x[j - 1]) * (dd[j - 1] - 0.8) / (dd[j - 1] - dd[j])
    assert abs(r80 - R) <= max(p.grid.dx, 0.01 * R)


def test_energy_balance(c1_run):
    # all energy between E0 and E_cut is deposited (nothing leaves this box):
    # int D dx dy = E0 - E_cut per proton (per cm in 2D) up to the O(dt) energy rule
    p, res = c1_run
    E = res["dose"].sum() * p.grid.dx * p.grid.dy
    assert abs(E - (p.beams[0].E0 - p.options.e_cut)) < 0.01 * p.beams[0].E0


def test_collided_part_is_a_small_positive_share(c1_run):
    p, res = c1_run
    frac = res["dose_c"].sum() / res["dose_u"].sum()
    assert 0.01 < frac < 0.5
