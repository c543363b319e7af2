"""GPU parity of the plan objective and its beam-weight gradient (the
library's dlra_plan_objective) against the reference's closed form."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import adjoint
from oracle import solver as ref
from workloads import configs
from workloads.plan import centre_target, synthetic_plan

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_04484_amd as dl
    return dl, torch


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,nb,seed", [(50_000, 9, 5), (50_001, 1, 6), (777, 64, 7), (1, 3, 8)])
def test_synthetic_plan_matches_reference(n, nb, seed):
    dl, torch = _gpu()
    say(f"plan objective n={n} nb={nb}")
    doses, w, target, dhat, lam = synthetic_plan(n, nb, seed=seed)
    J, g = dl.binding.plan_objective(torch.from_numpy(doses).cuda(), w,
                                     torch.from_numpy(target).cuda(), dhat, lam)
    J_ref = adjoint.objective(doses, w, target, dhat, lam)
    g_ref = adjoint.weight_gradient(doses, w, target, dhat, lam)
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
    assert np.abs(g - g_ref).max() <= 1e-12 * np.abs(g_ref).max()


def test_gradient_equals_central_difference_on_the_gpu():
    # J is quadratic in w: the central difference of the library's own J is
    # its derivative up to rounding
    dl, torch = _gpu()
    say("plan objective: central differences")
    doses, w, target, dhat, lam = synthetic_plan(20_000, 4, seed=9)
    d_t, t_t = torch.from_numpy(doses).cuda(), torch.from_numpy(target).cuda()
    _, g = dl.binding.plan_objective(d_t, w, t_t, dhat, lam)
    h = 0.125
    for b in range(len(w)):
        e = np.zeros_like(w)
        e[b] = h
        Jp, _ = dl.binding.plan_objective(d_t, w + e, t_t, dhat, lam)
        Jm, _ = dl.binding.plan_objective(d_t, w - e, t_t, dhat, lam)
        assert abs((Jp - Jm) / (2 * h) - g[b]) <= 1e-9 * max(1.0, abs(g[b]))


def test_plan_of_transport_doses():
    # three beams of the small 3D phantom (+x, -y, +y): per-beam doses from
    # the library and from the reference, then the objective on each side
    dl, torch = _gpu()
    say("plan objective on transport doses")
    p = configs.small_3d(n=8, r=6)
    b0 = p.beams[0]
    L = p.grid.ny * p.grid.dy
    mid = 0.5 * L
    beams = [b0,
             dataclasses.replace(b0, E0=22.0, sigma_E=0.22, pos=(mid, L, mid), dir=(0.0, -1.0, 0.0)),
             dataclasses.replace(b0, E0=28.0, sigma_E=0.28, pos=(mid - 0.05, 0.0, mid),
                                 dir=(0.0, 1.0, 0.0))]
    p = dataclasses.replace(p, beams=beams)
    target = centre_target(p.grid, 0.1)
    gpu_doses, ref_doses = [], []
    for b in range(len(beams)):
        s = dl.BeamSolver(p, b)
        s.raytrace()
        s.run()
        gpu_doses.append(s.dose())
        s.close()
        ref_doses.append(ref.run_beam_dlra(p, beams[b])["dose"])
    ref_doses = np.stack(ref_doses)
    dhat = adjoint.unit_weight_level(ref_doses, target)   # a shared input
    w = np.array([1.0, 0.7, 1.3])
    J, g = dl.binding.plan_objective(torch.stack(gpu_doses).contiguous(), w,
                                     torch.from_numpy(target).cuda(), dhat, 0.1)
    J_ref = adjoint.objective(ref_doses, w, target, dhat, 0.1)
    g_ref = adjoint.weight_gradient(ref_doses, w, target, dhat, 0.1)
    assert abs(J - J_ref) <= 1e-8 * abs(J_ref)
    assert np.abs(g - g_ref).max() <= 1e-8 * np.abs(g_ref).max()
