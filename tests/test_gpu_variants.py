"""GPU parity of the method's variants and of the library's boundary, through
the C ABI against the CPU reference on the same seeded inputs:

  * Fokker-Planck collisions (Sec. 2.1, Sec. 3.1);
  * non-uniform energy grids (proportional, constant CFL, user; Sec. 6);
  * the twelve-element material decomposition (Sec. 2.1);
  * a joint source of two beams in one collided solve (Sec. 4.3);
  * checkpoints (bitwise resume), the accumulated plan dose, and error flags
    raised by kernels surfacing at the next synchronising call.

Bars as in test_gpu_parity: FP64 relative L2 error of the deposited energy
<= 1e-10, mixed precision <= 1e-4.
"""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import coeffs
from oracle import solver as ref
from workloads import configs

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_04484_amd as dl
    return dl


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _beam_dose(dl, p, b=0):
    s = dl.BeamSolver(p, b)
    s.raytrace()
    s.run()
    d = s.dose().cpu().numpy()
    s.close()
    return d


VARIANTS = {
    "fokker_planck_2d": lambda: configs.small_2d(mats="slab", r=6, collision="fokker_planck"),
    "fokker_planck_3d": lambda: configs.small_3d(n=8, r=6, collision="fokker_planck"),
    "egrid_proportional": lambda: configs.small_2d(mats="slab", r=6, egrid="proportional"),
    "egrid_cfl": lambda: configs.small_2d(mats="slab", r=6, egrid="cfl"),
    "egrid_cfl_3d": lambda: configs.small_3d(n=8, r=6, egrid="cfl"),
    "elements_2d": lambda: configs.to_elements(configs.small_2d(mats="slab", r=6)),
    "elements_3d": lambda: configs.to_elements(configs.small_3d(n=8, r=6)),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_dose_parity_fp64(name):
    dl = _gpu()
    p = VARIANTS[name]()
    say(f"variant parity {name} (n_mat {p.materials.n_mat})")
    got = _beam_dose(dl, p)
    want = ref.run_beam_dlra(p, p.beams[0])["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-10


def test_user_energy_grid_parity():
    dl = _gpu()
    p = configs.small_2d(mats="slab", r=6)
    E = coeffs.energy_edges(p, p.beams)
    # a graded user grid between the same end points: denser at low energy
    t = np.linspace(0.0, 1.0, p.options.n_steps + 1)
    pts = tuple(E[-1] + (E[0] - E[-1]) * (1.0 - t) ** 1.5)
    pu = p.with_options(egrid="user", egrid_points=pts)
    say("user energy grid parity")
    got = _beam_dose(dl, pu)
    want = ref.run_beam_dlra(pu, pu.beams[0])["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-10


def test_variant_mixed_precision():
    dl = _gpu()
    p = configs.to_elements(configs.small_3d(n=10, N=5, r=12, precision="mixed", aug_tol=1e-4,
                                             floor_tol=1e-5, egrid="cfl"))
    say("twelve elements, CFL grid, mixed precision")
    got = _beam_dose(dl, p)
    want = ref.run_beam_dlra(p.with_options(precision="fp64"), p.beams[0])["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_joint_two_beam_source(precision):
    dl = _gpu()
    kw = dict(precision="mixed", aug_tol=1e-4, floor_tol=1e-5) if precision == "mixed" else {}
    p = configs.small_joint_2d(**kw)
    say(f"joint two-beam source, {precision}")
    s = dl.Solver(p)
    s.raytrace()
    ps, Du = s.uncollided()
    s.run()
    got = s.dose().cpu().numpy()
    s.close()
    want = ref.run_joint_dlra(p.with_options(precision="fp64"))
    if precision == "fp64":
        edges = coeffs.energy_edges(p, p.beams)
        ps_ref, Du_ref = ref.joint_uncollided(p, edges)
        assert np.abs(ps - ps_ref).max() <= 1e-12 * np.abs(ps_ref).max()
        assert np.abs(Du - Du_ref).max() <= 1e-12 * np.abs(Du_ref).max()
    err = rel(got, want["dose"])
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= (1e-10 if precision == "fp64" else 1e-4)


def test_plan_dose_accumulates_in_the_library():
    # separately solved beams at their weights, summed by dose_deposit's
    # accumulate flag, against the reference's weighted sum of beam doses
    dl = _gpu()
    p = configs.small_joint_2d()
    say("plan dose of separately solved beams")
    got = dl.solve(p).cpu().numpy()
    want = sum(b.weight * ref.run_beam_dlra(p, b)["dose"] for b in p.beams)
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("name,precision", [("slab2d", "fp64"), ("random3d", "mixed")])
def test_checkpoint_resume_is_bitwise(name, precision):
    dl = _gpu()
    import torch
    if name == "slab2d":
        p = configs.small_2d(mats="slab", rank_mode="adaptive", r=4, r_min=2, r_max=12,
                             trunc_tol=1e-4, precision=precision)
    else:
        p = configs.small_3d(n=8, r=6, precision=precision)
    say(f"checkpoint resume {name} {precision}")
    k = p.options.n_steps // 2
    a = dl.BeamSolver(p, 0)
    a.raytrace()
    a.run(k)
    blob = a.save()
    a.run(p.options.n_steps - k)
    full = a.dose()
    a.close()
    b = dl.BeamSolver(p, 0)
    b.raytrace()
    b.load(blob)
    assert b.state()[3] == k
    b.run(p.options.n_steps - k)
    resumed = b.dose()
    b.close()
    assert torch.equal(full, resumed)


def test_checkpoint_of_another_problem_is_rejected():
    dl = _gpu()
    a = dl.BeamSolver(configs.small_2d(r=6), 0)
    blob = a.save()
    a.close()
    b = dl.BeamSolver(configs.small_2d(nx=18, r=6), 0)
    with pytest.raises(dl.DlraError) as e:
        b.load(blob)
    assert e.value.code == -1
    with pytest.raises(dl.DlraError):
        b.load(blob[:10])
    b.close()


def test_non_finite_state_surfaces_at_sync():
    # a NaN in an injected S propagates through the step; the kernel's flag
    # is reported by the next synchronising call (dlra_sync and dose_deposit)
    # and cleared once reported
    dl = _gpu()
    p = configs.small_2d(mats="slab", r=6)
    say("non-finite state flag")
    s = dl.BeamSolver(p, 0)
    s.raytrace()
    s.run(2)
    U, S, V, k = s.state()
    S[0, 0] = np.nan
    s.set_state(U, S, V, k)
    s.step()
    with pytest.raises(dl.DlraError) as e:
        s.sync()
    assert e.value.code == -4
    s.sync()   # reported once, then cleared
    s.set_state(U, S, V, k)
    s.step()
    with pytest.raises(dl.DlraError) as e:
        s.dose()
    assert e.value.code == -4
    s.close()


def test_substep_limit_is_a_cfl_error():
    dl = _gpu()
    p = configs.small_2d(mats="slab", r=6)
    s = dl.BeamSolver(p, 0)
    most = max(s.substeps(k) for k in range(p.options.n_steps))
    s.close()
    assert most >= 2
    say(f"CFL limit below {most} substeps")
    q = p.with_options(n_sub_max=most - 1)
    with pytest.raises(dl.DlraError) as e:
        dl.BeamSolver(q, 0)
    assert e.value.code == -5
    s = dl.BeamSolver(p.with_options(n_sub_max=most), 0)
    s.close()


def test_set_uncollided_feeds_the_source():
    # a seeded synthetic uncollided table handed to the library and to the
    # reference gives the same step
    dl = _gpu()
    from oracle import dlra
    p = configs.small_2d(mats="slab", r=6)
    n, k = p.grid.n, 3
    rng = np.random.default_rng(21)
    psi = np.abs(rng.standard_normal(n))
    s = dl.BeamSolver(p, 0)
    s.set_uncollided(0, k, psi, np.zeros(n))
    st0 = dlra.initial_state(p, coeffs.step_coeffs(p, p.beams[0], 0).g)
    st0 = dataclasses.replace(st0, k=k)
    s.set_state(st0.U, st0.S, st0.V, k)
    s.step(sync=True)
    U, S, V, _ = s.state()
    dose_c = s.dose(flags=2).cpu().numpy()
    s.close()
    c = coeffs.step_coeffs(p, p.beams[0], k)
    nxt = dlra.step(st0, c, ref.streaming_split(p), p, psi)
    assert rel(U @ S @ V.T, nxt.U @ nxt.S @ nxt.V.T) <= 1e-11
    assert rel(dose_c, nxt.dose_c) <= 1e-11


# ---------------------------------------------------------------- oblique beams

OBLIQUE = {
    "oblique2d_30": lambda **k: configs.small_oblique_2d(angle_deg=30.0, **k),
    "oblique2d_135": lambda **k: configs.small_oblique_2d(angle_deg=135.0, mats="random", **k),
    "oblique3d": lambda **k: configs.small_oblique_3d(**k),
}


@pytest.mark.parametrize("name", list(OBLIQUE))
def test_oblique_raytrace_parity(name):
    # one ray per target cell from the domain entry, cut at faces and at the
    # perpendicular foot of every traversed cell's centre (Sec. 3.2)
    dl = _gpu()
    from oracle import raytrace
    p = OBLIQUE[name]()
    say(f"oblique ray tracer {name}")
    s = dl.BeamSolver(p, 0)
    s.raytrace()
    ps, Du = s.uncollided()
    s.close()
    ps_ref, Du_ref = raytrace.Tracer(p, p.beams[0]).trace()
    e1 = np.abs(ps - ps_ref).max() / np.abs(ps_ref).max()
    e2 = np.abs(Du - Du_ref).max() / np.abs(Du_ref).max()
    say(f"  max error psibar {e1:.3e}, Du {e2:.3e}")
    assert e1 <= 1e-12 and e2 <= 1e-12


# group counts around the wave kernel's two groups per lane: odd (the last
# lane half empty) and beyond 128 groups (one thread per ray, scratch rows)
RAY_GROUPS = {
    "oblique2d_33_groups": lambda: configs.small_oblique_2d(angle_deg=60.0, n_groups=33),
    "oblique2d_160_groups": lambda: configs.small_oblique_2d(angle_deg=30.0, n_groups=160),
    "axis2d_160_groups": lambda: configs.small_2d(nx=16, ny=14, N=3, n_steps=10, mats="slab",
                                                  r=6, dx=0.05, n_groups=160),
}


@pytest.mark.parametrize("name", list(RAY_GROUPS))
def test_raytrace_group_counts(name):
    dl = _gpu()
    from oracle import raytrace
    p = RAY_GROUPS[name]()
    say(f"ray tracer group count {name}")
    s = dl.BeamSolver(p, 0)
    s.raytrace()
    ps, Du = s.uncollided()
    s.close()
    ps_ref, Du_ref = raytrace.Tracer(p, p.beams[0]).trace()
    e1 = np.abs(ps - ps_ref).max() / np.abs(ps_ref).max()
    e2 = np.abs(Du - Du_ref).max() / np.abs(Du_ref).max()
    say(f"  max error psibar {e1:.3e}, Du {e2:.3e}")
    assert e1 <= 1e-12 and e2 <= 1e-12


@pytest.mark.parametrize("name", list(OBLIQUE))
def test_oblique_full_run_parity(name):
    dl = _gpu()
    p = OBLIQUE[name]()
    say(f"oblique full run {name}")
    got = _beam_dose(dl, p)
    want = ref.run_beam_dlra(p, p.beams[0])["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-10


def test_oblique_mixed_precision():
    dl = _gpu()
    p = configs.small_oblique_3d(precision="mixed", aug_tol=1e-4, floor_tol=1e-5)
    say("oblique 3D mixed precision")
    got = _beam_dose(dl, p)
    want = ref.run_beam_dlra(p.with_options(precision="fp64"), p.beams[0])["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-4


def test_joint_arc_of_oblique_beams():
    # three oblique beams of different energies and weights in one joint solve
    dl = _gpu()
    p = configs.small_arc_2d()
    say("joint arc of three oblique beams")
    s = dl.Solver(p)
    s.raytrace()
    s.run()
    got = s.dose().cpu().numpy()
    s.close()
    want = ref.run_joint_dlra(p)["dose"]
    err = rel(got, want)
    say(f"  rel-L2 dose error {err:.3e}")
    assert err <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["c1", "small3d_mixed"])
def test_graph_runs_match_eager_steps_bitwise(name):
    """Steps recorded and launched as HIP graphs (several graphs, with eager
    steps and synchronisations between them) give bitwise the doses and state
    of plain steps after every graph."""
    dl = _gpu()
    import torch
    if name == "c1":
        p = configs.c1(n_steps=40)
    else:
        p = configs.small_3d(n=8, r=6, precision="mixed", n_steps=24)
    say(f"graph runs {name}")
    plan = [("graph", 7), ("eager", 2), ("graph", 1), ("graph", 12), ("eager", 1)]
    n_total = sum(k for _, k in plan)
    assert n_total <= p.options.n_steps
    a = dl.BeamSolver(p, 0)
    a.raytrace()
    want = []
    for _, k in plan:
        a.run(k)
        want.append((a.dose().clone(), a.state()))
    a.close()
    b = dl.BeamSolver(p, 0)
    b.raytrace()
    for (how, k), (dose, state) in zip(plan, want):
        if how == "graph":
            b.run_graph(k)
        else:
            b.run(k)
        b.sync()
        got = b.dose()
        assert torch.equal(got, dose), how
        for x, y in zip(b.state(), state):
            if isinstance(x, int):
                assert x == y
            else:
                assert np.array_equal(x, y)
    b.close()


@pytest.mark.gpu
def test_graph_run_needs_fixed_rank():
    dl = _gpu()
    p = configs.small_2d(mats="slab", rank_mode="adaptive", r=4, r_min=2, r_max=12)
    s = dl.BeamSolver(p, 0)
    s.raytrace()
    with pytest.raises(RuntimeError, match="fixed rank"):
        s.run_graph(2)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("batch", [2, 0])
def test_grouped_batch_solve_matches_one_by_one(batch):
    """Separate beams solved in groups through the batch scheduler (batch = 2,
    or as many as fit the free memory) add up to bitwise the one-by-one dose."""
    dl = _gpu()
    import torch
    p = configs.small_arc_2d(n_beams=3)
    say(f"grouped batch solve, batch={batch}")
    one = dl.solve(p, batch=1)
    grouped = dl.solve(p, batch=batch)
    assert torch.equal(one, grouped)
    assert dl.binding.batch_group_size(p) >= 1


def test_roof_probes_give_plausible_rates():
    # the achievable-throughput probes run and report positive rates below
    # twice the vendor peaks (FP32 157.3, FP64 78.6 TFLOP/s), and reject bad
    # arguments
    _gpu()
    from paper_2508_04484_amd import binding
    peaks = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "fp32_fma": 157.3, "fp64_fma": 78.6}
    for kind, peak in peaks.items():
        rate = binding.roof_probe(kind, 2000)
        say(f"  {kind}: {rate:.1f} TFLOP/s")
        assert 0.0 < rate < 2.0 * peak
    lib = binding.load()
    import ctypes as C
    out = C.c_double(0.0)
    assert lib.dlra_roof_probe(4, 10, C.byref(out)) == -1
    assert lib.dlra_roof_probe(0, 0, C.byref(out)) == -1
    assert lib.dlra_roof_probe(0, 10, None) == -1
