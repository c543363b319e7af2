"""Throughput of the DLRA proton-transport energy step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]

Default workload (c3): 128^3 voxels of 1 mm, Gaussian-random-field density
0.2..1.9 g/cm^3 mixed from water/bone/air, one 150 MeV pencil beam
(sigma 5 mm), P_15 (256 moments), fixed rank 30, 250 energy steps, FP32
stencil/projections with FP64 QR/SVD/truncation.  Inputs are generated
(seeded) and resident in HBM before timing.  A "step" is one energy step
(dlra_step: streaming BUG with RK4 substeps, collided scattering, uncollided
source, truncation, dose).  The uncollided ray tracer runs once before the
timed region and is reported separately.

Prints one JSON line (value = energy-steps/s over the K timed steps), with a
roofline entry for the dominant kernel (the K-step stencil stage, timed live
with HIP events on the library's stream) and the CPU reference timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DLRA energy-steps/s at 128³ r=30; beams/s batched vs plain; adjoint/fwd"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}   # dense FP32 / FP64 matrix peaks
KSTAGE_SOURCE = os.path.join(ROOT, "paper_2508_04484_amd", "csrc", "kernels_tall.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kstage_traffic_c3.json")   # per-config name


def source_sha():
    import hashlib
    with open(KSTAGE_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _counter_rows(path):
    """Rows of a rocprofv3 counter_collection.csv (a file or a directory holding one)."""
    import csv
    import glob
    if os.path.isdir(path):
        hits = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
        if not hits:
            raise SystemExit(f"no counter_collection.csv under {path}")
        path = hits[0]
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_counters(fetch_path, write_path, probe_mib, config, out_path):
    """HBM bytes per K-stage launch from a FETCH_SIZE and a WRITE_SIZE pass
    (KiB per dispatch), each scaled so that the largest copy kernel of the run
    (the known-size probe copy of probe_mib MiB) reads and writes exactly its
    size; writes the summary that measured_traffic() reads."""
    import statistics

    def per_kernel(rows, ctr):
        by = {}
        for r in rows:
            if r.get("Counter_Name") == ctr:
                by.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return by

    probe = probe_mib * 1024 * 1024
    out = {"config": config, "source_sha256": source_sha(), "probe_bytes": probe}
    total = 0.0
    for ctr, path in (("FETCH_SIZE", fetch_path), ("WRITE_SIZE", write_path)):
        by = per_kernel(_counter_rows(path), ctr)
        # the benchmarked stage kernel: the K-stage instance with the most dispatches
        stage = sorted((v for k, v in by.items() if "k_kstage" in k), key=len, reverse=True)
        copies = [max(v) for k, v in by.items() if "copyBuffer" in k]
        if not stage or not copies:
            raise SystemExit(f"{ctr}: stage kernel or probe copy missing in {path}")
        kib = statistics.mean(stage[0])
        scale = probe / (max(copies) * 1024.0)
        out[ctr] = {"stage_kib_per_dispatch": kib, "dispatches": len(stage[0]),
                    "probe_kib": max(copies), "scale": scale,
                    "stage_bytes_per_launch": kib * 1024.0 * scale}
        total += kib * 1024.0 * scale
    out["bytes_per_launch"] = total
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def summarize_sq(path, out_path):
    """Per-launch SQ counters of the K-step stage from one rocprofv3 --pmc pass
    (counter_collection.csv): matrix-core busy share of the busy CU cycles and
    instruction counts per launch; writes a short text summary."""
    import statistics
    rows = _counter_rows(path)
    # the benchmarked stage kernel: the K-stage instance with the most dispatches
    names = {}
    for r in rows:
        n = r.get("Kernel_Name", "")
        if "k_kstage" in n:
            names[n] = names.get(n, 0) + 1
    stage = max(names, key=names.get) if names else None
    by = {}
    for r in rows:
        if r.get("Kernel_Name", "") == stage:
            by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not by:
        raise SystemExit(f"no K-stage rows in {path}")
    mean = {k: statistics.mean(v) for k, v in by.items()}
    lines = ["counter                          mean per launch   launches"]
    for k in sorted(mean):
        lines.append(f"{k:32s} {mean[k]:16.4g} {len(by[k]):10d}")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and "GRBM_GUI_ACTIVE" in mean:
        # matrix-core busy cycles summed over the 256 CUs x 4 SIMDs, against
        # the kernel's active cycles
        lines.append(f"matrix cores busy / (GPU active cycles x 1024 SIMDs): "
                     f"{mean['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024.0 * mean['GRBM_GUI_ACTIVE']):.3f}")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and "SQ_BUSY_CU_CYCLES" in mean:
        lines.append(f"matrix cores busy / (4 x CU busy cycles): "
                     f"{mean['SQ_VALU_MFMA_BUSY_CYCLES'] / (4.0 * mean['SQ_BUSY_CU_CYCLES']):.3f}")
    if "SQ_INSTS_MFMA" in mean and "SQ_INSTS_VALU" in mean:
        lines.append(f"VALU (non-MFMA) per MFMA instruction: "
                     f"{(mean['SQ_INSTS_VALU'] - mean['SQ_INSTS_MFMA']) / mean['SQ_INSTS_MFMA']:.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def measured_traffic(config):
    """HBM bytes per K-stage launch from the committed counter summary, or None
    when it is missing, for another workload, or older than the kernel source."""
    try:
        with open(TRAFFIC_FILE.replace("_c3", f"_{config}")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("config") != config or t.get("source_sha256") != source_sha():
        return None
    return t.get("bytes_per_launch")


def kstage_algorithmic(problem):
    """(flops, bytes, flops with the differences) of one K-step RK4 stage over
    all cells.  Flops: the contraction of the 2*dim one-sided difference
    vectors with the r x r couplings, 2 ndk r^2 per cell (12 n r^2 per stage
    in 3D, a quarter of the 48 n r^2 per substep of the cost model); the
    differences (4 ndk r) and the stage combine (2 r) are given separately.
    Bytes: read the stage input, K0 and s, write the stage output."""
    g, o = problem.grid, problem.options
    ndk = 2 * g.dim
    r = o.r if o.rank_mode == "fixed" else o.r_max
    b = 8 if o.precision == "fp64" else 4
    flops = g.n * (2 * ndk * r * r)
    flops_all = g.n * (2 * ndk * r * r + 4 * ndk * r + 2 * r)
    nbytes = g.n * (3 * r + 1) * b
    return flops, nbytes, flops_all


# Algorithmic work of the ray tracer per energy group: one Crank-Nicolson
# substep forms (M + h/2 A) c (three 3x3 blocks, 54 flops) and solves the
# block-tridiagonal system with a stored factorisation (forward 39, backward
# 21 flops): 114 flops; one factorisation mixes the three blocks of n_mat
# materials (54 n_mat flops) and forms L E, the 3x3 inverse and Dinv U
# (150 flops).
RAY_FLOPS_PER_SUBSTEP_GROUP = 114
RAY_WAVE_GROUPS = 128   # up to this many groups one wave marches a ray (no scratch)


def ray_factor_flops_per_group(n_mat):
    return 150 + 54 * n_mat


def raytrace_roofline(problem, work, kernel_ms):
    """FP64-ALU roofline of the ray tracer from its work counts and duration,
    with the bytes it must write (uncollided tables and D_u)."""
    substeps, factors, rays = work
    G = problem.options.n_groups
    flops = G * (substeps * RAY_FLOPS_PER_SUBSTEP_GROUP
                 + factors * ray_factor_flops_per_group(problem.materials.n_mat))
    b = 8 if problem.options.precision == "fp64" else 4
    out_cells = problem.grid.n   # upper bound: every cell gets a table
    nbytes = out_cells * (problem.options.n_steps * b + 8)
    t = kernel_ms / 1000.0
    achieved = flops / t / 1e12
    wave = G <= RAY_WAVE_GROUPS
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": 78.6, "unit": "TFLOP/s",
           "frac": round(achieved / 78.6, 4),
           "kernel": "k_raytrace_wave" if wave else "k_raytrace",
           "ms": round(kernel_ms, 3), "rays": rays, "cn_substeps": substeps,
           "factorizations": factors, "algorithmic_flops": flops,
           "output_bytes_upper": nbytes, "output_gbs": round(nbytes / t / 1e9, 1),
           "note": "per group: 114 flops per CN substep, 150 + 54 n_mat per factorisation "
                   "(sequential block LU; the wave kernel's cyclic reduction does more)"}
    if not wave:
        out["scratch_gbs_model"] = round(substeps * G * 42 * 8 / t / 1e9, 1)
    return out


def cpu_baseline(problem, budget_planes=32, window=None):
    """Time one reference (CPU, FP64) step on a z-slab of the phantom from a
    seeded random rank-r state at the step whose substep count is closest to
    the run's mean, and scale to the whole phantom."""
    import dataclasses

    import numpy as np

    from oracle import coeffs, dlra, solver
    from workloads.problem import Grid

    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    g = problem.grid
    o = problem.options
    window = list(window) if window is not None else None
    nzs = min(budget_planes, g.nz)
    z0 = (g.nz - nzs) // 2
    sub = Grid(g.nx, g.ny, nzs, g.dx, g.dy, g.dz)
    plane = g.nx * g.ny
    w = problem.materials.w[:, z0 * plane:(z0 + nzs) * plane].copy()
    mats = dataclasses.replace(problem.materials, w=w)
    beam = dataclasses.replace(problem.beams[0], pos=(0.0, problem.beams[0].pos[1],
                                                      0.5 * nzs * g.dz))
    p = dataclasses.replace(problem, grid=sub, materials=mats, beams=[beam],
                            options=o.with_(precision="fp64"))
    nsub = [coeffs.step_coeffs(problem, problem.beams[0], k).n_sub for k in range(o.n_steps)]
    if window is not None:   # the GPU's timed steps: scale to their substeps
        nsub = [nsub[k] for k in window]
    mean_nsub = sum(nsub) / len(nsub)
    k = min(range(o.n_steps), key=lambda j: abs(nsub[j] - mean_nsub))
    rng = np.random.default_rng(7)
    r = o.r
    U, _ = np.linalg.qr(rng.standard_normal((sub.n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((p.m, r)))
    S = np.diag(np.logspace(0, -6, r))
    st = dlra.State(U, S, V, np.zeros(sub.n), k)
    c = coeffs.step_coeffs(p, beam, k)
    x = (np.arange(sub.n) % g.nx + 0.5) * g.dx
    psi = np.exp(-x)                                      # synthetic uncollided source
    Apm = solver.streaming_split(p)
    t0 = time.perf_counter()
    dlra.step(st, c, Apm, p, psi)
    dt = time.perf_counter() - t0
    scale = (g.n / sub.n) * (mean_nsub / c.n_sub)
    return {
        "value": 1.0 / (dt * scale), "unit": "energy-steps/s", "cores": int(threads),
        "kind": "oracle",
        "sample": (f"one FP64 reference step (k={k}, n_sub={c.n_sub}) on a "
                   f"{g.nx}x{g.ny}x{nzs} slab of the phantom from a seeded random rank-{r} "
                   f"state with a synthetic source, {dt:.2f} s, scaled by cells "
                   f"x{g.n / sub.n:.0f} and substeps x{mean_nsub / c.n_sub:.3f} "
                   f"(mean n_sub {mean_nsub:.2f} of the GPU's timed steps)"),
    }


def cpu_baseline_2d(problem, window, budget_s=15.0):
    """The FP64 reference on the whole 2D problem from the first energy step,
    as many steps as fit in about budget_s seconds, scaled to the substeps of
    the GPU's timed steps."""
    import numpy as np

    from oracle import coeffs, dlra, solver
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    o = problem.options
    beam = problem.beams[0]
    edges = coeffs.energy_edges(problem, [beam])
    t0 = time.perf_counter()
    psibar, Du = solver.uncollided(problem, beam, edges=edges)
    t_ray = time.perf_counter() - t0
    Apm = solver.streaming_split(problem)
    st = dlra.initial_state(problem, coeffs.step_coeffs(problem, beam, 0, edges).g)
    nsub, k, t_steps = [], 0, 0.0
    while k < o.n_steps and (k == 0 or t_steps < budget_s):
        c = coeffs.step_coeffs(problem, beam, k, edges)
        t0 = time.perf_counter()
        st = dlra.step(st, c, Apm, problem, psibar[k])
        t_steps += time.perf_counter() - t0
        nsub.append(c.n_sub)
        k += 1
    gpu_nsub = [coeffs.step_coeffs(problem, beam, j, edges).n_sub for j in window]
    scale = (sum(gpu_nsub) / len(gpu_nsub)) / (sum(nsub) / len(nsub))
    return {"value": k / t_steps / scale, "unit": "energy-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"FP64 reference steps 0..{k - 1} of the whole problem ({t_steps:.2f} s, "
                       f"mean n_sub {sum(nsub) / len(nsub):.2f}), scaled to the mean n_sub of "
                       f"the GPU's timed steps (x{scale:.3f}); its ray tracer took {t_ray:.2f} s")}


def bench_plan(problem, args):
    """c5's nine oblique beams on the slab phantom: the plan dose solved as
    separate beams through the batch scheduler, and as one joint collided
    solve (Sec. 4.3), each timed with its ray traces; then the plan objective
    and its exact gradient over the beam weights on the separate doses."""
    import numpy as np
    import torch

    import paper_2508_04484_amd as dl
    from workloads.plan import centre_target
    B = len(problem.beams)
    o = problem.options
    g = problem.grid
    # warm-up
    s = dl.BeamSolver(problem, 0)
    s.raytrace()
    s.step()
    s.sync()
    s.close()
    torch.cuda.synchronize()
    solvers = [dl.Solver(problem, [b], stream=torch.cuda.Stream()) for b in range(B)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dl.run_batch(solvers)
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    print(f"separate beams (batched): {t_sep:.2f} s", file=sys.stderr, flush=True)
    total = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    for sv in solvers:
        sv.dose(dl.binding.DOSE_UNCOLLIDED | dl.binding.DOSE_COLLIDED | dl.binding.DOSE_ACCUMULATE,
                 out=total)
    doses = torch.stack([sv.dose() for sv in solvers]).contiguous()
    for sv in solvers:
        sv.close()
    j = dl.Solver(problem)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    j.raytrace()
    j.run()
    torch.cuda.synchronize()
    t_joint = time.perf_counter() - t0
    joint = j.dose()
    j.close()
    print(f"joint solve: {t_joint:.2f} s", file=sys.stderr, flush=True)
    target = torch.from_numpy(centre_target(g, 1.0)).cuda()
    tmask = target.bool()
    dhat = float(total[tmask].mean()) if bool(tmask.any()) else 1.0
    w = np.array([b.weight for b in problem.beams])
    dl.binding.plan_objective(doses, w, target, dhat, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        J, grad = dl.binding.plan_objective(doses, w, target, dhat, 0.1)
    t_grad = (time.perf_counter() - t0) / 20
    diff = float(torch.linalg.norm(joint - total) / torch.linalg.norm(total))
    out = {
        "metric": "plan of 9 beams: separate (batched) vs joint solve",
        "value": round(B / t_sep, 5), "unit": "beams/s", "n_gpus": 1, "steps": o.n_steps,
        "warmup": 1, "ms_per_step": round(1000.0 * t_sep / o.n_steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if o.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": (f"{problem.name}: {g.nx}x{g.ny} cells of {g.dx * 10:g} mm, "
                                f"{B} oblique beams {problem.beams[0].E0:.0f}.."
                                f"{problem.beams[-1].E0:.0f} MeV every 40 deg, P_{o.pn_degree}, "
                                f"adaptive rank <= {o.r_max}, {o.n_steps} steps, {o.precision}")},
        "separate_s": round(t_sep, 3), "joint_s": round(t_joint, 3),
        "joint_over_separate_time": round(t_joint / t_sep, 4),
        "joint_vs_separate_rel_l2_dose": diff,
        "weight_gradient": {"ms": round(1000.0 * t_grad, 4), "J": J,
                            "dJ_dw": [round(float(x), 6) for x in grad]},
    }
    print(json.dumps(out), flush=True)


def bench_batch(problem, args):
    """beams/s of B beams of a treatment plan: one after another through the
    single-beam path (plain) and all together through the batch scheduler
    (each beam on its own stream, one host thread per beam).  Per beam: ray
    trace + all energy steps; inputs resident before timing; doses checked
    bitwise equal between the two runs."""
    import numpy as np
    import torch

    import paper_2508_04484_amd as dl
    B = max(1, min(args.beams, len(problem.beams)))
    idx = list(range(B))
    # warm-up (code objects, allocator): one beam, a few steps
    s = dl.BeamSolver(problem, 0)
    s.raytrace()
    for _ in range(min(3, problem.options.n_steps)):
        s.step()
    s.sync()
    s.close()
    del s
    torch.cuda.synchronize()
    plain_dose = []
    t_plain = 0.0
    for b in idx:
        s = dl.BeamSolver(problem, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.raytrace()
        s.run()
        torch.cuda.synchronize()
        dt_b = time.perf_counter() - t0
        t_plain += dt_b
        print(f"plain beam {b}: {problem.beams[b].E0:.1f} MeV, {dt_b:.2f} s", file=sys.stderr,
              flush=True)
        plain_dose.append(s.dose().cpu())
        s.close()
        del s
        torch.cuda.empty_cache()
    solvers = dl.batch_solvers(problem, idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_steps = problem.options.n_steps
    for k0 in range(0, n_steps, 50):   # chunks of 50 energy steps (progress lines)
        dl.run_batch(solvers, n_steps=min(50, n_steps - k0))
        print(f"batched: steps {k0}..{min(k0 + 50, n_steps) - 1} done, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"batched: {B} beams, {t_batch:.2f} s", file=sys.stderr, flush=True)
    same = all(torch.equal(s.dose().cpu(), plain_dose[b]) for b, s in enumerate(solvers))
    # plan objective over the beam weights and its exact gradient (the adjoint
    # of the linear dose map) on the batched doses: target = the central 2 cm
    # cube, prescription = mean target dose at unit weights, lam = 0.1
    from workloads.plan import centre_target
    doses = torch.stack([s.dose() for s in solvers]).contiguous()
    target = torch.from_numpy(centre_target(problem.grid, 1.0)).cuda()
    tmask = target.bool()
    dhat = float(doses.sum(0)[tmask].mean()) if bool(tmask.any()) else 1.0
    w = np.ones(B)
    dl.binding.plan_objective(doses, w, target, dhat, 0.1)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_rep = 20
    for _ in range(n_rep):
        J, grad = dl.binding.plan_objective(doses, w, target, dhat, 0.1)
    t_grad = (time.perf_counter() - t0) / n_rep
    for s in solvers:
        s.close()
    o = problem.options
    g = problem.grid
    out = {
        "metric": "beams/s batched vs plain",
        "value": round(B / t_batch, 5),
        "unit": "beams/s",
        "n_gpus": 1,
        "steps": o.n_steps,
        "warmup": 1,
        "ms_per_step": round(1000.0 * t_batch / o.n_steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if o.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{problem.name}: {B} of the plan's beams on {g.nx}x{g.ny}x{g.nz} "
                                f"voxels of {g.dx * 10:g} mm, P_{o.pn_degree}, adaptive rank "
                                f"[{o.r_min}, {o.r_max}], {o.n_steps} energy steps per beam, "
                                f"{o.precision}"),
                   "beams": B,
                   "energies_MeV": [round(problem.beams[b].E0, 1) for b in idx]},
        "plain_beams_per_s": round(B / t_plain, 5),
        "batched_over_plain": round(t_plain / t_batch, 4),
        "plain_s": round(t_plain, 3), "batched_s": round(t_batch, 3),
        "doses_bitwise_equal": bool(same),
        "weight_gradient": {"ms": round(1000.0 * t_grad, 4),
                            "over_batched_forward": t_grad / t_batch,
                            "J": J, "dJ_dw": [round(float(x), 6) for x in grad],
                            "note": "exact gradient over beam weights only; the voxel-density "
                                    "adjoint (reverse sweep) is not built"},
    }
    print(json.dumps(out), flush=True)


def fp64_check(problem, K, dose_mixed):
    """Relative L2 difference of the deposited energy after K steps between the
    benchmarked mixed-precision run and the same run through the library's
    FP64 path (which matches the FP64 reference to 1e-10 on the test cases)."""
    import numpy as np

    import paper_2508_04484_amd as dl
    p64 = problem.with_options(precision="fp64")
    s = dl.BeamSolver(p64, 0)
    s.raytrace()
    t0 = time.perf_counter()
    s.run(K)
    t = time.perf_counter() - t0
    d64 = s.dose().cpu().numpy()
    s.close()
    return {"rel_l2_dose": float(np.linalg.norm(dose_mixed - d64) / np.linalg.norm(d64)),
            "steps": K, "fp64_run_s": round(t, 3),
            "note": "mixed (FP32 storage/stencil/projections) against the library's FP64 path"}


def achievable_roofs():
    """Achievable roofs of this GPU, quoted beside the vendor peaks the
    roofline fractions use: the library's throughput probes (dlra_roof_probe:
    independent MFMA or FMA chains over every CU) and a 512 MiB
    device-to-device copy (bytes read + written over the best of three).  A
    failure is reported in place of the numbers."""
    import torch

    import paper_2508_04484_amd as dl
    try:
        res = {}
        for kind, iters in (("fp32_mfma", 40000), ("fp64_mfma", 20000), ("fp32_fma", 200000),
                            ("fp64_fma", 200000)):
            res[f"{kind}_tflops"] = round(dl.binding.roof_probe(kind, iters), 2)
        a = torch.ones(512 << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        res["copy_tbs"] = round(2.0 * a.numel() * 4 / (best * 1e-3) / 1e12, 3)
        del a, b
        res["vendor_peaks"] = {"fp32_tflops": 157.3, "fp64_tflops": 78.6, "hbm_tbs": 8.0}
        return res
    except Exception as e:   # reported, not fatal: the line's other numbers stand
        return {"error": str(e)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=250)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c4_axis", "c5"])
    ap.add_argument("--beams", type=int, default=8,
                    help="c4, c4_axis: number of the plan's beams timed plain and batched")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the second timing of the steps as one HIP graph (fixed rank)")
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the FP64 run of the timed steps that states the relative L2 "
                         "dose difference of a mixed-precision run (done by default)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the K-stage HBM-traffic summary from two rocprofv3 --pmc "
                         "passes (FETCH_SIZE, WRITE_SIZE) of this script run with "
                         "--copy-probe-mib, then exit")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("PMC_CSV", "OUT_TXT"),
                    help="write the K-stage SQ-counter summary of one rocprofv3 --pmc pass, "
                         "then exit")
    args = ap.parse_args()
    if args.summarize_sq:
        summarize_sq(*args.summarize_sq)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, max(args.copy_probe_mib, 1),
                           args.config, TRAFFIC_FILE.replace("_c3", f"_{args.config}"))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2508_04484_amd as dl
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    problem = configs.CONFIGS[args.config]()
    o = problem.options
    if args.config in ("c4", "c4_axis"):
        return bench_batch(problem, args)
    if args.config == "c5":
        return bench_plan(problem, args)
    K = min(args.steps, o.n_steps)

    # warm-up: a separate solver runs W steps (code objects, allocator,
    # caches); every phase of its steps is timed, for the phase breakdown
    # (the events themselves add a few microseconds per phase)
    warm_prof, warm_steps = None, 0
    if args.warmup > 0:
        s = dl.BeamSolver(problem, 0)
        s.raytrace()
        s.sync()
        s.profile(True)
        warm_steps = min(args.warmup, o.n_steps)
        for _ in range(warm_steps):
            s.step()
        s.sync()
        warm_prof = s.profile_read()
        s.profile(False)
        s.close()
        del s
        torch.cuda.synchronize()

    # the timed solver records only the light events: the step, the ray
    # tracer and one pair around each step's K-step RK4 loop
    s = dl.BeamSolver(problem, 0)
    s.profile(True, light=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.raytrace()
    s.sync()
    t_ray = time.perf_counter() - t0
    prof_ray = s.profile_read()["raytrace"]
    ray_work = s.raytrace_work()
    s.profile(True, light=True)   # reset counters for the timed region
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(K):
        s.step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    nsub = [s.substeps(k) for k in range(K)]
    check64 = o.precision == "mixed" and not args.no_fp64_check
    s_dose = s.dose().cpu().numpy() if check64 else None
    eager_dose = s.dose() if (o.rank_mode == "fixed" and not args.no_graph) else None
    s.close()

    # the same K steps recorded and launched as one HIP graph (fixed rank):
    # recording, instantiation and launch all inside the timed region
    graph = None
    if eager_dose is not None:
        s = dl.BeamSolver(problem, 0)
        s.raytrace()
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run_graph(K)
        s.sync()
        wall_g = time.perf_counter() - t0
        graph = {"value": round(K / wall_g, 4), "ms_per_step": round(1000.0 * wall_g / K, 3),
                 "speedup_vs_eager": round(wall / wall_g, 4),
                 "dose_bitwise_equal": bool(torch.equal(s.dose(), eager_dose)),
                 "note": "dlra_run_graph: the K steps recorded once (both streams) and "
                         "launched as one graph; recording and instantiation timed"}
        s.close()
        del eager_dose

    ms_step = 1000.0 * wall / K
    flops, nbytes, flops_all = kstage_algorithmic(problem)
    ks_ms, ks_n = prof["kstage"]
    avg = ks_ms / max(ks_n, 1) / 1000.0
    achieved_flops = flops / avg / 1e12
    achieved_gbs = nbytes / avg / 1e9
    # the stage contraction runs on the matrix cores (FP32 MFMA in mixed mode)
    peak = MFMA_PEAK_TFLOPS[o.precision]
    frac_mfma = achieved_flops / peak
    frac_hbm = achieved_gbs / HBM_PEAK_GBS
    traffic = measured_traffic(args.config)
    if frac_mfma >= frac_hbm:
        roof = {"bound": "mfma", "achieved": round(achieved_flops, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(frac_mfma, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(frac_hbm, 4), "traffic": traffic}
    roof.update({"kernel": "K-step RK4 stage (k_kstage_*)", "avg_launch_ms": round(avg * 1e3, 4),
                 "launches": ks_n, "algorithmic_flops_per_launch": flops,
                 "algorithmic_bytes_per_launch": nbytes,
                 "hbm_frac": round(frac_hbm, 4), "mfma_frac": round(frac_mfma, 4),
                 "frac_incl_differences": round(flops_all / avg / 1e12 / peak, 4)})
    g = problem.grid
    out = {
        "metric": METRIC,
        "value": round(K / wall, 4),
        "unit": "energy-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if o.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{problem.name}: {g.nx}x{g.ny}x{g.nz} voxels of {g.dx * 10:g} mm, "
                         f"{problem.beams[0].E0:g} MeV pencil beam, P_{o.pn_degree} "
                         f"({problem.m} moments), rank {o.r} ({o.rank_mode}), "
                         f"{o.n_steps} energy steps, {o.precision}"),
            "cells": g.n, "moments": problem.m, "rank": o.r, "energy_steps_total": o.n_steps,
            "timed_steps": f"0..{K - 1}", "mean_rk4_substeps": round(sum(nsub) / len(nsub), 3),
        },
        "rk4_substeps_per_s": round(sum(nsub) / wall, 2),
        "graph": graph,
        "event_ms_per_step": round(ev0.elapsed_time(ev1) / K, 3),
        "raytrace_ms": round(1000.0 * t_ray, 2),
        "raytrace_kernel_ms": round(prof_ray[0], 2),
        "phase_ms_per_step": None if warm_prof is None else {
            k: round(v[0] / warm_steps, 3) for k, v in warm_prof.items()
            if k not in ("raytrace",) and v[1] > 0},
        "phase_steps": (f"0..{warm_steps - 1} of the warm-up solver, every phase timed"
                        if warm_prof is not None else None),
        "kstage_timing": "one event pair per step around its RK4 loop (launch gaps included)",
        "roofline": roof,
        "raytrace_roofline": raytrace_roofline(problem, ray_work, prof_ray[0]),
    }
    if check64:
        out["mixed_vs_fp64"] = fp64_check(problem, K, s_dose)
    if not args.no_cpu_baseline and args.config == "c3":
        out["cpu_baseline"] = cpu_baseline(problem, window=range(K))
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_2d(problem, window=range(K))
    out["achievable"] = achievable_roofs()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
