"""Seeded synthetic workloads.

The paper's phantoms come from CT Hounsfield units and Monte Carlo data that
are not available (Sec. 4); these stand-ins keep the paper's structure (water
boxes, heterogeneous slabs, mixture fractions per voxel, Gaussian pencil
beams with 1% energy spread, Sec. 4) at the sizes of the benchmark workloads:

  c1  2D water 64x64 cells of 1 mm, 70 MeV beam (sigma 3 mm) along +x,
      P_7 (64 moments), 100 energy steps, fixed rank 10, FP64
  c2  2D 200x200 cells of 0.5 mm, water with a 10 mm bone slab (1.85 g/cm^3)
      and a 20 mm lung slab (0.26 g/cm^3), boundary voxels 50/50 mixtures,
      150 MeV beam (sigma 4 mm), P_21 (484 moments), 300 steps, adaptive rank
      (relative tail 1e-4, r <= 40)
  c3  3D 128^3 cells of 1 mm, density from a seeded Gaussian random field
      (correlation length 8 mm) mapped to water/bone/air mixtures with
      densities 0.2..1.9, 150 MeV beam (sigma 5 mm), P_15 (256 moments),
      fixed rank 30, 250 steps, mixed precision
  c4  c3's phantom with 64 beams: energies U[70, 230] MeV, axial angles
      U[0, 2 pi), spot sigma U[3, 6] mm, adaptive ranks in [10, 50]
  c4_axis  c4 with the beam directions snapped to the nearest axial grid axis
  c5  c2's phantom with 9 beams of 100 + 10 b MeV at 40 b degrees aimed at the
      centre (adjoint workload)
  c2_elements, c3_elements  c2 / c3 with every voxel decomposed into the
      paper's twelve elements (12 base materials)
  two_beams  the paper's two-beam case on c1's grid: two perpendicular 70 MeV
      beams in water in one joint collided solve

Every random draw uses numpy's PCG64 with the stated seed.  Nothing here
implements any part of the transport method.
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
import math

import numpy as np
from scipy.special import ndtr

from . import materials as M
from .problem import Beam, Grid, Materials, Options, Problem


@functools.lru_cache(maxsize=16)
def _tables(names: tuple, n_leg: int):
    mats = [M.BASE_MATERIALS[n] for n in names]
    return M.build_tables(mats, n_leg)


def make_materials(names, w, pn_degree):
    e, S, T, G0, dG = _tables(tuple(names), pn_degree + 2)
    return Materials(tuple(names), np.ascontiguousarray(w, dtype=np.float64),
                     e.copy(), S.copy(), T.copy(), G0.copy(), dG.copy())


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------- phantoms

def water_box(grid: Grid, density=1.0):
    return np.full((1, grid.n), density, dtype=np.float64)


def slab_phantom(grid: Grid, slabs, background="water", bg_density=1.0):
    """Slabs along x: list of (name, density, x0, x1) in cm.  Each voxel's
    partial density is the volume-fraction-weighted density of what covers it."""
    names = [background] + [s[0] for s in slabs]
    uniq = list(dict.fromkeys(names))
    w = np.zeros((len(uniq), grid.nz, grid.ny, grid.nx))
    x_lo = np.arange(grid.nx) * grid.dx
    x_hi = x_lo + grid.dx
    covered = np.zeros(grid.nx)
    for name, rho, a, b in slabs:
        frac = np.clip(np.minimum(x_hi, b) - np.maximum(x_lo, a), 0.0, None) / grid.dx
        w[uniq.index(name)] += rho * frac[None, None, :]
        covered += frac
    w[uniq.index(background)] += bg_density * (1.0 - covered)[None, None, :]
    w[np.abs(w) < 1e-12] = 0.0
    return tuple(uniq), w.reshape(len(uniq), -1)


def gaussian_random_field(shape, spacing, corr_len, seed):
    """Periodic Gaussian random field with covariance exp(-d^2/(2 l^2)),
    normalised to zero mean and unit variance (FFT filter of white noise)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal(shape)
    ks = [2.0 * math.pi * np.fft.fftfreq(n, d=spacing) for n in shape]
    K2 = sum(np.meshgrid(*[k**2 for k in ks], indexing="ij"))
    filt = np.exp(-0.25 * K2 * corr_len**2)
    g = np.real(np.fft.ifftn(np.fft.fftn(white) * filt))
    g -= g.mean()
    g /= g.std()
    return g


def random_phantom(grid: Grid, seed=3, corr_len=0.8, rho_min=0.2, rho_max=1.9):
    """Water/bone/air mixtures: rho = rho_min + (rho_max - rho_min) Phi(g);
    rho <= 1 mixes air (0.0012) and water by volume, rho > 1 water and bone
    (rho_max)."""
    shape = (grid.nz, grid.ny, grid.nx)
    g = gaussian_random_field(shape, grid.dx, corr_len, seed)
    rho = rho_min + (rho_max - rho_min) * ndtr(g)
    rho = rho.ravel()
    rho_air, rho_w, rho_b = M.AIR.density, 1.0, rho_max
    w = np.zeros((3, grid.n))  # water, bone, air
    lo = rho <= 1.0
    fw = (rho[lo] - rho_air) / (rho_w - rho_air)
    w[0, lo] = fw * rho_w
    w[2, lo] = (1.0 - fw) * rho_air
    hi = ~lo
    fb = (rho[hi] - rho_w) / (rho_b - rho_w)
    w[0, hi] = (1.0 - fb) * rho_w
    w[1, hi] = fb * rho_b
    return ("water", "bone", "air"), w


# ---------------------------------------------------------------- configs

def beam_along_x(E0, spot_sigma, y0, z0=0.0, weight=1.0):
    return Beam(E0=E0, sigma_E=0.01 * E0, spot_sigma=spot_sigma, weight=weight,
                pos=(0.0, y0, z0), dir=(1.0, 0.0, 0.0))


def c1(**opt) -> Problem:
    grid = Grid(64, 64, 1, 0.1, 0.1, 0.1)
    o = Options(pn_degree=7, n_steps=100, rank_mode="fixed", r=10, precision="fp64").with_(**opt)
    mats = make_materials(("water",), water_box(grid), o.pn_degree)
    return Problem(grid, mats, [beam_along_x(70.0, 0.3, 3.2)], o, name="c1")


def c2(**opt) -> Problem:
    grid = Grid(200, 200, 1, 0.05, 0.05, 0.05)
    o = Options(pn_degree=21, n_steps=300, rank_mode="adaptive", r=40, r_min=2, r_max=40,
                trunc_tol=1e-4, precision="fp64").with_(**opt)
    names, w = slab_phantom(grid, [("bone", 1.85, 3.025, 4.025), ("lung", 0.26, 5.025, 7.025)])
    mats = make_materials(names, w, o.pn_degree)
    return Problem(grid, mats, [beam_along_x(150.0, 0.4, 5.0)], o, name="c2")


def c3(**opt) -> Problem:
    grid = Grid(128, 128, 128, 0.1, 0.1, 0.1)
    # mixed precision: drop and floor tolerances above the FP32 rounding level
    # (the FP64 defaults 1e-6 / 1e-7 would admit rounding noise as directions)
    o = Options(pn_degree=15, n_steps=250, rank_mode="fixed", r=30, r_max=30,
                precision="mixed", aug_tol=1e-4, floor_tol=1e-5).with_(**opt)
    names, w = random_phantom(grid, seed=3)
    mats = make_materials(names, w, o.pn_degree)
    return Problem(grid, mats, [beam_along_x(150.0, 0.5, 6.4, 6.4)], o, name="c3",
                   meta={"phantom_sha256": sha256(w)})


def aimed_beam(E0, spot, angle, center, radius):
    d = (math.cos(angle), math.sin(angle), 0.0)
    pos = (center[0] - radius * d[0], center[1] - radius * d[1], center[2])
    return Beam(E0=E0, sigma_E=0.01 * E0, spot_sigma=spot, pos=pos, dir=d)


def c4(n_beams=64, **opt) -> Problem:
    p = c3(**opt)
    rng = np.random.Generator(np.random.PCG64(4))
    E = rng.uniform(70.0, 230.0, n_beams)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_beams)
    spot = rng.uniform(0.3, 0.6, n_beams)
    c = (6.4, 6.4, 6.4)
    beams = [aimed_beam(E[b], spot[b], ang[b], c, 10.0) for b in range(n_beams)]
    o = p.options.with_(rank_mode="adaptive", r=10, r_min=10, r_max=50, trunc_tol=1e-4).with_(**opt)
    return Problem(p.grid, p.materials, beams, o, name="c4", meta=p.meta)


def c4_axis(n_beams=64, **opt) -> Problem:
    """c4 with every beam direction snapped to the nearest grid axis of the
    axial plane (+x, +y, -x, -y), entering at the centre of that face; the
    energies, spot sizes and rank options are c4's draws."""
    p = c4(n_beams=n_beams, **opt)
    rng = np.random.Generator(np.random.PCG64(4))
    rng.uniform(70.0, 230.0, n_beams)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_beams)
    c = (6.4, 6.4, 6.4)
    axes = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    beams = []
    for b, beam in enumerate(p.beams):
        ux, uy = axes[int(round(ang[b] / (math.pi / 2.0))) % 4]
        pos = (c[0] - 6.4 * ux, c[1] - 6.4 * uy, c[2])
        beams.append(Beam(E0=beam.E0, sigma_E=beam.sigma_E, spot_sigma=beam.spot_sigma,
                          pos=pos, dir=(ux, uy, 0.0)))
    return Problem(p.grid, p.materials, beams, p.options, name="c4_axis", meta=p.meta)


def c5(**opt) -> Problem:
    p = c2(**opt)
    c = (5.0, 5.0, 0.0)
    beams = [aimed_beam(100.0 + 10.0 * b, 0.4, math.radians(40.0 * b), c, 6.0) for b in range(9)]
    return Problem(p.grid, p.materials, beams, p.options, name="c5")


def to_elements(problem: Problem) -> Problem:
    """The same phantom decomposed into the paper's twelve elements (Sec. 2.1):
    every voxel's compound partial densities become elemental partial densities
    (mass fractions of the compounds), with per-element tables."""
    names, w = M.element_weights(problem.materials.names, problem.materials.w)
    mats = make_materials(names, w, problem.options.pn_degree)
    return Problem(problem.grid, mats, problem.beams, problem.options,
                   name=problem.name + "_elements", meta=dict(problem.meta))


def c2_elements(**opt) -> Problem:
    """c2's slab phantom with the twelve-element decomposition."""
    return to_elements(c2(**opt))


def c3_elements(**opt) -> Problem:
    """c3's random phantom with the twelve-element decomposition."""
    return to_elements(c3(**opt))


def two_beams(**opt) -> Problem:
    """The paper's two-beam case (Sec. 4.3) on c1's grid: 2D water 64 x 64 cells
    of 1 mm, two perpendicular 70 MeV beams (sigma 3 mm), one along +x through
    the centre row and one along +y through the centre column, in one joint
    collided solve (P_7, fixed rank 10, 100 energy steps, FP64)."""
    p = c1(**opt)
    L = p.grid.nx * p.grid.dx
    b2 = Beam(E0=70.0, sigma_E=0.7, spot_sigma=0.3, pos=(0.5 * L + 0.013, 0.0, 0.0),
              dir=(0.0, 1.0, 0.0))
    return Problem(p.grid, p.materials, [p.beams[0], b2], p.options, name="two_beams")


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c4_axis": c4_axis, "c5": c5,
           "c2_elements": c2_elements, "c3_elements": c3_elements, "two_beams": two_beams}


# ---------------------------------------------------------------- small cases

def small_2d(nx=16, ny=12, N=3, E0=30.0, n_steps=12, spot=0.15, mats="water", r=6,
             seed=None, dx=0.05, **opt) -> Problem:
    """Small 2D case for tests: either water, or (mats="slab") water/bone/lung
    slabs, or (mats="random") a seeded random water/bone/air field."""
    grid = Grid(nx, ny, 1, dx, dx, dx)
    o = Options(pn_degree=N, n_steps=n_steps, rank_mode="fixed", r=r, r_max=max(r, 2),
                precision="fp64").with_(**opt)
    if mats == "water":
        names, w = ("water",), water_box(grid)
    elif mats == "slab":
        L = nx * dx
        names, w = slab_phantom(grid, [("bone", 1.85, 0.30 * L, 0.45 * L),
                                       ("lung", 0.26, 0.60 * L, 0.80 * L)])
    elif mats == "random":
        names, w = random_phantom(grid, seed=0 if seed is None else seed, corr_len=4 * dx)
    else:
        raise ValueError(mats)
    m = make_materials(names, w, o.pn_degree)
    return Problem(grid, m, [beam_along_x(E0, spot, 0.5 * ny * dx + 0.013)], o, name="small_2d")


def small_joint_2d(nx=14, ny=14, N=3, n_steps=10, mats="slab", r=8, dx=0.05, E=(25.0, 20.0),
                   weights=(1.0, 0.7), **opt) -> Problem:
    """Small 2D case with two perpendicular beams (+x and +y) of different
    energies and weights, for joint-source tests."""
    p = small_2d(nx=nx, ny=ny, N=N, n_steps=n_steps, mats=mats, r=r, dx=dx, E0=E[0], **opt)
    b1 = dataclasses.replace(p.beams[0], weight=weights[0])
    b2 = Beam(E0=E[1], sigma_E=0.01 * E[1], spot_sigma=0.15, weight=weights[1],
              pos=(0.5 * nx * dx - 0.021, 0.0, 0.0), dir=(0.0, 1.0, 0.0))
    return Problem(p.grid, p.materials, [b1, b2], p.options, name="small_joint_2d")


def small_3d(n=8, N=3, E0=25.0, n_steps=8, spot=0.15, mats="random", r=6, dx=0.05,
             **opt) -> Problem:
    grid = Grid(n, n, n, dx, dx, dx)
    o = Options(pn_degree=N, n_steps=n_steps, rank_mode="fixed", r=r, r_max=max(r, 2),
                precision="fp64").with_(**opt)
    if mats == "water":
        names, w = ("water",), water_box(grid)
    else:
        names, w = random_phantom(grid, seed=1, corr_len=3 * dx)
    m = make_materials(names, w, o.pn_degree)
    c = 0.5 * n * dx
    return Problem(grid, m, [beam_along_x(E0, spot, c + 0.011, c - 0.007)], o, name="small_3d")


def small_oblique_2d(angle_deg=30.0, nx=16, ny=14, N=3, E0=25.0, n_steps=10, mats="slab", r=6,
                     dx=0.05, n_groups=32, **opt) -> Problem:
    """Small 2D case with one beam at an oblique angle in the plane, aimed at
    the grid centre from outside (one ray per target cell)."""
    p = small_2d(nx=nx, ny=ny, N=N, E0=E0, n_steps=n_steps, mats=mats, r=r, dx=dx,
                 n_groups=n_groups, **opt)
    c = (0.5 * nx * dx + 0.004, 0.5 * ny * dx - 0.006, 0.0)
    b = aimed_beam(E0, 0.15, math.radians(angle_deg), c, nx * dx)
    return Problem(p.grid, p.materials, [b], p.options, name="small_oblique_2d")


def small_oblique_3d(n=8, N=3, E0=25.0, n_steps=8, r=6, dx=0.05, n_groups=32,
                     direction=(0.8, 0.5, 0.33), **opt) -> Problem:
    """Small 3D random phantom with one beam along an oblique (non-planar)
    direction through the grid centre."""
    p = small_3d(n=n, N=N, E0=E0, n_steps=n_steps, r=r, dx=dx, n_groups=n_groups, **opt)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    c = np.full(3, 0.5 * n * dx) + np.array([0.003, -0.005, 0.002])
    pos = tuple(c - n * dx * d)
    b = Beam(E0=E0, sigma_E=0.01 * E0, spot_sigma=0.15, pos=pos, dir=tuple(d))
    return Problem(p.grid, p.materials, [b], p.options, name="small_oblique_3d")


def small_arc_2d(n_beams=3, nx=16, ny=16, N=3, n_steps=10, mats="slab", r=8, dx=0.05,
                 n_groups=32, **opt) -> Problem:
    """Small 2D case with several beams of different energies and weights aimed
    at the centre from angles spread over the plane (a reduced arc of the
    adjoint configuration's beams)."""
    p = small_2d(nx=nx, ny=ny, N=N, n_steps=n_steps, mats=mats, r=r, dx=dx, n_groups=n_groups,
                 **opt)
    c = (0.5 * nx * dx + 0.003, 0.5 * ny * dx - 0.002, 0.0)
    beams = []
    for b in range(n_beams):
        E = 22.0 + 3.0 * b
        bm = aimed_beam(E, 0.15, math.radians(40.0 * b + 5.0), c, nx * dx)
        beams.append(dataclasses.replace(bm, weight=1.0 - 0.2 * b))
    return Problem(p.grid, p.materials, beams, p.options, name="small_arc_2d")

