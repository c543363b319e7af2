"""Problem description shared by the solver binding and its checker.

A problem is: a structured grid (cells x-fastest, Sec. 3.3.2), per-voxel partial
densities of the base materials (Sec. 2.1, eq. mixXS), per-material energy
tables, pencil beams (Gaussian spot, Gaussian energy spread, Sec. 4) and the
method options (P_N degree, energy steps, rank control).  These containers hold
data only; none of the method's arithmetic lives here.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float   # cm
    dy: float
    dz: float

    @property
    def dim(self) -> int:
        return 2 if self.nz == 1 else 3

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def centers(self):
        """Cell-centre coordinates (n, 3), cm, cell index i + nx*(j + ny*k)."""
        x = (np.arange(self.nx) + 0.5) * self.dx
        y = (np.arange(self.ny) + 0.5) * self.dy
        z = (np.arange(self.nz) + 0.5) * self.dz if self.dim == 3 else np.zeros(1)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


@dataclass
class Materials:
    names: tuple
    w: np.ndarray        # (n_mat, n) partial densities, g/cm^3
    e: np.ndarray        # (n_e,) table energies, MeV, ascending
    S: np.ndarray        # (n_mat, n_e) mass stopping power, MeV cm^2/g
    T: np.ndarray        # (n_mat, n_e) mass straggling, MeV^2 cm^2/g
    G0: np.ndarray       # (n_mat, n_e) total cross section G_0, cm^2/g
    dG: np.ndarray       # (n_mat, n_e, n_leg) G_0 - G_l, cm^2/g (dG[..., 0] = 0)

    @property
    def n_mat(self) -> int:
        return self.w.shape[0]

    def density(self):
        return self.w.sum(axis=0)


@dataclass
class Beam:
    E0: float                      # mean energy, MeV
    sigma_E: float                 # energy spread, MeV
    spot_sigma: float              # lateral Gaussian sigma, cm
    weight: float = 1.0
    pos: tuple = (0.0, 0.0, 0.0)   # a point on the beam axis (cm)
    dir: tuple = (1.0, 0.0, 0.0)   # unit direction of flight


@dataclass
class Options:
    pn_degree: int = 7
    n_steps: int = 100
    rank_mode: str = "fixed"       # "fixed" | "adaptive"
    r: int = 10                    # fixed rank (and initial rank cap)
    r_min: int = 2
    r_max: int = 40
    precision: str = "fp64"        # "fp64" | "mixed"
    e_cut: float = 1.0             # MeV
    e_max_sigmas: float = 5.0      # E_max = E0 + e_max_sigmas * sigma_E
    trunc_tol: float = 1e-4        # relative L1 tail tolerance (adaptive)
    aug_tol: float = 1e-6          # basis-augmentation drop tolerance (relative)
    floor_tol: float = 1e-7        # singular-value floor for kept directions
    fill_tol: float = 1e-2         # acceptance threshold for filler directions
    nu_max: float = 0.0            # CFL number; 0 -> 0.45 (2D) / 0.35 (3D)
    n_sub_max: int = 0             # bound on RK4 substeps per energy step (0: none)
    ray_h_max: float = 0.01        # cm, ray-tracer step bound (Sec. 3.2)
    n_groups: int = 128            # DG energy groups of the ray tracer (Sec. 3.2)
    beam_cut_sigmas: float = 8.0   # rays are traced where d_perp <= cut * spot sigma
    collision: str = "boltzmann"   # "boltzmann" | "fokker_planck" (Sec. 2.1)
    egrid: str = "uniform"         # "uniform" | "proportional" | "cfl" | "user"
    egrid_points: tuple = ()       # n_steps + 1 descending energies (egrid = "user")

    def cfl(self, dim: int) -> float:
        if self.nu_max > 0:
            return self.nu_max
        return 0.45 if dim == 2 else 0.35

    def with_(self, **kw) -> "Options":
        return replace(self, **kw)


@dataclass
class Problem:
    grid: Grid
    materials: Materials
    beams: list
    options: Options
    name: str = "problem"
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return (self.options.pn_degree + 1) ** 2

    def with_options(self, **kw) -> "Problem":
        return replace(self, options=self.options.with_(**kw))

    def single_beam(self, b: int) -> "Problem":
        return replace(self, beams=[self.beams[b]])
