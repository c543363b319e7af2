"""Base materials and per-material energy tables (inputs to the transport solver).

The solver consumes, for every base material i and every table energy E_e:

  S[i, e]     mass stopping power                      MeV cm^2 / g
  T[i, e]     mass straggling coefficient              MeV^2 cm^2 / g
  G0[i, e]    total cross section G_0 = Sigma_t               cm^2 / g
  dG[i, e, l] G_0 - G_l, with G_l = 2*pi*int P_l(mu) Sigma_s dmu  cm^2 / g, l < n_leg

The Legendre moments are handed over as G_0 plus the differences G_0 - G_l:
the screened-Rutherford peak makes G_0 some 1e8 times larger than those
differences, and the transport-corrected operator of the method only ever uses
differences of moments (self-scattering G_l - G_0, in-scattering G_l - G_{N+1},
removal G_0 - G_{N+1}), so this form keeps every input at full precision.

and mixes them per voxel with partial densities w_i(x) (g/cm^3), following the
mixture rule of the paper (Sec. 2.1, eq. mixXS, Bragg additivity).  The paper
takes stopping powers from a Monte Carlo code and straggling / elastic
scattering from physics models (Sec. 2.1.1).  The Monte Carlo tables are not
available, so all three quantities here come from closed-form physics models:

* stopping power: the Bethe formula without shell or density corrections;
* straggling: the Bohr term with the Williams-type ionisation correction of
  Sec. 2.1.1 (the leading "1 +" of the Bohr term is restored);
* elastic scattering: the screened Rutherford cross section with the Moliere
  screening angle of Sec. 2.1.1 (eq. elasticXS), including the centre-of-mass
  to laboratory factor tau_lab.

These tables are inputs: the solver and its checker read the same arrays, so
the physics fidelity does not enter any parity comparison.  Nothing in this
module is part of the discretised method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# physical constants (CODATA 2018 values, MeV / cm units)
ME_C2 = 0.51099895000        # electron rest energy, MeV
MP_C2 = 938.27208816         # proton rest energy, MeV
ALPHA = 1.0 / 137.035999084  # fine-structure constant
HBAR_C = 197.3269804e-13     # MeV cm
N_AVOGADRO = 6.02214076e23   # 1/mol
K_BETHE = 0.307075           # 4 pi N_A r_e^2 m_e c^2, MeV cm^2 / mol

# The twelve elements of the paper's tissue model (Sec. 2.1): Z, A (g/mol),
# mean excitation energy I (eV).
ELEMENTS = {
    "H": (1, 1.008, 19.2),
    "C": (6, 12.011, 81.0),
    "N": (7, 14.007, 82.0),
    "O": (8, 15.999, 95.0),
    "Na": (11, 22.990, 149.0),
    "Mg": (12, 24.305, 156.0),
    "P": (15, 30.974, 173.0),
    "S": (16, 32.06, 180.0),
    "Cl": (17, 35.45, 174.0),
    "Ar": (18, 39.948, 188.0),
    "K": (19, 39.098, 190.0),
    "Ca": (20, 40.078, 191.0),
}


@dataclass(frozen=True)
class BaseMaterial:
    """A compound base material: elemental mass fractions, nominal density and
    compound mean excitation energy."""

    name: str
    density: float                 # g/cm^3 (nominal, informational)
    fractions: tuple               # ((element, mass fraction), ...)
    i_ev: float                    # compound mean excitation energy, eV

    def z_over_a(self) -> float:
        return sum(f * ELEMENTS[e][0] / ELEMENTS[e][1] for e, f in self.fractions)


# Compositions: ICRU-style compounds built from the paper's element set.
WATER = BaseMaterial("water", 1.0, (("H", 0.111894), ("O", 0.888106)), 75.0)
BONE = BaseMaterial(
    "bone", 1.85,
    (("H", 0.034), ("C", 0.155), ("N", 0.042), ("O", 0.435), ("Na", 0.001),
     ("Mg", 0.002), ("P", 0.103), ("S", 0.003), ("Ca", 0.225)),
    106.4,
)
LUNG = BaseMaterial(
    "lung", 0.26,
    (("H", 0.103), ("C", 0.105), ("N", 0.031), ("O", 0.749), ("Na", 0.002),
     ("P", 0.002), ("S", 0.003), ("Cl", 0.003), ("K", 0.002)),
    75.3,
)
AIR = BaseMaterial(
    "air", 0.0012,
    (("C", 0.000124), ("N", 0.755268), ("O", 0.231781), ("Ar", 0.012827)),
    85.7,
)
BASE_MATERIALS = {m.name: m for m in (WATER, BONE, LUNG, AIR)}

# The twelve elements themselves as base materials (the paper's decomposition,
# Sec. 2.1): mass fraction one, the element's own mean excitation energy.
ELEMENT_MATERIALS = {e: BaseMaterial(e, 0.0, ((e, 1.0),), v[2]) for e, v in ELEMENTS.items()}
BASE_MATERIALS.update(ELEMENT_MATERIALS)


def element_weights(names, w):
    """Partial densities of the twelve elements (12 x n, g/cm^3, in ELEMENTS
    order) of voxels given as partial densities w (n_mat x n) of the compound
    base materials `names`: w_e(x) = sum_c w_c(x) f_{c,e} with f the compound's
    elemental mass fractions."""
    els = list(ELEMENTS)
    out = np.zeros((len(els), np.asarray(w).shape[1]))
    for c, name in enumerate(names):
        for el, f in BASE_MATERIALS[name].fractions:
            out[els.index(el)] += f * np.asarray(w)[c]
    return tuple(els), out


def kinematics(E):
    """Proton kinetic energy E (MeV) -> (beta^2, gamma, p c in MeV)."""
    E = np.asarray(E, dtype=np.float64)
    gamma = 1.0 + E / MP_C2
    beta2 = 1.0 - 1.0 / gamma**2
    pc = np.sqrt(E * (E + 2.0 * MP_C2))
    return beta2, gamma, pc


def stopping_power(mat: BaseMaterial, E):
    """Bethe mass stopping power (MeV cm^2/g), no shell/density corrections."""
    beta2, gamma, _ = kinematics(E)
    ratio = ME_C2 / MP_C2
    bg2 = beta2 * gamma**2
    wmax = 2.0 * ME_C2 * bg2 / (1.0 + 2.0 * gamma * ratio + ratio**2)
    I = mat.i_ev * 1e-6
    L = 0.5 * np.log(2.0 * ME_C2 * bg2 * wmax / I**2) - beta2
    return K_BETHE * mat.z_over_a() / beta2 * L


def straggling(mat: BaseMaterial, E):
    """Bohr straggling with the ionisation correction, MeV^2 cm^2/g (floored at 0)."""
    beta2, _, _ = kinematics(E)
    I = mat.i_ev * 1e-6
    mv2 = ME_C2 * beta2
    corr = 1.0 + (4.0 * I / (3.0 * mv2)) * np.log(2.0 * mv2 / I)
    return np.maximum(K_BETHE * ME_C2 * mat.z_over_a() * corr, 0.0)


def _legendre_all(lmax, x):
    """P_0..P_lmax at points x (three-term recurrence); shape (lmax+1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    P = np.empty((lmax + 1,) + x.shape)
    P[0] = 1.0
    if lmax >= 1:
        P[1] = x
    for l in range(1, lmax):
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
    return P


def _gl_panels(a, b, n_panels, n_pts):
    xg, wg = np.polynomial.legendre.leggauss(n_pts)
    edges = np.linspace(a, b, n_panels + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    x = (0.5 * (lo + hi) + 0.5 * (hi - lo) * xg[None, :]).ravel()
    w = (0.5 * (hi - lo) * wg[None, :]).ravel()
    return x, w


def legendre_moments(mat: BaseMaterial, E, n_leg: int):
    """(G_0(E), G_0(E) - G_l(E)) with G_l = 2 pi int_{-1}^{1} P_l(mu) Sigma_s(E, mu) dmu,
    l < n_leg, cm^2/g.

    Screened Rutherford per element j (mass fraction f_j):
      Sigma_s = f_j N_A / A_j * Z_j^2 alpha^2 / (k^2 beta^2) * tau_lab(mu) / (1 - mu + chi_j/2)^2
    with k = p / hbar, chi_j = chi0_j^2 (1.13 + 3.76 a_j^2), chi0_j = 1.13 alpha Z^(1/3) m_e c / p,
    a_j = Z_j alpha / beta.  The peak at mu = 1 has width ~1e-10, so the integral
    is taken in t = ln(1 - mu + chi/2).  G_0 and the differences G_0 - G_l are
    integrated separately (the latter with integrand (1 - P_l) that vanishes at
    mu = 1) so that G_l keeps full relative accuracy in its differences.
    """
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    g0_out = np.zeros(E.size)
    dg_out = np.zeros((E.size, n_leg))
    beta2, _, pc = kinematics(E)
    k2 = (pc / HBAR_C) ** 2
    for ie in range(E.size):
        g0 = 0.0
        diff = np.zeros(n_leg)
        for el, frac in mat.fractions:
            Z, A, _ = ELEMENTS[el]
            ratio = 1.0 / A  # m_p / m_i with the nucleon-mass simplification of Sec. 2.1.1
            chi0 = 1.13 * ALPHA * Z ** (1.0 / 3.0) * ME_C2 / pc[ie]
            a2 = (Z * ALPHA) ** 2 / beta2[ie]
            c = 0.5 * chi0**2 * (1.13 + 3.76 * a2)
            pref = frac * N_AVOGADRO / A * Z**2 * ALPHA**2 / (k2[ie] * beta2[ie])
            t, wt = _gl_panels(math.log(c), math.log(2.0 + c), 240, 8)
            one_minus_mu = np.exp(t) - c
            mu = 1.0 - one_minus_mu
            tau = (1.0 + 2.0 * mu * ratio + ratio**2) ** 1.5 / (1.0 + mu * ratio)
            # int f(mu) / (1-mu+c)^2 dmu = int f(mu(t)) e^{-t} dt
            base = pref * tau * np.exp(-t) * wt
            g0 += 2.0 * math.pi * base.sum()
            P = _legendre_all(n_leg - 1, mu)
            # 1 - P_l(mu) evaluated stably near mu = 1 through the recurrence
            # values; the loss of digits is bounded by the t-substitution.
            diff += 2.0 * math.pi * ((1.0 - P) * base[None, :]).sum(axis=1)
        g0_out[ie] = g0
        dg_out[ie] = diff
    dg_out[:, 0] = 0.0
    return g0_out, dg_out


def energy_grid(e_min=0.5, e_max=300.0, n=320):
    """Log-spaced table energies (MeV)."""
    return np.geomspace(e_min, e_max, n)


def build_tables(materials, n_leg, e_tab=None):
    """Tables for a list of BaseMaterial: (e, S, T, G0, dG) with shapes
    (n_e,), (n_mat, n_e), (n_mat, n_e), (n_mat, n_e), (n_mat, n_e, n_leg)."""
    e = energy_grid() if e_tab is None else np.asarray(e_tab, dtype=np.float64)
    S = np.stack([stopping_power(m, e) for m in materials])
    T = np.stack([straggling(m, e) for m in materials])
    mom = [legendre_moments(m, e, n_leg) for m in materials]
    G0 = np.stack([g for g, _ in mom])
    dG = np.stack([d for _, d in mom])
    return e, S, T, G0, dG
