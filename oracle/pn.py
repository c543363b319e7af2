"""Angular P_N algebra (Sec. 3.3.1 and Sec. 3.3.2).

Real spherical harmonics m_l^k up to degree N in the paper's ordering
p = l^2 + l + k (0-based), m = (N+1)^2 moments.  With the associated Legendre
functions carrying the Condon-Shortley phase, the paper's definition reduces to
  m_l^0 = N_l^0 P_l(mu),
  m_l^k = sqrt(2) N_l^k Pbar_l^k(mu) cos(k phi)      (k > 0),
  m_l^k = sqrt(2) N_l^|k| Pbar_l^|k|(mu) sin(|k| phi) (k < 0),
with N_l^k = sqrt((2l+1)/(4 pi) (l-k)!/(l+k)!) and Pbar without that phase.
Directions: Omega = (sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi, mu).

A_d = int m m^T Omega_d dOmega (Sec. 3.3.1), evaluated with a product rule
(Gauss-Legendre in mu, trapezoid in phi) that is exact for the polynomial
integrand; A_d = V_d Lambda_d V_d^T and A_d^{+/-} = V_d Lambda_d^{+/-} V_d^T with
Lambda^+ = max(0, lambda), Lambda^- = min(0, lambda) (Sec. 3.3.2).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import lpmv


def n_moments(N: int) -> int:
    return (N + 1) ** 2


def degree_order(N: int):
    """(l[p], k[p]) for p = l^2 + l + k."""
    ls, ks = [], []
    for l in range(N + 1):
        for k in range(-l, l + 1):
            ls.append(l)
            ks.append(k)
    return np.array(ls), np.array(ks)


def real_sh(N: int, mu, phi):
    """Real spherical harmonics at directions (mu, phi): shape (npts, m)."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    out = np.empty((mu.size, n_moments(N)))
    for l in range(N + 1):
        for k in range(-l, l + 1):
            a = abs(k)
            norm = math.sqrt((2 * l + 1) / (4.0 * math.pi)
                             * math.factorial(l - a) / math.factorial(l + a))
            pbar = (-1.0) ** a * lpmv(a, l, mu)
            if k == 0:
                v = norm * pbar
            elif k > 0:
                v = math.sqrt(2.0) * norm * pbar * np.cos(k * phi)
            else:
                v = math.sqrt(2.0) * norm * pbar * np.sin(a * phi)
            out[:, l * l + l + k] = v
    return out


def direction_to_angles(omega):
    """Unit vector -> (mu, phi)."""
    o = np.asarray(omega, dtype=np.float64)
    o = o / np.linalg.norm(o)
    mu = np.clip(o[2], -1.0, 1.0)
    phi = math.atan2(o[1], o[0])
    return mu, phi


def beam_moments(N: int, omega):
    """T_M = m(Omega_in) (Sec. 3.3.1)."""
    mu, phi = direction_to_angles(omega)
    return real_sh(N, mu, phi)[0]


def sphere_rule(N: int, extra: int = 0):
    """Product quadrature exact for polynomials of degree <= 2N+1+extra."""
    nmu = N + 2 + extra
    nphi = 2 * N + 4 + 2 * extra
    xm, wm = np.polynomial.legendre.leggauss(nmu)
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    MU, PH = np.meshgrid(xm, ph, indexing="ij")
    W = np.repeat(wm, nphi) * (2.0 * math.pi / nphi)
    return MU.ravel(), PH.ravel(), W


def streaming_matrices(N: int, extra: int = 0):
    """[A_x, A_y, A_z] = int m m^T Omega_d dOmega."""
    mu, phi, w = sphere_rule(N, extra)
    Y = real_sh(N, mu, phi)
    s = np.sqrt(1.0 - mu**2)
    om = [s * np.cos(phi), s * np.sin(phi), mu]
    return [(Y * (w * o)[:, None]).T @ Y for o in om]


def split_matrix(A):
    """(A^+, A^-) from the eigen-decomposition of the symmetric A."""
    A = 0.5 * (A + A.T)
    lam, V = np.linalg.eigh(A)
    Ap = (V * np.maximum(lam, 0.0)) @ V.T
    Am = (V * np.minimum(lam, 0.0)) @ V.T
    return Ap, Am


def split_streaming(N: int, dim: int):
    """[(A_d^+, A_d^-) for d < dim]."""
    return [split_matrix(A) for A in streaming_matrices(N)[:dim]]
