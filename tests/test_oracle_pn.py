"""Pins of the angular algebra against textbook facts (Sec. 3.3.1, Sec. 3.3.2)."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_gegenbauer

from oracle import pn


@pytest.mark.parametrize("N", [1, 3, 7])
def test_real_sh_orthonormal(N):
    mu, phi, w = pn.sphere_rule(N, extra=3)
    Y = pn.real_sh(N, mu, phi)
    assert np.abs((Y * w[:, None]).T @ Y - np.eye(pn.n_moments(N))).max() < 1e-13


@pytest.mark.parametrize("N", [1, 3, 7, 15])
def test_Az_three_term_recurrence(N):
    # mu Y_l^k = a(l,k) Y_{l+1}^k + a(l-1,k) Y_{l-1}^k with
    # a(l,k) = sqrt(((l+1)^2 - k^2) / ((2l+1)(2l+3)))  (textbook recurrence)
    Az = pn.streaming_matrices(N)[2]
    m = pn.n_moments(N)
    ref = np.zeros((m, m))
    for l in range(N):
        for k in range(-l, l + 1):
            a = math.sqrt(((l + 1) ** 2 - k * k) / ((2 * l + 1) * (2 * l + 3)))
            p, q = l * l + l + k, (l + 1) ** 2 + (l + 1) + k
            ref[p, q] = ref[q, p] = a
    assert np.abs(Az - ref).max() < 1e-13


@pytest.mark.parametrize("N", [1, 3, 7])
def test_streaming_spectra_are_gauss_nodes(N):
    # The |k| block of A_z is the Jacobi matrix of the weight (1-mu^2)^|k|:
    # its eigenvalues are the zeros of the Gegenbauer polynomial
    # C_{N+1-|k|}^{(|k|+1/2)} (Legendre nodes for k = 0).
    ref = []
    for k in range(-N, N + 1):
        n = N + 1 - abs(k)
        x, _ = roots_gegenbauer(n, abs(k) + 0.5)
        ref.extend(x)
    ref = np.sort(ref)
    A = pn.streaming_matrices(N)
    for d in range(3):
        lam = np.linalg.eigvalsh(A[d])
        # rotation invariance of the degree <= N space: equal spectra for x, y, z
        assert np.abs(np.sort(lam) - ref).max() < 1e-12
    x0, _ = np.polynomial.legendre.leggauss(N + 1)
    assert abs(np.max(np.linalg.eigvalsh(A[2])) - x0.max()) < 1e-13


@pytest.mark.parametrize("N", [3, 7])
def test_eigen_split(N):
    for A in pn.streaming_matrices(N):
        Ap, Am = pn.split_matrix(A)
        assert np.abs(Ap + Am - A).max() < 1e-13
        assert np.linalg.eigvalsh(Ap).min() > -1e-13
        assert np.linalg.eigvalsh(Am).max() < 1e-13
        assert np.abs(Ap @ Am).max() < 1e-13


def test_beam_moments_first_degree():
    # l = 1 real harmonics are sqrt(3/(4 pi)) (Omega_y, Omega_z, Omega_x)
    om = np.array([0.3, -0.5, 0.8])
    om /= np.linalg.norm(om)
    T = pn.beam_moments(3, om)
    assert abs(T[0] - 1.0 / math.sqrt(4 * math.pi)) < 1e-15
    c = math.sqrt(3.0 / (4.0 * math.pi))
    assert np.allclose(T[1:4], c * np.array([om[1], om[2], om[0]]), atol=1e-14)


def test_addition_theorem():
    rng = np.random.default_rng(0)
    N = 7
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    Ta, Tb = pn.beam_moments(N, a), pn.beam_moments(N, b)
    ell, _ = pn.degree_order(N)
    for l in range(N + 1):
        lhs = np.sum(Ta[ell == l] * Tb[ell == l])
        rhs = (2 * l + 1) / (4 * math.pi) * eval_legendre(l, float(a @ b))
        assert abs(lhs - rhs) < 1e-13
