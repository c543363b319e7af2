"""Pins of the reference DLRA step (Sec. 2.2, Sec. 3.3.3) against the full-rank
step and closed forms."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import coeffs, dlra, fullrank, linalg, pn, solver
from workloads import configs


def _synthetic_source(problem, seed=0):
    rng = np.random.default_rng(seed)
    return rng.random((problem.options.n_steps, problem.grid.n))


def test_dlra_equals_full_rank_at_full_rank():
    # r = n = m: U and V span everything, the BUG steps are exact and the low-
    # rank step is the full-rank step up to round-off.
    p = configs.small_2d(nx=4, ny=4, N=3, r=16, n_steps=5, mats="slab", aug_tol=1e-12,
                         floor_tol=1e-14)
    ps = _synthetic_source(p)
    Du = np.zeros(p.grid.n)
    a = solver.run_beam_dlra(p, p.beams[0], psibar=ps, Du=Du)
    b = solver.run_beam_fullrank(p, p.beams[0], psibar=ps, Du=Du)
    st = a["state"]
    u_lr = st.U @ st.S @ st.V.T
    assert np.linalg.norm(u_lr - b["u"]) / np.linalg.norm(b["u"]) < 1e-11
    assert np.linalg.norm(a["dose_c"] - b["dose_c"]) / np.linalg.norm(b["dose_c"]) < 1e-11


def test_first_step_from_zero_is_the_source():
    # From u = 0 streaming and self-scattering do nothing; one explicit Euler
    # source step gives U S V^T = dt sum_i q_i g_i^T exactly (n_mat <= r; drop
    # tolerances below the source's smallest relative singular value, ~1e-7 here).
    p = configs.small_2d(mats="slab", r=6, aug_tol=1e-12, floor_tol=1e-14)
    ps = _synthetic_source(p, 1)
    Apm = solver.streaming_split(p)
    c = coeffs.step_coeffs(p, p.beams[0], 0)
    st = dlra.initial_state(p, c.g)
    st = dlra.step(st, c, Apm, p, ps[0])
    w = p.materials.w
    ref = c.dt * (w.T * ps[0][:, None]) @ c.g.T
    assert np.linalg.norm(st.U @ st.S @ st.V.T - ref) / np.linalg.norm(ref) < 1e-13
    # bases stay orthonormal
    assert np.abs(st.U.T @ st.U - np.eye(6)).max() < 1e-13
    assert np.abs(st.V.T @ st.V - np.eye(6)).max() < 1e-13


def test_dose_linear_in_source_strength():
    # relative truncation and relative drop rules make the step homogeneous of degree 1
    p = configs.small_2d(mats="slab", r=6, rank_mode="adaptive", r_min=2, r_max=10)
    ps = _synthetic_source(p, 2)
    Du = np.zeros(p.grid.n)
    a = solver.run_beam_dlra(p, p.beams[0], psibar=ps, Du=Du)["dose_c"]
    b = solver.run_beam_dlra(p, p.beams[0], psibar=3.7 * ps, Du=Du)["dose_c"]
    assert np.linalg.norm(b - 3.7 * a) / np.linalg.norm(b) < 1e-12


def test_collided_step_reduces_to_diagonal_division():
    # with U = I the implicit-Euler L-step is the per-(x,p) division of the full-rank step
    p = configs.small_2d(nx=4, ny=2, N=2, r=8, mats="slab")
    rng = np.random.default_rng(3)
    c = coeffs.step_coeffs(p, p.beams[0], 2)
    U = np.eye(8)
    S = rng.standard_normal((8, 8))
    V, _ = np.linalg.qr(rng.standard_normal((9, 8)))
    U2, St, Vt = dlra.collided(U, S, V, c, p.materials.w, 2, p.options)
    u = U @ S @ V.T
    ell, _ = pn.degree_order(2)
    wa = p.materials.w.T @ c.a
    ref = u / (1.0 - c.dt * c.s[:, None] * wa[:, ell])
    assert np.abs(U2 @ St @ Vt.T - ref).max() < 1e-12


def test_truncation_rules():
    rng = np.random.default_rng(4)
    opts = configs.small_2d().options.with_(rank_mode="adaptive", r_min=2, r_max=9,
                                            trunc_tol=1e-3)
    P0, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    Q0, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    sig = np.array([1.0, 0.5, 0.2, 1e-2, 5e-4, 2e-4, 1e-5, 1e-6, 1e-8, 0.0])
    S = P0[:, :10] @ np.diag(sig) @ Q0.T
    P, S1, Q = linalg.truncate(S, opts, 0)
    # tail(4) = 5e-4 + 2e-4 + ... = 7.11e-4 <= 1e-3 * 1.71..., tail(3) > it
    assert S1.shape == (4, 4)
    assert np.allclose(np.diag(S1), sig[:4], atol=1e-14)
    assert np.abs(P.T @ P - np.eye(4)).max() < 1e-13
    # fixed rank above the numerical rank: floor keeps 8 directions, fills 2
    opts2 = opts.with_(rank_mode="fixed", floor_tol=1e-7)
    P, S1, Q = linalg.truncate(S, opts2, 10)
    assert np.count_nonzero(np.diag(S1)) == 8
    assert np.abs(P.T @ P - np.eye(10)).max() < 1e-13
    assert np.abs(Q.T @ Q - np.eye(10)).max() < 1e-13
    assert np.linalg.norm(P @ S1 @ Q.T - S) < 1.01e-8


def test_rank_convergence_towards_full_rank():
    # the low-rank dose approaches the full-rank dose as the rank grows
    p = configs.small_2d(nx=10, ny=8, N=3, n_steps=8, mats="slab")
    ps = _synthetic_source(p, 5)
    Du = np.zeros(p.grid.n)
    ref = solver.run_beam_fullrank(p, p.beams[0], psibar=ps, Du=Du)["dose_c"]
    errs = []
    for r in (2, 6, 16):
        q = p.with_options(r=r, r_max=r)
        d = solver.run_beam_dlra(q, q.beams[0], psibar=ps, Du=Du)["dose_c"]
        errs.append(np.linalg.norm(d - ref) / np.linalg.norm(ref))
    assert errs[2] < errs[1] < errs[0]


def test_full_rank_mirror_symmetry():
    # a beam on the symmetry line of a symmetric phantom gives a symmetric dose
    p = configs.small_2d(nx=10, ny=8, N=3, n_steps=6, mats="slab")
    b = dataclasses.replace(p.beams[0], pos=(0.0, 0.5 * 8 * 0.05, 0.0))
    p = dataclasses.replace(p, beams=[b])
    res = solver.run_beam_fullrank(p, b)
    D = res["dose"].reshape(8, 10)
    assert np.abs(D - D[::-1]).max() <= 1e-11 * np.abs(D).max()
