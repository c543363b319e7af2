"""One energy step of the DLRA integrator for the collided equation.

Follows Sec. 3.3.3 with the augmented BUG integrator of Sec. 2.2 (eq. KLS):

1. streaming (eq. split-streaming), RK4 with n_sub substeps:
     K1 from K(0) = U S,  L1 from L(0) = V S^T  (both with the old U, V);
     Uhat = [U | orth((I - UU^T) K1)], Vhat = [V | orth((I - VV^T) L1)];
     S1 from S(0) = (Uhat^T U) S (V^T Vhat) = [[S, 0], [0, 0]];
     truncation -> (U^1/2, S^1/2, V^1/2)
2. collided self-scattering, L-step only, implicit Euler (Sec. 3.3.3 item 1):
     (I - dt sum_i a_{il} M_i) L1[p, :]^T = L0[p, :]^T for every p of degree l,
     M_i = U^T diag(w_i s) U, L0 = V S^T; QR with completion -> (V~, S~)
3. uncollided in-scattering source, explicit Euler (items 2-4), starting from
   (U^1/2, S~, V~), source term sum_i (w_i psi_u) g_i^T (summed over the beams
   of a joint source) with
   g_i = (G_l - G_{N+1}) T_M (no 1/S factor: the collided equation of
   eq. final_collided_multmat sources the untransformed psi_u):
     K = U S~ + dt sum_i q_i (V~^T g_i)^T,  L = V~ S~^T + dt sum_i g_i (U^T q_i)^T,
     Uhat, Vhat by augmentation, Shat = [[S~, 0], [0, 0]] + dt sum_i (Uhat^T q_i)(Vhat^T g_i)^T,
     truncation -> (U^1, S^1, V^1)
4. deposited energy (collided part): D_c += dt sqrt(4 pi) U S V[0, :]^T, the
   right-endpoint rule for int int psi~ dOmega dE (m_0^0 = 1/sqrt(4 pi)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import linalg, pn
from . import transport as tr


@dataclass
class State:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    dose_c: np.ndarray
    k: int = 0
    log: list = field(default_factory=list)


def initial_state(problem, g0):
    """S = 0 (no collided flux at E_max) with deterministic orthonormal bases:
    U has unit vectors at cells floor((j + 1/2) n / r); V starts from the
    in-scattering source directions g_i of the first step (ordered CGS2, drop
    below aug_tol * ||g||_F), completed with the unit moment vectors e_0, e_1, ...
    With V spanning the g_i the first uncollided step reproduces the source
    dt sum_i q_i g_i^T exactly."""
    o = problem.options
    n, m = problem.grid.n, problem.m
    r = o.r if o.rank_mode == "fixed" else o.r_min
    U = np.zeros((n, r))
    for j in range(r):
        U[int((j + 0.5) * n / r), j] = 1.0
    V, _ = linalg.qr_complete(g0, np.eye(m), r, o.aug_tol, o.fill_tol)
    return State(U, np.zeros((r, r)), V, np.zeros(n))


def rank_target(opts, r_now):
    return opts.r if opts.rank_mode == "fixed" else r_now


def streaming(U, S, V, c, Apm, grid, opts):
    dim = grid.dim
    r = U.shape[1]
    Bpm = tr.galerkin_angular(V, Apm)
    Cbf = tr.projections(U, U, c.s, grid, dim)
    K1 = tr.rk4(lambda K: tr.kstep_rhs(K, c.s, Bpm, grid), U @ S, c.h, c.n_sub)
    L1 = tr.rk4(lambda L: tr.lstep_rhs(L, Apm, Cbf), V @ S.T, c.h, c.n_sub)
    Uh = linalg.augment(U, K1, opts.aug_tol)
    Vh = linalg.augment(V, L1, opts.aug_tol)
    Ch = tr.projections(Uh, Uh, c.s, grid, dim)
    Bh = tr.galerkin_angular(Vh, Apm)
    S0 = np.zeros((Uh.shape[1], Vh.shape[1]))
    S0[:r, :r] = S
    S1 = tr.rk4(lambda X: tr.sstep_rhs(X, Ch, Bh), S0, c.h, c.n_sub)
    P, Sn, Q = linalg.truncate(S1, opts, rank_target(opts, r))
    return Uh @ P, Sn, Vh @ Q, (Uh.shape[1] - r, Vh.shape[1] - r)


def collided(U, S, V, c, w, N, opts):
    r = U.shape[1]
    ell, _ = pn.degree_order(N)
    M = [U.T @ ((w[i] * c.s)[:, None] * U) for i in range(w.shape[0])]
    L0 = V @ S.T
    L1 = np.empty_like(L0)
    for l in range(N + 1):
        A = np.eye(r) - c.dt * sum(c.a[i, l] * M[i] for i in range(w.shape[0]))
        rows = ell == l
        L1[rows] = np.linalg.solve(A, L0[rows].T).T
    Vt, St = linalg.qr_complete(L1, V, r, opts.aug_tol, opts.fill_tol)
    return U, St, Vt


def source_factors(w, psibars, gs):
    """Q (n x n_src) and G (m x n_src) with Q G^T = sum_b sum_i (w_i o psi_b) g_{i,b}^T:
    the in-scattering source of one or several beams (a joint source, the
    two-beam case of Sec. 4.3), columns beam-major."""
    Q = np.concatenate([(w * ps[None, :]).T for ps in psibars], axis=1)
    G = np.concatenate(gs, axis=1)
    return Q, G


def uncollided(U, St, Vt, dt, Q, G, opts):
    """Explicit-Euler K, L and S steps of the source Q G^T (Sec. 3.3.3 items 2-4)."""
    r = U.shape[1]
    Ku = U @ St + dt * Q @ (Vt.T @ G).T
    Lu = Vt @ St.T + dt * G @ (U.T @ Q).T
    Uh = linalg.augment(U, Ku, opts.aug_tol)
    Vh = linalg.augment(Vt, Lu, opts.aug_tol)
    Sh = np.zeros((Uh.shape[1], Vh.shape[1]))
    Sh[:r, :r] = St
    Sh += dt * (Uh.T @ Q) @ (Vh.T @ G).T
    P, Sn, Qv = linalg.truncate(Sh, opts, rank_target(opts, r))
    return Uh @ P, Sn, Vh @ Qv, (Uh.shape[1] - r, Vh.shape[1] - r)


def step(state, c, Apm, problem, psibar_k, sources=None):
    """Advance `state` by energy step c.k in place-free fashion; returns a new
    State.  The source is that of one beam (psibar_k with c.g), or the factor
    pair `sources` = (Q, G) of source_factors for several beams."""
    g, o = problem.grid, problem.options
    w = problem.materials.w
    Q, G = source_factors(w, [psibar_k], [c.g]) if sources is None else sources
    U, S, V, aug1 = streaming(state.U, state.S, state.V, c, Apm, g, o)
    r_half = U.shape[1]
    U, St, Vt = collided(U, S, V, c, w, o.pn_degree, o)
    U, S, V, aug2 = uncollided(U, St, Vt, c.dt, Q, G, o)
    dose_c = state.dose_c + c.dt * math.sqrt(4.0 * math.pi) * (U @ (S @ V[0, :]))
    log = state.log + [dict(k=c.k, n_sub=c.n_sub, r_half=r_half, r=U.shape[1],
                            aug_stream=aug1, aug_source=aug2)]
    return State(U, S, V, dose_c, state.k + 1, log)
