"""Basis augmentation, rank truncation and completion (Sec. 2.2, Sec. 3.3.3).

Readings (the paper gives "a QR decomposition" and "a truncated SVD"):
  * augmentation  [B | orth_tau((I - B B^T) X)]: the new directions are the
    left singular vectors of the projected residual whose singular values
    exceed tau_aug * ||X||_F (two projection passes);
  * truncation  S = P Sigma Q^T; adaptive rank = smallest r1 with
    sum_{j >= r1} sigma_j <= theta * sum_j sigma_j (relative L1 tail),
    clamped to [r_min, r_max]; fixed rank r1 = r;
  * floor  only directions with sigma_j > tau_floor * sigma_1 keep their
    singular vectors; the remaining r1 - kept columns are filled, in order,
    from the previous basis (the unit vectors of the augmented coordinates),
    each orthogonalised twice and accepted when its residual exceeds
    fill_tol; the filled columns carry zero coefficients;
  * collided QR with completion  columns of L1 in order (accepted when the
    twice-orthogonalised residual exceeds tau_aug * ||L1||_F), then columns of
    the old basis V (accepted above fill_tol) until r columns; S~ = L1^T V~.
"""
from __future__ import annotations

import numpy as np


def project_out(X, B):
    """(I - B B^T) X with two classical Gram-Schmidt passes."""
    if B.shape[1] == 0:
        return X.copy()
    R = X - B @ (B.T @ X)
    return R - B @ (B.T @ R)


def orth_tau(R, thresh):
    if R.shape[1] == 0:
        return np.zeros((R.shape[0], 0))
    Ur, sig, _ = np.linalg.svd(R, full_matrices=False)
    return Ur[:, sig > thresh]


def augment(B, X, tol):
    """[B | orth_tau((I - B B^T) X, tol ||X||_F)]."""
    R = project_out(X, B)
    new = orth_tau(R, tol * np.linalg.norm(X))
    return np.hstack([B, new])


def _cgs2_append(Q, v, thresh):
    """Orthogonalise v twice against the columns of Q; return the normalised
    residual, or None if its norm does not exceed thresh."""
    if Q:
        B = np.stack(Q, axis=1)
        v = v - B @ (B.T @ v)
        v = v - B @ (B.T @ v)
    nv = np.linalg.norm(v)
    if nv > thresh:
        return v / nv
    return None


def fill_columns(Pk, dim, need, accept):
    """Columns of Pk followed by `need` fillers drawn in order from e_0..e_{dim-1}."""
    Q = [Pk[:, j].copy() for j in range(Pk.shape[1])]
    added = 0
    for j in range(dim):
        if added == need:
            break
        e = np.zeros(dim)
        e[j] = 1.0
        v = _cgs2_append(Q, e, accept)
        if v is not None:
            Q.append(v)
            added += 1
    if added != need:
        raise RuntimeError("basis completion ran out of candidates")
    return np.stack(Q, axis=1) if Q else np.zeros((dim, 0))


def truncation_rank(sig, opts, r_fixed):
    pmin = sig.size
    if opts.rank_mode == "fixed":
        return min(r_fixed, pmin)
    total = sig.sum()
    tail = np.concatenate([np.cumsum(sig[::-1])[::-1], [0.0]])
    r1 = int(np.argmax(tail <= opts.trunc_tol * total))
    return int(min(max(r1, opts.r_min), opts.r_max, pmin))


def truncate(Shat, opts, r_fixed):
    """Truncated SVD with the floor rule: returns (P', S', Q') with
    Uhat P', S', Vhat Q' the new factors."""
    pu, pv = Shat.shape
    P, sig, Qt = np.linalg.svd(Shat, full_matrices=True)
    r1 = truncation_rank(sig, opts, r_fixed)
    kept = 0
    if sig.size and sig[0] > 0.0:
        kept = int(np.count_nonzero(sig[:r1] > opts.floor_tol * sig[0]))
    Pf = fill_columns(P[:, :kept], pu, r1 - kept, opts.fill_tol)
    Qf = fill_columns(Qt.T[:, :kept], pv, r1 - kept, opts.fill_tol)
    S1 = np.zeros((r1, r1))
    S1[np.arange(kept), np.arange(kept)] = sig[:kept]
    return Pf, S1, Qf


def qr_complete(L1, V, r, tol, accept):
    """Orthonormal V~ (m x r) spanning the columns of L1, completed from V;
    S~ = L1^T V~."""
    Q = []
    thr = tol * np.linalg.norm(L1)
    for j in range(L1.shape[1]):
        if len(Q) == r:
            break
        v = _cgs2_append(Q, L1[:, j].copy(), thr)
        if v is not None:
            Q.append(v)
    for j in range(V.shape[1]):
        if len(Q) == r:
            break
        v = _cgs2_append(Q, V[:, j].copy(), accept)
        if v is not None:
            Q.append(v)
    if len(Q) != r:
        raise RuntimeError("collided QR completion ran out of candidates")
    Vt = np.stack(Q, axis=1)
    return Vt, L1.T @ Vt
