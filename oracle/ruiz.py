"""Modified Ruiz equilibration (Algorithm 2, Section 3.3).

Computes c > 0 and positive diagonal D (n), E (m) with
    P̄ = c·D P D,  q̄ = c·D q,  Ā = E A D,  l̄ = E l,  ū = E u.

Readings where the paper is silent or inconsistent:
* The matrix-scaling step of Algorithm 2 rebuilds P̄ and q̄ from the unscaled
  data without the cost factor c accumulated so far, which breaks P̄ = cDPD
  after the first pass; here P̄ ← c·DPD and q̄ ← c·Dq, so the stated relation
  holds after every pass.
* ε_equil is not given: at most ``iters`` (10) passes, stopping after a pass
  whose δ satisfies ‖1 − δ‖∞ ≤ 1e-3.
* δ_i = 1/√‖M_i‖∞ is undefined for an empty column: a norm below 1e-4 is
  taken as 1 and norms are capped at 1e4. The same guard is applied to the
  denominator of γ = 1/max(mean_i ‖P̄_i‖∞, ‖q̄‖∞).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NORM_MIN = 1e-4
NORM_MAX = 1e4
EPS_EQUIL = 1e-3


def _guard(v):
    v = np.asarray(v, dtype=np.float64).copy()
    v[v < NORM_MIN] = 1.0
    return np.minimum(v, NORM_MAX)


def col_inf_norms(M: sp.spmatrix) -> np.ndarray:
    M = sp.csc_matrix(M)
    out = np.zeros(M.shape[1])
    if M.nnz:
        out = np.asarray(abs(M).max(axis=0).todense()).ravel()
    return out


def row_inf_norms(M: sp.spmatrix) -> np.ndarray:
    return col_inf_norms(sp.csr_matrix(M).T)


def ruiz(P_full: sp.csr_matrix, q: np.ndarray, A: sp.csr_matrix, iters: int = 10):
    """Return (D, E, c, P̄, q̄, Ā, passes) following Algorithm 2."""
    n = A.shape[1]
    m = A.shape[0]
    c = 1.0
    D = np.ones(n)
    E = np.ones(m)
    P = sp.csr_matrix(P_full, dtype=np.float64)
    A = sp.csr_matrix(A, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Pb, qb, Ab = P.copy(), q.copy(), A.copy()
    passes = 0
    for _ in range(iters):
        passes += 1
        # column ∞-norms of M = [[P̄, Āᵀ], [Ā, 0]]
        norm_x = np.maximum(col_inf_norms(Pb), col_inf_norms(Ab))
        norm_z = row_inf_norms(Ab)
        delta = 1.0 / np.sqrt(_guard(np.concatenate([norm_x, norm_z])))
        D = delta[:n] * D
        E = delta[n:] * E
        Dm = sp.diags(D)
        Em = sp.diags(E)
        Pb = (c * (Dm @ P @ Dm)).tocsr()
        qb = c * D * q
        Ab = (Em @ A @ Dm).tocsr()
        mean_p = float(np.mean(col_inf_norms(Pb))) if n else 0.0
        g = _guard([max(mean_p, float(np.max(np.abs(qb))) if n else 0.0)])[0]
        gamma = 1.0 / g
        Pb = (gamma * Pb).tocsr()
        qb = gamma * qb
        c = gamma * c
        if np.max(np.abs(1.0 - delta)) <= EPS_EQUIL:
            break
    return D, E, c, Pb, qb, Ab, passes


def no_scaling(P_full, q, A):
    n, m = A.shape[1], A.shape[0]
    return (np.ones(n), np.ones(m), 1.0, sp.csr_matrix(P_full, dtype=np.float64),
            np.asarray(q, dtype=np.float64).copy(), sp.csr_matrix(A, dtype=np.float64), 0)
