"""Reduced KKT system and preconditioned conjugate gradient (Sections 4, 6.3).

Reduced KKT system with R = ρ̄I (Section 6.3, eq. kkt_red_sc):
    K x̃ = b,   K = P + σI + ρ̄AᵀA,   b = σx − q + Aᵀ(ρ̄z − y),
applied matrix-free as  w = ρ̄Ax,  Kx = Px + σx + Aᵀw.
Jacobi preconditioner (Section 6.3.1): diag(M) = diag(P) + σ·1 + ρ̄·diag(AᵀA),
with (AᵀA)_ii the squared 2-norm of column i of A.

PCG (Algorithm 3, following Nocedal & Wright's Algorithm 5.3 that the paper
cites). The step length is printed with a leading minus sign; with r = Kx − b
and p⁰ = −y⁰ the exact line search of Section 4.1, α = −rᵀp / pᵀKp, equals
+rᵀy / pᵀKp, which is what is used here (the printed sign would step uphill).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def reduced_kkt_matvec(P, A, sigma, rho):
    P = sp.csr_matrix(P)
    A = sp.csr_matrix(A)
    At = A.T.tocsr()

    def K(v):
        w = rho * (A @ v)
        return P @ v + sigma * v + At @ w

    return K


def reduced_kkt_dense(P, A, sigma, rho):
    P = sp.csr_matrix(P).toarray()
    A = sp.csr_matrix(A).toarray()
    return P + sigma * np.eye(P.shape[0]) + rho * (A.T @ A)


def reduced_rhs(A, q, sigma, rho, x, z, y):
    return sigma * x - q + sp.csr_matrix(A).T @ (rho * z - y)


def jacobi_diag(P, A, sigma, rho):
    P = sp.csr_matrix(P)
    A = sp.csc_matrix(A)
    colsq = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    return P.diagonal() + sigma + rho * colsq


def pcg(K, b, x0, minv, eps, max_iter, relative=True, norm=np.inf):
    """Algorithm 3. Stops when ‖r‖ ≤ ε‖b‖ (relative) or ‖r‖ ≤ ε (absolute).

    Returns (x, iterations, final ‖r‖, history of ‖r‖).
    """
    x = np.array(x0, dtype=np.float64)
    r = K(x) - b
    y = minv * r
    p = -y
    ry = float(r @ y)
    bn = np.linalg.norm(b, norm)
    thresh = eps * bn if relative else eps
    hist = [np.linalg.norm(r, norm)]
    k = 0
    while hist[-1] > thresh and k < max_iter:
        Kp = K(p)
        alpha = ry / float(p @ Kp)
        x = x + alpha * p
        r = r + alpha * Kp
        y = minv * r
        ry_new = float(r @ y)
        beta = ry_new / ry
        p = -y + beta * p
        ry = ry_new
        k += 1
        hist.append(np.linalg.norm(r, norm))
    return x, k, hist[-1], hist
