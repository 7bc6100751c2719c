"""The identity behind the right-hand-side pass that starts from the previous PCG solve.

The reduced system of eq. kkt_red_sc has K = P̄ + σI + ĀᵀRĀ and b = σx − q̄ + Āᵀ(Rz − y). A PCG
solve of K'x̃ = b' leaves x̃ and its residual r' = K'x̃ − b'. When ρ̄ changes by γ (R = γR', for
R = ρ̄I and for R = diag(ρ_i) alike), with z̃ = Āx̃:

    ĀᵀRz̃ = γ(r' + b' − P̄x̃ − σx̃),
    b    = σx − q̄ + γ(r' + b' − P̄x̃ − σx̃) − Āᵀ(R(z̃ − z) + y),
    r⁰   = Kx̃ − b = P̄x̃ + σ(x̃ − x) + q̄ + Āᵀ(R(z̃ − z) + y).

These are checked in float64 against the oracle's operator and right-hand side, on random
problems, so that the formulas the device pass evaluates are pinned to the definitions.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pcg as o_pcg


def random_problem(seed, n=40, m=30, eq_rows=8):
    rng = np.random.default_rng(seed)
    F = sp.random(n, n, density=0.2, random_state=rng)
    P = (F @ F.T + sp.eye(n)).tocsr()
    A = sp.random(m, n, density=0.3, random_state=rng, data_rvs=rng.standard_normal).tocsr()
    eq = np.zeros(m, bool)
    eq[rng.choice(m, eq_rows, replace=False)] = True
    q = rng.standard_normal(n)
    x, xt = rng.standard_normal(n), rng.standard_normal(n)
    z, y = rng.standard_normal(m), rng.standard_normal(m)
    return P, A, eq, q, x, xt, z, y


def kkt(P, A, sigma, R):
    return (P + sigma * sp.eye(P.shape[0]) + A.T @ sp.diags(R) @ A).tocsr()


def rhs(A, q, sigma, R, x, z, y):
    return sigma * x - q + A.T @ (R * z - y)


@pytest.mark.parametrize("vector_r", [False, True])
@pytest.mark.parametrize("rho_old, rho", [(0.3, 0.3), (0.3, 0.7), (2.0, 0.05)])
def test_rhs_from_previous_solve(vector_r, rho_old, rho):
    P, A, eq, q, x, xt, z, y = random_problem(1 + int(vector_r))
    sigma = 1e-6
    scale = np.where(eq, 1e3, 1.0) if vector_r else np.ones(A.shape[0])
    R_old, R = rho_old * scale, rho * scale
    gamma = rho / rho_old
    # the previous solve: any right-hand side b', and the residual its PCG left at x̃
    x_prev, z_prev, y_prev = x + 0.1, z - 0.2, y + 0.3
    b_prev = rhs(A, q, sigma, R_old, x_prev, z_prev, y_prev)
    r_prev = kkt(P, A, sigma, R_old) @ xt - b_prev
    zt = A @ xt
    g = R * (zt - z) + y
    s1, s2 = P @ xt, A.T @ g
    b_rec = sigma * x - q + gamma * ((r_prev + b_prev) - s1 - sigma * xt) - s2
    r0 = s1 + sigma * (xt - x) + q + s2
    b_def = rhs(A, q, sigma, R, x, z, y)
    size = np.abs(b_def).max() + np.abs(gamma * (r_prev + b_prev)).max() + np.abs(s2).max()
    assert np.abs(b_rec - b_def).max() <= 1e-13 * size
    Kx = kkt(P, A, sigma, R) @ xt
    assert np.abs(r0 - (Kx - b_def)).max() <= 1e-13 * (np.abs(Kx).max() + np.abs(b_def).max())


def test_scalar_case_matches_the_oracle_operator():
    """With R = ρ̄I the operator and right-hand side are the oracle's own (reduced_kkt_matvec,
    reduced_rhs), so the identity holds for the oracle's definitions, not only for this file's."""
    P, A, _, q, x, xt, z, y = random_problem(7)
    sigma, rho_old, rho = 1e-6, 0.4, 1.3
    K_old = o_pcg.reduced_kkt_matvec(P, A, sigma, rho_old)
    b_prev = o_pcg.reduced_rhs(A, q, sigma, rho_old, x - 1.0, z + 0.5, y)
    r_prev = K_old(xt) - b_prev
    s1 = P @ xt
    s2 = A.T @ (rho * (A @ xt - z) + y)
    b_rec = sigma * x - q + (rho / rho_old) * ((r_prev + b_prev) - s1 - sigma * xt) - s2
    b_def = o_pcg.reduced_rhs(A, q, sigma, rho, x, z, y)
    assert np.abs(b_rec - b_def).max() <= 1e-12 * max(1.0, np.abs(b_def).max())


def test_planted_mistakes_fail_the_identity():
    """Plausible slips in the formula (γ dropped, σx̃ dropped, γ applied to the Āᵀ term as well,
    the Āᵀ term's sign flipped) each miss the defined b by far more than the tolerance above."""
    P, A, _, q, x, xt, z, y = random_problem(3)
    sigma, rho_old, rho = 1e-6, 0.3, 0.7
    R_old, R = rho_old * np.ones(A.shape[0]), rho * np.ones(A.shape[0])
    gamma = rho / rho_old
    b_prev = rhs(A, q, sigma, R_old, x + 0.1, z - 0.2, y + 0.3)
    r_prev = kkt(P, A, sigma, R_old) @ xt - b_prev
    s1, s2 = P @ xt, A.T @ (R * (A @ xt - z) + y)
    b_def = rhs(A, q, sigma, R, x, z, y)
    size = np.abs(b_def).max() + np.abs(gamma * (r_prev + b_prev)).max() + np.abs(s2).max()
    slips = {
        "gamma dropped": sigma * x - q + ((r_prev + b_prev) - s1 - sigma * xt) - s2,
        "sigma*xt dropped": sigma * x - q + gamma * ((r_prev + b_prev) - s1) - s2,
        "gamma on s2": sigma * x - q + gamma * ((r_prev + b_prev) - s1 - sigma * xt) - gamma * s2,
        "s2 sign": sigma * x - q + gamma * ((r_prev + b_prev) - s1 - sigma * xt) + s2,
    }
    for name, b in slips.items():
        assert np.abs(b - b_def).max() > 1e3 * 1e-13 * size, name
