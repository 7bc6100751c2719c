"""Seeded synthetic QP instances in OSQP form  min ½xᵀPx + qᵀx  s.t.  l ≤ Ax ≤ u.

This module only draws random data and writes the problem classes of the
paper's benchmark section (Section 7.1: Random, Lasso, Portfolio, SVM) in the
standard form of Section 2, eq. (qp). It holds none of the solver's arithmetic
and imports neither the solver binding nor the oracle, so both sides (and the
tests) can draw identical inputs from it.

Output convention (the OSQP input convention, Section 6.2): P is returned as
the upper triangle (diagonal included) in CSC, A in CSC, q/l/u as float64
vectors, ±inf for absent bounds.

Sparsity patterns are i.i.d. Bernoulli(d): the linearised positions of the
nonzeros are drawn by geometric gap skipping, which realises exactly one
independent Bernoulli(d) trial per entry at O(nnz) cost.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class QP:
    name: str
    P_triu: sp.csc_matrix      # upper triangle of P incl. diagonal, CSC
    q: np.ndarray
    A: sp.csc_matrix           # m×n, CSC
    l: np.ndarray
    u: np.ndarray
    meta: dict

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    def P_full(self) -> sp.csr_matrix:
        T = self.P_triu.tocsr()
        return (T + sp.triu(T, k=1).T).tocsr()


def _bernoulli_positions(rng, rows: int, cols: int, d: float) -> tuple[np.ndarray, np.ndarray]:
    """Row/column indices (row-major sorted) of an i.i.d. Bernoulli(d) pattern."""
    total = rows * cols
    if d <= 0.0 or total == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if d >= 1.0:
        pos = np.arange(total, dtype=np.int64)
    else:
        expect = total * d
        chunks = []
        last = -1
        while True:
            k = int(expect + 6.0 * math.sqrt(expect) + 64) if not chunks else int(0.05 * expect + 1024)
            gaps = rng.geometric(d, size=k).astype(np.int64)
            p = last + np.cumsum(gaps)
            chunks.append(p)
            last = int(p[-1])
            if last >= total:
                break
        pos = np.concatenate(chunks)
        pos = pos[pos < total]
    return pos // cols, pos % cols


def sprandn(rng, rows: int, cols: int, d: float, mean=0.0, var=1.0, row_mean=None) -> sp.csr_matrix:
    """rows×cols CSR with Bernoulli(d) pattern and N(mean, var) values.

    ``row_mean`` (length rows) overrides ``mean`` per row.
    """
    r, c = _bernoulli_positions(rng, rows, cols, d)
    vals = rng.standard_normal(r.size) * math.sqrt(var)
    if row_mean is not None:
        vals += np.asarray(row_mean, dtype=np.float64)[r]
    else:
        vals += mean
    indptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=rows), out=indptr[1:])
    return sp.csr_matrix((vals, c.astype(np.int32), indptr), shape=(rows, cols))


def _finish(name, P_full, q, A, l, u, meta) -> QP:
    P_triu = sp.triu(sp.csr_matrix(P_full), format="csc")
    P_triu.sort_indices()
    A = sp.csc_matrix(A)
    A.sort_indices()
    P_triu.indices = P_triu.indices.astype(np.int32)
    P_triu.indptr = P_triu.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    meta = dict(meta)
    meta.update(n=A.shape[1], m=A.shape[0], nnz_P_full=int(sp.csr_matrix(P_full).nnz),
                nnz_P_triu=int(P_triu.nnz), nnz_A=int(A.nnz))
    return QP(name, P_triu, np.ascontiguousarray(q, np.float64), A,
              np.ascontiguousarray(l, np.float64), np.ascontiguousarray(u, np.float64), meta)


def random_qp(n: int, m: int, dens_M: float, dens_A: float, seed: int) -> QP:
    """Random class: P = MMᵀ + 1e-2·I, A Bernoulli, q ~ N(0,1), l = −U[0,1], u = U[0,1]."""
    rng = np.random.default_rng(seed)
    M = sprandn(rng, n, n, dens_M)
    P = (M @ M.T + 1e-2 * sp.identity(n, format="csr")).tocsr()
    A = sprandn(rng, m, n, dens_A)
    q = rng.standard_normal(n)
    l = -rng.random(m)
    u = rng.random(m)
    return _finish("random", P, q, A, l, u, dict(seed=seed, dens_M=dens_M, dens_A=dens_A))


def lasso_qp(n_feat: int, m_data: int, dens: float, seed: int) -> QP:
    """Lasso class: min ‖Ad·x − b‖² + λ‖x‖₁ in OSQP form over (x, y, t).

    min yᵀy + λ1ᵀt  s.t.  y = Ad·x − b,  −t ≤ x ≤ t.
    """
    rng = np.random.default_rng(seed)
    Ad = sprandn(rng, m_data, n_feat, dens)
    v = rng.standard_normal(n_feat) * math.sqrt(1.0 / n_feat)
    v[rng.choice(n_feat, n_feat // 2, replace=False)] = 0.0
    b = Ad @ v + rng.standard_normal(m_data)
    lam = float(np.max(np.abs(Ad.T @ b))) / 5.0
    n, m = n_feat, m_data
    In = sp.identity(n, format="csr")
    Im = sp.identity(m, format="csr")
    P = sp.block_diag((sp.csr_matrix((n, n)), 2.0 * Im, sp.csr_matrix((n, n))), format="csr")
    q = np.concatenate([np.zeros(n), np.zeros(m), lam * np.ones(n)])
    A = sp.bmat([[Ad, -Im, None], [In, None, -In], [In, None, In]], format="csc")
    inf = np.inf
    l = np.concatenate([b, -inf * np.ones(n), np.zeros(n)])
    u = np.concatenate([b, np.zeros(n), inf * np.ones(n)])
    return _finish("lasso", P, q, A, l, u, dict(seed=seed, n_feat=n_feat, m_data=m_data, dens=dens, lam=lam))


def portfolio_qp(n_assets: int, k_factors: int, dens: float, seed: int, gamma: float = 1.0) -> QP:
    """Portfolio class: min xᵀDx + yᵀy − μᵀx/γ  s.t.  y = Fᵀx, 1ᵀx = 1, x ≥ 0."""
    rng = np.random.default_rng(seed)
    F = sprandn(rng, n_assets, k_factors, dens)
    Dd = rng.random(n_assets) * math.sqrt(k_factors)
    mu = rng.standard_normal(n_assets)
    n, k = n_assets, k_factors
    P = sp.block_diag((sp.diags(2.0 * Dd), 2.0 * sp.identity(k)), format="csr")
    q = np.concatenate([-mu / gamma, np.zeros(k)])
    A = sp.bmat([[F.T, -sp.identity(k)],
                 [sp.csr_matrix(np.ones((1, n))), None],
                 [sp.identity(n), None]], format="csc")
    l = np.concatenate([np.zeros(k), [1.0], np.zeros(n)])
    u = np.concatenate([np.zeros(k), [1.0], np.inf * np.ones(n)])
    return _finish("portfolio", P, q, A, l, u, dict(seed=seed, n_assets=n, k_factors=k, dens=dens, gamma=gamma))


def svm_qp(n_points: int, n_feat: int, dens: float, seed: int, lam: float = 1.0) -> QP:
    """SVM class: min xᵀx + λ Σ max(0, b_i a_iᵀx + 1) over (x, t).

    min xᵀx + λ1ᵀt  s.t.  t ≥ diag(b)·Ad·x + 1,  t ≥ 0  (the hinge sign as the
    paper prints it). The first half of the points has label +1 and entries
    N(+1/n_feat, 1/n_feat), the second half label −1 and N(−1/n_feat, 1/n_feat).
    """
    rng = np.random.default_rng(seed)
    half = n_points // 2
    b = np.concatenate([np.ones(half), -np.ones(n_points - half)])
    Ad = sprandn(rng, n_points, n_feat, dens, var=1.0 / n_feat, row_mean=b / n_feat)
    n, N = n_feat, n_points
    P = sp.block_diag((2.0 * sp.identity(n), sp.csr_matrix((N, N))), format="csr")
    q = np.concatenate([np.zeros(n), lam * np.ones(N)])
    A = sp.bmat([[sp.diags(b) @ Ad, -sp.identity(N)],
                 [None, sp.identity(N)]], format="csc")
    l = np.concatenate([-np.inf * np.ones(N), np.zeros(N)])
    u = np.concatenate([-np.ones(N), np.inf * np.ones(N)])
    return _finish("svm", P, q, A, l, u, dict(seed=seed, n_points=N, n_feat=n, dens=dens, lam=lam))


def control_qp(nx: int, nu: int, horizon: int, dens: float, seed: int) -> QP:
    """Control class (Section 7.1): min x_Tᵀ Q_T x_T + Σ_{t<T} x_tᵀQx_t + u_tᵀRu_t subject to
    x_0 = x_init, x_{t+1} = A x_t + B u_t, −x̲ ≤ x_t ≤ x̄, −u̲ ≤ u_t ≤ ū, over the stacked
    variables (x_0, …, x_T, u_0, …, u_{T−1}).

    Data: A = 0.95·I + Δ with Δ Bernoulli(dens), entries N(0, 0.03²/(nx·dens)) (spectral radius
    of Δ about 0.03, so A is contractive); B Bernoulli(dens) N(0, 1); Q = diag(U[0, 10]) with a
    fifth of its entries zeroed; Q_T = 10·Q + I; R = 0.1·I; x̄ = x̲ = 2 + U[0, 2];
    ū = u̲ = 1 + U[0, 1]; x_init ~ U[−1, 1]. With A contractive, u = 0 keeps every |x_t| below
    the bounds, so every instance is feasible. The objective has no ½, so
    P = 2·blockdiag(Q, …, Q, Q_T, R, …, R).
    """
    rng = np.random.default_rng(seed)
    T = horizon
    Ad = (0.95 * sp.identity(nx, format="csr")
          + sprandn(rng, nx, nx, dens, var=0.0009 / (nx * dens))).tocsr()
    Bd = sprandn(rng, nx, nu, dens)
    qd = rng.random(nx) * 10.0
    qd[rng.choice(nx, nx // 5, replace=False)] = 0.0
    Q = sp.diags(qd)
    QT = sp.diags(10.0 * qd + 1.0)
    R = 0.1 * sp.identity(nu)
    P = 2.0 * sp.block_diag([Q] * T + [QT] + [R] * T, format="csr")
    nX, nU = nx * (T + 1), nu * T
    n = nX + nU
    q = np.zeros(n)
    # x_0 = x_init; x_{t+1} − A x_t − B u_t = 0
    Ix = sp.identity(nx, format="csr")
    Sx = sp.kron(sp.eye(T + 1, k=-1), -Ad) + sp.kron(sp.identity(T + 1), Ix)  # rows t: x_t − A x_{t−1}
    Su = sp.kron(sp.vstack([sp.csr_matrix((1, T)), sp.identity(T)]), -Bd)      # rows t ≥ 1: − B u_{t−1}
    Aeq = sp.hstack([Sx, Su]).tocsr()
    xbar = 2.0 + 2.0 * rng.random(nx)
    ubar = 1.0 + rng.random(nu)
    x0 = 2.0 * rng.random(nx) - 1.0
    beq = np.concatenate([x0, np.zeros(nx * T)])
    Abox = sp.hstack([sp.csr_matrix((nx * T + nU, nx)), sp.identity(nx * T + nU)]).tocsr()
    A = sp.vstack([Aeq, Abox], format="csc")
    lbox = np.concatenate([np.tile(-xbar, T), np.tile(-ubar, T)])
    ubox = np.concatenate([np.tile(xbar, T), np.tile(ubar, T)])
    l = np.concatenate([beq, lbox])
    u = np.concatenate([beq, ubox])
    return _finish("control", P, q, A, l, u, dict(seed=seed, nx=nx, nu=nu, horizon=T, dens=dens))


def equality_qp(n: int, m: int, dens_M: float, dens_A: float, seed: int) -> QP:
    """Equality class (Section 7.1): min ½xᵀPx + qᵀx  s.t.  Ax = b, with the random class's
    P = MMᵀ + 1e-2·I and A, q ~ N(0, 1), and b = A·x₀ for x₀ ~ N(0, 1) (consistent)."""
    rng = np.random.default_rng(seed)
    M = sprandn(rng, n, n, dens_M)
    P = (M @ M.T + 1e-2 * sp.identity(n, format="csr")).tocsr()
    A = sprandn(rng, m, n, dens_A)
    q = rng.standard_normal(n)
    b = A @ rng.standard_normal(n)
    return _finish("equality", P, q, A, b, b.copy(), dict(seed=seed, dens_M=dens_M, dens_A=dens_A))


def huber_qp(n_feat: int, m_data: int, dens: float, seed: int, M: float = 1.0) -> QP:
    """Huber class (Section 7.1): min Σ φ_hub(a_iᵀx − b_i), φ_hub(v) = v² for |v| ≤ M and
    M(2|v| − M) otherwise, as the QP over (x, w, r, s):

        min wᵀw + 2M·1ᵀ(r + s)  s.t.  Ad·x − w − r + s = b,  r ≥ 0,  s ≥ 0

    (for a residual v the inner minimum over w + r − s = v is v² when |v| ≤ M and 2M|v| − M²
    otherwise). Data: Ad Bernoulli(dens) N(0, 1); x_true ~ N(0, 1/n_feat); b = Ad·x_true + ε with
    ε ~ N(0, 1/4) on 95% of the points and N(0, 10²) on the other 5% (outliers)."""
    rng = np.random.default_rng(seed)
    Ad = sprandn(rng, m_data, n_feat, dens)
    x_true = rng.standard_normal(n_feat) * math.sqrt(1.0 / n_feat)
    noise = 0.5 * rng.standard_normal(m_data)
    out = rng.random(m_data) < 0.05
    noise[out] = 10.0 * rng.standard_normal(int(out.sum()))
    b = Ad @ x_true + noise
    n, m = n_feat, m_data
    Im = sp.identity(m, format="csr")
    P = sp.block_diag((sp.csr_matrix((n, n)), 2.0 * Im, sp.csr_matrix((2 * m, 2 * m))), format="csr")
    q = np.concatenate([np.zeros(n + m), 2.0 * M * np.ones(2 * m)])
    A = sp.bmat([[Ad, -Im, -Im, Im],
                 [None, None, Im, None],
                 [None, None, None, Im]], format="csc")
    l = np.concatenate([b, np.zeros(2 * m)])
    u = np.concatenate([b, np.inf * np.ones(2 * m)])
    return _finish("huber", P, q, A, l, u, dict(seed=seed, n_feat=n, m_data=m, dens=dens, M=M))


def primal_infeasible_qp(n: int, m: int, dens: float, seed: int) -> QP:
    """Random class whose longest row a of A is moved to the end and doubled under disjoint
    bounds, a·x ∈ [1, 2] (row m − 1) and a·x ∈ [3, 4] (row m), so that no x is feasible; every
    fourth other row has u = +∞. With m < n the rows of A other than the copy are independent
    (almost surely), so Aᵀy = 0 (Section 2.1) forces y onto the two copies:
    y ∝ e_{m−1} − e_m, the only certificate direction."""
    base = random_qp(n, m, dens, dens, seed)
    A = sp.csr_matrix(base.A)
    r = int(np.argmax(np.diff(A.indptr)))  # the longest row (non-empty)
    rest = np.delete(np.arange(m), r)
    A2 = sp.vstack([A[rest], A[r], A[r]]).tocsr()
    l = np.concatenate([base.l[rest], [1.0, 3.0]])
    u = np.concatenate([base.u[rest], [2.0, 4.0]])
    u[:m - 1:4] = np.inf
    return _finish("primal_infeasible", base.P_full(), base.q, A2, l, u,
                   dict(seed=seed, dens=dens, rows=(m - 1, m)))


def dual_infeasible_qp(n: int, m: int, dens: float, seed: int) -> QP:
    """Random class in which variable j (drawn) appears neither in P nor in A, except in one last
    row x_j ≥ 0 (u = +∞), and has q_j = −1: the objective decreases without bound along e_j
    (Pe_j = 0, qᵀe_j < 0, Ae_j ≥ 0 on that row), and P is positive definite on the other
    variables, so e_j is the only certificate direction (Section 2.1)."""
    base = random_qp(n, m, dens, dens, seed)
    rng = np.random.default_rng(seed + 1)
    j = int(rng.integers(n))
    keep = np.ones(n)
    keep[j] = 0.0
    Dk = sp.diags(keep)
    P = (Dk @ base.P_full() @ Dk).tocsr()
    P.eliminate_zeros()
    A = (sp.csr_matrix(base.A) @ Dk).tocsr()
    A.eliminate_zeros()
    ej = sp.csr_matrix(([1.0], ([0], [j])), shape=(1, n))
    A2 = sp.vstack([A, ej]).tocsr()
    q = base.q.copy()
    q[j] = -1.0
    l = np.concatenate([base.l, [0.0]])
    u = np.concatenate([base.u, [np.inf]])
    return _finish("dual_infeasible", P, q, A2, l, u, dict(seed=seed, dens=dens, var=j))


# The five benchmark workloads and their scaled-down parity variants.
# Instance j of workload i uses seed 1000·i + j.
WORKLOADS = {
    "random_c0": lambda j=0: random_qp(200, 400, 0.15, 0.15, 1000 * 0 + j),
    "lasso_c1": lambda j=0: lasso_qp(10_000, 100_000, 0.01, 1000 * 1 + j),
    "random_c2": lambda j=0: random_qp(100_000, 1_000_000, 4.47e-5, 2e-4, 1000 * 2 + j),
    "portfolio_c3": lambda j=0: portfolio_qp(100_000, 1_000, 0.5, 1000 * 3 + j),
    "svm_c4": lambda j=0: svm_qp(1_000_000, 10_000, 0.01, 1000 * 4 + j),
}

# The three further classes of Section 7.1 at sizes of the same order (n + m ≈ 2·10⁵–6·10⁶,
# 10⁷–2·10⁷ entries of A); instance j uses seed 1000·i + j with i = 10, 11, 12.
MORE = {
    "control_large": lambda j=0: control_qp(2000, 1000, 30, 0.1, 1000 * 10 + j),
    "equality_large": lambda j=0: equality_qp(100_000, 50_000, 4.47e-5, 4e-4, 1000 * 11 + j),
    "huber_large": lambda j=0: huber_qp(10_000, 1_000_000, 1e-3, 1000 * 12 + j),
}

# Scaled-down variants with the same generators and per-row densities, sized so
# that the oracle's direct solve finishes in seconds.
SMALL = {
    "random_small": lambda j=0: random_qp(300, 600, 0.10, 0.10, 1000 * 5 + j),
    "lasso_small": lambda j=0: lasso_qp(200, 2_000, 0.05, 1000 * 6 + j),
    "random2_small": lambda j=0: random_qp(1_000, 10_000, 4.4e-3, 2e-2, 1000 * 7 + j),
    "portfolio_small": lambda j=0: portfolio_qp(2_000, 20, 0.5, 1000 * 8 + j),
    "svm_small": lambda j=0: svm_qp(4_000, 100, 0.1, 1000 * 9 + j),
    "control_small": lambda j=0: control_qp(20, 10, 10, 0.3, 1000 * 13 + j),
    "equality_small": lambda j=0: equality_qp(500, 250, 0.02, 0.02, 1000 * 14 + j),
    "huber_small": lambda j=0: huber_qp(100, 2_000, 0.05, 1000 * 15 + j),
}


def make(name: str, j: int = 0) -> QP:
    if name in WORKLOADS:
        return WORKLOADS[name](j)
    if name in MORE:
        return MORE[name](j)
    return SMALL[name](j)
