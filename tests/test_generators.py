"""Seeded input generators: shapes, densities, value distributions, reproducibility."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1912_04263_amd import problems as pr


def test_bernoulli_pattern_density_and_moments():
    rng = np.random.default_rng(0)
    M = pr.sprandn(rng, 2000, 500, 0.02)
    assert M.nnz == pytest.approx(2000 * 500 * 0.02, rel=0.03)
    assert abs(M.data.mean()) < 0.03 and M.data.std() == pytest.approx(1.0, rel=0.03)
    M.sum_duplicates()
    assert M.has_sorted_indices
    counts = np.diff(M.indptr)  # Binomial(500, 0.02) per row
    assert counts.mean() == pytest.approx(10.0, rel=0.05)
    assert counts.var() == pytest.approx(500 * 0.02 * 0.98, rel=0.15)


def test_reproducible_and_seed_dependent():
    a, b, c = pr.make("random_c0", 0), pr.make("random_c0", 0), pr.make("random_c0", 1)
    assert (a.A != b.A).nnz == 0 and np.array_equal(a.q, b.q)
    assert not np.array_equal(a.q, c.q)


@pytest.mark.parametrize("name", list(pr.SMALL) + ["random_c0"])
def test_problem_structure(name):
    p = pr.make(name)
    assert p.P_triu.shape == (p.n, p.n) and p.A.shape == (p.m, p.n)
    T = p.P_triu.tocoo()
    assert np.all(T.row <= T.col)
    assert np.all(p.l <= p.u)
    P = p.P_full().toarray() if p.n <= 5000 else None
    if P is not None:
        assert np.allclose(P, P.T)
        assert np.linalg.eigvalsh(P).min() > -1e-9
    assert p.P_triu.indices.dtype == np.int32 and p.A.indptr.dtype == np.int32


def test_lasso_structure():
    p = pr.lasso_qp(50, 400, 0.1, 9)
    n, m = 50, 400
    assert p.n == 2 * n + m and p.m == m + 2 * n
    # P = blkdiag(0, 2I, 0); equality rows first, then −t ≤ x ≤ t
    d = p.P_full().diagonal()
    assert np.all(d[:n] == 0) and np.all(d[n:n + m] == 2) and np.all(d[n + m:] == 0)
    assert np.array_equal(p.l[:m], p.u[:m])
    assert np.all(np.isinf(p.l[m:m + n])) and np.all(np.isinf(p.u[m + n:]))


def test_svm_labels_and_means():
    p = pr.svm_qp(4000, 100, 0.2, 3)
    N = 4000
    Ad = sp.csr_matrix(p.A)[:N, :100]
    # rows are diag(b)·Ad, whose entries then all have mean +1/n_feat
    assert Ad.data.mean() == pytest.approx(1.0 / 100, rel=0.1)
    assert np.all(p.u[:N] == -1.0) and np.all(p.l[N:] == 0.0)


def test_infeasible_generators_structure():
    p = pr.primal_infeasible_qp(60, 40, 0.15, 7)
    i, j = p.meta["rows"]
    A = p.A.tocsr()
    assert (A[i] != A[j]).nnz == 0 and A[i].nnz > 0
    assert (p.l[i], p.u[i], p.l[j], p.u[j]) == (1.0, 2.0, 3.0, 4.0)
    assert np.linalg.matrix_rank(A.toarray()) == p.m - 1  # independent rows apart from the copy
    d = pr.dual_infeasible_qp(60, 80, 0.15, 8)
    v = d.meta["var"]
    assert d.P_full()[:, v].nnz == 0 and d.q[v] == -1.0
    col = d.A.tocsc()[:, v]
    assert col.nnz == 1 and col.indices[0] == d.m - 1 and d.l[-1] == 0.0 and d.u[-1] == np.inf
    assert np.linalg.eigvalsh(np.delete(np.delete(d.P_full().toarray(), v, 0), v, 1)).min() > 0


def test_control_instances_are_feasible_with_zero_input():
    p = pr.control_qp(20, 10, 10, 0.3, 5)
    nx, nu, T = 20, 10, 10
    A = p.A.tocsr()
    # u = 0: propagate x with the dynamics rows themselves (x_{t+1} solves row block t + 1)
    x = np.zeros(p.n)
    x[:nx] = p.l[:nx]
    Ad = -A[nx:2 * nx, :nx].toarray()  # rows x_1 − A x_0
    for t in range(T):
        x[(t + 1) * nx:(t + 2) * nx] = Ad @ x[t * nx:(t + 1) * nx]
    Ax = A @ x
    assert np.all(Ax >= p.l - 1e-12) and np.all(Ax <= p.u + 1e-12)
    assert p.P_full().shape == (p.n, p.n) and np.all(p.P_full().diagonal() >= 0)


def test_huber_qp_objective_is_the_huber_loss():
    p = pr.huber_qp(30, 200, 0.2, 6)
    n, m, M = 30, 200, p.meta["M"]
    rng = np.random.default_rng(0)
    x = rng.standard_normal(n)
    A = p.A.tocsr()
    v = A[:m, :n] @ x - p.l[:m]  # residuals a_iᵀx − b_i
    w = np.clip(v, -M, M)
    r = np.maximum(v - M, 0.0)
    s = np.maximum(-v - M, 0.0)
    z = np.concatenate([x, w, r, s])
    Az = A @ z
    assert np.allclose(Az[:m], p.l[:m]) and np.all(Az[m:] >= 0)
    obj = 0.5 * z @ (p.P_full() @ z) + p.q @ z
    huber = np.where(np.abs(v) <= M, v ** 2, M * (2 * np.abs(v) - M))
    assert obj == pytest.approx(huber.sum(), rel=1e-12)


def test_equality_instances_are_consistent():
    p = pr.equality_qp(500, 250, 0.02, 0.02, 7)
    assert np.array_equal(p.l, p.u)
    x, *_ = np.linalg.lstsq(p.A.toarray(), p.l, rcond=None)
    assert np.allclose(p.A @ x, p.l, atol=1e-8)
