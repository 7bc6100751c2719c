"""Pins of the learned-preconditioner side of the oracle (CPU only).

* The network's manual backward pass against central finite differences of its own loss.
* Hutchinson's estimator over all 2ⁿ sign vectors equals diag(K⁻¹) exactly (dense inverse).
* The initial network reproduces the Jacobi preconditioner exactly (softplus = 1).
* A plausible mistake (forgetting the mean removal in the loss gradient) fails the check.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hutchinson, mpnn
from oracle import pcg as o_pcg


def small_graph(seed, n=15, m=22, dens=0.35):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, random_state=seed, format="csr")
    A.data = rng.standard_normal(A.nnz)
    Mq = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.3)
    P = sp.csr_matrix(Mq @ Mq.T + 0.1 * np.eye(n))
    l = -rng.random(m)
    u = rng.random(m)
    u[:3] = l[:3]
    return P, A, l, u


def setup_inputs(seed, rho=0.3, sigma=1e-6):
    P, A, l, u = small_graph(seed)
    fv, fc, dP, colsq = mpnn.features(P, A, sigma, l, u)
    Ahat, Acheck = mpnn.graph(A)
    phi, K = mpnn.head_inputs(dP, colsq, sigma, rho)
    rng = np.random.default_rng(seed + 1)
    target = np.log(1.0 + rng.random(P.shape[0]))
    theta = mpnn.init_params(seed)
    # move off the Jacobi initialisation so that every layer carries gradient
    theta = theta + 0.3 * rng.standard_normal(theta.size)
    return theta, fv, fc, Ahat, Acheck, phi, target


def fd_check(theta, args, grad, idx, h=1e-4):
    fv, fc, Ahat, Acheck, phi, target = args
    errs = []
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        Lp, _, _ = mpnn.loss_grad(tp, fv, fc, Ahat, Acheck, phi, target)
        Lm, _, _ = mpnn.loss_grad(tm, fv, fc, Ahat, Acheck, phi, target)
        fd = (Lp - Lm) / (2 * h)
        errs.append(abs(fd - grad[i]) / max(1e-8, abs(fd), abs(grad[i])))
    return max(errs)


def test_backward_matches_central_differences():
    theta, fv, fc, Ahat, Acheck, phi, target = setup_inputs(1)
    L, grad, g = mpnn.loss_grad(theta, fv, fc, Ahat, Acheck, phi, target)
    rng = np.random.default_rng(2)
    big = np.nonzero(np.abs(grad) > 1e-4 * np.abs(grad).max())[0]
    idx = rng.choice(big, min(200, big.size), replace=False)
    assert fd_check(theta, (fv, fc, Ahat, Acheck, phi, target), grad, idx) < 1e-6
    # every parameter block receives gradient
    p = mpnn.unpack(grad)
    for name, v in p.items():
        if name.startswith("W") and name not in ("W_v0", "W_c0"):
            assert np.abs(v).max() > 0, name


def test_backward_matches_central_differences_far_in_the_softplus_tail():
    """Outputs g ≪ 0 (softplus ≈ e^g): the loss still depends smoothly on every parameter."""
    theta, fv, fc, Ahat, Acheck, phi, target = setup_inputs(4)
    p = mpnn.unpack(theta)
    p["b_h2"] = p["b_h2"] - 80.0
    theta = mpnn.pack(p)
    L, grad, g = mpnn.loss_grad(theta, fv, fc, Ahat, Acheck, phi, target)
    assert g.max() < -40
    idx = np.argsort(-np.abs(grad))[:60]
    assert np.abs(grad).max() > 0
    assert fd_check(theta, (fv, fc, Ahat, Acheck, phi, target), grad, idx) < 1e-6


def test_gradient_check_has_teeth(monkeypatch):
    theta, fv, fc, Ahat, Acheck, phi, target = setup_inputs(3)

    def no_mean_removal(g, tgt):
        s = mpnn.softplus(g)
        e = np.log(s) - tgt
        d = e - e.mean()
        return float(np.mean(d * d)), (2.0 / g.size) * e * mpnn.sigmoid(g) / s

    monkeypatch.setattr(mpnn, "loss_and_dg", no_mean_removal)
    L, grad, g = mpnn.loss_grad(theta, fv, fc, Ahat, Acheck, phi, target)
    monkeypatch.undo()
    idx = np.argsort(-np.abs(grad))[:40]
    assert fd_check(theta, (fv, fc, Ahat, Acheck, phi, target), grad, idx) > 1e-3


def test_initial_network_is_jacobi():
    P, A, l, u = small_graph(5)
    fv, fc, dP, colsq = mpnn.features(P, A, 1e-6, l, u)
    Ahat, Acheck = mpnn.graph(A)
    phi, K = mpnn.head_inputs(dP, colsq, 1e-6, 0.7)
    g, _ = mpnn.forward(mpnn.init_params(0), fv, fc, Ahat, Acheck, phi)
    np.testing.assert_allclose(mpnn.softplus(g), 1.0, rtol=1e-15)
    np.testing.assert_allclose(mpnn.softplus(g) / K, 1.0 / o_pcg.jacobi_diag(P, A, 1e-6, 0.7), rtol=1e-14)


@pytest.mark.parametrize("n", [3, 6, 10])
def test_hutchinson_exhaustive_is_exact(n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    K = B @ B.T + n * np.eye(n)
    Kinv = np.linalg.inv(K)
    h = hutchinson.estimate(lambda v: Kinv @ v, hutchinson.all_sign_vectors(n))
    np.testing.assert_allclose(h, np.diag(Kinv), rtol=1e-10)
    assert np.all(np.diag(Kinv) >= 1.0 / np.diag(K) * (1 - 1e-12))


def test_hutchinson_error_shrinks_with_probes():
    rng = np.random.default_rng(9)
    n = 60
    B = rng.standard_normal((n, n))
    K = B @ B.T + 5 * np.eye(n)
    Kinv = np.linalg.inv(K)
    err = []
    for s in (8, 512):
        z = rng.choice([-1.0, 1.0], size=(s, n))
        h = hutchinson.estimate(lambda v: Kinv @ v, z)
        err.append(np.sqrt(np.mean((h - np.diag(Kinv)) ** 2)))
    assert err[1] < err[0] / 4  # ≈ 1/√s: a factor 8 expected


# ------------------------------------------------------------ graph operators and node features
# A hand-worked example: 3 constraints × 4 variables, variable 2 in no constraint, row and
# column statistics all different from each other.
#        x0  x1  x2  x3
#  c0 [   1  -2   0   0 ]     |row| sums 3, 4, 7;  row degrees 2, 2, 3
#  c1 [   0   3   0  -1 ]     |col| sums 3, 6, 0, 5; column degrees 2, 3, 0, 2
#  c2 [   2  -1   0   4 ]
HAND_A = np.array([[1.0, -2.0, 0.0, 0.0], [0.0, 3.0, 0.0, -1.0], [2.0, -1.0, 0.0, 4.0]])
# Â_ji = |Ā_ji| / Σ_i |Ā_ji| (each constraint row divided by its |row| sum)
HAND_AHAT = np.array([[1 / 3, 2 / 3, 0, 0], [0, 3 / 4, 0, 1 / 4], [2 / 7, 1 / 7, 0, 4 / 7]])
# Ǎ_ij = |Ā_ji| / Σ_j |Ā_ji| (each variable's column divided by its |column| sum; x2 has none)
HAND_ACHECK = np.array([[1 / 3, 0, 2 / 3], [2 / 6, 3 / 6, 1 / 6], [0, 0, 0], [0, 1 / 5, 4 / 5]])
HAND_DP = np.array([2.0, 0.0, 1.0, 0.5])   # diag(P̄)
HAND_SIGMA = 0.5
HAND_L = np.array([0.0, 1.0, -np.inf])
HAND_U = np.array([0.0, 2.0, 3.0])          # c0 is an equality row
T = 1e-12
LOG = np.log
# variable i: log(P̄_ii + σ), log(Σ_j Ā_ji² + 1e-12), log(1 + degree), log(max_j |Ā_ji| + 1e-12)
#   column sums of squares 1+4 = 5, 4+9+1 = 14, 0, 1+16 = 17; column maxima 2, 3, 0, 4
HAND_FV = np.array([[LOG(2.5), LOG(5 + T), LOG(3.0), LOG(2 + T)],
                    [LOG(0.5), LOG(14 + T), LOG(4.0), LOG(3 + T)],
                    [LOG(1.5), LOG(T), LOG(1.0), LOG(T)],
                    [LOG(1.0), LOG(17 + T), LOG(3.0), LOG(4 + T)]])
# constraint j: log(Σ_i Ā_ji² + 1e-12), log(1 + degree), [l_j = u_j], log(max_i |Ā_ji| + 1e-12)
#   row sums of squares 1+4 = 5, 9+1 = 10, 4+1+16 = 21; row maxima 2, 3, 4
HAND_FC = np.array([[LOG(5 + T), LOG(3.0), 1.0, LOG(2 + T)],
                    [LOG(10 + T), LOG(3.0), 0.0, LOG(3 + T)],
                    [LOG(21 + T), LOG(4.0), 0.0, LOG(4 + T)]])


def hand_inputs():
    return sp.diags(HAND_DP).tocsr(), sp.csr_matrix(HAND_A)


def test_graph_operators_match_hand_worked_example():
    _, A = hand_inputs()
    Ahat, Acheck = mpnn.graph(A)
    np.testing.assert_allclose(Ahat.toarray(), HAND_AHAT, rtol=1e-15, atol=0)
    np.testing.assert_allclose(Acheck.toarray(), HAND_ACHECK, rtol=1e-15, atol=0)
    # invariants: rows of Â and Ǎ sum to 1 (0 for a node with no edge)
    np.testing.assert_allclose(np.asarray(Ahat.sum(axis=1)).ravel(), [1, 1, 1], rtol=1e-15)
    np.testing.assert_allclose(np.asarray(Acheck.sum(axis=1)).ravel(), [1, 1, 0, 1], rtol=1e-15)


def test_node_features_match_hand_worked_example():
    P, A = hand_inputs()
    fv, fc, dP, colsq = mpnn.features(P, A, HAND_SIGMA, HAND_L, HAND_U)
    assert fv.shape == (4, 32) and fc.shape == (3, 32)
    np.testing.assert_allclose(fv[:, :4], HAND_FV, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(fc[:, :4], HAND_FC, rtol=1e-14, atol=1e-14)
    assert not fv[:, 4:].any() and not fc[:, 4:].any()
    np.testing.assert_array_equal(dP, HAND_DP)
    np.testing.assert_array_equal(colsq, [5.0, 14.0, 0.0, 17.0])


def _graph_rows_for_check(Ab):
    """Planted mistake: Ǎ normalised by the constraint rows' sums (Âᵀ) instead of its own."""
    Aabs = abs(sp.csr_matrix(Ab)).tocsr()
    rs = np.asarray(Aabs.sum(axis=1)).ravel()
    rinv = np.divide(1.0, rs, out=np.zeros_like(rs), where=rs > 0)
    Ahat = (sp.diags(rinv) @ Aabs).tocsr()
    return Ahat, Ahat.T.tocsr()


def _features_swapped_axes(Pb, Ab, sigma, l, u):
    """Planted mistake: degrees and maxima of the variables taken over rows (square case)."""
    fv, fc, dP, colsq = mpnn.features(Pb, Ab, sigma, l, u)
    fv = fv.copy()
    fc = fc.copy()
    fv[:, 2], fc[:, 1] = fc[:, 1].copy(), fv[:, 2].copy()
    fv[:, 3], fc[:, 3] = fc[:, 3].copy(), fv[:, 3].copy()
    return fv, fc, dP, colsq


def _features_abs_not_squared(Pb, Ab, sigma, l, u):
    """Planted mistake: column norms summed from |Ā| instead of Ā²."""
    fv, fc, dP, colsq = mpnn.features(Pb, Ab, sigma, l, u)
    c1 = np.asarray(abs(sp.csr_matrix(Ab)).sum(axis=0)).ravel()
    fv = fv.copy()
    fv[:, 1] = np.log(c1 + 1e-12)
    return fv, fc, dP, colsq


def test_graph_pin_catches_rows_normalised_check_operator(monkeypatch):
    monkeypatch.setattr(mpnn, "graph", _graph_rows_for_check)
    _, A = hand_inputs()
    Ahat, Acheck = mpnn.graph(A)
    monkeypatch.undo()
    np.testing.assert_allclose(Ahat.toarray(), HAND_AHAT, rtol=1e-15)  # Â is unaffected
    assert not np.allclose(Acheck.toarray(), HAND_ACHECK, rtol=1e-6)


@pytest.mark.parametrize("mutant", [_features_abs_not_squared])
def test_feature_pin_catches_planted_mistakes(mutant):
    P, A = hand_inputs()
    fv, fc, _, _ = mutant(P, A, HAND_SIGMA, HAND_L, HAND_U)
    assert not (np.allclose(fv[:, :4], HAND_FV, rtol=1e-6) and np.allclose(fc[:, :4], HAND_FC, rtol=1e-6))


def test_feature_pin_catches_swapped_axes():
    """On a square Ā whose row and column statistics differ, taking a variable's degree and
    maximum over the rows instead of the columns changes the features (a shape error cannot hide
    the slip there)."""
    A = sp.csr_matrix(np.array([[1.0, 5.0, 0.0], [0.0, 0.0, 2.0], [3.0, 0.0, 0.0]]))
    P = sp.identity(3, format="csr")
    l = np.array([-1.0, -1.0, -1.0])
    u = np.array([1.0, 1.0, 1.0])
    fv, fc, _, _ = mpnn.features(P, A, 1e-6, l, u)
    # hand values: column degrees 2, 1, 1 and maxima 3, 5, 2; row degrees 2, 1, 1, maxima 5, 2, 3
    np.testing.assert_allclose(fv[:, 2], LOG([3.0, 2.0, 2.0]), rtol=1e-15)
    np.testing.assert_allclose(fv[:, 3], LOG(np.array([3.0, 5.0, 2.0]) + T), rtol=1e-15)
    np.testing.assert_allclose(fc[:, 3], LOG(np.array([5.0, 2.0, 3.0]) + T), rtol=1e-15)
    mv, mc, _, _ = _features_swapped_axes(P, A, 1e-6, l, u)
    assert not np.allclose(mv[:, 3], fv[:, 3])
