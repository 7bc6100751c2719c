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
