"""Infeasibility detection (Section 3.1) of the HIP path against the oracle. Needs an MI355X.

Every instance here has a certificate direction that is unique up to a positive factor (the
closed forms below; the generators document theirs), so the normalised certificates are
compared with it directly, besides the status being compared with the oracle's. Tolerance:
a difference that passes the test at ε = 1e-4 still carries the not yet converged part of
δ^k, so the direction is compared to 1e-2 in ∞-norm.
"""
import functools
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import admm as o_admm
from paper_1912_04263_amd import problems as pr
from paper_1912_04263_amd import qpg

pytestmark = pytest.mark.gpu
INF = np.inf


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


# name: P (dense), q, A (dense), l, u, expected status, expected certificate
TINY = {
    "x_ge_1_and_x_le_0": ([[0.0]], [0.0], [[1.0], [1.0]], [1.0, -INF], [INF, 0.0], "primal_infeasible",
                          [-1.0, 1.0]),
    "contradicting_equalities": ([[1.0, 0.0], [0.0, 1.0]], [0.0, 0.0], [[1.0, 1.0], [1.0, 1.0]], [1.0, 2.0],
                                 [1.0, 2.0], "primal_infeasible", [1.0, -1.0]),
    "unbounded_ray": ([[1.0, 0.0], [0.0, 0.0]], [0.0, -1.0], [[0.0, 1.0]], [0.0], [INF], "dual_infeasible",
                      [0.0, 1.0]),
    "unbounded_lp_with_equality": ([[0.0, 0.0], [0.0, 0.0]], [-1.0, -1.0],
                                   [[1.0, -1.0], [1.0, 0.0], [0.0, 1.0]], [0.0, 0.0, 0.0],
                                   [0.0, INF, INF], "dual_infeasible", [1.0, 1.0]),
}


def _gpu(P_full, q, A, l, u, precision):
    P_triu = sp.triu(sp.csr_matrix(P_full), format="csc")
    with qpg.Solver(P_triu, q, sp.csc_matrix(A), l, u, precision=precision) as s:
        info = s.solve()
        dx, dy = s.certificate() if info.status.endswith("infeasible") else (None, None)
    return info, dx, dy


@pytest.mark.parametrize("precision", [qpg.QPG_FP64, qpg.QPG_MIXED])
@pytest.mark.parametrize("name", list(TINY))
def test_tiny_closed_form(name, precision):
    P, q, A, l, u, status, cert = TINY[name]
    say("infeasible tiny", name, "precision", precision)
    P, A = np.array(P), np.array(A)
    q, l, u = np.array(q), np.array(l), np.array(u)
    o = o_admm.solve(sp.csr_matrix(P), q, sp.csr_matrix(A), l, u, eps_abs=1e-3, eps_rel=1e-3, check_every=5)
    assert o.status == status
    info, dx, dy = _gpu(P, q, A, l, u, precision)
    assert info.status == status
    got = dy if status == "primal_infeasible" else dx
    np.testing.assert_allclose(got, cert, atol=1e-2)
    np.testing.assert_allclose(got, o.certificate, atol=1e-2)


CASES = {
    "primal_60x40": lambda: pr.primal_infeasible_qp(60, 40, 0.15, 7),
    "dual_60x80": lambda: pr.dual_infeasible_qp(60, 80, 0.15, 8),
    "primal_3000x2000": lambda: pr.primal_infeasible_qp(3000, 2000, 0.01, 11),
    "dual_3000x6000": lambda: pr.dual_infeasible_qp(3000, 6000, 0.01, 12),
}


@functools.lru_cache(maxsize=None)
def generated(name):
    qp = CASES[name]()
    o = o_admm.solve(qp.P_full(), qp.q, sp.csr_matrix(qp.A), qp.l, qp.u, eps_abs=1e-3, eps_rel=1e-3,
                     check_every=5, max_iter=4000)
    return qp, o


@pytest.mark.parametrize("precision", [qpg.QPG_FP64, qpg.QPG_MIXED])
@pytest.mark.parametrize("name", list(CASES))
def test_generated_instances(name, precision):
    say("infeasible generated", name, "precision", precision)
    qp, o = generated(name)
    kind = "primal" if name.startswith("primal") else "dual"
    assert o.status == kind + "_infeasible"
    info, dx, dy = _gpu(qp.P_full(), qp.q, qp.A, qp.l, qp.u, precision)
    assert info.status == o.status
    if kind == "primal":
        want = np.zeros(qp.m)
        want[list(qp.meta["rows"])] = [1.0, -1.0]
        got = dy
    else:
        want = np.zeros(qp.n)
        want[qp.meta["var"]] = 1.0
        got = dx
    np.testing.assert_allclose(got, want, atol=1e-2)
    np.testing.assert_allclose(got, o.certificate, atol=1e-2)


def test_certificate_of_a_solved_problem_is_refused():
    p = pr.make("random_c0")
    say("certificate refused on random_c0")
    with qpg.Solver.from_qp(p) as s:
        assert s.solve().status == "solved"
        with pytest.raises(qpg.QpgError) as e:
            s.certificate()
        assert e.value.code == qpg.QPG_ERR_STATE


def test_detection_off_runs_to_the_cap():
    P, q, A, l, u, _, _ = TINY["x_ge_1_and_x_le_0"]
    say("infeasibility tests off")
    with qpg.Solver(sp.csc_matrix(np.array(P)), np.array(q), sp.csc_matrix(np.array(A)), np.array(l),
                    np.array(u), eps_prim_inf=0.0, eps_dual_inf=0.0, max_iter=200) as s:
        assert s.solve().status == "max_iter_reached"
