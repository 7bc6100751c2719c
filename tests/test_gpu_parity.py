"""Parity of the HIP path (through the C ABI) with the CPU oracle. Needs an MI355X.

Tolerances:
* SpMV FP64: max_i |Δ_i| / (|M||x|)_i ≤ 1e-12 (the device's reduction order costs at most
  ≈ rowlen·2⁻⁵³ relative to (|M||x|)_i; the oracle sums in extended precision).
* SpMV FP32: ≤ 1e-5 on the same scale (inputs rounded to 2⁻²⁴, accumulation in float).
* Final answer at eps_abs = eps_rel = 1e-5: |f − f*| ≤ 1e-4·max(1, |f*|) and
  ‖x − x*‖∞ ≤ 1e-3·‖x*‖∞ against the oracle run to 1e-9; the residuals of the returned point,
  recomputed in float64, within 1.01·eps (plus, in mixed precision, the forward error bound
  (k + 2)·2⁻²⁴·(|M||v|)_i of the float dot products the solver's own test used). Portfolio
  and control instances are compared at eps 1e-7: the method itself (the oracle's exact-solve
  ADMM) stopped at 1e-5 is 3.5e-4 (portfolio) and 2.3e-4 (control) off in objective on them, and
  stopped at 1e-6 portfolio is still ≈1e-3 off in x (measured: 0.98e-3 in FP64), so only a
  tighter stop separates implementation error from the method's own.
* Iterate trace with a near-exact PCG (fixed relative tolerance 1e-13) against the oracle's
  direct KKT solves: 1e-8 relative.
"""
import functools
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import admm as o_admm
from oracle import kkt as o_kkt
from oracle import pcg as o_pcg
from oracle import ruiz as o_ruiz
from oracle import spmv as o_spmv
from paper_1912_04263_amd import problems as pr
from paper_1912_04263_amd import qpg

pytestmark = pytest.mark.gpu

PROBLEMS = ["random_c0", "random_small", "lasso_small", "portfolio_small", "svm_small", "random2_small",
            "control_small", "equality_small", "huber_small"]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@functools.lru_cache(maxsize=None)
def problem(name):
    return pr.make(name)


@functools.lru_cache(maxsize=None)
def oracle_solution(name):
    p = problem(name)
    return o_admm.solve(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, eps_abs=1e-9, eps_rel=1e-9,
                        max_iter=50000)


def spmv_err(M, x, y):
    M = sp.csr_matrix(M)
    ref = o_spmv.spmv(M.indptr, M.indices, M.data, x)
    scale = o_spmv.spmv_abs(M.indptr, M.indices, M.data, x)
    d = np.abs(y - ref)
    zero = scale == 0
    assert np.all(d[zero] == 0)
    return float(np.max(d[~zero] / scale[~zero])) if np.any(~zero) else 0.0


def skewed_problem(seed=0):
    """Rows of length 0, 1, 7, 300, 3000 (one workgroup), 40000 (split into chunks)."""
    rng = np.random.default_rng(seed)
    n = 50000
    lens = [0, 1, 7, 300, 3000, 40000, 2, 0, 5] + [3] * 5000
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = np.sort(rng.choice(n, L, replace=False))
        rows.append(np.full(L, i))
        cols.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = sp.csc_matrix((rng.standard_normal(r.size), (r, c)), shape=(len(lens), n))
    d = rng.uniform(0.5, 2.0, n)
    P = sp.diags(d).tocsc()
    q = rng.standard_normal(n)
    m = len(lens)
    return P, q, A, -np.ones(m), np.ones(m)


# ------------------------------------------------------------------------------ SpMV
@pytest.mark.parametrize("name", PROBLEMS + ["skewed"])
def test_spmv_fp64_matches_oracle(name):
    say("spmv fp64", name)
    if name == "skewed":
        P, q, A, l, u = skewed_problem()
    else:
        p = problem(name)
        P, q, A, l, u = p.P_triu, p.q, p.A, p.l, p.u
    Pf = sp.csr_matrix(sp.triu(P) + sp.triu(P, 1).T)
    rng = np.random.default_rng(1)
    with qpg.Solver(P, q, A, l, u, scaling_iters=0) as s:
        x = rng.standard_normal(s.n)
        y = rng.standard_normal(s.m)
        assert spmv_err(A, x, s.apply(qpg.QPG_OP_A, x)) <= 1e-12
        assert spmv_err(sp.csr_matrix(A).T, y, s.apply(qpg.QPG_OP_AT, y)) <= 1e-12
        assert spmv_err(Pf, x, s.apply(qpg.QPG_OP_P, x)) <= 1e-12
        # bitwise reproducible
        assert np.array_equal(s.apply(qpg.QPG_OP_A, x), s.apply(qpg.QPG_OP_A, x))


@pytest.mark.parametrize("name", ["lasso_small", "skewed"])
def test_spmv_fp32_error_bound(name):
    say("spmv fp32", name)
    if name == "skewed":
        P, q, A, l, u = skewed_problem(2)
    else:
        p = problem(name)
        P, q, A, l, u = p.P_triu, p.q, p.A, p.l, p.u
    rng = np.random.default_rng(3)
    with qpg.Solver(P, q, A, l, u, scaling_iters=0, precision="mixed") as s:
        x = rng.standard_normal(s.n)
        assert spmv_err(A, x, s.apply(qpg.QPG_OP_A, x, qpg.QPG_MIXED)) <= 1e-5
        y = rng.standard_normal(s.m)
        assert spmv_err(sp.csr_matrix(A).T, y, s.apply(qpg.QPG_OP_AT, y, qpg.QPG_MIXED)) <= 1e-5


def scaled_data(s, p):
    D, E, c = s.scaling()
    Pb = (c * sp.diags(D) @ p.P_full() @ sp.diags(D)).tocsr()
    Ab = (sp.diags(E) @ sp.csr_matrix(p.A) @ sp.diags(D)).tocsr()
    return D, E, c, Pb, Ab


@pytest.mark.parametrize("name", ["random_c0", "lasso_small", "svm_small"])
def test_scaling_and_kkt_operator_match_oracle(name):
    say("ruiz + K operator", name)
    p = problem(name)
    with qpg.Solver.from_qp(p) as s:
        D, E, c, Pb, Ab = scaled_data(s, p)
        Do, Eo, co, *_ = o_ruiz.ruiz(p.P_full(), p.q, sp.csr_matrix(p.A), 10)
        np.testing.assert_allclose(D, Do, rtol=1e-12)
        np.testing.assert_allclose(E, Eo, rtol=1e-12)
        assert c == pytest.approx(co, rel=1e-12)
        s.set_rho(0.37)
        v = np.random.default_rng(4).standard_normal(s.n)
        K = o_pcg.reduced_kkt_matvec(Pb, Ab, 1e-6, 0.37)
        ref = K(v)
        got = s.apply(qpg.QPG_OP_K, v)
        scale = np.abs(Pb) @ np.abs(v) + 1e-6 * np.abs(v) + 0.37 * (abs(Ab).T @ (abs(Ab) @ np.abs(v)))
        assert np.max(np.abs(got - ref) / scale) <= 1e-11


# ------------------------------------------------------------------------------ PCG
@pytest.mark.parametrize("name", ["random_c0", "lasso_small", "portfolio_small"])
def test_pcg_matches_oracle(name):
    say("pcg", name)
    p = problem(name)
    with qpg.Solver.from_qp(p) as s:
        D, E, c, Pb, Ab = scaled_data(s, p)
        rho = 0.1
        s.set_rho(rho)
        b = np.random.default_rng(5).standard_normal(s.n)
        K = o_pcg.reduced_kkt_matvec(Pb, Ab, 1e-6, rho)
        minv = 1.0 / o_pcg.jacobi_diag(Pb, Ab, 1e-6, rho)
        for eps in (1e-3, 1e-8):
            xo, ko, rno, _ = o_pcg.pcg(K, b, np.zeros(s.n), minv, eps, 2000)
            xg, kg, rng_, broke = s.pcg(b, eps=eps, max_iter=2000)
            assert not broke
            assert abs(kg - ko) <= max(1, ko // 50), (kg, ko)
            assert rng_ <= eps * np.max(np.abs(b)) * (1 + 1e-6)
            if kg == ko:
                np.testing.assert_allclose(xg, xo, rtol=0, atol=1e-8 * np.max(np.abs(xo)))


def test_pcg_pins_on_gpu():
    say("pcg pins")
    rng = np.random.default_rng(6)
    n = 3000
    d = rng.uniform(0.5, 4.0, n)
    P = sp.diags(d).tocsc()
    A = sp.csc_matrix((0, n))
    with qpg.Solver(P, np.zeros(n), A, np.zeros(0), np.zeros(0), scaling_iters=0) as s:
        b = rng.standard_normal(n)
        x, k, rn, broke = s.pcg(b, eps=1e-14, max_iter=50)
        assert k == 1 and not broke  # diagonal K with the Jacobi preconditioner: one step
        np.testing.assert_allclose(x, b / (d + 1e-6), rtol=1e-14)
        x2, k2, _, _ = s.pcg(b, x0=x, eps=1e-12, max_iter=50)
        assert k2 == 0  # warm start at the solution


# ------------------------------------------------------------------------------ ADMM
@pytest.mark.parametrize("name", ["random_c0", "lasso_small"])
def test_admm_iterates_match_oracle_trace(name):
    say("admm trace", name)
    p = problem(name)
    K = 20
    ref = o_admm.solve(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, eps_abs=0.0, eps_rel=0.0,
                       max_iter=K, adaptive_rho=False, record=K)
    for k in (1, 2, 5, 20):
        st = qpg.default_settings(rho_update_every=0, pcg_eps_fixed=1e-13, pcg_max_iter=3000,
                                  check_every=10000, max_iter=k)
        with qpg.Solver.from_qp(p, settings=st) as s:
            s.solve()
            xk, zk, yk = ref.trace[k - 1]
            for got, want in ((s.x(), xk), (s.z(), zk), (s.y(), yk)):
                assert np.max(np.abs(got - want)) <= 1e-8 * max(1.0, np.max(np.abs(want))), k


@pytest.mark.parametrize("name", ["svm_small", "control_small"])
def test_admm_iterates_across_a_rho_update_match_oracle_trace(name):
    """ρ̄ changes at iteration 10 on both sides (Section 3.4). Iteration 1 forms its right-hand
    side directly; every later one from the previous solve's residual and right-hand side, and
    iteration 11 with the factor ρ̄_new/ρ̄_old; the iterates before and after must match."""
    say("admm trace across a rho update", name)
    p = problem(name)
    K = 20
    ref = o_admm.solve(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, eps_abs=0.0, eps_rel=0.0,
                       max_iter=K, adaptive_rho=True, rho_interval=10, record=K)
    assert ref.rho_updates == 1 and ref.rho != 0.1
    for k in (2, 10, 11, 15, 20):
        st = qpg.default_settings(rho_update_every=10, check_every=5, pcg_eps_fixed=1e-13,
                                  pcg_max_iter=5000, max_iter=k)
        with qpg.Solver.from_qp(p, settings=st) as s:
            info = s.solve()
            if 10 <= k < K:  # (the check at k = K may update ρ̄ again, after the iterate)
                assert info.rho_updates == 1
                assert abs(info.rho_final - ref.rho) <= 1e-9 * ref.rho
            xk, zk, yk = ref.trace[k - 1]
            for got, want in ((s.x(), xk), (s.z(), zk), (s.y(), yk)):
                assert np.max(np.abs(got - want)) <= 1e-8 * max(1.0, np.max(np.abs(want))), k


@pytest.mark.parametrize("name", ["lasso_small", "huber_small", "portfolio_small"])
def test_admm_iterates_with_vector_rho_match_oracle_trace(name):
    """R = diag(ρ_i), ρ_i = 10³ρ̄ on equality rows (eq. rho_vec): the GPU's K, Jacobi diagonal and
    updates against the oracle's direct solves with the same R."""
    say("admm trace, vector rho", name)
    p = problem(name)
    assert np.any(p.l == p.u)
    K = 10
    ref = o_admm.solve(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, eps_abs=0.0, eps_rel=0.0,
                       max_iter=K, adaptive_rho=False, record=K, r_mode="vector")
    for k in (1, 3, 10):
        st = qpg.default_settings(rho_update_every=0, pcg_eps_fixed=1e-13, pcg_max_iter=5000,
                                  check_every=10000, max_iter=k, rho_vector=1)
        with qpg.Solver.from_qp(p, settings=st) as s:
            s.solve()
            xk, zk, yk = ref.trace[k - 1]
            for got, want in ((s.x(), xk), (s.z(), zk), (s.y(), yk)):
                assert np.max(np.abs(got - want)) <= 1e-8 * max(1.0, np.max(np.abs(want))), k


@pytest.mark.parametrize("name", ["lasso_small", "equality_small"])
def test_vector_rho_operator_and_final_answer(name):
    say("vector rho operator + answer", name)
    p = problem(name)
    ref = oracle_solution(name)
    with qpg.Solver.from_qp(p, eps_abs=1e-5, eps_rel=1e-5, max_iter=20000, rho_vector=1) as s:
        D, E, c, Pb, Ab = scaled_data(s, p)
        s.set_rho(0.37)
        eq = (p.l == p.u).astype(float)
        r = 0.37 * (1.0 + 999.0 * eq)
        v = np.random.default_rng(7).standard_normal(s.n)
        want = Pb @ v + 1e-6 * v + Ab.T @ (r * (Ab @ v))
        got = s.apply(qpg.QPG_OP_K, v)
        scale = np.abs(Pb) @ np.abs(v) + 1e-6 * np.abs(v) + abs(Ab).T @ (r * (abs(Ab) @ np.abs(v)))
        assert np.max(np.abs(got - want) / scale) <= 1e-11
        info = s.solve()
        assert info.status == "solved"
        assert abs(info.obj_val - ref.obj) <= 1e-4 * max(1.0, abs(ref.obj))
        assert np.max(np.abs(s.x() - ref.x)) <= 1e-3 * np.max(np.abs(ref.x))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", PROBLEMS)
def test_final_answer_matches_oracle(name, precision):
    say("final answer", name, precision)
    p = problem(name)
    ref = oracle_solution(name)
    assert ref.status == "solved"
    eps = 1e-7 if name.startswith(("portfolio", "control")) else 1e-5
    with qpg.Solver.from_qp(p, eps_abs=eps, eps_rel=eps, max_iter=20000, precision=precision) as s:
        info = s.solve()
        assert info.status == "solved", info
        x = s.x()
        fs = ref.obj
        assert abs(info.obj_val - fs) <= 1e-4 * max(1.0, abs(fs))
        assert np.max(np.abs(x - ref.x)) <= 1e-3 * np.max(np.abs(ref.x))
        # the reported objective is the objective of the returned x
        f = o_kkt.objective(p.P_full(), p.q, x)
        assert abs(f - info.obj_val) <= 1e-6 * max(1.0, abs(f))
        y, z = s.y(), s.z()
        rep = o_kkt.kkt_report(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, x, y, z)
        eps_p = eps + eps * max(rep["norms"]["Ax"], rep["norms"]["z"])
        eps_d = eps + eps * max(rep["norms"]["Px"], rep["norms"]["Aty"], rep["norms"]["q"])
        slack_p = slack_d = 0.0
        if precision == "mixed":
            # the solver's own residuals are float sums of float products: the exact residual of
            # the returned point may exceed them by the dot-product bound (k + 2)·2⁻²⁴·(|M||v|)_i
            A = sp.csr_matrix(p.A)
            P = sp.csr_matrix(p.P_full())
            u = 2.0 ** -24
            kA = np.diff(A.indptr) + 2
            kB = np.diff(P.indptr) + np.diff(sp.csc_matrix(A).indptr) + 2
            slack_p = float(np.max(u * kA * (abs(A) @ np.abs(x) + np.abs(z)))) if p.m else 0.0
            slack_d = float(np.max(u * kB * (abs(P) @ np.abs(x) + abs(A).T @ np.abs(y) + np.abs(p.q))))
        assert rep["prim"] <= 1.01 * eps_p + slack_p and rep["dual"] <= 1.01 * eps_d + slack_d
        # z and the scaled bounds are held in float in mixed precision
        box_tol = 1e-6 if precision == "mixed" else 1e-9
        assert rep["box"] <= box_tol * (1 + rep["norms"]["z"])


def test_closed_form_box_on_gpu():
    say("closed form box")
    rng = np.random.default_rng(31)
    n = 5000
    pd = rng.uniform(0.1, 5, n)
    q = rng.standard_normal(n) * 3
    l, u = -rng.random(n), rng.random(n)
    with qpg.Solver(sp.diags(pd).tocsc(), q, sp.identity(n, format="csc"), l, u, eps_abs=1e-9,
                    eps_rel=1e-9, pcg_eps_min=1e-13, max_iter=20000) as s:
        assert s.solve().status == "solved"
        x = np.clip(-q / pd, l, u)
        np.testing.assert_allclose(s.x(), x, atol=1e-7)
        np.testing.assert_allclose(s.y(), -(pd * x + q), atol=1e-7)


def test_unconstrained_without_constraints():
    say("m = 0")
    p = problem("random_c0")
    n = p.n
    with qpg.Solver(p.P_triu, p.q, sp.csc_matrix((0, n)), np.zeros(0), np.zeros(0), eps_abs=1e-9,
                    eps_rel=1e-9, pcg_eps_min=1e-13, max_iter=20000) as s:
        assert s.solve().status == "solved"
        P = p.P_full().toarray()
        np.testing.assert_allclose(s.x(), -np.linalg.solve(P, p.q), rtol=1e-6, atol=1e-6)


def test_verbose_reports_setup_phases_and_checks(capfd):
    say("verbose output")
    p = problem("lasso_small")
    with qpg.Solver.from_qp(p, verbose=1, max_iter=5) as s:
        s.solve()
    err = capfd.readouterr().err
    for phase in ("host checks", "A in CSR (host)", "index uploads", "value uploads", "equilibration (device)", "work lists",
                  "work-list uploads", "values into SELL order", "vectors, preconditioner"):
        assert f"qpg setup  {phase}" in err, phase
    assert "qpg     5  prim" in err


def test_repeat_solves_are_bitwise_identical():
    say("determinism")
    p = problem("lasso_small")
    with qpg.Solver.from_qp(p) as s:
        i1 = s.solve()
        x1, y1 = s.x(), s.y()
        i2 = s.solve()
        assert np.array_equal(x1, s.x()) and np.array_equal(y1, s.y())
        assert i1.iter == i2.iter and i1.pcg_iter_total == i2.pcg_iter_total


def sampled_spmv_check(p, rows=200, seed=7):
    """Sampled rows of Ā x, Āᵀ y, P x against exact rational row sums (unscaled data)."""
    rng = np.random.default_rng(seed)
    A = sp.csr_matrix(p.A)
    At = sp.csr_matrix(p.A.T)
    Pf = p.P_full()
    with qpg.Solver.from_qp(p, scaling_iters=0) as s:
        x = rng.standard_normal(s.n)
        y = rng.standard_normal(s.m)
        for M, v, op in ((A, x, qpg.QPG_OP_A), (At, y, qpg.QPG_OP_AT), (Pf, x, qpg.QPG_OP_P)):
            out = s.apply(op, v)
            for i in rng.choice(M.shape[0], min(rows, M.shape[0]), replace=False):
                a, b = M.indptr[i], M.indptr[i + 1]
                ex = o_spmv.row_exact(M.indptr, M.indices, M.data, v, i)
                sc = float(np.abs(M.data[a:b]) @ np.abs(v[M.indices[a:b]]))
                assert abs(out[i] - ex) <= 1e-12 * sc, (op, i)


def kkt_certificate(p, eps, **kw):
    """The optimality conditions (eq. opt_cond) at the returned point, measured by the oracle on the
    unscaled data:
    * primal and dual residuals within the termination test (1.01·eps_prim, 1.01·eps_dual);
    * l ≤ z ≤ u, and complementarity y₋ᵀ(z − l) = y₊ᵀ(z − u) = 0, up to the rounding of the
      projection (z is a projection and y changes sign only where z sits on a bound): 1e-9
      relative in FP64, 1e-6 in mixed precision (z and the bounds held in float);
    * no multiplier on an infinite bound;
    * the duality gap xᵀPx + qᵀx + uᵀy₊ + lᵀy₋, which equals xᵀr_dual − yᵀr_prim when
      complementarity holds exactly, within ‖x‖₁·eps_dual + ‖y‖₁·eps_prim (with the same 1%
      slack and a rounding term);
    * the reported objective equal to ½xᵀPx + qᵀx of the returned x."""
    with qpg.Solver.from_qp(p, eps_abs=eps, eps_rel=eps, max_iter=40000, **kw) as s:
        info = s.solve()
        say("full size", p.name, kw, info)
        assert info.status == "solved"
        x, y, z = s.x(), s.y(), s.z()
        rep = o_kkt.kkt_report(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, x, y, z)
        eps_p = eps + eps * max(rep["norms"]["Ax"], rep["norms"]["z"])
        eps_d = eps + eps * max(rep["norms"]["Px"], rep["norms"]["Aty"], rep["norms"]["q"])
        say("certificate", p.name, {k: v for k, v in rep.items() if k != "norms"})
        assert rep["prim"] <= 1.01 * eps_p and rep["dual"] <= 1.01 * eps_d
        rnd = 1e-6 if kw.get("precision") == "mixed" else 1e-9
        zs = max(1.0, float(np.max(np.abs(z))) if z.size else 1.0)
        ys = max(1.0, float(np.max(np.abs(y))) if y.size else 1.0)
        assert rep["box"] <= rnd * zs
        assert rep["comp"] <= rnd * zs * ys
        assert rep["inf_mult"] <= rnd * ys
        gap_tol = 1.01 * (float(np.sum(np.abs(x))) * eps_d + float(np.sum(np.abs(y))) * eps_p) \
            + rnd * zs * float(np.sum(np.abs(y))) + 1e-9 * max(1.0, abs(rep["obj"]))
        assert rep["gap"] <= gap_tol, (rep["gap"], gap_tol)
        assert abs(info.obj_val - rep["obj"]) <= 1e-6 * max(1.0, abs(rep["obj"]))
        return info, rep


def test_full_size_lasso_sampled_spmv_and_kkt_certificate():
    """The bench workload at full size (Ad 100000×10000, 1%): sampled rows of every SpMV against
    exact row sums, and the optimality certificate of the returned solution."""
    say("lasso full size")
    p = problem("lasso_c1")
    rng = np.random.default_rng(7)
    with qpg.Solver.from_qp(p, eps_abs=1e-5, eps_rel=1e-5, scaling_iters=0) as s:
        A = sp.csr_matrix(p.A)
        At = sp.csr_matrix(p.A.T)
        x = rng.standard_normal(s.n)
        y = rng.standard_normal(s.m)
        ax = s.apply(qpg.QPG_OP_A, x)
        aty = s.apply(qpg.QPG_OP_AT, y)
        for i in rng.choice(s.m, 300, replace=False):
            ex = o_spmv.row_exact(A.indptr, A.indices, A.data, x, i)
            sc = float(np.abs(A[i].data) @ np.abs(x[A[i].indices])) if A[i].nnz else 0.0
            assert abs(ax[i] - ex) <= 1e-12 * sc
        for i in rng.choice(s.n, 300, replace=False):
            ex = o_spmv.row_exact(At.indptr, At.indices, At.data, y, i)
            sc = float(np.abs(At[i].data) @ np.abs(y[At[i].indices])) if At[i].nnz else 0.0
            assert abs(aty[i] - ex) <= 1e-12 * sc
    with qpg.Solver.from_qp(p, eps_abs=1e-5, eps_rel=1e-5, max_iter=20000) as s:
        info = s.solve()
        say("lasso full size solve", info)
        assert info.status == "solved"
        rep = o_kkt.kkt_report(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, s.x(), s.y(), s.z())
        eps_p = 1e-5 + 1e-5 * max(rep["norms"]["Ax"], rep["norms"]["z"])
        eps_d = 1e-5 + 1e-5 * max(rep["norms"]["Px"], rep["norms"]["Aty"], rep["norms"]["q"])
        assert rep["prim"] <= 1.01 * eps_p and rep["dual"] <= 1.01 * eps_d


@pytest.mark.slow
@pytest.mark.parametrize("name, eps, kw", [
    ("random_c2", 1e-5, {}),
    ("portfolio_c3", 1e-6, {}),
    ("svm_c4", 1e-5, {}),
    ("svm_c4", 1e-5, {"precision": "mixed"}),
])
def test_full_size_sampled_spmv_and_kkt_certificate(name, eps, kw):
    """The remaining benchmark workloads at full size: sampled SpMV rows against exact sums, and
    the optimality certificate (primal and dual residuals within the termination test, measured
    by the oracle on the unscaled data) of the returned solution."""
    say("full size", name, kw)
    p = problem(name)
    if not kw:
        sampled_spmv_check(p, rows=100)
    kkt_certificate(p, eps, **kw)


@pytest.mark.parametrize("name", ["lasso_small", "huber_small"])
def test_pcg_tolerance_schedule_final_answer(name):
    """The ε(k) schedule (settings.pcg_eps_schedule = 1) changes only how accurately each step is
    solved: the final answer still matches the oracle."""
    say("eps schedule", name)
    p = problem(name)
    ref = oracle_solution(name)
    with qpg.Solver.from_qp(p, eps_abs=1e-5, eps_rel=1e-5, max_iter=20000, pcg_eps_schedule=1) as s:
        info = s.solve()
        assert info.status == "solved"
        assert abs(info.obj_val - ref.obj) <= 1e-4 * max(1.0, abs(ref.obj))
        assert np.max(np.abs(s.x() - ref.x)) <= 1e-3 * np.max(np.abs(ref.x))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_is_bitwise_reproducible(precision):
    """Speculative ADMM iterations (launched between checks without waiting for the host) and
    the resumption after a PCG solve that needs more iterations than predicted leave the result
    independent of timing: two solves agree bitwise."""
    say("reproducible solve", precision)
    p = problem("lasso_small")
    with qpg.Solver.from_qp(p, eps_abs=1e-6, eps_rel=1e-6, max_iter=20000, precision=precision) as s:
        i1 = s.solve()
        x1, y1 = s.x(), s.y()
        i2 = s.solve()
        assert (i1.iter, i1.pcg_iter_total) == (i2.iter, i2.pcg_iter_total)
        assert np.array_equal(x1, s.x()) and np.array_equal(y1, s.y())


def _edge_qp(seed):
    """Small random QPs with the structure the kernels special-case: empty rows and columns of A,
    an all-zero P column (a variable only in constraints), equality rows, one-sided and free
    bounds, and rows much longer than the others."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(20, 300))
    m = int(rng.integers(4, 400))
    M = sp.random(n, n, density=float(rng.uniform(0.01, 0.2)), random_state=rng, format="csr")
    P = (M @ M.T + 1e-2 * sp.identity(n)).tolil()
    j = int(rng.integers(n - 1))
    P[j, :] = 0.0
    P[:, j] = 0.0
    P = P.tocsr()
    A = sp.random(m, n, density=float(rng.uniform(0.005, 0.1)), random_state=rng, format="lil")
    A[0, :] = 0.0                                        # empty row
    A[1, :] = rng.standard_normal(n)                     # a full row
    A[:, n - 1] = 0.0                                    # empty column (kept bounded by P)
    A[m - 1, :] = 0.0
    A[m - 1, j] = 1.0                                    # the P-free variable, bounded in [0, 1]
    A = A.tocsr()
    q = rng.standard_normal(n)
    l = -rng.random(m) - 0.1
    u = rng.random(m) + 0.1
    eq = rng.random(m) < 0.1
    l[eq] = u[eq] = 0.0                                  # equality rows
    free = rng.random(m) < 0.1
    l[free] = -np.inf                                    # one-sided rows
    l[m - 1], u[m - 1] = 0.0, 1.0
    return sp.triu(P, format="csc"), q, sp.csc_matrix(A), l, u


@pytest.mark.parametrize("seed", range(8))
def test_edge_structure_final_answers(seed):
    P_triu, q, A, l, u = _edge_qp(seed)
    say("edge structure", seed, A.shape)
    Pf = sp.csr_matrix(P_triu + sp.triu(P_triu, 1).T)
    ref = o_admm.solve(Pf, q, sp.csr_matrix(A), l, u, eps_abs=1e-9, eps_rel=1e-9, max_iter=50000)
    assert ref.status == "solved"
    for precision in ("fp64", "mixed"):
        with qpg.Solver(P_triu, q, A, l, u, eps_abs=1e-6, eps_rel=1e-6, max_iter=20000, precision=precision) as s:
            info = s.solve()
            assert info.status == "solved", (precision, info)
            assert abs(info.obj_val - ref.obj) <= 1e-4 * max(1.0, abs(ref.obj)), precision
            assert np.max(np.abs(s.x() - ref.x)) <= 1e-3 * max(1.0, np.max(np.abs(ref.x))), precision


def test_mixed_precision_falls_back_to_fp64_on_stagnation():
    """eps 1e-9 is out of FP32's reach: after 20 checks without progress the solve continues in
    FP64 from the FP32 iterates and ends at the oracle's answer."""
    say("fallback: stagnation")
    p = problem("lasso_small")
    ref = oracle_solution("lasso_small")
    with qpg.Solver.from_qp(p, eps_abs=1e-9, eps_rel=1e-9, max_iter=20000, precision="mixed",
                            pcg_eps_min=1e-12) as s:
        info = s.solve()
        assert info.fallback_events == 1 and info.precision_used == "fp64"
        assert info.status == "solved"
        assert np.max(np.abs(s.x() - ref.x)) <= 1e-6 * max(1.0, np.max(np.abs(ref.x)))


def test_mixed_precision_falls_back_after_three_capped_pcg_solves():
    """A PCG cap of one iteration under a fixed tight tolerance caps every solve; in FP32 the
    third capped solve in a row (seen by the host through the speculation's abort flag) moves the
    solve to FP64, which keeps going with capped solves."""
    say("fallback: capped PCG")
    p = problem("random_c0")
    with qpg.Solver.from_qp(p, precision="mixed", pcg_max_iter=1, pcg_eps_fixed=1e-12, max_iter=400) as s:
        info = s.solve()
        assert info.fallback_events == 1 and info.precision_used == "fp64"
        assert info.iter >= 3 and info.pcg_iter_max == 1
        # the iteration that requested the fallback runs again in FP64
        assert info.pcg_iter_total <= info.iter + info.fallback_events


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_indefinite_p_ends_in_a_numerical_error(precision):
    """With P negative definite, pᵀKp < 0 in the first PCG step: a breakdown, reported as a
    status (after the FP64 retry in mixed precision) rather than a wrong answer."""
    say("pcg breakdown", precision)
    n = 50
    P = sp.diags(np.full(n, -10.0)).tocsc()
    rng = np.random.default_rng(8)
    with qpg.Solver(P, rng.standard_normal(n), sp.identity(n, format="csc"), -np.ones(n), np.ones(n),
                    precision=precision, scaling_iters=0) as s:
        info = s.solve()
        assert info.status == "numerical_error"
        assert info.fallback_events == (1 if precision == "mixed" else 0)


@pytest.mark.parametrize("passes", [0, 1, 3])
@pytest.mark.parametrize("name", ["svm_small", "portfolio_small", "huber_small"])
def test_device_equilibration_pass_by_pass(name, passes):
    """Ruiz equilibration on the device (Algorithm 2) after 0, 1 and 3 passes against the oracle's,
    including the pass count, and the equilibrated matrices themselves through the operators."""
    say("device ruiz", name, passes)
    p = problem(name)
    Do, Eo, co, Pbo, qbo, Abo, npass = o_ruiz.ruiz(p.P_full(), p.q, sp.csr_matrix(p.A), passes)
    with qpg.Solver.from_qp(p, scaling_iters=passes) as s:
        D, E, c = s.scaling()
        np.testing.assert_allclose(D, Do, rtol=1e-12)
        np.testing.assert_allclose(E, Eo, rtol=1e-12)
        assert c == pytest.approx(co, rel=1e-12)
        assert s.info().scaling_passes == npass
        v = np.random.default_rng(9).standard_normal(s.n)
        for op, M in ((qpg.QPG_OP_A, Abo), (qpg.QPG_OP_P, Pbo)):
            got = s.apply(op, v)
            scale = np.abs(M) @ np.abs(v)
            assert np.max(np.abs(got - M @ v) / np.maximum(scale, 1e-300)) <= 1e-11
