"""OSQP's ADMM (Algorithm 1, Section 3) with the direct KKT solve (eq. kkt).

Each iteration, on the Ruiz-scaled problem (Algorithm 2):
  1. solve  [P̄+σI  Āᵀ; Ā  −R⁻¹] [x̃; ν] = [σx − q̄; z − R⁻¹y]          (eq. kkt)
  2. z̃ = z + R⁻¹(ν − y)
  3. x ← αx̃ + (1−α)x
  4. z ← Π_[l̄,ū](αz̃ + (1−α)z + R⁻¹y)
  5. y ← y + R(αz̃ + (1−α)z − z_new)
and stops when the unscaled residuals meet the relative test of Section 3.1, or when the
iterate differences δx = x^k − x^{k−1}, δy = y^k − y^{k−1} certify infeasibility (Section 3,
Section 3.1; ``infeasibility``).

``linsys="pcg"`` replaces the direct solve by the route of Section 6.3: R = ρ̄I, the reduced
system (eq. kkt_red_sc) solved with Algorithm 3 (``oracle.pcg``) to a tight relative tolerance,
warm-started from the previous x̃, and z̃ = Āx̃. With an exact solve both routes produce the
same iterates; this mode only exists to time the method on the host at sizes the direct
factorisation cannot reach.

R is ρ̄I (the choice Section 6.3 makes for the GPU solver) or OSQP's vector
ρ_i = ρ̄ on inequalities and 10³ρ̄ on equalities (eq. rho_vec); the solution
does not depend on R. The KKT matrix is factored once and again only when ρ̄
changes (Section 3.2, 3.4). The sparse LU used for the factorisation is a
library primitive; no ordering or factorisation is re-implemented here (``dense_degree`` only
eliminates the densest rows last, by block elimination with the library's sparse and dense LU).

Scaled variables (Section 3.3): x̄ = D⁻¹x, ȳ = cE⁻¹y, and z̄ = Ez. (The paper
prints z̄ = E⁻¹z, which contradicts Ā = EAD and l̄ = El; z̄ = Āx̄ = EAx = Ez is
the consistent reading.) Unscaled residuals are r_prim = E⁻¹r̄_prim and
r_dual = c⁻¹D⁻¹r̄_dual.

ρ̄ estimate (Section 3.4 names only "the ratio of primal and dual residual
norms"): ρ̄·√[(‖r̄_p‖∞ / max(‖Āx̄‖∞, ‖z̄‖∞)) / (‖r̄_d‖∞ / max(‖P̄x̄‖∞, ‖Āᵀȳ‖∞, ‖q̄‖∞))]
on scaled quantities, clipped to [1e-6, 1e6]. Because every change costs a
refactorisation, the oracle applies it only when the estimate differs from
ρ̄ by more than a factor 5, and at most every ``rho_interval`` iterations.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ruiz as _ruiz

RHO_MIN, RHO_MAX = 1e-6, 1e6
INF = 1e20


def infeasibility(dx, dy, P_full, q, A, l, u, eps_pinf, eps_dinf, tiny=1e-30):
    """Infeasibility tests of Section 3.1 on the unscaled differences dx (n) and dy (m).

    Primal (certificate conditions of Section 2.1, Aᵀȳ = 0 and lᵀȳ₋ + uᵀȳ₊ < 0): dy is first
    projected so that no term of the support function is infinite (dy_i ≤ 0 where u_i = +∞,
    dy_i ≥ 0 where l_i = −∞); then ‖Aᵀdy‖∞ ≤ ε_pinf‖dy‖∞ and lᵀdy₋ + uᵀdy₊ < −ε_pinf‖dy‖∞,
    the infinite bounds contributing nothing.
    Dual (conditions Px̄ = 0, qᵀx̄ < 0 and the sign pattern of Ax̄): ‖P dx‖∞ ≤ ε_dinf‖dx‖∞,
    qᵀdx < −ε_dinf‖dx‖∞, and (A dx)_i within ±ε_dinf‖dx‖∞ for finite l_i and u_i, ≥ −ε_dinf‖dx‖∞
    for u_i = +∞, ≤ ε_dinf‖dx‖∞ for l_i = −∞.
    The tests are the paper's, with every tolerance relative to ‖δ‖∞ (the paper's are absolute;
    normalising makes them independent of how fast the iterates diverge). A test whose tolerance
    is 0 is skipped. Returns (status, certificate normalised to ‖·‖∞ = 1) or None.
    """
    l_inf = l <= -INF
    u_inf = u >= INF
    if eps_pinf > 0 and dy.size:
        d = np.where(u_inf, np.minimum(dy, 0.0), dy)
        d = np.where(l_inf, np.maximum(d, 0.0), d)
        nrm = float(np.max(np.abs(d)))
        if nrm > tiny:
            atd = A.T @ d
            support = float(np.sum(np.where(u_inf, 0.0, u) * np.maximum(d, 0.0))
                            + np.sum(np.where(l_inf, 0.0, l) * np.minimum(d, 0.0)))
            if float(np.max(np.abs(atd))) <= eps_pinf * nrm and support < -eps_pinf * nrm:
                return "primal_infeasible", d / nrm
    if eps_dinf > 0:
        nrm = float(np.max(np.abs(dx)))
        if nrm > tiny:
            tol = eps_dinf * nrm
            if float(np.max(np.abs(P_full @ dx))) <= tol and float(q @ dx) < -tol:
                adx = A @ dx
                ok = np.where(l_inf & u_inf, True,
                              np.where(u_inf, adx >= -tol,
                                       np.where(l_inf, adx <= tol, np.abs(adx) <= tol)))
                if bool(np.all(ok)):
                    return "dual_infeasible", dx / nrm
    return None


@dataclasses.dataclass
class AdmmResult:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    obj: float
    iters: int
    status: str
    prim_res: float
    dual_res: float
    rho: float
    rho_updates: int
    trace: list
    scaling: tuple
    factor_time: float = 0.0
    iter_time: float = 0.0
    certificate: np.ndarray | None = None  # normalised δy (primal) or δx (dual infeasibility)


def kkt_matrix(Pb, Ab, sigma, rvec):
    n = Pb.shape[0]
    return sp.bmat([[Pb + sigma * sp.identity(n), Ab.T],
                    [Ab, -sp.diags(1.0 / rvec)]], format="csc")


class KKTSolver:
    """Factor the quasi-definite KKT matrix once; solve many right-hand sides.

    With ``dense_degree`` = 0 the whole matrix goes to the library's sparse LU (its minimum-degree
    order on AᵀA + A, diagonal pivots). With ``dense_degree`` > 0 the nodes of more than that many
    neighbours (the dense rows of the portfolio class, 5·10⁴ and 10⁵ entries, on which the
    library's ordering and symbolic factorisation do not finish) are eliminated last, by block
    Gaussian elimination of the same matrix:
        K = [K_SS  K_SD; K_DS  K_DD],   C = K_DD − K_DS K_SS⁻¹ K_SD  (dense),
        K_SS u = r_S,  C x_D = r_D − K_DS u,  x_S = u − K_SS⁻¹ K_SD x_D,
    with K_SS by the library's sparse LU and C by a dense LU. Both are exact solves of eq. kkt up to
    round-off (quasi-definiteness makes K_SS and C nonsingular, Section 3.2)."""

    def __init__(self, Pb, Ab, sigma, rvec, dense_degree=0):
        K = kkt_matrix(Pb, Ab, sigma, rvec)
        self.K = K
        self.dense = None
        if dense_degree > 0:
            deg = np.diff(sp.csr_matrix(K).indptr)
            D = np.nonzero(deg > dense_degree)[0]
            if D.size:
                S = np.nonzero(deg <= dense_degree)[0]
                Kr = sp.csr_matrix(K)
                self.dense = (S, D)
                self.lu = self._splu(Kr[S][:, S].tocsc())
                K_SD = np.ascontiguousarray(Kr[S][:, D].toarray())
                self.K_DS = Kr[D][:, S].tocsr()
                self.W = np.ascontiguousarray(self.lu.solve(K_SD))   # K_SS⁻¹ K_SD, |S|×|D|
                C = Kr[D][:, D].toarray() - K_SD.T @ self.W          # K_DS = K_SDᵀ (K symmetric)
                del K_SD
                import scipy.linalg as sla
                self.C = sla.lu_factor(C)
                self._lu_solve_dense = sla.lu_solve
                return
        self.lu = self._splu(K)

    @staticmethod
    def _splu(K):
        try:
            lu = spla.splu(K, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                           options=dict(SymmetricMode=True))
            t = np.ones(K.shape[0])
            if not np.all(np.isfinite(lu.solve(t))):
                raise RuntimeError
            return lu
        except Exception:
            return spla.splu(K)

    def _solve_once(self, rhs):
        if self.dense is None:
            return self.lu.solve(rhs)
        S, D = self.dense
        u = self.lu.solve(rhs[S])
        xd = self._lu_solve_dense(self.C, rhs[D] - self.K_DS @ u)
        out = np.empty_like(rhs)
        out[D] = xd
        out[S] = u - self.W @ xd
        return out

    def solve(self, rhs):
        sol = self._solve_once(rhs)
        # one step of iterative refinement keeps the solve at round-off level
        return sol - self._solve_once(self.K @ sol - rhs)


class ReducedPCGSolver:
    """Exact-to-tolerance solve of eq. kkt via the reduced system and Algorithm 3 (R = ρ̄I)."""

    def __init__(self, Pb, Ab, sigma, rvec, tol):
        from . import pcg as _pcg
        self.n = Pb.shape[0]
        self.rho = float(rvec[0]) if rvec.size else 1.0
        self.A = sp.csr_matrix(Ab)
        self.At = self.A.T.tocsr()
        self.K = _pcg.reduced_kkt_matvec(Pb, Ab, sigma, self.rho)
        self.minv = 1.0 / _pcg.jacobi_diag(Pb, Ab, sigma, self.rho)
        self.sigma = sigma
        self.tol = tol
        self.xt = np.zeros(self.n)
        self.pcg_iters = 0
        self._pcg = _pcg.pcg

    def solve(self, rhs):
        # rhs = [σx − q̄; z − R⁻¹y]  ⇒  b = σx − q̄ + Āᵀ(ρ̄z − y) = rhs_x + ρ̄Āᵀ rhs_z
        b = rhs[:self.n] + self.rho * (self.At @ rhs[self.n:])
        self.xt, k, _, _ = self._pcg(self.K, b, self.xt, self.minv, self.tol, 10 * self.n + 100)
        self.pcg_iters += k
        zt = self.A @ self.xt
        # return (x̃, ν) with ν chosen so that z + R⁻¹(ν − y) = z̃, i.e. ν = ρ̄(z̃ − rhs_z)
        return np.concatenate([self.xt, self.rho * (zt - rhs[self.n:])])


def admm_step(kkt, qb, lb, ub, rvec, sigma, alpha, x, z, y):
    """One iteration of Algorithm 1 on the scaled problem."""
    n = x.shape[0]
    sol = kkt.solve(np.concatenate([sigma * x - qb, z - y / rvec]))
    xt = sol[:n]
    nu = sol[n:]
    zt = z + (nu - y) / rvec
    x_new = alpha * xt + (1.0 - alpha) * x
    v = alpha * zt + (1.0 - alpha) * z
    z_new = np.minimum(np.maximum(v + y / rvec, lb), ub)
    y_new = y + rvec * (v - z_new)
    return x_new, z_new, y_new


def rho_vector(l, u, rho_bar, mode):
    if mode == "scalar":
        return np.full(l.shape[0], rho_bar)
    eq = np.abs(u - l) < 1e-12 * np.maximum(1.0, np.abs(l))
    return np.where(eq, 1e3 * rho_bar, rho_bar)


def solve(P_full, q, A, l, u, *, rho=0.1, sigma=1e-6, alpha=1.6, eps_abs=1e-9, eps_rel=1e-9,
          max_iter=20000, scaling_iters=10, r_mode="scalar", adaptive_rho=True, rho_interval=100,
          check_every=1, record=0, x0=None, z0=None, y0=None, linsys="direct",
          pcg_tol=1e-12, eps_pinf=1e-4, eps_dinf=1e-4, progress=None, dense_degree=0) -> AdmmResult:
    """``progress``, if given, is called as progress(k, prim, dual, eps_prim, eps_dual, rho) after
    every residual check (reporting only; it does not change the iteration)."""
    import time

    P_full = sp.csr_matrix(P_full, dtype=np.float64)
    A = sp.csr_matrix(A, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    l = np.maximum(np.asarray(l, dtype=np.float64), -INF)
    u = np.minimum(np.asarray(u, dtype=np.float64), INF)
    n, m = A.shape[1], A.shape[0]

    if scaling_iters > 0:
        D, E, c, Pb, qb, Ab, _ = _ruiz.ruiz(P_full, q, A, scaling_iters)
    else:
        D, E, c, Pb, qb, Ab, _ = _ruiz.no_scaling(P_full, q, A)
    lb = E * l
    ub = E * u
    Abt = Ab.T.tocsr()

    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64) / D
    z = np.zeros(m) if z0 is None else E * np.asarray(z0, dtype=np.float64)
    y = np.zeros(m) if y0 is None else c * np.asarray(y0, dtype=np.float64) / E

    rho_bar = rho
    if linsys == "pcg":
        r_mode = "scalar"
    rvec = rho_vector(lb, ub, rho_bar, r_mode)

    def factor(rv):
        if linsys == "pcg":
            return ReducedPCGSolver(Pb, Ab, sigma, rv, pcg_tol)
        return KKTSolver(Pb, Ab, sigma, rv, dense_degree)

    t0 = time.perf_counter()
    kkt = factor(rvec)
    factor_time = time.perf_counter() - t0
    rho_updates = 0
    last_update = 0
    trace = []
    status = "max_iter_reached"
    it = 0
    pr = dr = np.inf
    t1 = time.perf_counter()
    cert = None
    for it in range(1, max_iter + 1):
        x_prev, y_prev = x, y
        x, z, y = admm_step(kkt, qb, lb, ub, rvec, sigma, alpha, x, z, y)
        if it <= record:
            trace.append((D * x, z / E, E * y / c))
        if it % check_every:
            continue
        Ax = Ab @ x
        Px = Pb @ x
        Aty = Abt @ y
        rp_s = Ax - z
        rd_s = Px + qb + Aty
        # unscaled residuals and normalisers
        pr = float(np.max(np.abs(rp_s / E))) if m else 0.0
        dr = float(np.max(np.abs(rd_s / D))) / c
        nAx = float(np.max(np.abs(Ax / E))) if m else 0.0
        nz = float(np.max(np.abs(z / E))) if m else 0.0
        nPx = float(np.max(np.abs(Px / D))) / c
        nAty = float(np.max(np.abs(Aty / D))) / c
        nq = float(np.max(np.abs(qb / D))) / c
        eps_p = eps_abs + eps_rel * max(nAx, nz)
        eps_d = eps_abs + eps_rel * max(nPx, nAty, nq)
        if progress is not None:
            progress(it, pr, dr, eps_p, eps_d, rho_bar)
        if pr <= eps_p and dr <= eps_d:
            status = "solved"
            break
        # unscaled differences: δx = D δx̄, δy = E δȳ / c
        found = infeasibility(D * (x - x_prev), E * (y - y_prev) / c, P_full, q, A, l, u,
                              eps_pinf, eps_dinf)
        if found is not None:
            status, cert = found
            break
        if adaptive_rho and it - last_update >= rho_interval:
            num = float(np.max(np.abs(rp_s))) / max(float(np.max(np.abs(Ax))) if m else 0.0,
                                                     float(np.max(np.abs(z))) if m else 0.0, 1e-10)
            den = float(np.max(np.abs(rd_s))) / max(float(np.max(np.abs(Px))), float(np.max(np.abs(Aty))),
                                                     float(np.max(np.abs(qb))), 1e-10)
            est = float(np.clip(rho_bar * np.sqrt(num / max(den, 1e-300)), RHO_MIN, RHO_MAX))
            if est > 5.0 * rho_bar or est < rho_bar / 5.0:
                rho_bar = est
                rvec = rho_vector(lb, ub, rho_bar, r_mode)
                t0 = time.perf_counter()
                prev = getattr(kkt, "xt", None)
                kkt = factor(rvec)
                if prev is not None:
                    kkt.xt = prev
                factor_time += time.perf_counter() - t0
                rho_updates += 1
                last_update = it
    iter_time = time.perf_counter() - t1
    xs = D * x
    ys = E * y / c
    zs = z / E
    obj = 0.5 * float(xs @ (P_full @ xs)) + float(q @ xs)
    return AdmmResult(xs, ys, zs, obj, it, status, pr, dr, rho_bar, rho_updates, trace,
                      (D, E, c), factor_time, iter_time, cert)
