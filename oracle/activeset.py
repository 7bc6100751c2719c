"""Brute-force solution of tiny QPs by active-set enumeration.

An independent route to the optimum of eq. (qp), used to pin the ADMM oracle:
every constraint is set inactive, active at l_i or active at u_i (equalities
l_i = u_i are always active). For each choice S the equality-constrained QP
    min ½xᵀPx + qᵀx  s.t.  A_S x = b_S
is solved through its KKT system [P A_Sᵀ; A_S 0][x; y_S] = [−q; b_S], and the
candidate is kept when it satisfies the optimality conditions of Section 2.1:
l ≤ Ax ≤ u and the sign rule of the multipliers (y_i ≥ 0 only at an upper
bound, y_i ≤ 0 only at a lower bound, y_i = 0 if inactive). With P ≻ 0 the
surviving x is unique.
"""
from __future__ import annotations

import itertools

import numpy as np

INF = 1e20


def solve(P, q, A, l, u, tol=1e-9):
    P = np.asarray(P, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n, m = A.shape[1], A.shape[0]
    choices = []
    for i in range(m):
        if abs(u[i] - l[i]) <= 0.0:
            choices.append(("eq",))
        else:
            c = ["free"]
            if l[i] > -INF:
                c.append("lo")
            if u[i] < INF:
                c.append("up")
            choices.append(tuple(c))
    best = None
    for combo in itertools.product(*choices):
        act = [i for i, s in enumerate(combo) if s != "free"]
        rhs_b = np.array([l[i] if combo[i] in ("lo", "eq") else u[i] for i in act])
        k = len(act)
        K = np.zeros((n + k, n + k))
        K[:n, :n] = P
        if k:
            As = A[act]
            K[:n, n:] = As.T
            K[n:, :n] = As
        rhs = np.concatenate([-q, rhs_b])
        try:
            sol = np.linalg.solve(K, rhs)
        except np.linalg.LinAlgError:
            continue
        if not np.all(np.isfinite(sol)) or np.max(np.abs(K @ sol - rhs)) > 1e-8 * (1 + np.max(np.abs(rhs))):
            continue
        x = sol[:n]
        y = np.zeros(m)
        y[act] = sol[n:]
        Ax = A @ x
        scale = 1.0 + np.max(np.abs(Ax)) if m else 1.0
        if np.any(Ax < l - tol * scale) or np.any(Ax > u + tol * scale):
            continue
        ok = True
        for i, s in enumerate(combo):
            if s == "lo" and y[i] > tol:
                ok = False
            if s == "up" and y[i] < -tol:
                ok = False
        if not ok:
            continue
        obj = 0.5 * x @ P @ x + q @ x
        if best is None or obj < best[2] - 1e-12:
            best = (x, y, obj)
    if best is None:
        raise RuntimeError("no KKT point found")
    return best
