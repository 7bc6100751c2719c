"""Objective, residuals and optimality conditions of the QP (Section 2.1, 3.1).

Optimality (eq. opt_cond): Ax − z = 0; Px + q + Aᵀy = 0; l ≤ z ≤ u;
y₋ᵀ(z − l) = 0 and y₊ᵀ(z − u) = 0, with y₊ = max(y, 0), y₋ = min(y, 0).
Residuals (Section 3.1): r_prim = Ax − z, r_dual = Px + q + Aᵀy.
Relative tolerances (the paper only says they are relative to the iterate
scale; OSQP's published form is used):
    ε_prim = ε_abs + ε_rel·max(‖Ax‖∞, ‖z‖∞)
    ε_dual = ε_abs + ε_rel·max(‖Px‖∞, ‖Aᵀy‖∞, ‖q‖∞).
Duality gap (derived from the Lagrange dual of eq. qp): for a point with
Px + q + Aᵀy = 0 the dual value is −½xᵀPx − uᵀy₊ − lᵀy₋, so
    gap = xᵀPx + qᵀx + uᵀy₊ + lᵀy₋   (only finite bounds can carry a multiplier).
"""
from __future__ import annotations

import numpy as np

INF = 1e20  # |bound| ≥ 1e20 is treated as infinite


def _inf(v):
    return float(np.max(np.abs(v))) if np.size(v) else 0.0


def objective(P_full, q, x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * float(x @ (P_full @ x)) + float(q @ x)


def residuals(P_full, q, A, x, z, y):
    Ax = A @ x
    Px = P_full @ x
    Aty = A.T @ y
    rp = Ax - z
    rd = Px + q + Aty
    return dict(prim=_inf(rp), dual=_inf(rd), Ax=_inf(Ax), z=_inf(z), Px=_inf(Px), Aty=_inf(Aty), q=_inf(q))


def tolerances(res, eps_abs, eps_rel):
    eps_p = eps_abs + eps_rel * max(res["Ax"], res["z"])
    eps_d = eps_abs + eps_rel * max(res["Px"], res["Aty"], res["q"])
    return eps_p, eps_d


def kkt_report(P_full, q, A, l, u, x, y, z=None):
    """Violation of each optimality condition at (x, z, y); z defaults to Π_[l,u](Ax)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Ax = A @ x
    if z is None:
        z = np.minimum(np.maximum(Ax, l), u)
    res = residuals(P_full, q, A, x, z, y)
    lf = np.where(np.abs(l) >= INF, 0.0, l)
    uf = np.where(np.abs(u) >= INF, 0.0, u)
    yp = np.maximum(y, 0.0)
    ym = np.minimum(y, 0.0)
    box = max(_inf(np.maximum(l - z, 0.0)), _inf(np.maximum(z - u, 0.0)))
    # a multiplier on an infinite bound is a violation by itself
    inf_mult = max(_inf(yp[u >= INF]), _inf(ym[l <= -INF]))
    comp = max(_inf(ym * np.where(np.abs(l) >= INF, 0.0, z - lf)),
               _inf(yp * np.where(np.abs(u) >= INF, 0.0, z - uf)))
    gap = float(x @ (P_full @ x)) + float(q @ x) + float(uf @ yp) + float(lf @ ym)
    return dict(prim=res["prim"], dual=res["dual"], box=box, comp=comp, inf_mult=inf_mult,
                gap=abs(gap), obj=objective(P_full, q, x), norms=res)
