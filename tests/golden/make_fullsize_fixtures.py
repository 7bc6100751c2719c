"""Write the oracle's answers for the full-size benchmark workloads (test fixtures).

Calls only the oracle (oracle/admm.py: Algorithm 1 with the direct solve of eq. kkt, or, where
the factorisation does not fit the CPU time, its reduced-KKT PCG route solved to 1e-12 relative,
which gives the same iterates) and the seeded generators. Nothing here comes from the HIP path.

For each workload it stores, in tests/golden/fullsize_<workload>.npz:
  x      the independent block of the minimiser (float32; the rest follows from it):
           random_c0     all of x
           lasso_c1      the 10⁴ feature weights (y = Ad·x − b and t = |x| at the optimum)
           random_c2     all of x
           portfolio_c3  the 10⁵ asset weights (the factor block is y = Fᵀx)
           svm_c4        the 10⁴ feature weights (t = max(0, diag(b)Ad·x + 1) at the optimum)
  meta   JSON: f* (float64), the oracle's status, iterations, final residuals and tolerances,
         the route, and a digest of the generated problem so that a changed generator is caught.

  python tests/golden/make_fullsize_fixtures.py lasso_c1 [--eps 1e-8] [--route direct|pcg]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import admm  # noqa: E402
from paper_1912_04263_amd import problems  # noqa: E402

BLOCK = {"random_c0": None, "lasso_c1": 10_000, "random_c2": None, "portfolio_c3": 100_000, "svm_c4": 10_000}
ROUTE = {"random_c0": "direct", "lasso_c1": "direct", "random_c2": "pcg", "portfolio_c3": "direct", "svm_c4": "pcg"}
# the library's own fill-reducing order does not finish on the portfolio class's dense KKT rows
# (the 10³ factor rows of 5·10⁴ entries and the budget row): those nodes are eliminated last,
# by block elimination (oracle.admm.KKTSolver)
DENSE_DEGREE = {"portfolio_c3": 2000}


def problem_digest(p) -> str:
    h = hashlib.sha256()
    for a in (p.P_triu.indptr, p.P_triu.indices, p.P_triu.data, p.q, p.A.indptr, p.A.indices, p.A.data,
              p.l, p.u):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def path_for(name):
    return os.path.join(HERE, f"fullsize_{name}.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(BLOCK))
    ap.add_argument("--eps", type=float, default=1e-8)
    ap.add_argument("--route", choices=["direct", "pcg"], default=None)
    ap.add_argument("--max-iter", type=int, default=100_000)
    ap.add_argument("--rho-interval", type=int, default=100)
    ap.add_argument("--check-every", type=int, default=5)
    args = ap.parse_args()
    route = args.route or ROUTE[args.workload]

    t0 = time.time()
    p = problems.make(args.workload)
    digest = problem_digest(p)
    print(f"{args.workload}: n={p.n} m={p.m} nnz(A)={p.A.nnz} generated in {time.time() - t0:.1f}s; "
          f"route {route}, eps {args.eps:g}", flush=True)
    last = [time.time()]

    def progress(k, pr, dr, ep, ed, rho):
        if time.time() - last[0] > 60:
            last[0] = time.time()
            print(f"  k={k} prim {pr:.3e} ({ep:.1e}) dual {dr:.3e} ({ed:.1e}) rho {rho:.3e} "
                  f"[{time.time() - t0:.0f}s]", flush=True)

    r = admm.solve(p.P_full(), p.q, sp.csr_matrix(p.A), p.l, p.u, eps_abs=args.eps, eps_rel=args.eps,
                   max_iter=args.max_iter, linsys=route, rho_interval=args.rho_interval,
                   check_every=args.check_every, progress=progress,
                   dense_degree=DENSE_DEGREE.get(args.workload, 0))
    k = BLOCK[args.workload] or p.n
    meta = {"workload": args.workload, "f_star": r.obj, "status": r.status, "iters": r.iters,
            "prim_res": r.prim_res, "dual_res": r.dual_res, "eps": args.eps, "route": route,
            "rho_final": r.rho, "rho_updates": r.rho_updates, "check_every": args.check_every,
            "dense_degree": DENSE_DEGREE.get(args.workload, 0),
            "block": k, "problem_sha256": digest,
            "x_inf_norm": float(np.max(np.abs(r.x[:k]))), "seconds": time.time() - t0,
            "factor_seconds": r.factor_time}
    np.savez_compressed(path_for(args.workload), x=r.x[:k].astype(np.float32), meta=json.dumps(meta))
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
