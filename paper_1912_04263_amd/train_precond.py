"""Train the learned diagonal preconditioner of one problem family on generated QPs, on the GPU.

Pipeline (every numeric step runs in the library's device kernels):
  1. draw the training instances of the family at a training size (seeds 50000 + i; the
     portfolio default: n = 20,000 assets, k = 200 factors, 50% dense factor matrix) and set each
     up on the device (Ruiz scaling included);
  2. Hutchinson targets: for each instance and ρ̄ ∈ rhos, s Rademacher probes (drawn here and
     passed in), each K⁻¹z by the solver's own PCG; ĥ clamped at 1/K_ii; target log(ĥ K_ii);
  3. Adam on the mean-removed log-error loss, one (instance, ρ̄) pair per step, shuffled epochs;
  4. evaluation on held-out instances (seeds 60000 + i): loss, PCG iterations with the learned
     diagonal vs Jacobi on random right-hand sides, and full solves (ADMM + PCG) with both.
Writes the float32 parameters and a JSON summary.

Training sizes per family keep the benchmark instances' per-row structure at a fraction of their
size: portfolio 20,000 × 200 factors at 50%; random n = 5,000, m = 50,000 with about 20 entries per
row of A and of P; Lasso 1,000 features × 10,000 data rows at 10% (100 entries per data row);
SVM 20,000 points × 1,000 features at 10% (100 entries per point).

  python -m paper_1912_04263_amd.train_precond --family portfolio --out weights/portfolio_h32.f32
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import problems, qpg


# training-size generators of the other families (same per-row structure as the benchmark sizes)
FAMILIES = {
    "random": lambda seed: problems.random_qp(5_000, 50_000, 4.47 / 5_000, 20.0 / 5_000, seed),
    "lasso": lambda seed: problems.lasso_qp(1_000, 10_000, 0.1, seed),
    "svm": lambda seed: problems.svm_qp(20_000, 1_000, 0.1, seed),
}


def log(*a):
    print(*a, flush=True)


def targets(solver, rhos, probes, seed, eps, max_iter):
    rng = np.random.default_rng(seed)
    out = []
    for rho in rhos:
        z = rng.choice(np.array([-1, 1], dtype=np.int8), size=(probes, solver.n))
        h = solver.hutchinson(z, rho, eps=eps, max_iter=max_iter)
        K = solver.kdiag(rho)
        out.append((rho, np.log(np.maximum(h, 1.0 / K) * K).astype(np.float32)))
    return out


def pcg_iterations(problem, weights, rhos, seed, eps=1e-6):
    """Mean PCG iterations to ‖r‖∞ ≤ eps‖b‖∞ on random b: (Jacobi, learned)."""
    rng = np.random.default_rng(seed)
    sj = qpg.Solver.from_qp(problem)
    sl = qpg.Solver.from_qp(problem, precond="learned", precond_weights=weights)
    res = []
    for rho in rhos:
        b = rng.standard_normal(problem.n)
        sj.set_rho(rho)
        sl.set_rho(rho)
        _, kj, _, _ = sj.pcg(b, eps=eps, max_iter=5000)
        _, kl, _, _ = sl.pcg(b, eps=eps, max_iter=5000)
        res.append((rho, kj, kl))
    sj.close()
    sl.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="portfolio", choices=["portfolio", *sorted(FAMILIES)])
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--heldout", type=int, default=16)
    ap.add_argument("--n-assets", type=int, default=20000)
    ap.add_argument("--k-factors", type=int, default=200)
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--rhos", default="0.01,0.1,1,10")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--hutch-eps", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", required=True)
    ap.add_argument("--summary", default=None)
    args = ap.parse_args(argv)
    rhos = [float(r) for r in args.rhos.split(",")]
    t0 = time.time()

    def make(seed):
        if args.family == "portfolio":
            return problems.portfolio_qp(args.n_assets, args.k_factors, 0.5, seed)
        return FAMILIES[args.family](seed)

    # 1–2: instances and targets
    train = []
    for i in range(args.instances):
        p = make(50000 + i)
        s = qpg.Solver.from_qp(p)
        train.append((s, targets(s, rhos, args.probes, 7_000_000 + i, args.hutch_eps, 2000)))
        if i % 16 == 0 or i == args.instances - 1:
            log(f"[train] targets {i + 1}/{args.instances}  {time.time() - t0:.0f}s")
    held = []
    for i in range(args.heldout):
        p = make(60000 + i)
        s = qpg.Solver.from_qp(p)
        held.append((p, s, targets(s, rhos, args.probes, 8_000_000 + i, args.hutch_eps, 2000)))
    log(f"[train] held-out targets done  {time.time() - t0:.0f}s")

    # 3: training
    net = qpg.Net(None, seed=args.seed, bf16=True)

    def heldout_loss():
        return float(np.mean([net.loss_grad(s, rho, t, want_grad=False)[0] for _, s, tt in held for rho, t in tt]))

    hist = [heldout_loss()]
    log(f"[train] epoch 0 held-out loss {hist[-1]:.4f}")
    pairs = [(k, j) for k in range(len(train)) for j in range(len(rhos))]
    rng = np.random.default_rng(args.seed)
    steps = args.epochs * len(pairs)
    step = 0
    for ep in range(1, args.epochs + 1):
        tl = []
        for idx in rng.permutation(len(pairs)):
            k, j = pairs[idx]
            s, tt = train[k]
            rho, t = tt[j]
            lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * step / steps))  # cosine decay
            loss, _ = net.loss_grad(s, rho, t, want_grad=False)
            net.adam_step(lr)
            tl.append(loss)
            step += 1
        hist.append(heldout_loss())
        log(f"[train] epoch {ep} train loss {np.mean(tl):.4f} held-out loss {hist[-1]:.4f}  {time.time() - t0:.0f}s")
    w = net.params()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    w.astype("<f4").tofile(args.out)
    for s, _ in train:
        s.close()

    # 4: held-out evaluation
    it = []
    solves = []
    for i, (p, s, _) in enumerate(held):
        it += pcg_iterations(p, w, rhos, 9_000_000 + i)
        if i < 8:
            r = {}
            for name, kw in (("jacobi", {}), ("learned", dict(precond="learned", precond_weights=w))):
                sv = qpg.Solver.from_qp(p, eps_abs=1e-3, eps_rel=1e-3, **kw)
                sv.solve()
                info = sv.solve()
                r[name] = dict(iter=info.iter, pcg=info.pcg_iter_total, solve_s=info.solve_time,
                               obj=info.obj_val, trials=info.precond_trials, won=info.precond_learned_chosen)
                sv.close()
            solves.append(r)
            log(f"[eval] held-out {i}: jacobi {r['jacobi']}  learned {r['learned']}")
        s.close()
    it = np.array(it)
    summary = {
        "family": args.family,
        "instances": args.instances, "heldout": args.heldout, "n_assets": args.n_assets,
        "k_factors": args.k_factors, "probes": args.probes, "rhos": rhos, "epochs": args.epochs,
        "lr": args.lr, "heldout_loss": hist,
        "pcg_iters_random_rhs": {"jacobi_mean": float(it[:, 1].mean()), "learned_mean": float(it[:, 2].mean()),
                                 "per_rho": {str(r): [float(it[it[:, 0] == r, 1].mean()), float(it[it[:, 0] == r, 2].mean())]
                                             for r in rhos}},
        "solves": solves,
        "train_seconds": time.time() - t0,
    }
    log("[eval] PCG iterations on random right-hand sides (jacobi, learned):",
        summary["pcg_iters_random_rhs"]["jacobi_mean"], summary["pcg_iters_random_rhs"]["learned_mean"])
    if args.summary:
        with open(args.summary, "w") as fh:
            json.dump(summary, fh, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
