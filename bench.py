"""Benchmark: QP time-to-solution and ADMM iterations/s at eps 1e-3, PCG kernel HBM GB/s.

One step = one complete solve (Algorithm 1 with the reduced-KKT PCG step, every kernel of the
hot path) of the device-resident problem from a cold start (x = z = y = 0, initial ρ̄) to
eps_abs = eps_rel = 1e-3. The problem is set up (validated, equilibrated, copied to HBM) once,
before the timed region. Prints one JSON line.

  python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload lasso_c1] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP time-to-solution & ADMM iter/s at eps 1e-3; PCG HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_b_bytes(n, m, nnz_b, s):
    """Algorithmic bytes of one launch of the PCG K-matvec second half, Kp = P̄p + σp + Āᵀw and
    pᵀKp: matrix values and column indices once, row pointers and split points, the gathered
    vectors p (n) and w (m) once each, Kp written once."""
    return nnz_b * (s + 4) + 4 * (n + 1) + 4 * n + (n + m) * s + n * s


def spmv_b_stream_bytes(n, m, nnz_b, s):
    """Algorithmic bytes of the stream kernel of that pass alone (segment sums of [P̄ | Āᵀ][p; w]):
    matrix values and 32-bit column indices once, the gathered vectors p (n) and w (m) once."""
    return nnz_b * (s + 4) + (n + m) * s


def stream_bytes_moved(layout, s):
    """Bytes the stream kernel actually reads and writes in its layout: values and 16-bit column
    offsets in windowed tiles, values and 32-bit columns elsewhere (padding included), chunk
    descriptors and slot numbers, the two planes of segment sums written."""
    return (layout["windowed_positions"] * (s + 2) + layout["plain_positions"] * (s + 4)
            + layout["chunks"] * (16 + 64 * 4) + layout["slots"] * 2 * s)


def spmv_a_bytes(n, m, nnz_a, s):
    """w = ρ̄Āp: Ā values and indices once, row pointers, p gathered once, w written once."""
    return nnz_a * (s + 4) + 4 * (m + 1) + n * s + m * s


def pcg_update_bytes(n, m, s):
    """x̃ += αp, r += αKp, rᵀM⁻¹r, ‖r‖∞: read x̃, p, r, Kp, M⁻¹; write x̃, r. z̃ += αw/ρ̄ (the
    tracked Āx̃): read z̃, w; write z̃."""
    return 7 * n * s + 3 * m * s


def pcg_dir_bytes(n, s):
    """p = −M⁻¹r + βp: read r, M⁻¹, p; write p."""
    return 4 * n * s


def csrc_digest():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1912_04263_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None when
    there is no measurement for this workload/precision or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"spmv_B_stream_{workload}_{precision}.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("csrc_sha256") != csrc_digest():
        return None
    return d["traffic_bytes_per_launch"]


def cpu_baseline(problem, iters):
    """The oracle timed on this host: ADMM with its float64 reduced-KKT PCG solves."""
    import scipy.sparse as sp

    from oracle import admm as o_admm

    r = o_admm.solve(problem.P_full(), problem.q, sp.csr_matrix(problem.A), problem.l, problem.u,
                     eps_abs=0.0, eps_rel=0.0, max_iter=iters, linsys="pcg", adaptive_rho=False)
    rate = r.iters / r.iter_time
    return {"value": rate, "unit": "ADMM iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"{r.iters} ADMM iterations of the float64 oracle (numpy/scipy, one thread; linear "
                       f"step = reduced KKT system by its own PCG to 1e-12 relative, warm-started) on the "
                       f"same {problem.name} instance; Ruiz scaling not timed; {r.iter_time:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lasso_c1")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "learned"])
    ap.add_argument("--weights", default="portfolio_h32", help="learned-preconditioner weights name")
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--rho-update-every", type=int, default=10,
                    help="ρ̄ update cadence in ADMM iterations (0: constant ρ̄), for the cadence ablation")
    ap.add_argument("--check-every", type=int, default=5, help="termination check cadence (ablation)")
    ap.add_argument("--rho-vector", type=int, default=0, help="1: R = diag(ρ_i) (ablation)")
    ap.add_argument("--pcg-eps-schedule", type=int, default=0,
                    help="1: PCG tolerance decreasing with k instead of the residual rule (ablation)")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--ref-eps", type=float, default=0.0,
                    help="also solve to this tolerance (FP64/Jacobi, untimed) and report each "
                         "variant's objective error against it")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (reference for counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); multi-GPU sharding is a design note only, not implemented.",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_1912_04263_amd import problems, qpg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    p = problems.make(args.workload)
    log(f"[bench] generated {args.workload}: n={p.n} m={p.m} nnz(P)={p.meta['nnz_P_full']} "
        f"nnz(A)={p.meta['nnz_A']} in {time.perf_counter() - t0:.1f}s")

    weights = qpg.load_weights(args.weights)

    def run(precision, steps, warmup, precond=None):
        precond = precond or args.precond
        extra = dict(precond="learned", precond_weights=weights) if precond == "learned" else {}
        s = qpg.Solver.from_qp(p, eps_abs=args.eps, eps_rel=args.eps, precision=precision,
                               stream=stream, device=0, max_iter=20000,
                               rho_update_every=args.rho_update_every, check_every=args.check_every,
                               rho_vector=args.rho_vector, pcg_eps_schedule=args.pcg_eps_schedule,
                               **extra)
        setup = s.info().setup_time
        for _ in range(warmup):
            s.solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = [s.solve() for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return s, setup, infos, el

    if args.copy_calibration_mb > 0:
        nel = args.copy_calibration_mb * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration_mb} MiB read + written")
        del a, b

    s, setup_s, infos, elapsed = run(args.precision, args.steps, args.warmup)
    steps = max(1, args.steps)
    last = infos[-1] if infos else s.info()
    admm_iters = sum(i.iter for i in infos)
    log(f"[bench] {args.precision}/{args.precond}: {last.status} in {last.iter} ADMM / {last.pcg_iter_total} PCG "
        f"iterations ({last.infeas_checks} infeasibility checks), solve {elapsed / steps * 1e3:.2f} ms, "
        f"setup {setup_s:.2f} s, obj {last.obj_val:.10g}")

    prec_id = qpg.QPG_MIXED if args.precision == "mixed" else qpg.QPG_FP64
    sz = 4 if args.precision == "mixed" else 8
    n, m = p.n, p.m
    nnz_a = p.meta["nnz_A"]
    nnz_b = p.meta["nnz_P_full"] + nnz_a
    kernels = {}
    pcg_steps = ((qpg.QPG_KERNEL_SPMV_B, "spmv_B_Kp", spmv_b_bytes(n, m, nnz_b, sz)),
             (qpg.QPG_KERNEL_SPMV_A, "spmv_A_w", spmv_a_bytes(n, m, nnz_a, sz)),
             (qpg.QPG_KERNEL_PCG_UPDATE, "pcg_update", pcg_update_bytes(n, m, sz)),
             (qpg.QPG_KERNEL_PCG_DIR, "pcg_dir", pcg_dir_bytes(n, sz)))
    for kid, name, nbytes in pcg_steps:
        us = s.time_kernel(kid, args.kernel_reps, prec_id)
        kernels[name] = {"avg_us": us, "bytes": nbytes, "GBs": nbytes / us / 1e3}
    pcg_bytes = sum(k["bytes"] for k in kernels.values())
    pcg_us = sum(k["avg_us"] for k in kernels.values())
    # the dominant kernel: the stream kernel of the B pass, timed alone
    layout_b = s.spmv_layout(1)
    us = s.time_kernel(qpg.QPG_KERNEL_SPMV_B_STREAM, args.kernel_reps, prec_id)
    nbytes = spmv_b_stream_bytes(n, m, nnz_b, sz)
    moved = stream_bytes_moved(layout_b, sz)
    kernels["spmv_B_stream"] = {"avg_us": us, "bytes": nbytes, "GBs": nbytes / us / 1e3,
                                "bytes_moved": moved, "GBs_moved": moved / us / 1e3, "layout": layout_b}
    us_a = s.time_kernel(qpg.QPG_KERNEL_SPMV_A_STREAM, args.kernel_reps, prec_id)
    kernels["spmv_A_stream"] = {"avg_us": us_a, "layout": s.spmv_layout(0)}
    dom = kernels["spmv_B_stream"]
    prec_tag = "float" if args.precision == "mixed" else "double"
    roofline = {"bound": "hbm", "achieved": dom["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["GBs"] / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload, args.precision),
                "kernel": f"k_spmv<{prec_tag}, OpKp<{prec_tag}>> (segment sums of [P̄ | Āᵀ][p; w])",
                "bytes_per_launch": dom["bytes"], "avg_us": dom["avg_us"],
                "bytes_moved_per_launch": moved, "achieved_moved": dom["GBs_moved"],
                "pass_B": kernels["spmv_B_Kp"],
                "pcg_iteration": {"bytes": pcg_bytes, "kernel_us": pcg_us, "GBs": pcg_bytes / pcg_us / 1e3}}
    s.close()

    variants = []
    if not args.no_compare:
        for prec, pc in (("fp64", "jacobi"), ("mixed", "jacobi"), ("mixed", "learned"), ("fp64", "learned")):
            if (prec, pc) == (args.precision, args.precond):
                continue
            s2, su2, inf2, el2 = run(prec, max(1, args.steps // 2), 1, pc)
            last2 = inf2[-1]
            v = {"precision": prec, "precond": pc, "tts_ms": el2 / len(inf2) * 1e3,
                 "admm_iter_per_s": sum(i.iter for i in inf2) / el2, "admm_iters": last2.iter,
                 "pcg_iters": last2.pcg_iter_total, "infeas_checks": last2.infeas_checks,
                 "status": last2.status, "obj": last2.obj_val,
                 "precision_used": last2.precision_used, "precond_used": last2.precond_used,
                 "precond_trials_won": [last2.precond_learned_chosen, last2.precond_trials],
                 "setup_s": su2,
                 "obj_rel_diff_vs_main": abs(last2.obj_val - last.obj_val) / max(1.0, abs(last.obj_val))}
            variants.append(v)
            log(f"[bench] {prec}/{pc}: {v['status']} tts {v['tts_ms']:.2f} ms, {v['admm_iters']} ADMM / "
                f"{v['pcg_iters']} PCG, {v['infeas_checks']} infeasibility checks, obj {v['obj']:.10g}")
            s2.close()

    ref = None
    if args.ref_eps > 0:
        sr = qpg.Solver.from_qp(p, eps_abs=args.ref_eps, eps_rel=args.ref_eps, stream=stream, device=0,
                                max_iter=100000)
        ir = sr.solve()
        sr.close()
        ref = {"eps": args.ref_eps, "obj": ir.obj_val, "status": ir.status, "iters": ir.iter}
        scale = max(1.0, abs(ir.obj_val))
        for v in variants:
            v["obj_rel_err_vs_ref"] = abs(v["obj"] - ir.obj_val) / scale
        log(f"[bench] reference at eps {args.ref_eps}: {ir.status}, obj {ir.obj_val:.10g}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host ...")
        cpu = cpu_baseline(p, args.cpu_iters)
        log(f"[bench] cpu_baseline {cpu['value']:.3f} ADMM iter/s")

    out = {
        "metric": METRIC,
        "value": admm_iters / elapsed if admm_iters else None,
        "unit": "ADMM iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3 if args.steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "nnz_P": p.meta["nnz_P_full"], "nnz_A": nnz_a,
                   "eps_abs": args.eps, "eps_rel": args.eps, "precision": args.precision,
                   "preconditioner": args.precond, "rho_update_every": args.rho_update_every,
                   "check_every": args.check_every, "rho_vector": args.rho_vector,
                   "pcg_eps_schedule": args.pcg_eps_schedule,
                   "step": "one full solve from a cold start"},
        "tts_s": elapsed / steps if args.steps else None,
        "setup_s": setup_s,
        "status": last.status,
        "admm_iters": last.iter,
        "pcg_iters": last.pcg_iter_total,
        "infeas_checks": last.infeas_checks,
        "obj": last.obj_val,
        "kernels": kernels,
        "roofline": roofline,
        "variants": variants,
        "reference": ref,
        "obj_rel_err_vs_ref": (abs(last.obj_val - ref["obj"]) / max(1.0, abs(ref["obj"]))) if ref else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
