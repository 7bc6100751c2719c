"""Benchmark: QP time-to-solution and ADMM iterations/s at eps 1e-3, PCG kernel HBM GB/s.

One step = one complete solve (Algorithm 1 with the reduced-KKT PCG step, every kernel of the
hot path) of the device-resident problem from a cold start (x = z = y = 0, initial ρ̄) to
eps_abs = eps_rel = 1e-3. The problem is set up (validated, converted, equilibrated, copied to
HBM) once, before the timed region. Prints one JSON line.

Headline: the SVM workload (10⁶ points × 10⁴ features at 1%, 1.02·10⁸ matrix entries), the
largest of the five benchmark configurations and the one whose matrices (1.2–2.5 GB) cannot sit
in the 256 MB last-level cache, in FP32-bulk / FP64-reduction arithmetic with the Jacobi
preconditioner. Beside it, one entry per benchmark configuration (random 200×400, Lasso, large
random, portfolio, SVM) with every precision/preconditioner variant at eps 1e-3 and its objective
error against the oracle's minimiser (tests/golden/fullsize_<workload>.npz, where one has been
written). With --quality-sweep, every variant is also solved at eps 1e-4, 1e-5, 1e-6 until its
objective is within 1e-3 (relative) of a tight FP64 reference solve, and the time to that answer
quality is reported (minutes of GPU time on the portfolio workload).

  python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload svm_c4] [--precision mixed]
                  [--configs all|none|name,name,...] [--quality-sweep]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP time-to-solution & ADMM iter/s at eps 1e-3; PCG HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
CONFIGS = ["random_c0", "lasso_c1", "random_c2", "portfolio_c3", "svm_c4"]
VARIANTS = (("fp64", "jacobi"), ("mixed", "jacobi"), ("mixed", "learned"), ("fp64", "learned"))
# objective error that counts as "solved" when variants are compared at equal answer quality
EQUAL_QUALITY = 1e-3
QUALITY_EPS = (1e-3, 1e-4, 1e-5, 1e-6)
REF_EPS = {"portfolio_c3": 1e-7}  # tight FP64 reference solve per workload (default 1e-6)


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(problem, iters, small):
    """The oracle timed on this host: ADMM iterations/s on a bounded sample of the headline
    workload (its float64 reduced-KKT PCG route; the direct factorisation does not fit a bounded
    sample at this size), and the time-to-solution at eps 1e-3 of the 200×400 random QP with the
    direct KKT solve (factorisation included)."""
    import scipy.sparse as sp

    from oracle import admm as o_admm

    t = time.perf_counter()
    r = o_admm.solve(problem.P_full(), problem.q, sp.csr_matrix(problem.A), problem.l, problem.u,
                     eps_abs=0.0, eps_rel=0.0, max_iter=iters, linsys="pcg", adaptive_rho=False)
    total = time.perf_counter() - t
    t = time.perf_counter()
    r0 = o_admm.solve(small.P_full(), small.q, sp.csr_matrix(small.A), small.l, small.u,
                      eps_abs=1e-3, eps_rel=1e-3)
    tts0 = time.perf_counter() - t
    return {"value": r.iters / r.iter_time, "unit": "ADMM iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"{r.iters} ADMM iterations of the float64 oracle (numpy/scipy, one thread; "
                       f"linear step = reduced KKT system by its own PCG to 1e-12 relative, "
                       f"warm-started) on the same {problem.name} instance: {r.iter_time:.1f} s of "
                       f"iterations ({total:.1f} s with Ruiz scaling, which the rate excludes)"),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
            "random_c0_tts_s": tts0, "random_c0_status": r0.status, "random_c0_admm_iters": r0.iters,
            "random_c0_note": "oracle with its direct KKT solve (sparse LU, factorisation included), "
                              "eps_abs = eps_rel = 1e-3, one thread"}


def oracle_answer(workload):
    """f* and the status of the oracle's solve of a benchmark workload, from the stored fixture
    (written by tests/golden/make_fullsize_fixtures.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{workload}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
    return {"f_star": meta["f_star"], "eps": meta["eps"], "route": meta["route"], "status": meta["status"]}


def weights_for(workload, default):
    """Trained parameters of the learned preconditioner for a workload's problem family, or the
    given default set when that family has none."""
    from paper_1912_04263_amd import qpg
    family = workload.split("_")[0]
    path = os.path.join(qpg.WEIGHTS_DIR, f"{family}_h32.f32")
    name = f"{family}_h32" if os.path.exists(path) else default
    return name, qpg.load_weights(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="svm_c4")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "learned"])
    ap.add_argument("--weights", default="portfolio_h32",
                    help="learned-preconditioner weights when the workload's family has none")
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--rho-update-every", type=int, default=10,
                    help="ρ̄ update cadence in ADMM iterations (0: constant ρ̄), for the cadence ablation")
    ap.add_argument("--check-every", type=int, default=5, help="termination check cadence (ablation)")
    ap.add_argument("--rho-vector", type=int, default=0, help="1: R = diag(ρ_i) (ablation)")
    ap.add_argument("--pcg-eps-schedule", type=int, default=0,
                    help="1: PCG tolerance decreasing with k instead of the residual rule (ablation)")
    ap.add_argument("--spmv-tile-nnz", type=int, default=0,
                    help="matrix entries per SpMV workgroup with an LDS window (0: library default)")
    ap.add_argument("--spmv-plain-nnz", type=int, default=0,
                    help="matrix entries per SpMV workgroup without a window (0: library default)")
    ap.add_argument("--spmv-window-cols", type=int, default=0,
                    help="LDS gather window capacity in columns (0: library default)")
    ap.add_argument("--spmv-min-seg", type=int, default=0,
                    help="entries per row and column range for a multi-range work list (0: library default)")
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", default="all",
                    help="per-configuration entries: all, none, or a comma-separated list")
    ap.add_argument("--config-reps", type=int, default=3, help="timed solves per variant (mean)")
    ap.add_argument("--quality-sweep", action="store_true",
                    help="also solve each variant at tighter eps until its objective is within 1e-3 of a "
                         "tight FP64 reference (slow on the portfolio workload)")
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
    # the device and runtime start up here, once per process, not inside the first timed setup
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream

    def make(name):
        t0 = time.perf_counter()
        p = problems.make(name)
        log(f"[bench] generated {name}: n={p.n} m={p.m} nnz(P)={p.meta['nnz_P_full']} "
            f"nnz(A)={p.meta['nnz_A']} in {time.perf_counter() - t0:.1f}s")
        return p

    def solver(p, precision, precond, eps, weights=None, **kw):
        extra = dict(precond="learned", precond_weights=weights) if precond == "learned" else {}
        kw.setdefault("max_iter", 100000)
        kw.setdefault("spmv_tile_nnz", args.spmv_tile_nnz)
        kw.setdefault("spmv_plain_nnz", args.spmv_plain_nnz)
        kw.setdefault("spmv_window_cols", args.spmv_window_cols)
        kw.setdefault("spmv_min_seg", args.spmv_min_seg)
        return qpg.Solver.from_qp(p, eps_abs=eps, eps_rel=eps, precision=precision, stream=stream,
                                  device=0, **extra, **kw)

    def timed(s, steps, warmup):
        for _ in range(warmup):
            s.solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = [s.solve() for _ in range(steps)]
        torch.cuda.synchronize()
        return infos, time.perf_counter() - t

    def pcg_kernels(s, p, precision):
        prec_id = qpg.QPG_MIXED if precision == "mixed" else qpg.QPG_FP64
        sz = 4 if precision == "mixed" else 8
        n, m = p.n, p.m
        nnz_a = p.meta["nnz_A"]
        nnz_b = p.meta["nnz_P_full"] + nnz_a
        kernels = {}
        for kid, name, nbytes in ((qpg.QPG_KERNEL_SPMV_B, "spmv_B_Kp", spmv_b_bytes(n, m, nnz_b, sz)),
                                  (qpg.QPG_KERNEL_SPMV_A, "spmv_A_w", spmv_a_bytes(n, m, nnz_a, sz)),
                                  (qpg.QPG_KERNEL_PCG_UPDATE, "pcg_update", pcg_update_bytes(n, m, sz)),
                                  (qpg.QPG_KERNEL_PCG_DIR, "pcg_dir", pcg_dir_bytes(n, sz))):
            us = s.time_kernel(kid, args.kernel_reps, prec_id)
            kernels[name] = {"avg_us": us, "bytes": nbytes, "GBs": nbytes / us / 1e3,
                             "frac": nbytes / us / 1e3 / HBM_PEAK_GBS}
        pcg_bytes = sum(k["bytes"] for k in kernels.values())
        pcg_us = sum(k["avg_us"] for k in kernels.values())
        it = {"bytes": pcg_bytes, "kernel_us": pcg_us, "GBs": pcg_bytes / pcg_us / 1e3,
              "frac": pcg_bytes / pcg_us / 1e3 / HBM_PEAK_GBS}
        layout_b = s.spmv_layout(1)
        us = s.time_kernel(qpg.QPG_KERNEL_SPMV_B_STREAM, args.kernel_reps, prec_id)
        nbytes = spmv_b_stream_bytes(n, m, nnz_b, sz)
        moved = stream_bytes_moved(layout_b, sz)
        kernels["spmv_B_stream"] = {"avg_us": us, "bytes": nbytes, "GBs": nbytes / us / 1e3,
                                    "frac": nbytes / us / 1e3 / HBM_PEAK_GBS,
                                    "bytes_moved": moved, "GBs_moved": moved / us / 1e3, "layout": layout_b}
        us_a = s.time_kernel(qpg.QPG_KERNEL_SPMV_A_STREAM, args.kernel_reps, prec_id)
        kernels["spmv_A_stream"] = {"avg_us": us_a, "layout": s.spmv_layout(0)}
        return kernels, it

    if args.copy_calibration_mb > 0:
        nel = args.copy_calibration_mb * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration_mb} MiB read + written")
        del a, b

    # ------------------------------------------------------------------ headline
    p = make(args.workload)
    wname, weights = weights_for(args.workload, args.weights)
    s = solver(p, args.precision, args.precond, args.eps, weights,
               rho_update_every=args.rho_update_every, check_every=args.check_every,
               rho_vector=args.rho_vector, pcg_eps_schedule=args.pcg_eps_schedule)
    setup_s = s.info().setup_time
    infos, elapsed = timed(s, args.steps, args.warmup)
    steps = max(1, args.steps)
    last = infos[-1] if infos else s.info()
    admm_iters = sum(i.iter for i in infos)
    tts = elapsed / steps
    log(f"[bench] {args.workload} {args.precision}/{args.precond}: {last.status} in {last.iter} ADMM / "
        f"{last.pcg_iter_total} PCG iterations, solve {tts * 1e3:.2f} ms, setup {setup_s:.3f} s, "
        f"obj {last.obj_val:.10g}")
    kernels, pcg_it = pcg_kernels(s, p, args.precision)
    dom = kernels["spmv_B_stream"]
    prec_tag = "float" if args.precision == "mixed" else "double"
    roofline = {"bound": "hbm", "achieved": dom["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["GBs"] / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload, args.precision),
                "kernel": f"k_spmv<{prec_tag}, OpKp<{prec_tag}>> (segment sums of [P̄ | Āᵀ][p; w])",
                "bytes_per_launch": dom["bytes"], "avg_us": dom["avg_us"],
                "bytes_moved_per_launch": dom["bytes_moved"], "achieved_moved": dom["GBs_moved"],
                "pass_B": kernels["spmv_B_Kp"], "pass_A": kernels["spmv_A_w"],
                "pcg_iteration": pcg_it}
    s.close()
    log(f"[bench] dominant kernel {dom['avg_us']:.1f} us = {dom['GBs']:.0f} GB/s ({roofline['frac']:.3f}); "
        f"PCG iteration {pcg_it['kernel_us']:.1f} us = {pcg_it['GBs']:.0f} GB/s ({pcg_it['frac']:.3f})")

    head_orc = oracle_answer(args.workload)

    # ------------------------------------------------------------------ per configuration
    names = CONFIGS if args.configs == "all" else ([] if args.configs == "none" else args.configs.split(","))
    configs = {}
    for name in names:
        q = p if name == args.workload else make(name)
        wn, w = weights_for(name, args.weights)
        orc = oracle_answer(name)
        entry = {"n": q.n, "m": q.m, "nnz_P": q.meta["nnz_P_full"], "nnz_A": q.meta["nnz_A"],
                 "oracle": orc, "learned_weights": wn, "variants": {}}
        fref = None
        if args.quality_sweep:
            ref_eps = REF_EPS.get(name, 1e-6)
            with solver(q, "fp64", "jacobi", ref_eps) as sr:
                ir = sr.solve()
            fref = ir.obj_val
            entry["reference"] = {"eps": ref_eps, "obj": fref, "status": ir.status, "admm_iters": ir.iter}
            log(f"[bench] {name}: reference FP64/Jacobi at eps {ref_eps:g}: {ir.status}, {ir.iter} ADMM, "
                f"obj {fref:.10g}")
        for prec, pc in VARIANTS:
            v = {}
            for eps in (QUALITY_EPS if args.quality_sweep else (args.eps,)):
                with solver(q, prec, pc, eps, w) as sv:
                    inf, el = timed(sv, args.config_reps, 1)
                    setup = sv.info().setup_time
                    if eps == args.eps and pc == "jacobi":
                        kern, it = pcg_kernels(sv, q, prec)
                        v["pcg_iteration"] = it
                        v["spmv_B_stream"] = {k: kern["spmv_B_stream"][k] for k in ("avg_us", "GBs", "frac")}
                i = inf[-1]
                t_solve = el / len(inf)
                rec = {"status": i.status, "tts_s": t_solve, "setup_s": setup, "tts_with_setup_s": t_solve + setup,
                       "admm_iters": i.iter, "pcg_iters": i.pcg_iter_total, "admm_iter_per_s": i.iter / t_solve,
                       "obj": i.obj_val, "precision_used": i.precision_used, "precond_used": i.precond_used,
                       "precond_trials_won": [i.precond_learned_chosen, i.precond_trials]}
                if orc:
                    rec["obj_rel_err_vs_oracle"] = abs(i.obj_val - orc["f_star"]) / max(1.0, abs(orc["f_star"]))
                msg = f"obj err vs oracle {rec['obj_rel_err_vs_oracle']:.2e}" if orc else "no oracle answer stored"
                if fref is not None:
                    err = abs(i.obj_val - fref) / max(1.0, abs(fref))
                    rec["obj_rel_err_vs_ref"] = err
                    msg += f", vs reference {err:.2e}"
                if eps == args.eps:
                    v.update(rec)
                log(f"[bench]   {name} {prec}/{pc} eps {eps:g}: {i.status} {i.iter} ADMM / {i.pcg_iter_total} PCG, "
                    f"solve {t_solve * 1e3:.2f} ms, setup {setup:.3f} s, {msg}")
                if fref is not None and (rec["obj_rel_err_vs_ref"] <= EQUAL_QUALITY or eps == QUALITY_EPS[-1]):
                    v["equal_quality"] = {"obj_rel_err_target": EQUAL_QUALITY,
                                          "reached": rec["obj_rel_err_vs_ref"] <= EQUAL_QUALITY,
                                          "eps": eps, "tts_s": t_solve, "tts_with_setup_s": t_solve + setup,
                                          "obj_rel_err_vs_ref": rec["obj_rel_err_vs_ref"], "admm_iters": i.iter}
                    break
            entry["variants"][f"{prec}/{pc}"] = v
        configs[name] = entry
        if q is not p:
            del q

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host ...")
        cpu = cpu_baseline(p, args.cpu_iters, problems.make("random_c0"))
        log(f"[bench] cpu_baseline {cpu['value']:.4f} ADMM iter/s; random_c0 TTS {cpu['random_c0_tts_s']:.2f} s")

    n, m = p.n, p.m
    out = {
        "metric": METRIC,
        "value": admm_iters / elapsed if admm_iters else None,
        "unit": "ADMM iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tts * 1e3 if args.steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "nnz_P": p.meta["nnz_P_full"],
                   "nnz_A": p.meta["nnz_A"], "eps_abs": args.eps, "eps_rel": args.eps,
                   "precision": args.precision, "preconditioner": args.precond,
                   "learned_weights": wname if args.precond == "learned" else None,
                   "rho_update_every": args.rho_update_every, "check_every": args.check_every,
                   "rho_vector": args.rho_vector, "pcg_eps_schedule": args.pcg_eps_schedule,
                   "spmv_tile_nnz": args.spmv_tile_nnz, "spmv_plain_nnz": args.spmv_plain_nnz,
                   "spmv_window_cols": args.spmv_window_cols, "spmv_min_seg": args.spmv_min_seg,
                   "kernel_reps": args.kernel_reps,
                   "step": "one full solve from a cold start"},
        "tts_s": tts,
        "setup_s": setup_s,
        "tts_with_setup_s": tts + setup_s,
        "status": last.status,
        "admm_iters": last.iter,
        "pcg_iters": last.pcg_iter_total,
        "obj": last.obj_val,
        "obj_rel_err_vs_oracle": (abs(last.obj_val - head_orc["f_star"]) / max(1.0, abs(head_orc["f_star"]))
                                  if head_orc else None),
        "kernels": kernels,
        "roofline": roofline,
        "configs": configs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
