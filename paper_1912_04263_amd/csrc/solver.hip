// Solver object and C ABI: device memory, SpMV schedules, the ADMM loop of Algorithm 1 with the
// inexact reduced-KKT PCG step of Section 6.3, termination (Section 3.1), the PCG tolerance
// rule (Section 6.3.3) and the ρ̄ update (Section 3.4, 6.3.2).
#include <new>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

#include "ruiz.hpp"
#include "solver_internal.hpp"

using namespace qpg;

namespace {
thread_local std::string g_setup_error;
}  // namespace

void qpg_solver::alloc_prec64(const HostProblem& H) {
  Prec<double>& V = p64;
  place_raw(H);
  V.qb = upload(H.qb);
  V.lb = upload(H.lb);
  V.ub = upload(H.ub);
  V.x = alloc<double>((size_t)n + m);
  V.y = V.x + n;
  V.xt = alloc<double>(n);
  V.r = alloc<double>(n);
  V.p = alloc<double>((size_t)n + m);
  V.w = V.p + n;
  V.kp = alloc<double>(n);
  V.b = alloc<double>(n);
  V.dinv = alloc<double>(n);
  V.z = alloc<double>(m);
  V.zt = alloc<double>(m);
  V.ax = alloc<double>(m);
  V.bk = alloc<double>(n);
  V.g = alloc<double>(2 * ((size_t)n + m));
  V.dxy = alloc<double>((size_t)n + m);
  V.bg = alloc<double>(3 * (size_t)n);
  V.ready = true;
}

// Pinned staging for large host → device copies: kStageThreads host threads each own two
// buffers of kStagePiece bytes and copy every kStageThreads-th piece of the source into one of
// them while the DMA engine drains the other. One set per device, allocated on the first large
// copy and kept until the process ends: writing freshly pinned pages is slow (≈ 2.7 GB/s on first
// touch, against ≈ 78 GB/s for the copy into pages already touched), so the buffers are reused
// rather than allocated per setup. Copies to one device are serialised by its mutex.
constexpr int kStageThreads = 8;
constexpr size_t kStagePiece = size_t(8) << 20;
constexpr int kStageDevices = 64;

namespace {
struct StagingSet {
  std::mutex mu;
  void* buf[kStageThreads][2] = {};
  hipEvent_t done[kStageThreads][2] = {};
};
StagingSet g_staging[kStageDevices];

// allocates the set's missing buffers and events (S.mu held); a new buffer is written once, so
// that the first copy into it does not pay for the first touch of its pages
void ensure_staging(StagingSet& S) {
  for (int t = 0; t < kStageThreads; ++t)
    for (int b = 0; b < 2; ++b) {
      if (!S.done[t][b]) HIPCHK(hipEventCreateWithFlags(&S.done[t][b], hipEventDisableTiming));
      if (!S.buf[t][b]) {
        HIPCHK(hipHostMalloc(&S.buf[t][b], kStagePiece, hipHostMallocDefault));
        std::memset(S.buf[t][b], 0, kStagePiece);
      }
    }
}

// the staging set of a device, made ready ahead of the first large copy (run on a thread of its
// own during setup); a failure is left to the copy itself to report
void warm_staging(int device) {
  if (device < 0 || device >= kStageDevices) return;
  try {
    HIPCHK(hipSetDevice(device));
    StagingSet& S = g_staging[device];
    std::lock_guard<std::mutex> lock(S.mu);
    ensure_staging(S);
  } catch (...) {
  }
}
}  // namespace

void qpg_solver::copy_h2d(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (bytes < kStagePiece / 4 || device < 0 || device >= kStageDevices) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    if (bytes >= kStagePiece / 4) HIPCHK(hipStreamSynchronize(stream));  // the source may go on return
    return;
  }
  StagingSet& S = g_staging[device];
  std::lock_guard<std::mutex> lock(S.mu);
  ensure_staging(S);
  const size_t npieces = (bytes + kStagePiece - 1) / kStagePiece;
  const int T = (int)std::min<size_t>(kStageThreads, npieces);
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  std::exception_ptr err;
  std::mutex err_mu;
  auto work = [&](int t) {
    try {
      HIPCHK(hipSetDevice(device));
      int b = 0;
      for (size_t p = (size_t)t; p < npieces; p += (size_t)T, b ^= 1) {
        const size_t off = p * kStagePiece, len = std::min(kStagePiece, bytes - off);
        HIPCHK(hipEventSynchronize(S.done[t][b]));  // the DMA of this buffer's last piece is done
        std::memcpy(S.buf[t][b], s + off, len);
        HIPCHK(hipMemcpyAsync(d + off, S.buf[t][b], len, hipMemcpyHostToDevice, stream));
        HIPCHK(hipEventRecord(S.done[t][b], stream));
      }
    } catch (...) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (!err) err = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  th.reserve((size_t)T - 1);
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// Raw (unscaled) values of Ā and B on the device, from the caller's CSC values of A and the full
// P in CSR: Ā's values gathered through the CSR → CSC index map the host built with the pattern,
// B's rows assembled from P's rows and A's columns. The staging buffers are freed on return.
void qpg_solver::place_raw(const HostProblem& H) {
  Prec<double>& V = p64;
  const size_t nnz_a = H.a_src.size(), nnz_b = H.b_col.size();
  V.a_val = alloc<double>(nnz_a);
  V.b_val = alloc<double>(nnz_b);
  std::vector<void*> tmp;
  auto tmp_copy = [&](const void* src, size_t bytes) {
    void* d = nullptr;
    HIPCHK(hipMalloc(&d, std::max<size_t>(bytes, 1)));
    tmp.push_back(d);
    copy_h2d(d, src, bytes);
    return d;
  };
  try {
    const double* av = static_cast<const double*>(tmp_copy(H.a_csc_val, nnz_a * sizeof(double)));
    const int32_t* src = static_cast<const int32_t*>(tmp_copy(H.a_src.data(), nnz_a * sizeof(int32_t)));
    const int32_t* acp = static_cast<const int32_t*>(tmp_copy(H.a_colptr, ((size_t)n + 1) * sizeof(int32_t)));
    const int32_t* pp = static_cast<const int32_t*>(tmp_copy(H.p_ptr.data(), ((size_t)n + 1) * sizeof(int32_t)));
    const double* pv = static_cast<const double*>(tmp_copy(H.p_val.data(), H.p_val.size() * sizeof(double)));
    if (nnz_a) {
      const int g = (int)std::min<size_t>((nnz_a + kBlock - 1) / kBlock, 65536);
      hipLaunchKernelGGL(k_gather_values, dim3(g), dim3(kBlock), 0, stream, (int64_t)nnz_a, src, av, V.a_val);
    }
    const int gb = std::max(1, std::min((n + 3) / 4, 16384));
    hipLaunchKernelGGL(k_assemble_b, dim3(gb), dim3(kBlock), 0, stream, n, (const int32_t*)b_ptr,
                       (const int32_t*)b_split, pp, pv, acp, av, V.b_val);
    HIPCHK(hipStreamSynchronize(stream));
  } catch (...) {
    for (void* d : tmp) (void)hipFree(d);
    throw;
  }
  for (void* d : tmp) HIPCHK(hipFree(d));
}

// FP32 copies of the equilibrated device data (matrix values in CSR; the SELL copies are placed
// by place_values).
void qpg_solver::alloc_prec32() {
  Prec<float>& V = p32;
  auto cast = [&](const double* src, size_t count) {
    float* d = alloc<float>(count);
    if (count)
      hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for((int)count)), dim3(kBlock), 0, stream, (int)count,
                         d, src);
    return d;
  };
  V.a_val = cast(p64.a_val, (size_t)nnzA);
  V.b_val = cast(p64.b_val, (size_t)nnzB);
  V.qb = cast(p64.qb, n);
  V.lb = cast(p64.lb, m);
  V.ub = cast(p64.ub, m);
  V.x = alloc<float>((size_t)n + m);
  V.y = V.x + n;
  V.xt = alloc<float>(n);
  V.r = alloc<float>(n);
  V.p = alloc<float>((size_t)n + m);
  V.w = V.p + n;
  V.kp = alloc<float>(n);
  V.b = alloc<float>(n);
  V.dinv = alloc<float>(n);
  V.z = alloc<float>(m);
  V.zt = alloc<float>(m);
  V.bk = alloc<float>(n);
  V.g = alloc<float>(2 * ((size_t)n + m));
  V.dxy = alloc<float>((size_t)n + m);
  V.bg = alloc<float>(3 * (size_t)n);
  V.ready = true;
}

// Infeasibility tests of Section 3.1 on the norms of OpInfeasA / OpInfeasB, every tolerance
// relative to the ∞-norm of the difference tested (see the oracle's reading): primal first.
int qpg_solver::infeasibility_status() const {
  const double* nm = st_host->norms;
  const double tiny = 1e-30;
  const double ny = nm[17];
  if (s.eps_prim_inf > 0 && ny > tiny && nm[20] <= s.eps_prim_inf * ny && nm[18] < -s.eps_prim_inf * ny)
    return QPG_PRIMAL_INFEASIBLE;
  const double nx = nm[21], tol = s.eps_dual_inf * nx;
  if (s.eps_dual_inf > 0 && nx > tiny && nm[19] / c <= tol && nm[22] / c < -tol && nm[16] <= tol)
    return QPG_DUAL_INFEASIBLE;
  return QPG_UNSOLVED;
}

// The certificate directions: δx = Dδx̄ and δy ∝ Eδȳ, each scaled to ‖·‖∞ = 1.
template <typename T>
void qpg_solver::keep_certificate() {
  std::vector<T> d((size_t)n + m);
  HIPCHK(hipMemcpyAsync(d.data(), P<T>().dxy, d.size() * sizeof(T), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  cert_x.assign(n, 0.0);
  cert_y.assign(m, 0.0);
  double nx = 0.0, ny = 0.0;
  for (int i = 0; i < n; ++i) nx = std::max(nx, std::fabs(cert_x[i] = D[i] * (double)d[i]));
  for (int i = 0; i < m; ++i) ny = std::max(ny, std::fabs(cert_y[i] = E[i] * (double)d[n + i]));
  if (nx > 0)
    for (double& v : cert_x) v /= nx;
  if (ny > 0)
    for (double& v : cert_y) v /= ny;
  cert_valid = true;
}

// ADMM iterations k_start.. in precision T. Returns the last iteration index. status is set
// when the loop ends for a reason other than a precision fallback (fallback_request = 1).
template <typename T>
int qpg_solver::admm(int k_start, double& rho, double& eps_pcg, int& status,
                     int& fallback_request) {
  Prec<T>& V = P<T>();
  const double sigma = s.sigma, alpha = s.alpha;
  const bool fixed_eps = s.pcg_eps_fixed > 0;
  // Preconditioner policy. Jacobi (Section 6.3.1), or the learned diagonal: with trials on, the
  // first PCG solve and the first one after every ρ̄ change run with both preconditioners from the
  // same warm start, and the learned one is kept only if it needs fewer iterations (or, when both
  // hit the cap, ends with a smaller residual); a capped learned solve falls back to Jacobi.
  // A new trial is run only when ρ̄ has moved by more than a factor 2 since the last one, and
  // trials stop for the rest of the solve after the learned diagonal has lost two in a row.
  const bool infeas = s.eps_prim_inf > 0 || s.eps_dual_inf > 0;
  const bool learned_ok = (s.precond == QPG_PRECOND_LEARNED);
  bool trial = learned_ok && s.precond_trial;
  bool use_learned = learned_ok && !s.precond_trial;
  double rho_trial = rho;
  int lost_in_a_row = 0;
  if (use_learned)
    learned_dinv<T>(rho);
  else
    jacobi<T>(rho);
  int cap_streak = 0;
  double best_ratio = INFINITY;
  int since_best = 0;
  double tighten = 1.0;  // stall guard on the PCG tolerance (see below)
  // The infeasibility passes (Section 3.1) cost an Ā and a B pass per check. They run once the
  // residuals have stopped improving (kInfeasAfter checks without a 1% gain), which is where an
  // infeasible problem ends up; on a converging problem they would only add cost.
  constexpr int kInfeasAfter = 2;
  bool armed = false;
  // Speculation: an ADMM iteration without a check or a trial is launched without waiting for
  // its PCG solve. Its PCG runs a predicted number of iterations (the last count seen), then
  // k_after_pcg sets st->abort if the solve is unfinished, broke down or hit the cap; every later
  // kernel of the speculation is gated on that flag (the PCG kernels through `done`). The host
  // reads the state at the next check (or before a trial) and, after an abort, resumes at the
  // iteration that set it, whose state is exactly what its PCG iterations left. So the host
  // waits once per check instead of once per ADMM iteration.
  const int32_t* agate = &st->abort;
  constexpr int kSpecMaxPcg = 8;
  hipLaunchKernelGGL(k_spec_reset<DevState>, dim3(1), dim3(64), 0, stream, st);
  bool pending = false;  // speculative iterations launched since the last host read
  int last_cap_k = -2;
  auto finish = [&](int kk) {  // st_host is current at every return
    info.pcg_iter_total += st_host->pcg_sum;
    info.pcg_iter_max = std::max(info.pcg_iter_max, (int)st_host->pcg_max);
    last_precond_learned = use_learned;
    return kk;
  };
  // bookkeeping after the PCG solve of iteration kk (it iterations); true: stop the ADMM loop
  auto after_pcg = [&](int kk, int it) {
    const bool capped = it >= s.pcg_max_iter && st_host->rnorm > st_host->thresh;
    if (use_learned && (st_host->breakdown || capped)) {
      use_learned = false;  // runtime guard
      info.precond_switches++;
      jacobi<T>(rho);
    }
    info.pcg_iter_total += it;
    info.pcg_iter_max = std::max(info.pcg_iter_max, it);
    if (st_host->breakdown) {
      if (std::is_same<T, float>::value)
        fallback_request = 1;
      else
        status = QPG_NUMERICAL_ERROR;
      return true;
    }
    if (capped) {
      cap_streak = (kk == last_cap_k + 1) ? cap_streak + 1 : 1;
      last_cap_k = kk;
    }
    if (std::is_same<T, float>::value && cap_streak >= 3) {
      fallback_request = 1;
      return true;
    }
    return false;
  };
  // (a7)–(a8) z̃ = Āx̃ fused with relaxation, projection and dual update; x update. Between
  // checks z̃ = Āx̃ comes from the PCG iterations (z̃ += αĀp) and the update is a vector pass.
  // Āx̄ is tracked in FP64 in both precisions (p64.ax), so a check takes the primal residual
  // from the update as well. A check recomputes z̃ = Āx̃ by an Ā pass (which resets the rounding
  // drift of its recurrence) every kZtReset-th time in FP32 and never in FP64, where the drift
  // stays at rounding level; with R = diag(ρ_i), z̃ is not carried through PCG and every update
  // is an Ā pass.
  constexpr int kZtReset = std::is_same<T, float>::value ? 4 : 0;
  auto launch_update = [&](bool check, T* dxy, int kk) {
    double* ax = p64.ax;
    OpUpdate<T, false> upd{V.xt, V.x, V.z, V.y, V.zt, ax, V.g, V.lb, V.ub, escale,
                           (T)alpha, (T)rho, (T)(1.0 / rho), n, st, dxy, eqrow};
    const int g = grid_for(std::max(n, m));
    if (check) {
      OpUpdate<T, true> up{V.xt, V.x, V.z, V.y, V.zt, ax, V.g, V.lb, V.ub, escale, (T)alpha,
                           (T)rho, (T)(1.0 / rho), n, st, dxy, eqrow};
      const bool reset = eqrow || (kZtReset > 0 && (kk / s.check_every) % kZtReset == 0);
      if (reset) {
        finalize(up, spmv_A<T>(up, agate), agate);
      } else {
        up.zt = nullptr;  // s1 is z̃ itself
        hipLaunchKernelGGL((k_rows<T, OpUpdate<T, true>>), dim3(g), dim3(kBlock), 0, stream, m,
                           (const T*)V.zt, (const T*)nullptr, up, rb.partials, agate);
        finalize(up, g, agate);
      }
    } else if (eqrow) {
      spmv_A<T>(upd, agate);
    } else {
      upd.zt = nullptr;
      hipLaunchKernelGGL((k_rows<T, OpUpdate<T, false>>), dim3(g), dim3(kBlock), 0, stream, m,
                         (const T*)V.zt, (const T*)nullptr, upd, (double*)nullptr, agate);
    }
  };
  // after a host read that shows an abort: finish iteration j = abort_k (its PCG, then its
  // update) and return the iteration to continue from; −1 when the ADMM loop must stop
  auto resume = [&]() {
    const int j = st_host->abort_k, reason = st_host->abort_reason;
    info.spec_resumes++;
    hipLaunchKernelGGL(k_resume<DevState>, dim3(1), dim3(64), 0, stream, st, reason == 1 ? 1 : 0);
    const int it = reason == 1 ? pcg_loop<T>(rho, s.pcg_max_iter, true, st_host->iter) : st_host->iter;
    pending = false;
    if (after_pcg(j, it)) return -1;
    launch_update(false, nullptr, j);
    return j + 1;
  };
  // (a1)+(a2) right-hand side, ‖b‖∞ and the warm-started PCG residual: in one pass over B from
  // the previous solve's residual and right-hand side when they are in place (OpRhsRec), else
  // directly in two (OpRhsAt, OpRhsR0, after k_pairs). The recurrence
  // carries the error of b' (the gap between the recursive and the true residual of each solve)
  // into b, so b is recomputed directly every kRhsRefresh iterations; in FP64 the carried error
  // stays at rounding level, in FP32 the refresh bounds it.
  constexpr int kRhsRefresh = 50;
  double rho_b = 0.0;  // ρ̄ of the PCG solve whose x̃, r and bk are in place; 0: none
  // A check's dual-residual pass also forms B·g for the next iteration (when the window of
  // pairs fits in LDS and the check's PCG solve took at most kTrackedPcg steps): that
  // iteration's recurrence then runs as a vector pass.
  int bg_for = -1;     // the ADMM iteration whose B·g is in V.bg
  double bg_rho = 0.0;  // ρ̄ of that g
  auto rhs = [&](const int32_t* gate, int kk) {
    if (rho_b > 0.0 && kk % kRhsRefresh != 0) {
      OpRhsRec<T> rc{V.x, V.xt, V.qb, V.g, V.dinv, V.r, V.p, V.bk, (T)sigma, (T)(rho / rho_b),
                     s.pcg_max_iter, s.pcg_rel_test, eps_pcg, st};
      if (bg_for == kk) {
        const int gn = grid_for(n);
        if (rho == bg_rho) {
          hipLaunchKernelGGL((k_rows<T, OpRhsRec<T>>), dim3(gn), dim3(kBlock), 0, stream, n,
                             (const T*)V.bg, (const T*)V.bg + n, rc, rb.partials, gate);
          finalize(rc, gn, gate);
        } else {
          OpRhsRescaled<T> rs{rc, (const T*)V.bg + 2 * (size_t)n, (T)(rho / bg_rho)};
          hipLaunchKernelGGL((k_rows<T, OpRhsRescaled<T>>), dim3(gn), dim3(kBlock), 0, stream, n,
                             (const T*)V.bg, (const T*)V.bg + n, rs, rb.partials, gate);
          finalize(rs, gn, gate);
        }
      } else {
        finalize(rc, spmv_B<T>(rc, gate), gate);
      }
    } else {
      pairs<T>(rho);
      spmv_B<T>(OpRhsAt<T>{V.g + (size_t)n + m, V.bk}, gate);
      OpRhsR0<T> rr{V.x, V.xt, V.qb, V.g, V.dinv, V.r, V.p, V.bk, (T)sigma,
                    s.pcg_max_iter, s.pcg_rel_test, eps_pcg, st};
      finalize(rr, spmv_B<T>(rr, gate), gate);
    }
    rho_b = rho;
  };
  int k = k_start;
  int it = 0;
  while (k <= s.max_iter) {
    // PCG tolerance as a decreasing function of k (the alternative Section 6.3.3 attributes to
    // SCS), when chosen instead of the residual rule: ε_k = max(λ·(k + 1)^(−3/2), ε_min)
    if (!fixed_eps && s.pcg_eps_schedule == 1)
      eps_pcg = std::max(s.pcg_lambda * std::pow((double)k + 1.0, -1.5), s.pcg_eps_min);
    const bool check = (k % s.check_every == 0 || k == s.max_iter);
    if (trial) {
      if (pending) {  // read the speculation's outcome first
        hipLaunchKernelGGL(k_mirror<DevState>, dim3(1), dim3(64), 0, stream, (const DevState*)st, st_mirror_dev);
        sync_state();
        pending = false;
        if (st_host->abort) {
          k = resume();
          if (k < 0) return finish(st_host->abort_k);
          continue;
        }
      }
      copy(V.b, (const T*)V.xt, n);  // the warm start, kept for the second run
      learned_dinv<T>(rho);
      rho_b = 0.0;  // both runs start from the same warm start, with the right-hand side direct
      rhs(nullptr, k);
      const int it_l = pcg_loop<T>(rho, s.pcg_max_iter, true);
      const double rn_l = st_host->rnorm;
      const bool cap_l = it_l >= s.pcg_max_iter && rn_l > st_host->thresh;
      const bool broke_l = st_host->breakdown != 0;
      copy(V.xt, (const T*)V.b, n);
      spmv_A<T>(OpScaled<T>{V.xt, V.zt, (T)1});  // z̃ = Āx̃ of the restored warm start
      jacobi<T>(rho);
      rho_b = 0.0;
      rhs(nullptr, k);
      it = pcg_loop<T>(rho, s.pcg_max_iter, true);
      const bool cap_j = it >= s.pcg_max_iter && st_host->rnorm > st_host->thresh;
      use_learned = !broke_l && ((!cap_l && it_l < it) || (cap_l && cap_j && rn_l < st_host->rnorm));
      lost_in_a_row = use_learned ? 0 : lost_in_a_row + 1;
      rho_trial = rho;
      info.precond_trials++;
      if (use_learned) {
        info.precond_learned_chosen++;
        learned_dinv<T>(rho);
      }
      info.pcg_iter_total += it_l;
      trial = false;
      if (after_pcg(k, it)) return finish(k);
    } else if (!check && s.speculate && last_pcg <= kSpecMaxPcg) {
      // speculative: PCG with the predicted iteration count, no host read (only where PCG takes
      // few steps: there a host read is a large share of the iteration, and the predicted count
      // is rarely short; with tens of steps an abort costs more than the reads it saves)
      rhs(agate, k);
      const int b = std::max(1, std::min(last_pcg, s.pcg_max_iter));
      for (int i = 0; i < b; ++i) pcg_iteration<T>(rho, true, false, i, i == b - 1 ? k : -1);
      pending = true;
    } else {
      rhs(agate, k);
      // (a3)–(a6) PCG iterations
      it = pcg_loop<T>(rho, s.pcg_max_iter, true);
      if (st_host->abort) {  // a speculative iteration before this one needs the host
        k = resume();
        if (k < 0) return finish(st_host->abort_k);
        continue;
      }
      pending = false;
      if (after_pcg(k, it)) return finish(k);
    }
    T* dxy = (check && infeas && armed) ? V.dxy : nullptr;  // δx̄, δȳ of this step (Section 3.1)
    launch_update(check, dxy, k);
    if (!check) {
      ++k;
      continue;
    }
    // (a9) residuals and termination every check_every iterations. The update pass gave the
    // primal residual from the tracked Āx̄. In FP32 that recurrence also carries the rounding
    // drift of z̃ through the PCG iterations, so a solve that took more than kTrackedPcg PCG
    // iterations recomputes Āx̄ by an Ā pass, and a check that would stop the solve confirms the
    // primal residual by that pass first: drift can neither fake nor delay convergence there.
    {
      constexpr int kTrackedPcg = 4;
      const bool fp32 = std::is_same<T, float>::value;
      bool exact = !fp32;
      auto exact_prim = [&](bool mirror) {
        OpRPrim<T> rp{V.x, V.z, escale, st};
        finalize(rp, spmv_A<T>(rp), nullptr, mirror);
        exact = true;
      };
      if (!exact && it > kTrackedPcg) exact_prim(false);
      OpRDual<T> rd{V.x, V.y, V.qb, dscale, n, st};
      // with many PCG steps per ADMM step the saved B pass is a small share of the work
      if (pair_fits<T>() && k < s.max_iter && it <= kTrackedPcg) {
        finalize(rd, spmv_B_pair<T>(OpRDualRhs<T>{rd, V.g, V.bg}), nullptr, true);
        bg_for = k + 1;
        bg_rho = rho;
      } else {
        finalize(rd, spmv_B<T>(rd), nullptr, true);
      }
      sync_state();
      const double* nm = st_host->norms;
      double prim = nm[1], nAx = nm[3], nz = nm[5];
      const double dual = nm[7] / c, nPx = nm[9] / c, nAty = nm[11] / c;
      double eps_p = s.eps_abs + s.eps_rel * std::max(nAx, nz);
      const double eps_d = s.eps_abs + s.eps_rel * std::max(std::max(nPx, nAty), q_norm);
      if (!exact && prim <= eps_p && dual <= eps_d) {
        exact_prim(true);
        sync_state();
        prim = nm[1];
        nAx = nm[3];
        nz = nm[5];
        eps_p = s.eps_abs + s.eps_rel * std::max(nAx, nz);
      }
      info.prim_res = prim;
      info.dual_res = dual;
      info.obj_val = (0.5 * nm[12] + nm[13]) / c;
      info.iter = k;
      if (s.verbose)
        std::fprintf(stderr, "qpg %5d  prim %.3e (%.1e)  dual %.3e (%.1e)  rho %.3e  pcg %d  %s\n", k,
                     prim, eps_p, dual, eps_d, rho, it, std::is_same<T, float>::value ? "fp32" : "fp64");
      if (!(prim == prim) || !(dual == dual)) {
        if (std::is_same<T, float>::value)
          fallback_request = 1;
        else
          status = QPG_NUMERICAL_ERROR;
        return finish(k);
      }
      if (prim <= eps_p && dual <= eps_d) {
        status = QPG_SOLVED;
        return finish(k);
      }
      // infeasibility certificates from the differences of this step (Section 3, 3.1)
      if (dxy) {
        info.infeas_checks++;
        OpInfeasA<T> ia{V.dxy, V.lb, V.ub, escale, n, st};
        finalize(ia, spmv_A<T>(ia));
        OpInfeasB<T> ib{V.dxy, V.qb, dscale, st};
        finalize(ib, spmv_B<T>(ib), nullptr, true);
        sync_state();
        const int inf = infeasibility_status();
        if (s.verbose) {
          const double* q = st_host->norms;
          std::fprintf(stderr, "qpg        pinf: |Atdy|/|dy| %.2e  support/|dy| %.2e   dinf: |Pdx|/|dx| %.2e  "
                       "qdx/|dx| %.2e  Adx viol/|dx| %.2e\n", q[20] / q[17], q[18] / q[17], q[19] / c / q[21],
                       q[22] / c / q[21], q[16] / q[21]);
        }
        if (inf != QPG_UNSOLVED) {
          keep_certificate<T>();
          status = inf;
          return finish(k);
        }
      }
      // FP32 stagnation: no 1% improvement of the worse normalised residual in 20 checks
      const double ratio = std::max(prim / std::max(eps_p, 1e-300), dual / std::max(eps_d, 1e-300));
      if (ratio < 0.99 * best_ratio) {
        best_ratio = ratio;
        since_best = 0;
      } else if (++since_best >= 20 && std::is_same<T, float>::value) {
        fallback_request = 1;
        return finish(k);
      }
      armed = since_best >= kInfeasAfter;
      // PCG tolerance from the scaled residuals (Section 6.3.3). With the relative test
      // ‖r‖ ≤ ε‖b‖ the rule is capped at λ: a larger ε (residuals above 1/λ²) would let PCG stop
      // at zero iterations, freezing x̃ while ADMM stalls.
      // Stall guard (not in the paper): the rule keeps ε large while the residuals stay large,
      // which is what they do on an infeasible problem, and steps that inexact leave the
      // differences δx̄, δȳ of Section 3 too noisy to pass its tests. After 10 checks without a
      // 1% gain in the worse normalised residual, ε is divided by 10 at every second check.
      if (since_best >= 10 && since_best % 2 == 0) tighten = std::max(tighten * 0.1, 1e-12);
      if (!fixed_eps && s.pcg_eps_schedule == 0) {
        eps_pcg = s.pcg_lambda * std::sqrt(nm[0] * nm[6]);
        if (s.pcg_rel_test) eps_pcg = std::min(eps_pcg, s.pcg_lambda);
        eps_pcg = std::max(eps_pcg * tighten, s.pcg_eps_min);
      }
      // ρ̄ update (Section 3.4, every rho_update_every iterations, Section 6.3.2)
      if (s.rho_update_every > 0 && k % s.rho_update_every == 0) {
        const double num = nm[0] / std::max(std::max(nm[2], nm[4]), 1e-10);
        const double den = nm[6] / std::max(std::max(std::max(nm[8], nm[10]), qb_norm), 1e-10);
        if (den > 0 && num > 0) {
          double est = std::min(std::max(rho * std::sqrt(num / den), 1e-6), 1e6);
          if (est >= s.rho_update_gate * rho || est <= rho / s.rho_update_gate) {
            if (est != rho) {
              rho = est;
              info.rho_updates++;
              const bool moved = est > 2.0 * rho_trial || est < 0.5 * rho_trial;
              if (learned_ok && s.precond_trial && moved && lost_in_a_row < 2)
                trial = true;
              else if (use_learned)
                learned_dinv<T>(rho);
              else
                jacobi<T>(rho);
              pairs<T>(rho);  // g with the new ρ̄ (the check's B·g is rescaled to it)
            }
          }
        }
      }
    }
    ++k;
  }
  status = QPG_MAX_ITER_REACHED;
  return finish(std::min(k, s.max_iter));
}

int qpg_solver::solve() {
  auto t0 = std::chrono::steady_clock::now();
  info.status = QPG_UNSOLVED;
  cert_valid = false;
  have_out = false;
  info.iter = 0;
  info.pcg_iter_total = 0;
  info.pcg_iter_max = 0;
  info.rho_updates = 0;
  info.fallback_events = 0;
  info.precond_trials = 0;
  info.precond_learned_chosen = 0;
  info.precond_switches = 0;
  info.infeas_checks = 0;
  info.spec_resumes = 0;
  info.prim_res = info.dual_res = INFINITY;
  info.obj_val = NAN;
  double rho = s.rho;
  double eps_pcg = s.pcg_eps_fixed > 0 ? s.pcg_eps_fixed : s.pcg_lambda;
  int status = QPG_UNSOLVED;
  last_pcg = 1;
  bool use32 = (s.precision == QPG_MIXED);
  int k_end = 0;
  if (use32) {
    Prec<float>& V = p32;
    fill(V.x, n, 0.f);
    fill(V.xt, n, 0.f);
    fill(V.z, m, 0.f);
    fill(V.y, m, 0.f);
    fill(V.zt, m, 0.f);
    fill(p64.ax, m, 0.0);
    pairs<float>(rho);
    int fb = 0;
    k_end = admm<float>(1, rho, eps_pcg, status, fb);
    if (fb) {
      // continue in FP64 from the FP32 iterates
      info.fallback_events++;
      use32 = false;
      Prec<double>& W = p64;
      hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(kBlock), 0, stream, n, W.x, V.x);
      hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(kBlock), 0, stream, n, W.xt, V.xt);
      if (m > 0) {
        hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(m)), dim3(kBlock), 0, stream, m, W.z, V.z);
        hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(m)), dim3(kBlock), 0, stream, m, W.y, V.y);
      }
      // z̃ = Āx̃ and the tracked Āx are recomputed in FP64 from the converted iterates
      spmv_A<double>(OpScaled<double>{W.xt, W.zt, 1.0});
      spmv_A<double>(OpScaled<double>{W.x, W.ax, 1.0});
      pairs<double>(rho);
      int fb2 = 0;
      last_pcg = 1;
      k_end = admm<double>(k_end, rho, eps_pcg, status, fb2);
    }
  } else {
    Prec<double>& V = p64;
    fill(V.x, n, 0.0);
    fill(V.xt, n, 0.0);
    fill(V.z, m, 0.0);
    fill(V.y, m, 0.0);
    fill(V.zt, m, 0.0);
    fill(V.ax, m, 0.0);
    pairs<double>(rho);
    int fb = 0;
    k_end = admm<double>(1, rho, eps_pcg, status, fb);
  }
  info.status = status;
  info.rho_final = rho;
  info.precond_used = last_precond_learned ? QPG_PRECOND_LEARNED : QPG_PRECOND_JACOBI;
  info.precision_used = use32 ? QPG_MIXED : QPG_FP64;
  // unscaled iterates x = D x̄, z = E⁻¹ z̄, y = E ȳ / c, formed on the device and copied once into
  // pinned host memory
  const int gu = grid_for(n + m);
  if (use32)
    hipLaunchKernelGGL((k_unscale<float>), dim3(gu), dim3(kBlock), 0, stream, n, m, (const float*)p32.x,
                       (const float*)p32.y, (const float*)p32.z, (const double*)de, c, out_dev);
  else
    hipLaunchKernelGGL((k_unscale<double>), dim3(gu), dim3(kBlock), 0, stream, n, m, (const double*)p64.x,
                       (const double*)p64.y, (const double*)p64.z, (const double*)de, c, out_dev);
  HIPCHK(hipMemcpyAsync(out_host, out_dev, ((size_t)n + 2 * (size_t)m) * sizeof(double), hipMemcpyDeviceToHost,
                        stream));
  HIPCHK(hipStreamSynchronize(stream));
  HIPCHK(hipGetLastError());
  have_out = true;
  info.iter = k_end;
  info.solve_time = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return QPG_OK;
}

// =============================================================================== C ABI

namespace {

int device_error(qpg_solver* h, const HipError& e) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s failed: %s", e.what, hipGetErrorString(e.code));
  if (h) h->err = buf;
  else g_setup_error = buf;
  (void)hipGetLastError();
  return (e.code == hipErrorOutOfMemory) ? QPG_ERR_OOM : QPG_ERR_DEVICE;
}

template <typename T>
void to_device(qpg_solver* h, T* d, const double* src, int count) {
  std::vector<T> t(src, src + count);
  if (count) HIPCHK(hipMemcpyAsync(d, t.data(), count * sizeof(T), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
}

template <typename T>
void from_device(qpg_solver* h, double* dst, const T* d, int count) {
  std::vector<T> t(count);
  if (count) HIPCHK(hipMemcpyAsync(t.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < count; ++i) dst[i] = (double)t[i];
}

template <typename T>
int apply_impl(qpg_solver* h, int op, const double* in, double* out) {
  Prec<T>& V = h->P<T>();
  const int n = h->n, m = h->m;
  switch (op) {
    case QPG_OP_A:
      to_device<T>(h, V.p, in, n);
      h->spmv_A<T>(OpScaled<T>{V.p, V.w, (T)1});
      from_device<T>(h, out, V.w, m);
      break;
    case QPG_OP_AT:
      to_device<T>(h, V.w, in, m);
      h->spmv_B<T>(OpB<T>{nullptr, V.w, V.kp, n});
      from_device<T>(h, out, V.kp, n);
      break;
    case QPG_OP_P:
      to_device<T>(h, V.p, in, n);
      h->spmv_B<T>(OpB<T>{V.p, nullptr, V.kp, n});
      from_device<T>(h, out, V.kp, n);
      break;
    case QPG_OP_K:
      to_device<T>(h, V.p, in, n);
      h->spmv_A<T>(OpScaled<T>{V.p, V.w, (T)h->rho_cur, h->eqrow});
      h->spmv_B<T>(OpKp<T>{V.p, V.w, V.kp, (T)h->s.sigma, n, h->st});
      from_device<T>(h, out, V.kp, n);
      break;
    default:
      h->err = "qpg_apply: unknown operator";
      return QPG_ERR_ARG;
  }
  HIPCHK(hipGetLastError());
  return QPG_OK;
}

template <typename T>
int pcg_impl(qpg_solver* h, const double* b, const double* x0, double eps, int rel, int maxit,
             double* x, int32_t* iters, double* rnorm) {
  Prec<T>& V = h->P<T>();
  to_device<T>(h, V.b, b, h->n);
  to_device<T>(h, V.xt, x0, h->n);
  if (h->s.precond == QPG_PRECOND_LEARNED)
    h->learned_dinv<T>(h->rho_cur);
  else
    h->jacobi<T>(h->rho_cur);
  hipLaunchKernelGGL((k_absmax<T>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, h->n, (const T*)V.b,
                     h->rb.partials);
  h->finalize_fn<1, 1u>(FinThresh{h->st, eps, rel}, h->vgrid);
  h->last_pcg = 1;
  int it = h->pcg_solve<T>(h->rho_cur, maxit);
  from_device<T>(h, x, V.xt, h->n);
  if (iters) *iters = it;
  if (rnorm) *rnorm = h->st_host->rnorm;
  HIPCHK(hipGetLastError());
  return h->st_host->breakdown ? QPG_ERR_STATE : QPG_OK;
}

template <typename T>
int time_kernel_impl(qpg_solver* h, int kernel, int reps, double* avg_us) {
  Prec<T>& V = h->P<T>();
  auto launch = [&]() {
    switch (kernel) {
      case QPG_KERNEL_SPMV_A:
        h->spmv_A<T>(OpScaled<T>{V.p, V.w, (T)h->rho_cur, h->eqrow});
        break;
      case QPG_KERNEL_SPMV_B:
        h->spmv_B<T>(OpKp<T>{V.p, V.w, V.kp, (T)h->s.sigma, h->n, h->st});
        break;
      case QPG_KERNEL_SPMV_A_STREAM:
        h->spmv<T>(h->plan_a, INT32_MAX, 1, OpScaled<T>{V.p, V.w, (T)h->rho_cur, h->eqrow}, nullptr, false);
        break;
      case QPG_KERNEL_SPMV_B_STREAM:
        h->spmv<T>(h->plan_b, h->n, 2, OpKp<T>{V.p, V.w, V.kp, (T)h->s.sigma, h->n, h->st}, nullptr, false);
        break;
      case QPG_KERNEL_PCG_UPDATE:
        hipLaunchKernelGGL((k_pcg_update<T>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, h->n, V.xt,
                           V.r, V.p, V.kp, V.dinv, h->st, (const double*)h->rb.partials, h->plan_b.ncomb,
                           h->rb.vpartials, (const int32_t*)nullptr, h->m, V.zt, (const T*)V.w,
                           (T)(1.0 / h->rho_cur), 0);
        break;
      default:
        hipLaunchKernelGGL((k_pcg_dir<T>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, h->n, V.p,
                           (const T*)V.r, (const T*)V.dinv, h->st, (const double*)h->rb.vpartials, h->vgrid,
                           (const int32_t*)nullptr, 0, (DevState*)nullptr);
    }
  };
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  launch();
  HIPCHK(hipEventRecord(e0, h->stream));
  for (int i = 0; i < reps; ++i) launch();
  HIPCHK(hipEventRecord(e1, h->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  *avg_us = 1e3 * (double)ms / reps;
  return QPG_OK;
}

}  // namespace

TilePlan qpg_solver::plan_tiles(const std::vector<int32_t>& rowptr, const int32_t* col, int32_t nrows,
                               int32_t ncols) const {
  TileParams tp{win_cols, s.spmv_tile_nnz > 0 ? s.spmv_tile_nnz : kTileNnz,
                s.spmv_plain_nnz > 0 ? s.spmv_plain_nnz : kPlainNnz, kTileMaxRows,
                s.spmv_min_seg > 0 ? s.spmv_min_seg : kMinSeg,
                // the grid layout stages windows of 16384 columns for short rows: it pays in float
                // (64 KB of LDS per window), not in double (128 KB, one workgroup per CU)
                s.precision == QPG_MIXED,
                // the entries in SELL order are written on the device (upload_plan)
                false};
  return make_tiles(rowptr, col, nrows, ncols, tp);
}

// The work list on the device. The entries in SELL order (CSR index and column of every
// position) are written there from the lanes and the pattern's columns dcol, already on the
// device, instead of being built on the host and uploaded.
void qpg_solver::upload_plan(DevPlan& pl, TilePlan& t, const std::vector<int32_t>& rowptr, int32_t nrows,
                             const int32_t* dcol) {
  if (t.tiles.empty()) t.tiles.push_back(Tile{0, 0, 0, 0});
  if (t.comb.empty()) t.comb.push_back(CombItem{0, 0, 0, 0});
  pl.ncomb = (int32_t)t.comb.size();
  pl.comb = upload(t.comb);
  pl.ntiles = (int32_t)t.tiles.size();
  pl.tiles = upload(t.tiles);
  pl.chunks = upload(t.chunks);
  pl.segslot = upload(t.segslot);
  pl.rowslot = upload(t.rowslot);
  pl.slotidx = upload(t.slotidx);
  pl.tbase = upload(t.tbase);
  pl.nsrc = t.n_src;
  pl.src = alloc<int32_t>((size_t)t.n_src);
  pl.col16 = alloc<uint16_t>((size_t)t.n_c16);
  pl.col32 = alloc<int32_t>((size_t)t.n_c32);
  int32_t* lstart = upload(t.lstart);
  int32_t* llen = upload(t.llen);
  const int64_t nnz = (int64_t)rowptr[nrows] - rowptr[0];
  const int g = std::max(1, std::min(pl.ntiles, 65536));
  hipLaunchKernelGGL(k_sell_build, dim3(g), dim3(kBlock), 0, stream, (const Tile*)pl.tiles, pl.ntiles,
                     (const Chunk*)pl.chunks, (int64_t)t.chunks.size(), (const int32_t*)lstart,
                     (const int32_t*)llen, dcol, nnz, pl.src, t.n_src, pl.col16, t.n_c16, pl.col32, t.n_c32);
  HIPCHK(hipGetLastError());
  pl.nslot = t.nslot;
  pl.nrows = nrows;
  // B's slots hold four planes (the two-vector pass of the checks), Ā's two
  pl.slots = alloc<double>((&pl == &plan_b ? 4 : 2) * (size_t)std::max<int64_t>(t.nslot, 1));
  pl.max_wlen = t.max_wlen;
  int64_t staged = 0, wtiles = 0;
  for (const Tile& x : t.tiles) {
    staged += x.wlen;
    wtiles += x.wlen > 0;
  }
  const int64_t layout[8] = {nnz, t.n_c16, t.n_c32, (int64_t)t.tiles.size(), wtiles, staged, t.nslot,
                             (int64_t)t.chunks.size()};
  std::copy(layout, layout + 8, pl.layout);
  HIPCHK(hipStreamSynchronize(stream));  // t's host arrays go out of scope
  free_tracked(lstart);
  free_tracked(llen);
}

// Values in the plan's SELL order (zero in the padding), gathered on the device from the
// equilibrated CSR values through the plan's CSR index of every SELL position; FP32 copies cast
// from them.
void qpg_solver::place_values(DevPlan& pl, const double* csr_val, bool fp32) {
  const size_t count = (size_t)pl.nsrc;
  pl.val64 = alloc<double>(count);
  if (count) {
    const int g = (int)std::min<size_t>((count + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_gather_values, dim3(g), dim3(kBlock), 0, stream, (int64_t)count, (const int32_t*)pl.src,
                       csr_val, pl.val64);
  }
  if (fp32) {
    pl.val32 = alloc<float>(count);
    if (count)
      hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for((int)count)), dim3(kBlock), 0, stream,
                         (int)count, pl.val32, (const double*)pl.val64);
  }
  HIPCHK(hipStreamSynchronize(stream));
  free_tracked(pl.src);
  pl.src = nullptr;
}

// Modified Ruiz equilibration (Algorithm 2) of the uploaded raw problem, on the device (see
// ruiz.hpp); then diag(P̄), ‖Ā_i‖², l̄ = El, ū = Eu, D⁻¹, E⁻¹. Readings: P̄ ← c·DPD (so that
// P̄ = cDPD holds after every pass); stop after a pass whose δ satisfies ‖1 − δ‖∞ ≤ 1e-3, at most
// scaling_iters passes; norms below 1e-4 count as 1 and are capped at 1e4 (also for the
// denominator of γ). The host keeps D, E, c, ‖q̄‖∞, diag(P̄) and ‖Ā_i‖².
void qpg_solver::equilibrate() {
  Prec<double>& V = p64;
  const size_t nm = (size_t)n + m;
  double* work = nullptr;  // D, E, δ_D, δ_E, row norms of B and Ā, P̄ row norms
  HIPCHK(hipMalloc((void**)&work, (3 * nm + (size_t)n + 1) * sizeof(double)));
  double *Dd = work, *Ed = Dd + n, *dD = Ed + m, *dE = dD + n, *rB = dE + m, *rA = rB + n, *pB = rA + m;
  try {
    fill(Dd, (int)nm, 1.0);  // D and E
    hipLaunchKernelGGL(k_ruiz_init, dim3(1), dim3(64), 0, stream, st);
    auto rows_grid = [](int rows) { return std::max(1, std::min((rows + 3) / 4, 16384)); };
    const int gB = rows_grid(n), gA = rows_grid(m), gv = grid_for((int)nm), gn = grid_for(n);
    int passes = 0;
    while (passes < s.scaling_iters) {
      hipLaunchKernelGGL(k_ruiz_norms_B, dim3(gB), dim3(kBlock), 0, stream, n, (const int32_t*)b_ptr,
                         (const int32_t*)b_split, V.b_val, (const DevState*)st, rB);
      if (m)
        hipLaunchKernelGGL(k_ruiz_norms_A, dim3(gA), dim3(kBlock), 0, stream, m, (const int32_t*)a_ptr,
                           (const double*)V.a_val, rA);
      hipLaunchKernelGGL(k_ruiz_delta, dim3(gv), dim3(kBlock), 0, stream, n, m, (const double*)rB,
                         (const double*)rA, Dd, Ed, dD, dE, V.qb, (const DevState*)st, rb.partials);
      finalize_fn<2, 3u>(FinRuizDelta{st}, gv);
      hipLaunchKernelGGL(k_ruiz_scale_B, dim3(gB), dim3(kBlock), 0, stream, n, (const int32_t*)b_ptr,
                         (const int32_t*)b_split, (const int32_t*)b_col, V.b_val, (const double*)dD,
                         (const double*)dE, pB);
      if (m)
        hipLaunchKernelGGL(k_ruiz_scale_A, dim3(gA), dim3(kBlock), 0, stream, m, (const int32_t*)a_ptr,
                           (const int32_t*)a_col, V.a_val, (const double*)dD, (const double*)dE);
      hipLaunchKernelGGL(k_ruiz_pmean, dim3(gn), dim3(kBlock), 0, stream, n, (const double*)pB, rb.partials);
      finalize_fn<1, 0u>(FinRuizGamma{st, n}, gn, nullptr, true);
      sync_state();
      ++passes;
      if (st_host->norms[kRuizDev] <= 1e-3) break;
    }
    hipLaunchKernelGGL(k_ruiz_final_B, dim3(gB), dim3(kBlock), 0, stream, n, (const int32_t*)b_ptr,
                       (const int32_t*)b_split, (const int32_t*)b_col, V.b_val, (const DevState*)st,
                       (const uint8_t*)eqrow, diagP, colsq, colsq_eq);
    hipLaunchKernelGGL(k_ruiz_final_vec, dim3(gv), dim3(kBlock), 0, stream, n, m, V.qb, V.lb, V.ub,
                       (const double*)Dd, (const double*)Ed, dscale, escale, (const DevState*)st, rb.partials);
    finalize_fn<1, 1u>(FinRuizFinal{st}, gv, nullptr, true);
    sync_state();
    c = st_host->norms[kRuizC];
    qb_norm = st_host->norms[kRuizQmax];
    scaling_passes = passes;
    de = alloc<double>((size_t)n + m);
    HIPCHK(hipMemcpyAsync(de, Dd, ((size_t)n + m) * sizeof(double), hipMemcpyDeviceToDevice, stream));
    D.resize(n);
    E.resize(m);
    diagP_h.resize(n);
    colsq_h.resize(n);
    HIPCHK(hipMemcpyAsync(D.data(), Dd, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    if (m) HIPCHK(hipMemcpyAsync(E.data(), Ed, m * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(diagP_h.data(), diagP, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(colsq_h.data(), colsq, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
  } catch (...) {
    (void)hipFree(work);
    throw;
  }
  HIPCHK(hipFree(work));
}

extern "C" {

int qpg_time_kernel(qpg_solver* h, int32_t kernel, int32_t precision, int32_t reps, double* avg_us) {
  if (!h || !avg_us || reps < 1 || kernel < 0 || kernel > QPG_KERNEL_SPMV_B_STREAM) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    if (precision == QPG_FP64) return time_kernel_impl<double>(h, kernel, reps, avg_us);
    if (precision == QPG_MIXED && h->p32.ready) return time_kernel_impl<float>(h, kernel, reps, avg_us);
    h->err = "qpg_time_kernel: precision not available";
    return QPG_ERR_STATE;
  } catch (const HipError& e) {
    return device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_spmv_layout(const qpg_solver* h, int32_t matrix, int64_t out[8]) {
  if (!h || !out || (matrix != 0 && matrix != 1)) return QPG_ERR_ARG;
  const DevPlan& pl = matrix == 0 ? h->plan_a : h->plan_b;
  std::copy(pl.layout, pl.layout + 8, out);
  return QPG_OK;
}

int qpg_setup(qpg_solver** out, const qpg_csc* P_triu, const double* q, const qpg_csc* A,
              const double* l, const double* u, const qpg_settings* settings) {
  g_setup_error.clear();
  if (!out) {
    g_setup_error = "out: null";
    return QPG_ERR_ARG;
  }
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  // with settings->verbose, the time of each setup phase on stderr (the stream is synchronised
  // at every mark, so device work is charged to the phase that queued it)
  auto tmark = t0;
  auto mark = [&](const char* phase, hipStream_t st) {
    if (!settings || !settings->verbose) return;
    if (st) (void)hipStreamSynchronize(st);
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "qpg setup  %-34s %8.1f ms\n", phase,
                 std::chrono::duration<double, std::milli>(now - tmark).count());
    tmark = now;
  };
  HostProblem H;
  std::string msg;
  int rc;
  try {
    rc = prepare(P_triu, q, A, l, u, settings, &H, &msg, false);
  } catch (const std::bad_alloc&) {
    rc = QPG_ERR_OOM;
    msg = "host allocation failed";
  }
  if (rc) {
    g_setup_error = msg;
    return rc;
  }
  mark("host checks, full P, B = [P | A^T]", nullptr);
  qpg_solver* h = new (std::nothrow) qpg_solver();
  if (!h) {
    g_setup_error = "host allocation failed";
    return QPG_ERR_OOM;
  }
  h->s = *settings;
  h->n = H.n;
  h->m = H.m;
  h->device = settings->device;
  h->stream = static_cast<hipStream_t>(settings->stream);
  try {
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(resolve_noalloc_scratch(h->device));
    // SpMV work lists: the window capacity is capped so that a window of doubles fits in one
    // workgroup's LDS. They depend on the sparsity pattern only, so two host threads (Ā, B)
    // build them while the device equilibrates the values; B's starts while A is converted to
    // CSR.
    int lds_max = 0;
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->lds_max = lds_max;
    h->win_cols = settings->spmv_window_cols > 0 ? settings->spmv_window_cols : kWinCols;
    while (h->win_cols > 1024 && (size_t)h->win_cols * sizeof(double) + 1024 > (size_t)lds_max)
      h->win_cols >>= 1;
    TilePlan ta, tb;
    std::exception_ptr plan_err_a, plan_err_b;
    std::thread planner_a, planner_b, stager;
    struct Join {  // the planners read H: the threads are joined on every way out of this block
      std::thread& a;
      std::thread& b;
      std::thread& s;
      ~Join() {
        for (std::thread* t : {&a, &b, &s})
          if (t->joinable()) t->join();
      }
    } join{planner_a, planner_b, stager};
    // the uploads' pinned staging buffers (once per device and process) are made ready beside
    // the host's conversion of A
    stager = std::thread(warm_staging, h->device);
    planner_b = std::thread([&]() {
      try {
        tb = h->plan_tiles(H.b_ptr, H.b_col.data(), H.n, H.n + H.m);
      } catch (...) {
        plan_err_b = std::current_exception();
      }
    });
    prepare_a(A, &H);
    mark("A in CSR (host)", nullptr);
    planner_a = std::thread([&]() {
      try {
        ta = h->plan_tiles(H.a_ptr, H.a_col.data(), H.m, H.n);
      } catch (...) {
        plan_err_a = std::current_exception();
      }
    });
    Plan pa = make_plan(H.a_ptr, H.m);
    Plan pb = make_plan(H.b_ptr, H.n);
    for (Plan* pl : {&pa, &pb})
      if (pl->items.empty()) pl->items.push_back({0, 0, 0, 0, 0, 0, 0, 0});
    h->na_items = (int32_t)pa.items.size();
    h->nb_items = (int32_t)pb.items.size();
    h->vgrid = grid_for(h->n);
    h->nnzA = (int32_t)H.a_col.size();
    h->nnzB = (int32_t)H.b_col.size();
    h->a_ptr = h->upload(H.a_ptr);
    h->a_col = h->upload(H.a_col);
    h->b_ptr = h->upload(H.b_ptr);
    h->b_split = h->upload(H.b_split);
    h->b_col = h->upload(H.b_col);
    h->a_items = h->upload(pa.items);
    h->b_items = h->upload(pb.items);
    h->diagP = h->alloc<double>(H.n);
    h->colsq = h->alloc<double>(H.n);
    if (settings->rho_vector) {
      h->eqrow = h->upload(H.eqrow);
      h->colsq_eq = h->alloc<double>(H.n);
    }
    mark("index uploads", h->stream);
    h->dscale = h->alloc<double>(H.n);
    h->escale = h->alloc<double>(H.m);
    h->out_dev = h->alloc<double>((size_t)H.n + 2 * (size_t)H.m);
    HIPCHK(hipHostMalloc((void**)&h->out_host, ((size_t)H.n + 2 * (size_t)H.m) * sizeof(double),
                         hipHostMallocDefault));
    // partials hold up to max(work lists, vector grids) workgroups; the work-list counts are
    // known once the planner is done, so size them for the vector grids first
    int maxgrid = std::max(1024, std::max(h->na_items, h->nb_items));
    h->st = h->alloc<DevState>(1);
    HIPCHK(hipMemsetAsync(h->st, 0, sizeof(DevState), h->stream));
    HIPCHK(hipHostMalloc((void**)&h->st_host, sizeof(DevState), hipHostMallocMapped));
    std::memset(h->st_host, 0, sizeof(DevState));
    HIPCHK(hipHostGetDevicePointer((void**)&h->st_mirror_dev, h->st_host, 0));
    h->rb.partials = h->alloc<double>((size_t)maxgrid * kMaxSlots);
    h->rb.vpartials = h->alloc<double>((size_t)1024 * kMaxSlots);
    h->alloc_prec64(H);  // raw values, q, clamped bounds; vectors
    mark("value uploads", h->stream);
    h->equilibrate();
    mark("equilibration (device)", h->stream);
    planner_a.join();
    planner_b.join();
    if (plan_err_a) std::rethrow_exception(plan_err_a);
    if (plan_err_b) std::rethrow_exception(plan_err_b);
    mark("work lists (wait for the host thread)", nullptr);
    h->upload_plan(h->plan_a, ta, H.a_ptr, H.m, h->a_col);
    h->upload_plan(h->plan_b, tb, H.b_ptr, H.n, h->b_col);
    mark("work-list uploads", h->stream);
    if (std::max(h->plan_a.ncomb, h->plan_b.ncomb) > maxgrid) {
      maxgrid = std::max(h->plan_a.ncomb, h->plan_b.ncomb);
      h->rb.partials = h->alloc<double>((size_t)maxgrid * kMaxSlots);
    }
    if (settings->precision == QPG_MIXED) h->alloc_prec32();
    h->place_values(h->plan_a, h->p64.a_val, settings->precision == QPG_MIXED);
    h->place_values(h->plan_b, h->p64.b_val, settings->precision == QPG_MIXED);
    mark("values into SELL order", h->stream);
    for (double* v : {h->p64.x, h->p64.xt, h->p64.r, h->p64.p, h->p64.kp, h->p64.b}) h->fill(v, h->n, 0.0);
    for (double* v : {h->p64.z, h->p64.y, h->p64.w, h->p64.zt, h->p64.ax}) h->fill(v, h->m, 0.0);
    if (h->p32.ready) {
      for (float* v : {h->p32.x, h->p32.xt, h->p32.r, h->p32.p, h->p32.kp, h->p32.b}) h->fill(v, h->n, 0.f);
      for (float* v : {h->p32.z, h->p32.y, h->p32.w, h->p32.zt}) h->fill(v, h->m, 0.f);
    }
    h->q_norm = H.q_norm_unscaled;
    h->rho_cur = settings->rho;
    h->jacobi<double>(h->rho_cur);
    if (h->p32.ready) h->jacobi<float>(h->rho_cur);
    if (settings->precond == QPG_PRECOND_LEARNED) {
      h->precond_weights.assign(settings->precond_weights, settings->precond_weights + QPG_NET_NPARAMS);
      h->learned_prepare();  // graph and message-passing trunk: once per setup
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    mark("vectors, preconditioner", nullptr);
  } catch (const HipError& e) {
    int code = device_error(nullptr, e);
    delete h;
    return code;
  } catch (const std::bad_alloc&) {
    g_setup_error = "host allocation failed";
    delete h;
    return QPG_ERR_OOM;
  } catch (const std::exception& e) {
    g_setup_error = e.what();
    delete h;
    return QPG_ERR_HOST;
  }
  h->info.scaling_passes = h->scaling_passes;
  h->info.setup_time = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return QPG_OK;
}

int qpg_solve(qpg_solver* h) {
  if (!h) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    return h->solve();
  } catch (const HipError& e) {
    return device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_get_x(const qpg_solver* h, double* x) {
  if (!h || !x) return QPG_ERR_ARG;
  if (!h->have_out) return QPG_ERR_STATE;
  std::copy(h->out_host, h->out_host + h->n, x);
  return QPG_OK;
}

int qpg_get_y(const qpg_solver* h, double* y) {
  if (!h || (!y && h->m > 0)) return QPG_ERR_ARG;
  if (!h->have_out) return QPG_ERR_STATE;
  std::copy(h->out_host + h->n, h->out_host + h->n + h->m, y);
  return QPG_OK;
}

int qpg_get_z(const qpg_solver* h, double* z) {
  if (!h || (!z && h->m > 0)) return QPG_ERR_ARG;
  if (!h->have_out) return QPG_ERR_STATE;
  std::copy(h->out_host + h->n + h->m, h->out_host + h->n + 2 * (size_t)h->m, z);
  return QPG_OK;
}

int qpg_get_info(const qpg_solver* h, qpg_info* info) {
  if (!h || !info) return QPG_ERR_ARG;
  *info = h->info;
  return QPG_OK;
}

int qpg_get_scaling(const qpg_solver* h, double* D, double* E, double* c) {
  if (!h || !D || (!E && h->m > 0) || !c) return QPG_ERR_ARG;
  std::copy(h->D.begin(), h->D.end(), D);
  std::copy(h->E.begin(), h->E.end(), E);
  *c = h->c;
  return QPG_OK;
}

int qpg_get_certificate(const qpg_solver* h, double* dx, double* dy) {
  if (!h) return QPG_ERR_ARG;
  if (!h->cert_valid) return QPG_ERR_STATE;
  if (dx) std::copy(h->cert_x.begin(), h->cert_x.end(), dx);
  if (dy) std::copy(h->cert_y.begin(), h->cert_y.end(), dy);
  return QPG_OK;
}

int qpg_apply(qpg_solver* h, int32_t op, int32_t precision, const double* in, double* out) {
  if (!h || !in || !out) return QPG_ERR_ARG;
  if (op == QPG_OP_AT && h->m == 0) {
    std::fill(out, out + h->n, 0.0);
    return QPG_OK;
  }
  try {
    HIPCHK(hipSetDevice(h->device));
    if (precision == QPG_FP64) return apply_impl<double>(h, op, in, out);
    if (precision == QPG_MIXED) {
      if (!h->p32.ready) {
        h->err = "qpg_apply: float copies exist only when setup used QPG_MIXED";
        return QPG_ERR_STATE;
      }
      return apply_impl<float>(h, op, in, out);
    }
    h->err = "qpg_apply: bad precision";
    return QPG_ERR_ARG;
  } catch (const HipError& e) {
    return device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_pcg(qpg_solver* h, int32_t precision, const double* b, const double* x0, double eps,
            int32_t rel, int32_t max_iter, double* x, int32_t* iters, double* rnorm) {
  if (!h || !b || !x0 || !x || max_iter < 0 || !(eps >= 0)) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    if (precision == QPG_FP64) return pcg_impl<double>(h, b, x0, eps, rel, max_iter, x, iters, rnorm);
    if (precision == QPG_MIXED && h->p32.ready)
      return pcg_impl<float>(h, b, x0, eps, rel, max_iter, x, iters, rnorm);
    h->err = "qpg_pcg: precision not available";
    return QPG_ERR_STATE;
  } catch (const HipError& e) {
    return device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_set_rho(qpg_solver* h, double rho) {
  if (!h || !(rho > 0) || !std::isfinite(rho)) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    h->rho_cur = rho;
    h->jacobi<double>(rho);
    if (h->p32.ready) h->jacobi<float>(rho);
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (const HipError& e) {
    return device_error(h, e);
  } QPG_CATCH_HOST(h->err)
  return QPG_OK;
}

int qpg_cleanup(qpg_solver* h) {
  if (!h) return QPG_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return QPG_OK;
}

const char* qpg_error_string(int code) {
  switch (code) {
    case QPG_OK: return "ok";
    case QPG_ERR_ARG: return "invalid argument";
    case QPG_ERR_DATA: return "invalid problem data";
    case QPG_ERR_SIZE: return "problem too large for int32 indexing";
    case QPG_ERR_DEVICE: return "HIP device error";
    case QPG_ERR_OOM: return "out of memory";
    case QPG_ERR_STATE: return "invalid state";
    case QPG_ERR_HOST: return "host-side failure";
    default: return "unknown error";
  }
}

const char* qpg_last_error(const qpg_solver* h) {
  if (!h) return g_setup_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
