// The solver object shared by the translation units of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "qpg_internal.hpp"

using namespace qpg;

namespace qpg {

struct HipError {
  hipError_t code;
  const char* what;
};

#define HIPCHK(expr)                                         \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) throw HipError{e_, #expr};         \
  } while (0)

inline int grid_for(int n) {
  int g = (n + kBlock - 1) / kBlock;
  return std::max(1, std::min(g, 1024));
}

// Device arrays of one precision.
template <typename T>
struct Prec {
  T* a_val = nullptr;  // Ā values (CSR)
  T* b_val = nullptr;  // [P̄ | Āᵀ] values (CSR)
  T *qb = nullptr, *lb = nullptr, *ub = nullptr;
  T *x = nullptr, *z = nullptr, *y = nullptr, *xt = nullptr;  // ADMM iterates, PCG solution
  T *r = nullptr, *p = nullptr, *kp = nullptr, *b = nullptr, *dinv = nullptr;  // PCG (n)
  T* w = nullptr;   // ρ̄Āp (m)
  T* zt = nullptr;  // z̃ = Āx̃ of the last update pass (m)
  T* ax = nullptr;  // Āx tracked by its recurrence (m), FP64 only
  pair_t<T>* vw = nullptr;  // (ρ̄(z̃ − z) + y, ρ̄z − y) for the next right-hand side (m)
  bool ready = false;
};

struct LearnedState;  // learned-preconditioner data of a solver (learned.hip)
void destroy_learned(LearnedState* L);

}  // namespace qpg

struct qpg_solver {
  qpg_settings s{};
  int32_t n = 0, m = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;

  // structure shared by both precisions
  int32_t *a_ptr = nullptr, *a_col = nullptr, *b_ptr = nullptr, *b_split = nullptr,
          *b_col = nullptr;
  Item *a_items = nullptr, *b_items = nullptr, *b2_items = nullptr;
  int32_t na_items = 0, nb_items = 0, nb2_items = 0;
  int32_t nnzA = 0, nnzB = 0;
  double *diagP = nullptr, *colsq = nullptr, *dscale = nullptr, *escale = nullptr;  // D⁻¹, E⁻¹
  DevState* st = nullptr;
  DevState* st_host = nullptr;        // mapped pinned host memory, written by finalize kernels
  DevState* st_mirror_dev = nullptr;  // its device-side address
  RedBuf rb{};
  int32_t vgrid = 1;

  Prec<double> p64;
  Prec<float> p32;

  // host copies
  std::vector<double> D, E, diagP_h, colsq_h, x_out, y_out, z_out;
  double c = 1.0, q_norm = 0.0, qb_norm = 0.0;
  double rho_cur = 0.1;
  int32_t scaling_passes = 0;
  int32_t last_pcg = 1;
  bool last_precond_learned = false;
  qpg_info info{};
  std::string err;

  template <typename T>
  Prec<T>& P();

  template <typename T>
  T* alloc(size_t count) {
    void* ptr = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    allocs.push_back(ptr);
    return static_cast<T*>(ptr);
  }
  template <typename T>
  T* upload(const std::vector<T>& h) {
    T* d = alloc<T>(h.size());
    if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, stream));
    return d;
  }
  template <typename T, typename S>
  T* upload_as(const std::vector<S>& h) {
    std::vector<T> t(h.begin(), h.end());
    T* d = upload(t);
    HIPCHK(hipStreamSynchronize(stream));  // t goes out of scope
    return d;
  }

  qpg::LearnedState* learned = nullptr;  // created on first use of the learned preconditioner
  std::vector<float> precond_weights;     // network of QPG_PRECOND_LEARNED (copied at setup)

  void learned_prepare();
  template <typename T>
  void learned_dinv(double rho);

  ~qpg_solver() {
    if (learned) qpg::destroy_learned(learned);
    for (void* p : allocs) (void)hipFree(p);
    if (st_host) (void)hipHostFree(st_host);
  }

  // ----------------------------------------------------------------- launches
  // SpMV launches; the returned grid size is the number of partials a finalize must combine.
  template <typename T, class Op>
  int spmv_A(const Op& op, const int32_t* gate = nullptr) {
    hipLaunchKernelGGL((k_spmv<T, Op>), dim3(na_items), dim3(kBlock), 0, stream, a_items, a_ptr,
                       (const int32_t*)nullptr, a_col, P<T>().a_val, op, rb, gate);
    return na_items;
  }
  template <typename T, class Op>
  int spmv_B(const Op& op, const int32_t* gate = nullptr) {
    // two-product passes stage twice the products: they use the half-size work list
    const Item* items = Op::NV == 2 ? b2_items : b_items;
    const int ni = Op::NV == 2 ? nb2_items : nb_items;
    hipLaunchKernelGGL((k_spmv<T, Op>), dim3(ni), dim3(kBlock), 0, stream, items, b_ptr, b_split,
                       b_col, P<T>().b_val, op, rb, gate);
    return ni;
  }
  // Combine the partials of the previous launch (count workgroups) and run op's finalisation.
  template <class Op>
  void finalize(const Op& op, int count, const int32_t* gate = nullptr) {
    hipLaunchKernelGGL((k_finalize<Op::NS, Op::MAXMASK, Op>), dim3(1), dim3(kFinBlock), 0, stream,
                       (const double*)rb.partials, count, op, gate, (const DevState*)st, st_mirror_dev);
  }
  template <int NS, unsigned MASK, class Fin>
  void finalize_fn(const Fin& fin, int count, const int32_t* gate = nullptr) {
    hipLaunchKernelGGL((k_finalize<NS, MASK, Fin>), dim3(1), dim3(kFinBlock), 0, stream,
                       (const double*)rb.partials, count, fin, gate, (const DevState*)st, st_mirror_dev);
  }

  // Wait for the stream and read the device scalars. Every finalize kernel leaves a copy of
  // them in mapped host memory (st_host), so no copy is queued: the host polls the stream.
  void sync_state() {
    hipError_t e;
    while ((e = hipStreamQuery(stream)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) throw HipError{e, "hipStreamQuery"};
  }

  template <typename T>
  void jacobi(double rho) {
    hipLaunchKernelGGL((k_jacobi<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, P<T>().dinv, diagP,
                       colsq, s.sigma, rho);
  }

  // One PCG iteration (Algorithm 3), all on the device; skipped once st->done is set.
  template <typename T>
  void pcg_iteration(double rho) {
    Prec<T>& V = P<T>();
    const int32_t* gate = &st->done;
    spmv_A<T>(OpScaled<T>{V.p, V.w, (T)rho}, gate);
    OpKp<T> kp{V.p, V.w, V.kp, (T)s.sigma, n, st};
    finalize(kp, spmv_B<T>(kp, gate), gate);
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, V.xt, V.r, V.p,
                       V.kp, V.dinv, (const DevState*)st, rb.partials, gate);
    finalize_fn<2, 2u>(FinPcgUpdate{st}, vgrid, gate);
    hipLaunchKernelGGL((k_pcg_dir<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, V.p, V.r, V.dinv,
                       (const DevState*)st, gate);
  }

  // Run PCG iterations after the initialisation kernel until st->done. The first batch is one
  // shorter than the previous PCG solve took, so that iterations launched after convergence
  // (which exit at once) stay rare; then one iteration per host check. Returns the count.
  template <typename T>
  int pcg_loop(double rho, int maxit) {
    int issued = 0;
    int batch = std::max(1, std::min(last_pcg - 1, maxit));
    for (;;) {
      int k = std::min(batch, maxit - issued);
      for (int i = 0; i < k; ++i) pcg_iteration<T>(rho);
      issued += k;
      sync_state();
      if (st_host->done || issued >= maxit) break;
      batch = 1;
    }
    last_pcg = std::max(1, st_host->iter);
    return st_host->iter;
  }

  // PCG on K x̃ = b with b already in P<T>().b and the threshold in st; starts from P<T>().xt.
  template <typename T>
  int pcg_solve(double rho, int maxit) {
    Prec<T>& V = P<T>();
    spmv_A<T>(OpScaled<T>{V.xt, V.w, (T)rho});
    OpR0<T> r0{V.xt, V.w, V.b, V.dinv, V.r, V.p, (T)s.sigma, n, maxit, st};
    finalize(r0, spmv_B<T>(r0));
    return pcg_loop<T>(rho, maxit);
  }

  template <typename T>
  void pairs(double rho) {
    Prec<T>& V = P<T>();
    if (m > 0)
      hipLaunchKernelGGL((k_pairs<T>), dim3(grid_for(m)), dim3(kBlock), 0, stream, m, V.vw,
                         (const T*)V.zt, (const T*)V.z, (const T*)V.y, (T)rho);
  }

  template <typename T>
  void copy(T* dst, const T* src, int count) {
    if (count > 0)
      hipLaunchKernelGGL((k_cast<T, T>), dim3(grid_for(count)), dim3(kBlock), 0, stream, count, dst, src);
  }

  template <typename T>
  void fill(T* v, int count, T val) {
    if (count > 0)
      hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(count)), dim3(kBlock), 0, stream, count, v, val);
  }

  template <typename T>
  int admm(int k_start, double& rho, double& eps_pcg, int& status, int& fallback_request);

  int solve();
  void alloc_prec64(const HostProblem& H);
  void alloc_prec32(const HostProblem& H);
};

template <>
inline Prec<double>& qpg_solver::P<double>() {
  return p64;
}
template <>
inline Prec<float>& qpg_solver::P<float>() {
  return p32;
}
