// The solver object shared by the translation units of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <exception>
#include <new>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

// Host exceptions at the C ABI, after the HipError handler of an entry point: allocation
// failures and any other standard exception become error codes with the message kept in
// ERRSTR, so that no exception leaves an extern "C" function.
#define QPG_CATCH_HOST(ERRSTR)                  \
  catch (const std::bad_alloc&) {               \
    (ERRSTR) = "host allocation failed";       \
    return QPG_ERR_OOM;                         \
  }                                             \
  catch (const std::exception& e) {             \
    (ERRSTR) = e.what();                        \
    return QPG_ERR_HOST;                        \
  }
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
  // Vectors gathered by the B pass come in pairs of parts in one allocation (n then m entries),
  // so that column c of B = [P̄ | Āᵀ] reads element c of a single array.
  T *x = nullptr, *y = nullptr;  // ADMM iterates: x = xy, y = xy + n
  T *z = nullptr, *xt = nullptr;  // z (m), PCG solution x̃ (n)
  T *r = nullptr, *p = nullptr, *kp = nullptr, *b = nullptr, *dinv = nullptr;  // PCG (n); p = pw
  T* bk = nullptr;  // right-hand side b of the ADMM iteration's PCG solve (n)
  T* w = nullptr;   // ρ̄Āp (m) = pw + n
  T* zt = nullptr;  // z̃ = Āx̃ of the last update pass (m)
  T* ax = nullptr;  // Āx tracked by its recurrence (m), in the FP64 set only (both precisions use it)
  // vectors gathered by the right-hand-side pass, two planes of n + m: x̃ then ρ̄(z̃ − z) + y;
  // 0 then ρ̄z − y (plane 1 only for OpRhsR0, written by k_pairs)
  T* g = nullptr;
  T* dxy = nullptr;         // δx̄ (n), then δȳ (m): differences of the last checked ADMM step
  T* bg = nullptr;          // B·g from a check's dual-residual pass (P̄ part n, Āᵀ part n)
  bool ready = false;
};

// Device copy of a SpMV work list (TilePlan): the work list, the matrix in SELL order (values
// in both precisions), and the slots.
struct DevPlan {
  Tile* tiles = nullptr;
  int32_t ntiles = 0;
  Chunk* chunks = nullptr;
  int32_t* segslot = nullptr;
  int32_t* rowslot = nullptr;
  int32_t* slotidx = nullptr;
  int32_t* tbase = nullptr;
  CombItem* comb = nullptr;
  int32_t ncomb = 0;
  uint16_t* col16 = nullptr;
  int32_t* col32 = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  void* slots = nullptr;  // planes of nslot values: two of doubles (Ā), four of doubles (B, k_spmv2)
  int64_t nslot = 0;
  int32_t nrows = 0;
  int32_t max_wlen = 0;  // largest staged window, in columns
  int64_t layout[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // see qpg_spmv_layout
  int32_t* src = nullptr;  // CSR index of every SELL position, on the device until the values are placed
  int64_t nsrc = 0;
};

struct LearnedState;  // learned-preconditioner data of a solver (learned.hip)
void destroy_learned(LearnedState* L);
hipError_t resolve_noalloc_scratch(int device);  // learned.hip: scratch of qpg_hutchinson_noalloc

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
  Item *a_items = nullptr, *b_items = nullptr;  // row work lists of the learned SpMM
  int32_t na_items = 0, nb_items = 0;
  DevPlan plan_a, plan_b;  // SpMV work lists of Ā and B
  int32_t win_cols = 8192;  // LDS gather window capacity (columns)
  int lds_max = 0;          // dynamic LDS per workgroup on the device (bytes)
  int32_t nnzA = 0, nnzB = 0;
  double *diagP = nullptr, *colsq = nullptr, *dscale = nullptr, *escale = nullptr;  // D⁻¹, E⁻¹
  uint8_t* eqrow = nullptr;     // equality-row flags when R = diag(ρ_i) (eq. rho_vec), else null
  double* colsq_eq = nullptr;   // Σ over equality rows k of Ā_ki², per column (R = diag(ρ_i) only)
  DevState* st = nullptr;
  DevState* st_host = nullptr;        // mapped pinned host memory, written by finalize kernels
  DevState* st_mirror_dev = nullptr;  // its device-side address
  RedBuf rb{};
  int32_t vgrid = 1;

  Prec<double> p64;
  Prec<float> p32;

  // host copies
  std::vector<double> D, E, diagP_h, colsq_h;
  double* de = nullptr;        // D (n) then E (m) on the device
  double* out_dev = nullptr;   // unscaled x (n), y (m), z (m) of the last solve, on the device
  double* out_host = nullptr;  // the same in pinned host memory
  bool have_out = false;
  std::vector<double> cert_x, cert_y;  // normalised δx, δy of the last infeasibility check
  bool cert_valid = false;
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
  // frees a block from alloc before the solver ends
  void free_tracked(void* ptr) {
    auto it = std::find(allocs.begin(), allocs.end(), ptr);
    if (it == allocs.end()) return;
    allocs.erase(it);
    HIPCHK(hipFree(ptr));
  }
  template <typename T, class A>
  T* upload(const std::vector<T, A>& h) {
    T* d = alloc<T>(h.size());
    copy_h2d(d, h.data(), h.size() * sizeof(T));
    return d;
  }
  // Host → device copy on the stream. Large copies go through the device's pinned staging
  // buffers (host threads copy pieces into them while the DMA engine reads the others); the source
  // may be released on return. Small ones are queued directly from the source, which must then
  // stay valid until the stream has reached them.
  void copy_h2d(void* dst, const void* src, size_t bytes);
  template <typename T, typename S, class A>
  T* upload_as(const std::vector<S, A>& h) {
    qpg::hvec<T> t(h.size());
    qpg::parallel_chunks((int64_t)h.size(), 1 << 16, [&](int64_t, int64_t lo, int64_t hi) {
      for (int64_t k = lo; k < hi; ++k) t[k] = (T)h[k];
    });
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
    if (out_host) (void)hipHostFree(out_host);
  }

  // ----------------------------------------------------------------- launches
  // SpMV launches (k_spmv, then k_combine); the returned count is the number of workgroup
  // partials a finalize must combine. Segment sums go to the plan's slots and reduction partials
  // to rb.partials unless other buffers of the same sizes are given.
  template <typename T, class Op>
  int spmv(const DevPlan& pl, int nsplit, int planes, const Op& op, const int32_t* gate,
           bool combine = true, void* slots = nullptr, double* partials = nullptr) {
    T* sl = static_cast<T*>(slots ? slots : pl.slots);
    double* pa = partials ? partials : rb.partials;
    const size_t shmem = (size_t)pl.max_wlen * sizeof(T);
    // The dynamic LDS limit is a per-device attribute of each instantiation: raise it once per
    // device (always, for device ordinals beyond the table).
    constexpr int kDevTable = 64;
    static std::atomic<size_t> lds_allowed[kDevTable];
    const bool tab = device >= 0 && device < kDevTable;
    if (!tab || shmem > lds_allowed[device].load(std::memory_order_relaxed)) {
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv<T, Op>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
      if (tab) {
        size_t cur = lds_allowed[device].load(std::memory_order_relaxed);
        while (cur < shmem && !lds_allowed[device].compare_exchange_weak(cur, shmem)) {
        }
      }
    }
    const T* val = std::is_same<T, double>::value ? (const T*)pl.val64 : (const T*)pl.val32;
    hipLaunchKernelGGL((k_spmv<T, Op>), dim3(pl.ntiles), dim3(kSpmvBlock), shmem, stream, pl.tiles, pl.chunks,
                       pl.segslot, pl.col16, pl.col32, val, nsplit, op, sl, pl.nslot, planes, gate);
    if (!combine) return 0;
    hipLaunchKernelGGL((k_combine<T, Op>), dim3(pl.ncomb), dim3(kBlock), 0, stream, pl.comb, pl.rowslot,
                       pl.slotidx, pl.tbase, (const T*)sl, pl.nslot, planes, op, pa, gate);
    return pl.ncomb;
  }
  template <typename T, class Op>
  int spmv_A(const Op& op, const int32_t* gate = nullptr) {
    return spmv<T>(plan_a, INT32_MAX, 1, op, gate);
  }
  template <typename T, class Op>
  int spmv_B(const Op& op, const int32_t* gate = nullptr) {
    return spmv<T>(plan_b, n, 2, op, gate);
  }
  // One read of B for two gathered vectors (k_spmv2, then k_combine over four slot planes of
  // B's slots); false when its window of pairs would not fit in a workgroup's LDS.
  template <typename T>
  bool pair_fits() const {
    return (size_t)plan_b.max_wlen * sizeof(Pair<T>) <= (size_t)lds_max;
  }
  template <typename T, class Op>
  int spmv_B_pair(const Op& op, const int32_t* gate = nullptr) {
    const DevPlan& pl = plan_b;
    T* sl = static_cast<T*>(pl.slots);
    const size_t shmem = (size_t)pl.max_wlen * sizeof(Pair<T>);
    static std::atomic<size_t> lds_allowed[64];
    const bool tab = device >= 0 && device < 64;
    if (!tab || shmem > lds_allowed[device].load(std::memory_order_relaxed)) {
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv2<T, Op>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
      if (tab) {
        size_t cur = lds_allowed[device].load(std::memory_order_relaxed);
        while (cur < shmem && !lds_allowed[device].compare_exchange_weak(cur, shmem)) {
        }
      }
    }
    const T* val = std::is_same<T, double>::value ? (const T*)pl.val64 : (const T*)pl.val32;
    hipLaunchKernelGGL((k_spmv2<T, Op>), dim3(pl.ntiles), dim3(kSpmvBlock), shmem, stream, pl.tiles, pl.chunks,
                       pl.segslot, pl.col16, pl.col32, val, n, op, sl, pl.nslot, gate);
    hipLaunchKernelGGL((k_combine<T, Op>), dim3(pl.ncomb), dim3(kBlock), 0, stream, pl.comb, pl.rowslot,
                       pl.slotidx, pl.tbase, (const T*)sl, pl.nslot, 2, op, rb.partials, gate);
    return pl.ncomb;
  }
  // Combine the partials of the previous launch (count workgroups) and run op's finalisation.
  template <class Op>
  void finalize(const Op& op, int count, const int32_t* gate = nullptr, bool mirror = false) {
    hipLaunchKernelGGL((k_finalize<Op::NS, Op::MAXMASK, Op>), dim3(1), dim3(kFinBlock), 0, stream,
                       (const double*)rb.partials, count, op, gate, (const DevState*)st,
                       mirror ? st_mirror_dev : nullptr);
  }
  template <int NS, unsigned MASK, class Fin>
  void finalize_fn(const Fin& fin, int count, const int32_t* gate = nullptr, bool mirror = false) {
    hipLaunchKernelGGL((k_finalize<NS, MASK, Fin>), dim3(1), dim3(kFinBlock), 0, stream,
                       (const double*)rb.partials, count, fin, gate, (const DevState*)st,
                       mirror ? st_mirror_dev : nullptr);
  }

  // Wait for the stream and read the device scalars: the finalize kernel launched last before a
  // host read leaves a copy of them in mapped host memory (st_host), so no copy is queued and the
  // host polls the stream.
  void sync_state() {
    hipError_t e;
    while ((e = hipStreamQuery(stream)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) throw HipError{e, "hipStreamQuery"};
  }

  template <typename T>
  void jacobi(double rho) {
    hipLaunchKernelGGL((k_jacobi<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, P<T>().dinv, diagP,
                       colsq, s.sigma, rho, (const double*)colsq_eq);
  }

  // One PCG iteration (Algorithm 3), all on the device; skipped once st->done is set. With
  // track_zt, z̃ = Āx̃ is carried along (see k_pcg_update).
  template <typename T>
  void pcg_iteration(double rho, bool track_zt, bool mirror, int it, int spec_k = -1) {
    Prec<T>& V = P<T>();
    const int32_t* gate = &st->done;
    spmv_A<T>(OpScaled<T>{V.p, V.w, (T)rho, eqrow}, gate);
    OpKp<T> kp{V.p, V.w, V.kp, (T)s.sigma, n, st};
    const int nkp = spmv_B<T>(kp, gate);
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, V.xt, V.r, V.p,
                       V.kp, V.dinv, st, (const double*)rb.partials, nkp, rb.vpartials, gate, m,
                       (track_zt && !eqrow) ? V.zt : (T*)nullptr, (const T*)V.w, (T)(1.0 / rho), it);
    hipLaunchKernelGGL((k_pcg_dir<T>), dim3(vgrid), dim3(kBlock), 0, stream, n, V.p, (const T*)V.r,
                       (const T*)V.dinv, st, (const double*)rb.vpartials, vgrid, gate, it,
                       mirror ? st_mirror_dev : (DevState*)nullptr);
    if (spec_k >= 0) hipLaunchKernelGGL(k_after_pcg<DevState>, dim3(1), dim3(64), 0, stream, st, spec_k);
  }

  // Run PCG iterations after the initialisation kernel until st->done. The first batch is one
  // shorter than the previous PCG solve took, so that iterations launched after convergence
  // (which exit at once) stay rare; then batches of 2, 4 and 8 iterations per host check (fewer
  // round trips when the count has grown, at most 7 gated iterations wasted). Returns the count.
  // `start` iterations of this solve have run already (a solve resumed after a speculation).
  template <typename T>
  int pcg_loop(double rho, int maxit, bool track_zt = false, int start = 0) {
    int issued = start;
    int batch = std::max(1, std::min(last_pcg - 1, maxit));
    int more = 1;  // iterations per host read once the predicted count is spent: 2, 4, 8, 8, …
    for (;;) {
      int k = std::max(0, std::min(batch, maxit - issued));
      for (int i = 0; i < k; ++i)
        pcg_iteration<T>(rho, track_zt, i == k - 1, issued + i);
      if (k == 0) hipLaunchKernelGGL(k_mirror<DevState>, dim3(1), dim3(64), 0, stream, (const DevState*)st, st_mirror_dev);
      issued += k;
      sync_state();
      if (st_host->done || issued >= maxit) break;
      more = std::min(2 * more, 8);
      batch = more;
    }
    last_pcg = std::max(1, st_host->iter);
    return st_host->iter;
  }

  // PCG on K x̃ = b with b already in P<T>().b and the threshold in st; starts from P<T>().xt.
  template <typename T>
  int pcg_solve(double rho, int maxit) {
    Prec<T>& V = P<T>();
    spmv_A<T>(OpScaled<T>{V.xt, V.w, (T)rho, eqrow});
    OpR0<T> r0{V.xt, V.w, V.b, V.dinv, V.r, V.p, (T)s.sigma, n, maxit, st};
    finalize(r0, spmv_B<T>(r0));
    return pcg_loop<T>(rho, maxit);
  }

  template <typename T>
  void pairs(double rho) {
    Prec<T>& V = P<T>();
    hipLaunchKernelGGL((k_pairs<T>), dim3(grid_for(n + m)), dim3(kBlock), 0, stream, n, m, V.g,
                         (const T*)V.xt, (const T*)V.zt, (const T*)V.z, (const T*)V.y, (T)rho,
                         (const uint8_t*)eqrow);
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
  int infeasibility_status() const;
  template <typename T>
  void keep_certificate();

  int solve();
  TilePlan plan_tiles(const std::vector<int32_t>& rowptr, const int32_t* col, int32_t nrows,
                      int32_t ncols) const;
  void upload_plan(DevPlan& pl, TilePlan& t, const std::vector<int32_t>& rowptr, int32_t nrows,
                   const int32_t* dcol);
  void place_values(DevPlan& pl, const double* csr_val, bool fp32);
  void alloc_prec64(const HostProblem& H);
  void place_raw(const HostProblem& H);
  void alloc_prec32();
  void equilibrate();
};

template <>
inline Prec<double>& qpg_solver::P<double>() {
  return p64;
}
template <>
inline Prec<float>& qpg_solver::P<float>() {
  return p32;
}
