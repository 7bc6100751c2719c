// Learned diagonal preconditioner: graph construction, network forward/backward, training
// objects, Hutchinson targets and the learned M⁻¹ used by the solve.
//
// The preconditioner stays diagonal and strictly positive (M⁻¹_ii = softplus(g_i)/K_ii), so the
// PCG of Algorithm 3 is unchanged; only the Jacobi diagonal of Section 6.3.1 is replaced. The
// message-passing trunk does not depend on ρ̄ and runs once per setup; the head is re-evaluated
// when ρ̄ changes (Section 6.3.2 updates ρ̄ every 10 iterations).
#include <mutex>

#include "mpnn.hpp"
#include "solver_internal.hpp"

using namespace qpg;

struct qpg_net {
  int device = 0;
  int bf16 = 1;
  float* theta = nullptr;  // float32 master parameters (device)
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  int step = 0;
  std::string err;
  ~qpg_net() {
    for (float* p : {theta, grad, m1, m2})
      if (p) (void)hipFree(p);
  }
};

namespace qpg {

struct LearnedState {
  std::vector<void*> allocs;
  int n = 0, m = 0;
  float *fv = nullptr, *fc = nullptr;
  float *wA_hat = nullptr, *wA_chk = nullptr;  // on the Ā structure
  float *wB_hat = nullptr, *wB_chk = nullptr;  // on the B structure (Āᵀ part)
  float* hv[kRounds + 1] = {};
  float* hc[kRounds + 1] = {};
  float* av[kRounds + 1] = {};
  float* ac[kRounds + 1] = {};
  float *phi = nullptr, *u = nullptr, *g = nullptr, *dg = nullptr, *tgt = nullptr;
  double* e = nullptr;
  float *dhv = nullptr, *dhv2 = nullptr, *dav = nullptr, *dhc = nullptr, *dhc2 = nullptr,
        *dac = nullptr, *dU = nullptr;
  float* part = nullptr;
  int part_groups = 0;
  NetScalars* ns = nullptr;
  NetScalars* ns_host = nullptr;
  double* acc = nullptr;    // Hutchinson accumulator (n)
  int8_t* probe = nullptr;  // one probe (n)
  // inference network of the solve (settings.precond == QPG_PRECOND_LEARNED)
  float* theta_inf = nullptr;
  bool trunk_ready = false;

  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "hipMalloc (learned preconditioner)"};
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
};

void destroy_learned(LearnedState* L) {
  if (!L) return;
  for (void* p : L->allocs) (void)hipFree(p);
  if (L->ns_host) (void)hipHostFree(L->ns_host);
  delete L;
}

}  // namespace qpg

namespace {

int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Build the graph data of the scaled problem once: row statistics of Ā and Āᵀ, normalised
// edge weights on both CSR structures, node features; allocate activations.
LearnedState* ensure_graph(qpg_solver* h) {
  if (h->learned) return h->learned;
  LearnedState* L = new LearnedState();
  h->learned = L;
  const int n = h->n, m = h->m;
  L->n = n;
  L->m = m;
  hipStream_t st = h->stream;
  const int nnzA = std::max(1, h->nnzA), nnzB = std::max(1, h->nnzB);
  double *rsA = L->alloc<double>(m), *mxA = L->alloc<double>(m), *sqA = L->alloc<double>(m);
  double *rsB = L->alloc<double>(n), *mxB = L->alloc<double>(n), *sqB = L->alloc<double>(n);
  int32_t *dgA = L->alloc<int32_t>(m), *dgB = L->alloc<int32_t>(n);
  if (m > 0)
    hipLaunchKernelGGL(k_rowstats, dim3(div_up(m, kBlock)), dim3(kBlock), 0, st, m, (const int32_t*)h->a_ptr,
                       (const int32_t*)nullptr, (const double*)h->p64.a_val, rsA, mxA, sqA, dgA);
  hipLaunchKernelGGL(k_rowstats, dim3(div_up(n, kBlock)), dim3(kBlock), 0, st, n, (const int32_t*)h->b_ptr,
                     (const int32_t*)h->b_split, (const double*)h->p64.b_val, rsB, mxB, sqB, dgB);
  L->wA_hat = L->alloc<float>(nnzA);
  L->wA_chk = L->alloc<float>(nnzA);
  L->wB_hat = L->alloc<float>(nnzB);
  L->wB_chk = L->alloc<float>(nnzB);
  if (m > 0)
    hipLaunchKernelGGL(k_edge_weights, dim3(div_up(m, kBlock)), dim3(kBlock), 0, st, m,
                       (const int32_t*)h->a_ptr, (const int32_t*)nullptr, (const int32_t*)h->a_col,
                       (const double*)h->p64.a_val, 0, (const double*)rsA, (const double*)rsB, L->wA_hat,
                       L->wA_chk);
  hipLaunchKernelGGL(k_edge_weights, dim3(div_up(n, kBlock)), dim3(kBlock), 0, st, n, (const int32_t*)h->b_ptr,
                     (const int32_t*)h->b_split, (const int32_t*)h->b_col, (const double*)h->p64.b_val, n,
                     (const double*)rsB, (const double*)rsA, L->wB_chk, L->wB_hat);
  L->fv = L->alloc<float>((size_t)n * kH);
  L->fc = L->alloc<float>((size_t)m * kH);
  hipLaunchKernelGGL(k_features_v, dim3(div_up((long)n * kH, kBlock)), dim3(kBlock), 0, st, n,
                     (const double*)h->diagP, (const double*)h->colsq, (const int32_t*)dgB,
                     (const double*)mxB, h->s.sigma, L->fv);
  if (m > 0)
    hipLaunchKernelGGL((k_features_c<double>), dim3(div_up((long)m * kH, kBlock)), dim3(kBlock), 0, st, m,
                       (const double*)sqA, (const int32_t*)dgA, (const double*)mxA,
                       (const double*)h->p64.lb, (const double*)h->p64.ub, L->fc);
  for (int l = 0; l <= kRounds; ++l) {
    L->hv[l] = L->alloc<float>((size_t)n * kH);
    L->hc[l] = L->alloc<float>((size_t)m * kH);
    if (l > 0) {
      L->av[l] = L->alloc<float>((size_t)n * kH);
      L->ac[l] = L->alloc<float>((size_t)m * kH);
    }
  }
  L->phi = L->alloc<float>((size_t)n * kH);
  L->u = L->alloc<float>((size_t)n * kH);
  L->dU = L->alloc<float>((size_t)n * kH);
  L->g = L->alloc<float>(n);
  L->e = L->alloc<double>(n);
  L->dg = L->alloc<float>(n);
  L->tgt = L->alloc<float>(n);
  L->dhv = L->alloc<float>((size_t)n * kH);
  L->dhv2 = L->alloc<float>((size_t)n * kH);
  L->dav = L->alloc<float>((size_t)n * kH);
  L->dhc = L->alloc<float>((size_t)m * kH);
  L->dhc2 = L->alloc<float>((size_t)m * kH);
  L->dac = L->alloc<float>((size_t)m * kH);
  L->part_groups = std::max(1, std::min(256, div_up(std::max(n, m), 1024)));
  L->part = L->alloc<float>((size_t)L->part_groups * (64 * kH + kH));
  L->ns = L->alloc<NetScalars>(1);
  HIPCHK(hipHostMalloc((void**)&L->ns_host, sizeof(NetScalars), hipHostMallocDefault));
  L->acc = L->alloc<double>(n);
  L->probe = L->alloc<int8_t>(n);
  HIPCHK(hipGetLastError());
  return L;
}

void dense_fwd(qpg_solver* h, bool bf16, int N, const float* X1, const float* X2, const float* W,
               const float* b, float* Y) {
  if (N <= 0) return;
  if (bf16)
    hipLaunchKernelGGL(k_dense_fwd_mfma, dim3(div_up(N, 128)), dim3(kBlock), 0, h->stream, N, X1, X2, W, b, Y);
  else
    hipLaunchKernelGGL(k_dense_fwd_f32, dim3(div_up((long)N * kH, kBlock)), dim3(kBlock), 0, h->stream, N,
                       X1, X2, W, b, Y);
}

// Gradients of Y = relu([X1 X2] W + b): [W; b] written to gWb (K·32 + 32 floats, the parameter
// layout), dX1 (= or +=) and dX2 (=) when non-null.
void dense_bwd(qpg_solver* h, LearnedState* L, bool bf16, int N, const float* X1, const float* X2,
               const float* dY, const float* Y, const float* W, float* dX1, float* dX2, int acc,
               float* gWb) {
  const int K = X2 ? 64 : 32;
  const int width = K * kH + kH;
  if (N <= 0) {
    HIPCHK(hipMemsetAsync(gWb, 0, width * sizeof(float), h->stream));
    return;
  }
  const int G = std::max(1, std::min(L->part_groups, div_up(N, 256)));
  if (bf16)
    hipLaunchKernelGGL(k_dense_bwd_dw_mfma, dim3(G), dim3(kBlock), 0, h->stream, N, X1, X2, dY, Y, L->part);
  else
    hipLaunchKernelGGL(k_dense_bwd_dw_f32, dim3(G), dim3(kBlock), 0, h->stream, N, X1, X2, dY, Y, L->part);
  hipLaunchKernelGGL(k_part_reduce, dim3(div_up(width, kBlock)), dim3(kBlock), 0, h->stream,
                     (const float*)L->part, G, width, gWb);
  if (dX1) {
    if (bf16)
      hipLaunchKernelGGL(k_dense_bwd_dx_mfma, dim3(div_up(N, 128)), dim3(kBlock), 0, h->stream, N, dY, Y, W,
                         dX1, dX2, acc);
    else
      hipLaunchKernelGGL(k_dense_bwd_dx_f32, dim3(div_up((long)N * kH, kBlock)), dim3(kBlock), 0, h->stream,
                         N, dY, Y, W, dX1, dX2, acc);
  }
}

// Y (=|+=) Â X etc.: the SpMM over the Ā structure (m rows, gather from n×32) or over the Āᵀ
// part of B (n rows, gather from m×32).
void spmm_A(qpg_solver* h, const float* w, const float* X, float* Y, int acc) {
  hipLaunchKernelGGL(k_spmm32, dim3(h->na_items), dim3(kBlock), 0, h->stream, (const Item*)h->a_items,
                     (const int32_t*)h->a_ptr, (const int32_t*)nullptr, (const int32_t*)h->a_col, w, 0, X, Y, acc);
}
void spmm_B(qpg_solver* h, const float* w, const float* X, float* Y, int acc) {
  hipLaunchKernelGGL(k_spmm32, dim3(h->nb_items), dim3(kBlock), 0, h->stream, (const Item*)h->b_items,
                     (const int32_t*)h->b_ptr, (const int32_t*)h->b_split, (const int32_t*)h->b_col, w, h->n, X,
                     Y, acc);
}

// Message-passing trunk: h_v^L in L->hv[kRounds].
void trunk(qpg_solver* h, LearnedState* L, const float* th, bool bf16) {
  const int n = h->n, m = h->m;
  dense_fwd(h, bf16, n, L->fv, nullptr, th + NetOff::W_v0, th + NetOff::b_v0, L->hv[0]);
  dense_fwd(h, bf16, m, L->fc, nullptr, th + NetOff::W_c0, th + NetOff::b_c0, L->hc[0]);
  for (int l = 1; l <= kRounds; ++l) {
    if (m > 0) spmm_A(h, L->wA_hat, L->hv[l - 1], L->ac[l], 0);
    dense_fwd(h, bf16, m, L->hc[l - 1], L->ac[l], th + NetOff::W_c(l), th + NetOff::b_c(l), L->hc[l]);
    spmm_B(h, L->wB_chk, L->hc[l], L->av[l], 0);
    dense_fwd(h, bf16, n, L->hv[l - 1], L->av[l], th + NetOff::W_v(l), th + NetOff::b_v(l), L->hv[l]);
  }
}

// Head for a given ρ̄: u, g; and, if dinv is given, M⁻¹ = softplus(g) / K_ii in precision T.
template <typename T>
void head(qpg_solver* h, LearnedState* L, const float* th, bool bf16, double rho, T* dinv) {
  const int n = h->n;
  hipLaunchKernelGGL(k_phi, dim3(div_up((long)n * kH, kBlock)), dim3(kBlock), 0, h->stream, n,
                     (const double*)h->diagP, (const double*)h->colsq, h->s.sigma, rho, L->phi);
  dense_fwd(h, bf16, n, L->hv[kRounds], L->phi, th + NetOff::W_h1, th + NetOff::b_h1, L->u);
  hipLaunchKernelGGL((k_head_out<T>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, h->stream, n,
                     (const float*)L->u, th, L->g, dinv, (const double*)h->diagP,
                     (const double*)h->colsq, h->s.sigma, rho);
}

// Loss (mean-removed squared error of log s − target) and its gradient into `grad`.
double loss_backward(qpg_solver* h, LearnedState* L, const float* th, bool bf16, float* grad) {
  const int n = h->n, m = h->m;
  const int vg = h->vgrid;
  hipLaunchKernelGGL(k_loss_mean, dim3(vg), dim3(kBlock), 0, h->stream, n, (const float*)L->g,
                     (const float*)L->tgt, L->e, h->rb.partials);
  h->finalize_fn<1, 0u>(FinMeanE{L->ns, n}, vg);
  hipLaunchKernelGGL(k_loss_grad, dim3(vg), dim3(kBlock), 0, h->stream, n, (const double*)L->e,
                     (const float*)L->g, (const NetScalars*)L->ns, L->dg, h->rb.partials);
  h->finalize_fn<1, 0u>(FinLoss{L->ns, n}, vg);
  // head output layer
  const int G = std::max(1, std::min(L->part_groups, div_up(n, 256)));
  hipLaunchKernelGGL(k_head_out_bwd, dim3(G), dim3(kBlock), 0, h->stream, n, (const float*)L->u,
                     (const float*)L->dg, th, L->dU, L->part);
  hipLaunchKernelGGL(k_part_reduce, dim3(1), dim3(kBlock), 0, h->stream, (const float*)L->part, G, kH + 1,
                     grad + NetOff::w_h2);
  // head hidden layer: input [h_v^L, φ]; only the h_v^L part of the input gradient is needed
  dense_bwd(h, L, bf16, n, L->hv[kRounds], L->phi, L->dU, L->u, th + NetOff::W_h1, L->dhv, nullptr, 0,
            grad + NetOff::W_h1);
  float *dhv = L->dhv, *dhv2 = L->dhv2, *dhc = L->dhc, *dhc2 = L->dhc2;
  if (m > 0) HIPCHK(hipMemsetAsync(dhc, 0, (size_t)m * kH * sizeof(float), h->stream));
  for (int l = kRounds; l >= 1; --l) {
    // h_v^l = relu([h_v^{l−1}, a_v] W_vl + b_vl)
    dense_bwd(h, L, bf16, n, L->hv[l - 1], L->av[l], dhv, L->hv[l], th + NetOff::W_v(l), dhv2, L->dav, 0,
              grad + NetOff::W_v(l));
    // a_v = Ǎ h_c^l  ⇒  dh_c^l += Ǎᵀ da_v   (Ǎᵀ lives on the Ā structure)
    if (m > 0) spmm_A(h, L->wA_chk, L->dav, dhc, 1);
    // h_c^l = relu([h_c^{l−1}, a_c] W_cl + b_cl)
    dense_bwd(h, L, bf16, m, L->hc[l - 1], L->ac[l], dhc, L->hc[l], th + NetOff::W_c(l), dhc2, L->dac, 0,
              grad + NetOff::W_c(l));
    // a_c = Â h_v^{l−1}  ⇒  dh_v^{l−1} += Âᵀ da_c   (Âᵀ lives on the Āᵀ part of B)
    spmm_B(h, L->wB_hat, L->dac, dhv2, 1);
    std::swap(dhv, dhv2);
    std::swap(dhc, dhc2);
  }
  dense_bwd(h, L, bf16, n, L->fv, nullptr, dhv, L->hv[0], th + NetOff::W_v0, nullptr, nullptr, 0,
            grad + NetOff::W_v0);
  dense_bwd(h, L, bf16, m, L->fc, nullptr, dhc, L->hc[0], th + NetOff::W_c0, nullptr, nullptr, 0,
            grad + NetOff::W_c0);
  HIPCHK(hipMemcpyAsync(L->ns_host, L->ns, sizeof(NetScalars), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return L->ns_host->loss;
}

// Host-side parameter initialisation: uniform(±1/√fan_in) weights from a splitmix64 stream,
// zero biases, output layer at softplus = 1 (the Jacobi preconditioner).
void init_params(std::vector<float>& p, uint64_t seed) {
  p.assign(NetOff::total, 0.f);
  uint64_t x = seed;
  auto next = [&]() {
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int fan_in, int count) {
    const double a = 1.0 / std::sqrt((double)fan_in);
    for (int i = 0; i < count; ++i) p[off + i] = (float)((2.0 * next() - 1.0) * a);
  };
  fill(NetOff::W_v0, 32, 32 * kH);
  fill(NetOff::W_c0, 32, 32 * kH);
  for (int l = 1; l <= kRounds; ++l) {
    fill(NetOff::W_c(l), 64, 64 * kH);
    fill(NetOff::W_v(l), 64, 64 * kH);
  }
  fill(NetOff::W_h1, 64, 64 * kH);
  p[NetOff::b_h2] = (float)std::log(std::exp(1.0) - 1.0);
}

int net_error(qpg_net* net, const HipError& e) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s failed: %s", e.what, hipGetErrorString(e.code));
  if (net) net->err = buf;
  (void)hipGetLastError();
  return e.code == hipErrorOutOfMemory ? QPG_ERR_OOM : QPG_ERR_DEVICE;
}

}  // namespace

// ------------------------------------------------------------------- learned M⁻¹ in the solve

// Prepare the inference network of the solve: graph, weights, trunk (once per setup).
void qpg_solver::learned_prepare() {
  LearnedState* L = ensure_graph(this);
  if (!L->theta_inf) {
    L->theta_inf = L->alloc<float>(NetOff::total);
    HIPCHK(hipMemcpyAsync(L->theta_inf, precond_weights.data(), NetOff::total * sizeof(float),
                          hipMemcpyHostToDevice, stream));
  }
  if (!L->trunk_ready) {
    trunk(this, L, L->theta_inf, true);
    L->trunk_ready = true;
  }
}

template <typename T>
void qpg_solver::learned_dinv(double rho) {
  learned_prepare();
  head<T>(this, learned, learned->theta_inf, true, rho, P<T>().dinv);
}
template void qpg_solver::learned_dinv<double>(double);
template void qpg_solver::learned_dinv<float>(double);

// ------------------------------------------------------------ Hutchinson targets

namespace {

// Scratch of qpg_hutchinson_noalloc: the accumulator Σ_k z_k ∘ K⁻¹z_k (n doubles, then padding
// to 256 bytes) followed by one probe (n bytes). Every device the library runs on holds one copy
// for the life of the process; calls that overlap on one device share it and race.
__device__ __align__(256) unsigned char scratch[QPG_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::atomic<void*> g_scratch_addr[kScratchDevices];  // device address of `scratch`, per ordinal
std::mutex g_scratch_mu;

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  return g_scratch_addr[device].load(std::memory_order_acquire);
}

int hutchinson_check(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho, double eps,
                     int32_t max_iter, double* diag) {
  if (!h || !signs || nprobes < 1 || !diag || !(rho > 0) || !(eps >= 0) || max_iter < 1)
    return QPG_ERR_ARG;
  if (h->s.rho_vector) {
    h->err = "qpg_hutchinson: defined for R = rho*I (the handle was set up with rho_vector)";
    return QPG_ERR_STATE;
  }
  for (long k = 0; k < (long)nprobes * h->n; ++k)
    if (signs[k] != 1 && signs[k] != -1) {
      h->err = "qpg_hutchinson: probe entries must be +1 or -1";
      return QPG_ERR_ARG;
    }
  return QPG_OK;
}

// (1/s) Σ_k z_k ∘ K⁻¹z_k with K⁻¹z_k by the solver's Jacobi PCG from 0; acc (n doubles) and probe
// (n bytes) are device buffers the caller provides. ρ̄ and the Jacobi diagonal are restored.
int hutchinson_run(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho, double eps,
                   int32_t max_iter, double* diag, double* acc, int8_t* probe) {
  Prec<double>& V = h->p64;
  const int n = h->n;
  const double rho_saved = h->rho_cur;
  struct Restore {  // ρ̄ of the handle is restored on every way out
    qpg_solver* h;
    double rho;
    ~Restore() { h->rho_cur = rho; }
  } restore{h, rho_saved};
  h->rho_cur = rho;
  h->jacobi<double>(rho);
  h->fill(acc, n, 0.0);
  for (int k = 0; k < nprobes; ++k) {
    HIPCHK(hipMemcpyAsync(probe, signs + (size_t)k * n, n, hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL((k_probe_load<double>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, n,
                       (const int8_t*)probe, V.b);
    h->fill(V.xt, n, 0.0);
    hipLaunchKernelGGL((k_absmax<double>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, n,
                       (const double*)V.b, h->rb.partials);
    h->finalize_fn<1, 1u>(FinThresh{h->st, eps, 1}, h->vgrid);
    h->last_pcg = 1;
    h->pcg_solve<double>(rho, max_iter);
    hipLaunchKernelGGL((k_probe_acc<double>), dim3(h->vgrid), dim3(kBlock), 0, h->stream, n,
                       (const int8_t*)probe, (const double*)V.xt, acc);
  }
  HIPCHK(hipMemcpyAsync(diag, acc, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < n; ++i) diag[i] /= nprobes;
  h->jacobi<double>(rho_saved);
  HIPCHK(hipGetLastError());
  return QPG_OK;
}

int hutchinson_device_error(qpg_solver* h, const HipError& e) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s failed: %s", e.what, hipGetErrorString(e.code));
  h->err = buf;
  (void)hipGetLastError();
  return QPG_ERR_DEVICE;
}

}  // namespace

namespace qpg {

// Device address of the no-alloc scratch for the current device, looked up once per device at
// setup. Ordinals beyond the table keep no address (qpg_hutchinson_noalloc then fails with
// QPG_ERR_STATE on them).
hipError_t resolve_noalloc_scratch(int device) {
  if (device < 0 || device >= kScratchDevices) return hipSuccess;
  if (g_scratch_addr[device].load(std::memory_order_acquire)) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device].load(std::memory_order_relaxed)) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_addr[device].store(ptr, std::memory_order_release);
  return e;
}

}  // namespace qpg

// ================================================================================== C ABI

extern "C" {

int qpg_get_kdiag(const qpg_solver* h, double rho, double* kdiag) {
  if (!h || !kdiag || !(rho > 0)) return QPG_ERR_ARG;
  if (h->s.rho_vector) return QPG_ERR_STATE;  // K is defined here with R = ρ̄I
  for (int i = 0; i < h->n; ++i) kdiag[i] = h->diagP_h[i] + h->s.sigma + rho * h->colsq_h[i];
  return QPG_OK;
}

int qpg_hutchinson(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho, double eps,
                   int32_t max_iter, double* diag) {
  const int rc = hutchinson_check(h, signs, nprobes, rho, eps, max_iter, diag);
  if (rc) return rc;
  try {
    HIPCHK(hipSetDevice(h->device));
    LearnedState* L = ensure_graph(h);
    return hutchinson_run(h, signs, nprobes, rho, eps, max_iter, diag, L->acc, L->probe);
  } catch (const HipError& e) {
    return hutchinson_device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_hutchinson_noalloc(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho,
                           double eps, int32_t max_iter, double* diag) {
  const int rc = hutchinson_check(h, signs, nprobes, rho, eps, max_iter, diag);
  if (rc) return rc;
  const size_t acc_bytes = ((size_t)h->n * sizeof(double) + 255) / 256 * 256;
  if (acc_bytes + (size_t)h->n > (size_t)QPG_NOALLOC_SCRATCH_BYTES) {
    h->err = "qpg_hutchinson_noalloc: n exceeds the static scratch (QPG_NOALLOC_MAX_N)";
    return QPG_ERR_SIZE;
  }
  void* base = noalloc_scratch(h->device);
  if (!base) {
    h->err = "qpg_hutchinson_noalloc: no scratch address for this device";
    return QPG_ERR_STATE;
  }
  try {
    HIPCHK(hipSetDevice(h->device));
    unsigned char* b = static_cast<unsigned char*>(base);
    return hutchinson_run(h, signs, nprobes, rho, eps, max_iter, diag, reinterpret_cast<double*>(b),
                          reinterpret_cast<int8_t*>(b + acc_bytes));
  } catch (const HipError& e) {
    return hutchinson_device_error(h, e);
  } QPG_CATCH_HOST(h->err)
}

int qpg_net_create(qpg_net** out, const float* params, uint64_t seed, int32_t bf16, int32_t device) {
  if (!out) return QPG_ERR_ARG;
  *out = nullptr;
  qpg_net* net = new (std::nothrow) qpg_net();
  if (!net) return QPG_ERR_OOM;
  net->device = device;
  net->bf16 = bf16 ? 1 : 0;
  try {
    HIPCHK(hipSetDevice(device));
    const size_t bytes = NetOff::total * sizeof(float);
    for (float** p : {&net->theta, &net->grad, &net->m1, &net->m2}) HIPCHK(hipMalloc((void**)p, bytes));
    std::vector<float> init;
    if (params)
      init.assign(params, params + NetOff::total);
    else
      init_params(init, seed);
    HIPCHK(hipMemcpy(net->theta, init.data(), bytes, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(net->grad, 0, bytes));
    HIPCHK(hipMemset(net->m1, 0, bytes));
    HIPCHK(hipMemset(net->m2, 0, bytes));
  } catch (const HipError& e) {
    int code = net_error(net, e);
    delete net;
    return code;
  } catch (const std::bad_alloc&) {
    delete net;
    return QPG_ERR_OOM;
  } catch (const std::exception&) {
    delete net;
    return QPG_ERR_HOST;
  }
  *out = net;
  return QPG_OK;
}

int qpg_net_get_params(const qpg_net* net, float* params) {
  if (!net || !params) return QPG_ERR_ARG;
  if (hipSetDevice(net->device) != hipSuccess ||
      hipMemcpy(params, net->theta, NetOff::total * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return QPG_ERR_DEVICE;
  return QPG_OK;
}

int qpg_net_set_params(qpg_net* net, const float* params) {
  if (!net || !params) return QPG_ERR_ARG;
  if (hipSetDevice(net->device) != hipSuccess ||
      hipMemcpy(net->theta, params, NetOff::total * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return QPG_ERR_DEVICE;
  net->step = 0;
  return QPG_OK;
}

int qpg_net_forward(qpg_net* net, qpg_solver* h, double rho, float* g) {
  if (!net || !h || !(rho > 0)) return QPG_ERR_ARG;
  if (net->device != h->device) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    LearnedState* L = ensure_graph(h);
    trunk(h, L, net->theta, net->bf16);
    head<double>(h, L, net->theta, net->bf16, rho, (double*)nullptr);
    if (g) HIPCHK(hipMemcpyAsync(g, L->g, h->n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    return net_error(net, e);
  } QPG_CATCH_HOST(net->err)
  return QPG_OK;
}

int qpg_net_loss_grad(qpg_net* net, qpg_solver* h, double rho, const float* target, double* loss,
                      float* grad) {
  if (!net || !h || !target || !(rho > 0)) return QPG_ERR_ARG;
  if (net->device != h->device) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(h->device));
    LearnedState* L = ensure_graph(h);
    HIPCHK(hipMemcpyAsync(L->tgt, target, h->n * sizeof(float), hipMemcpyHostToDevice, h->stream));
    trunk(h, L, net->theta, net->bf16);
    head<double>(h, L, net->theta, net->bf16, rho, (double*)nullptr);
    const double l = loss_backward(h, L, net->theta, net->bf16, net->grad);
    if (loss) *loss = l;
    if (grad) {
      HIPCHK(hipMemcpyAsync(grad, net->grad, NetOff::total * sizeof(float), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    return net_error(net, e);
  } QPG_CATCH_HOST(net->err)
  return QPG_OK;
}

int qpg_net_adam_step(qpg_net* net, float lr) {
  if (!net || !(lr > 0)) return QPG_ERR_ARG;
  try {
    HIPCHK(hipSetDevice(net->device));
    net->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
    hipLaunchKernelGGL(k_adam, dim3(div_up(NetOff::total, kBlock)), dim3(kBlock), 0, 0, NetOff::total,
                       net->theta, (const float*)net->grad, net->m1, net->m2, lr, b1, b2, 1e-8f, c1, c2);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    return net_error(net, e);
  } QPG_CATCH_HOST(net->err)
  return QPG_OK;
}

int qpg_net_destroy(qpg_net* net) {
  if (!net) return QPG_OK;
  (void)hipSetDevice(net->device);
  delete net;
  return QPG_OK;
}

}  // extern "C"
