// Device kernels of the learned diagonal preconditioner: a message-passing network over the
// bipartite variable/constraint graph of Ā (hidden width 32), its training (backward pass, Adam)
// and the Hutchinson probe accumulation. Included by learned.hip only.
//
// Network (float32 parameters, one flat vector; dense layers run on bf16 MFMA with float32
// accumulation, or in plain float32 for validation):
//   h_v⁰ = relu(f_v W_v0 + b_v0),  h_c⁰ = relu(f_c W_c0 + b_c0)
//   round ℓ = 1..3:  a_c = Â h_v;  h_c = relu([h_c, a_c] W_cℓ + b_cℓ)
//                    a_v = Ǎ h_c;  h_v = relu([h_v, a_v] W_vℓ + b_vℓ)
//   head:  u = relu([h_v, φ(ρ̄)] W_h1 + b_h1);  g = u·w_h2 + b_h2;  M⁻¹_ii = softplus(g_i) / K_ii
// with Â = row-normalised |Ā| (m×n), Ǎ = row-normalised |Āᵀ| (n×m). softplus > 0 keeps the
// preconditioner SPD, and softplus = 1 is the Jacobi preconditioner of Section 6.3.1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qpg {

constexpr int kH = 32;
constexpr int kRounds = 3;

// Offsets in the flat parameter vector (row-major weights, [input][output]).
struct NetOff {
  static constexpr int W_v0 = 0;
  static constexpr int b_v0 = W_v0 + 32 * kH;
  static constexpr int W_c0 = b_v0 + kH;
  static constexpr int b_c0 = W_c0 + 32 * kH;
  static constexpr int r0 = b_c0 + kH;
  static constexpr int rsz = 2 * (2 * kH * kH + kH);
  static constexpr int W_c(int l) { return r0 + (l - 1) * rsz; }
  static constexpr int b_c(int l) { return W_c(l) + 2 * kH * kH; }
  static constexpr int W_v(int l) { return b_c(l) + kH; }
  static constexpr int b_v(int l) { return W_v(l) + 2 * kH * kH; }
  static constexpr int W_h1 = r0 + kRounds * rsz;
  static constexpr int b_h1 = W_h1 + 2 * kH * kH;
  static constexpr int w_h2 = b_h1 + kH;
  static constexpr int b_h2 = w_h2 + kH;
  static constexpr int total = b_h2 + 1;
};
static_assert(NetOff::total == 16705, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// float → bfloat16, round to nearest even.
__device__ __forceinline__ short f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float bf2f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

// x ≈ hi + lo with both parts bf16: a data operand carried at ~16 significant bits through the
// bf16 MFMA (weights stay single bf16).
__device__ __forceinline__ void split4(float4 v, bf16x4& hi, bf16x4& lo) {
  const float x[4] = {v.x, v.y, v.z, v.w};
  for (int t = 0; t < 4; ++t) {
    hi[t] = f2bf(x[t]);
    lo[t] = f2bf(x[t] - bf2f(hi[t]));
  }
}

__device__ __forceinline__ float softplusf(float g) { return fmaxf(g, 0.f) + log1pf(expf(-fabsf(g))); }

// ------------------------------------------------------------------------------------ SpMM
// Y[r, :] (=|+=) Σ_k w[k] · X[col[k] − coff, :] over the entries of row r from start[r] (or
// rowptr[r]) to rowptr[r+1]; 32 features, one 32-lane half-wavefront per row. Uses the SpMV work
// list of the matrix; a split long row is processed whole by the workgroup of its first chunk.
__global__ __launch_bounds__(kBlock) void k_spmm32(const Item* __restrict__ items,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ w, int coff,
                                                   const float* __restrict__ X,
                                                   float* __restrict__ Y, int accumulate) {
  const Item it = items[blockIdx.x];
  if (it.nchunk > 0 && it.chunk > 0) return;
  const int tid = threadIdx.x, lane = tid & 31, half = tid >> 5;  // 8 half-waves
  const bool single_long = (it.r1 == it.r0 + 1) && (it.nchunk > 0 || it.k1 - it.k0 > kStreamCap);
  if (!single_long) {
    for (int r = it.r0 + half; r < it.r1; r += kBlock / 32) {
      const int a = start ? start[r] : rowptr[r], b = rowptr[r + 1];
      float acc = 0.f;
#pragma unroll 4
      for (int k = a; k < b; ++k) acc += w[k] * X[(size_t)(col[k] - coff) * kH + lane];
      float* y = &Y[(size_t)r * kH + lane];
      *y = accumulate ? *y + acc : acc;
    }
  } else {
    __shared__ float part[kBlock / 32][kH];
    const int r = it.r0;
    const int a = start ? start[r] : rowptr[r], b = rowptr[r + 1];
    float acc = 0.f;
    for (int k = a + half; k < b; k += kBlock / 32) acc += w[k] * X[(size_t)(col[k] - coff) * kH + lane];
    part[half][lane] = acc;
    __syncthreads();
    if (tid < kH) {
      float s = 0.f;
      for (int h = 0; h < kBlock / 32; ++h) s += part[h][tid];
      float* y = &Y[(size_t)r * kH + tid];
      *y = accumulate ? *y + s : s;
    }
  }
}

// ------------------------------------------------------------------------------ dense layers
// Y = relu(X1 W[0:32] + X2 W[32:64] + b) (X2 may be null: K = 32). N rows, 32 outputs.

// bf16 MFMA: one wavefront per 32-row tile, v_mfma_f32_32x32x8 bf16 (K = 8 per instruction);
// activations and gradients enter as hi + lo bf16 pairs (two MFMAs), weights as one bf16.
// Fragment layout (64 lanes): A(32×8): lane l holds row l%32, k = 4(l/32)..+3; B(8×32): lane l
// holds column l%32, k = 4(l/32)..+3; C(32×32): lane l holds column l%32, rows
// 8(v/4) + 4(l/32) + v%4 for v = 0..15.
__device__ __forceinline__ int crow(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }

__global__ __launch_bounds__(kBlock) void k_dense_fwd_mfma(int N, const float* __restrict__ X1,
                                                           const float* __restrict__ X2,
                                                           const float* __restrict__ W,
                                                           const float* __restrict__ bias,
                                                           float* __restrict__ Y) {
  const int K = X2 ? 64 : 32;
  __shared__ bf16x4 wb[8][64];  // B fragments per k-block
  for (int e = threadIdx.x; e < (K / 8) * 64; e += kBlock) {
    const int kb = e >> 6, l = e & 63;
    bf16x4 f;
    for (int t = 0; t < 4; ++t) f[t] = f2bf(W[(8 * kb + 4 * (l >> 5) + t) * kH + (l & 31)]);
    wb[kb][l] = f;
  }
  __syncthreads();
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (blockIdx.x * (kBlock / 64) + wave) * 32;
  if (r0 >= N) return;
  const int row = r0 + (l & 31);
  floatx16 c = {};
  for (int kb = 0; kb < K / 8; ++kb) {
    const float* X = kb < 4 ? X1 : X2;
    const int c0 = 8 * (kb & 3) + 4 * (l >> 5);
    float4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < N) v = *reinterpret_cast<const float4*>(&X[(size_t)row * kH + c0]);
    bf16x4 ahi, alo;
    split4(v, ahi, alo);
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ahi, wb[kb][l], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(alo, wb[kb][l], c, 0, 0, 0);
  }
  const int j = l & 31;
  const float bj = bias[j];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = r0 + crow(v, l);
    if (r < N) Y[(size_t)r * kH + j] = fmaxf(c[v] + bj, 0.f);
  }
}

__global__ __launch_bounds__(kBlock) void k_dense_fwd_f32(int N, const float* __restrict__ X1,
                                                          const float* __restrict__ X2,
                                                          const float* __restrict__ W,
                                                          const float* __restrict__ bias,
                                                          float* __restrict__ Y) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N * kH) return;
  const int r = idx / kH, j = idx % kH;
  float s = bias[j];
  for (int k = 0; k < kH; ++k) s += X1[(size_t)r * kH + k] * W[k * kH + j];
  if (X2)
    for (int k = 0; k < kH; ++k) s += X2[(size_t)r * kH + k] * W[(kH + k) * kH + j];
  Y[idx] = fmaxf(s, 0.f);
}

// dX = (dY ∘ [Y > 0]) Wᵀ, split into dX1 (first 32 inputs) and dX2 (next 32; may be null).
// accumulate: dX1 += … instead of =.
__global__ __launch_bounds__(kBlock) void k_dense_bwd_dx_mfma(int N, const float* __restrict__ dY,
                                                              const float* __restrict__ Y,
                                                              const float* __restrict__ W,
                                                              float* __restrict__ dX1,
                                                              float* __restrict__ dX2,
                                                              int accumulate) {
  const int nh = dX2 ? 2 : 1;
  __shared__ bf16x4 wb[2][4][64];  // B[k = j][n = i] = W[i][j] for the two input halves
  for (int e = threadIdx.x; e < nh * 4 * 64; e += kBlock) {
    const int h = e >> 8, kb = (e >> 6) & 3, l = e & 63;
    bf16x4 f;
    for (int t = 0; t < 4; ++t) f[t] = f2bf(W[(h * kH + (l & 31)) * kH + 8 * kb + 4 * (l >> 5) + t]);
    wb[h][kb][l] = f;
  }
  __syncthreads();
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (blockIdx.x * (kBlock / 64) + wave) * 32;
  if (r0 >= N) return;
  const int row = r0 + (l & 31);
  bf16x4 ahi[4], alo[4];
  for (int kb = 0; kb < 4; ++kb) {
    const int c0 = 8 * kb + 4 * (l >> 5);
    float4 z = {0.f, 0.f, 0.f, 0.f};
    if (row < N) {
      const float4 d = *reinterpret_cast<const float4*>(&dY[(size_t)row * kH + c0]);
      const float4 y = *reinterpret_cast<const float4*>(&Y[(size_t)row * kH + c0]);
      z = {y.x > 0.f ? d.x : 0.f, y.y > 0.f ? d.y : 0.f, y.z > 0.f ? d.z : 0.f, y.w > 0.f ? d.w : 0.f};
    }
    split4(z, ahi[kb], alo[kb]);
  }
  const int j = l & 31;
  for (int h = 0; h < nh; ++h) {
    floatx16 c = {};
    for (int kb = 0; kb < 4; ++kb) {
      c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ahi[kb], wb[h][kb][l], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(alo[kb], wb[h][kb][l], c, 0, 0, 0);
    }
    float* dX = h == 0 ? dX1 : dX2;
    const int acc = h == 0 ? accumulate : 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = r0 + crow(v, l);
      if (r < N) {
        float* p = &dX[(size_t)r * kH + j];
        *p = acc ? *p + c[v] : c[v];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_dense_bwd_dx_f32(int N, const float* __restrict__ dY,
                                                             const float* __restrict__ Y,
                                                             const float* __restrict__ W,
                                                             float* __restrict__ dX1,
                                                             float* __restrict__ dX2,
                                                             int accumulate) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N * kH) return;
  const int r = idx / kH, i = idx % kH;
  float s1 = 0.f, s2 = 0.f;
  for (int j = 0; j < kH; ++j) {
    const float d = Y[(size_t)r * kH + j] > 0.f ? dY[(size_t)r * kH + j] : 0.f;
    s1 += d * W[i * kH + j];
    if (dX2) s2 += d * W[(kH + i) * kH + j];
  }
  dX1[idx] = accumulate ? dX1[idx] + s1 : s1;
  if (dX2) dX2[idx] = s2;
}

// Per-workgroup partial of dW = [X1 X2]ᵀ (dY ∘ [Y > 0]) (K×32) and db = Σ_rows (dY ∘ [Y > 0]),
// written to part[blockIdx][K·32 + 32]; rows are split evenly over the grid.
__global__ __launch_bounds__(kBlock) void k_dense_bwd_dw_mfma(int N, const float* __restrict__ X1,
                                                              const float* __restrict__ X2,
                                                              const float* __restrict__ dY,
                                                              const float* __restrict__ Y,
                                                              float* __restrict__ part) {
  const int K = X2 ? 64 : 32;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per_block = (N + gridDim.x - 1) / gridDim.x;
  const int rb = blockIdx.x * per_block, re = min(N, rb + per_block);
  floatx16 c1 = {}, c2 = {};
  float db = 0.f;
  const int j = l & 31;
  for (int base = rb + 8 * wave; base < re; base += 8 * (kBlock / 64)) {
    float4 x1 = {0.f, 0.f, 0.f, 0.f}, x2 = {0.f, 0.f, 0.f, 0.f}, d = {0.f, 0.f, 0.f, 0.f};
    float* px1 = &x1.x;
    float* px2 = &x2.x;
    float* pd = &d.x;
    for (int t = 0; t < 4; ++t) {
      const int r = base + 4 * (l >> 5) + t;
      if (r < re) {
        px1[t] = X1[(size_t)r * kH + j];
        if (X2) px2[t] = X2[(size_t)r * kH + j];
        pd[t] = Y[(size_t)r * kH + j] > 0.f ? dY[(size_t)r * kH + j] : 0.f;
      }
      db += pd[t];
    }
    // both operands are data: hi·hi + hi·lo + lo·hi
    bf16x4 a1h, a1l, bh, bl;
    split4(x1, a1h, a1l);
    split4(d, bh, bl);
    c1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1h, bh, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1h, bl, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1l, bh, c1, 0, 0, 0);
    if (X2) {
      bf16x4 a2h, a2l;
      split4(x2, a2h, a2l);
      c2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a2h, bh, c2, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a2h, bl, c2, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a2l, bh, c2, 0, 0, 0);
    }
  }
  db += __shfl_xor(db, 32, 64);
  __shared__ float acc[4][64 * kH + kH];
  for (int v = 0; v < 16; ++v) {
    acc[wave][crow(v, l) * kH + j] = c1[v];
    if (X2) acc[wave][(kH + crow(v, l)) * kH + j] = c2[v];
  }
  if (l < 32) acc[wave][K * kH + j] = db;
  __syncthreads();
  const int width = K * kH + kH;
  for (int e = threadIdx.x; e < width; e += kBlock)
    part[(size_t)blockIdx.x * width + e] = (acc[0][e] + acc[1][e]) + (acc[2][e] + acc[3][e]);
}

__global__ __launch_bounds__(kBlock) void k_dense_bwd_dw_f32(int N, const float* __restrict__ X1,
                                                             const float* __restrict__ X2,
                                                             const float* __restrict__ dY,
                                                             const float* __restrict__ Y,
                                                             float* __restrict__ part) {
  const int K = X2 ? 64 : 32;
  const int width = K * kH + kH;
  const int per_block = (N + gridDim.x - 1) / gridDim.x;
  const int rb = blockIdx.x * per_block, re = min(N, rb + per_block);
  for (int e = threadIdx.x; e < width; e += kBlock) {
    float s = 0.f;
    if (e < K * kH) {
      const int i = e / kH, j = e % kH;
      const float* X = i < kH ? X1 : X2;
      const int ii = i % kH;
      for (int r = rb; r < re; ++r) {
        const float d = Y[(size_t)r * kH + j] > 0.f ? dY[(size_t)r * kH + j] : 0.f;
        s += X[(size_t)r * kH + ii] * d;
      }
    } else {
      const int j = e - K * kH;
      for (int r = rb; r < re; ++r) s += Y[(size_t)r * kH + j] > 0.f ? dY[(size_t)r * kH + j] : 0.f;
    }
    part[(size_t)blockIdx.x * width + e] = s;
  }
}

// out[e] = Σ_g part[g·width + e] (workgroup order), for e < width.
__global__ __launch_bounds__(kBlock) void k_part_reduce(const float* __restrict__ part, int G,
                                                        int width, float* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= width) return;
  float s = 0.f;
  for (int g = 0; g < G; ++g) s += part[(size_t)g * width + e];
  out[e] = s;
}

// ------------------------------------------------------------------------------ head and loss
// φ (ρ̄-dependent head inputs, n×32): log(ρ̄‖Ā_i‖² + 1e-12) − log K_ii, log(P̄_ii + σ) − log K_ii.
__global__ __launch_bounds__(kBlock) void k_phi(int n, const double* __restrict__ diagP,
                                                const double* __restrict__ colsq, double sigma,
                                                double rho, float* __restrict__ phi) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n * kH) return;
  const int i = idx / kH, c = idx % kH;
  const double K = diagP[i] + sigma + rho * colsq[i];
  float v = 0.f;
  if (c == 0) v = (float)(log(rho * colsq[i] + 1e-12) - log(K));
  if (c == 1) v = (float)(log(diagP[i] + sigma) - log(K));
  phi[idx] = v;
}

// g = u·w_h2 + b_h2; optionally M⁻¹_ii = softplus(g_i) / K_ii into dinv (T). For M⁻¹, g is
// clamped to [−30, 30] so that softplus(g) ∈ [9e-14, 30] stays a normal positive float.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_head_out(int n, const float* __restrict__ u,
                                                     const float* __restrict__ theta,
                                                     float* __restrict__ g, T* __restrict__ dinv,
                                                     const double* __restrict__ diagP,
                                                     const double* __restrict__ colsq,
                                                     double sigma, double rho) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float acc = theta[NetOff::b_h2];
  for (int j = 0; j < kH; ++j) acc += u[(size_t)i * kH + j] * theta[NetOff::w_h2 + j];
  if (g) g[i] = acc;
  if (dinv) {
    const float gc = fminf(fmaxf(acc, -30.f), 30.f);
    dinv[i] = (T)((double)softplusf(gc) / (diagP[i] + sigma + rho * colsq[i]));
  }
}

__device__ __forceinline__ double softplus_d(double g) { return fmax(g, 0.0) + log1p(exp(-fabs(g))); }
__device__ __forceinline__ double sigmoid_d(double g) { return 1.0 / (1.0 + exp(-g)); }

// Loss, pass 1: e_i = log softplus(g_i) − t_i (double: no underflow for very negative g),
// partial sums of e.
__global__ __launch_bounds__(kBlock) void k_loss_mean(int n, const float* __restrict__ g,
                                                      const float* __restrict__ t,
                                                      double* __restrict__ e, double* partials) {
  double red[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double gi = (double)g[i];
    const double ls = gi < -30.0 ? gi + log1p(-0.5 * exp(gi)) : log(softplus_d(gi));
    const double ei = ls - (double)t[i];
    e[i] = ei;
    red[0] += ei;
  }
  publish<1, 0u>(red, partials);
}

struct NetScalars {
  double mean_e;
  double loss;
};

struct FinMeanE {
  NetScalars* ns;
  int n;
  __device__ void operator()(const double* t) const { ns->mean_e = t[0] / n; }
};
struct FinLoss {
  NetScalars* ns;
  int n;
  __device__ void operator()(const double* t) const { ns->loss = t[0] / n; }
};

// Loss, pass 2: d = e − ē, Σ d², dL/dg = (2/n) d σ(g)/softplus(g).
__global__ __launch_bounds__(kBlock) void k_loss_grad(int n, const double* __restrict__ e,
                                                      const float* __restrict__ g,
                                                      const NetScalars* ns, float* __restrict__ dg,
                                                      double* partials) {
  const double me = ns->mean_e;
  double red[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double d = e[i] - me;
    red[0] += d * d;
    const double gi = (double)g[i];
    const double ratio = gi < -30.0 ? 1.0 - 0.5 * exp(gi) : sigmoid_d(gi) / softplus_d(gi);
    dg[i] = (float)(2.0 / n * d * ratio);
  }
  publish<1, 0u>(red, partials);
}

// Head output backward: dU = dg ⊗ w_h2 (the relu mask is applied by the dense backward), and
// per-workgroup partials of dw_h2 = Σ_i dg_i u_i and db_h2 = Σ_i dg_i (width 33).
__global__ __launch_bounds__(kBlock) void k_head_out_bwd(int n, const float* __restrict__ u,
                                                         const float* __restrict__ dg,
                                                         const float* __restrict__ theta,
                                                         float* __restrict__ dU,
                                                         float* __restrict__ part) {
  __shared__ float acc[kBlock / kH][kH + 1];
  const int lane = threadIdx.x % kH, grp = threadIdx.x / kH;
  float sw = 0.f, sb = 0.f;
  const int stride = gridDim.x * (kBlock / kH);
  for (int i = blockIdx.x * (kBlock / kH) + grp; i < n; i += stride) {
    const float d = dg[i];
    dU[(size_t)i * kH + lane] = d * theta[NetOff::w_h2 + lane];
    sw += d * u[(size_t)i * kH + lane];
    if (lane == 0) sb += d;
  }
  acc[grp][lane] = sw;
  if (lane == 0) acc[grp][kH] = sb;
  __syncthreads();
  if (threadIdx.x <= kH) {
    float s = 0.f;
    for (int g2 = 0; g2 < kBlock / kH; ++g2) s += acc[g2][threadIdx.x];
    part[(size_t)blockIdx.x * (kH + 1) + threadIdx.x] = s;
  }
}

// Adam on the float32 master parameters.
__global__ __launch_bounds__(kBlock) void k_adam(int P, float* __restrict__ theta,
                                                 const float* __restrict__ grad,
                                                 float* __restrict__ m1, float* __restrict__ m2,
                                                 float lr, float b1, float b2, float eps, float c1,
                                                 float c2) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= P) return;
  const float gi = grad[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  theta[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// ------------------------------------------------------------------------------ graph build
// Per-row statistics of rows [start or rowptr, rowptr+1) of a CSR matrix (one thread per row):
// Σ|v|, max|v|, Σv², number of entries.
__global__ __launch_bounds__(kBlock) void k_rowstats(int nrows, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ start,
                                                     const double* __restrict__ val,
                                                     double* __restrict__ sum_abs,
                                                     double* __restrict__ max_abs,
                                                     double* __restrict__ sumsq,
                                                     int32_t* __restrict__ deg) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrows) return;
  const int a = start ? start[r] : rowptr[r], b = rowptr[r + 1];
  double s = 0.0, mx = 0.0, q = 0.0;
  for (int k = a; k < b; ++k) {
    const double v = fabs(val[k]);
    s += v;
    mx = v > mx ? v : mx;
    q += v * v;
  }
  sum_abs[r] = s;
  max_abs[r] = mx;
  sumsq[r] = q;
  deg[r] = b - a;
}

// Edge weights on one CSR structure: w_row[k] = |v| / rowsum[row], w_col[k] = |v| / colsum[col−coff].
__global__ __launch_bounds__(kBlock) void k_edge_weights(int nrows, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ start,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, int coff,
                                                         const double* __restrict__ rowsum,
                                                         const double* __restrict__ colsum,
                                                         float* __restrict__ w_row,
                                                         float* __restrict__ w_col) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrows) return;
  const int a = start ? start[r] : rowptr[r], b = rowptr[r + 1];
  const double rs = rowsum[r];
  for (int k = a; k < b; ++k) {
    const double v = fabs(val[k]);
    const double cs = colsum[col[k] - coff];
    w_row[k] = rs > 0 ? (float)(v / rs) : 0.f;
    w_col[k] = cs > 0 ? (float)(v / cs) : 0.f;
  }
}

// Node features (padded to 32 columns).
__global__ __launch_bounds__(kBlock) void k_features_v(int n, const double* __restrict__ diagP,
                                                       const double* __restrict__ colsq,
                                                       const int32_t* __restrict__ deg,
                                                       const double* __restrict__ maxabs,
                                                       double sigma, float* __restrict__ fv) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n * kH) return;
  const int i = idx / kH, c = idx % kH;
  float v = 0.f;
  if (c == 0) v = (float)log(diagP[i] + sigma);
  if (c == 1) v = (float)log(colsq[i] + 1e-12);
  if (c == 2) v = (float)log1p((double)deg[i]);
  if (c == 3) v = (float)log(maxabs[i] + 1e-12);
  fv[idx] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_features_c(int m, const double* __restrict__ rowsq,
                                                       const int32_t* __restrict__ deg,
                                                       const double* __restrict__ maxabs,
                                                       const T* __restrict__ lb,
                                                       const T* __restrict__ ub,
                                                       float* __restrict__ fc) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= m * kH) return;
  const int j = idx / kH, c = idx % kH;
  float v = 0.f;
  if (c == 0) v = (float)log(rowsq[j] + 1e-12);
  if (c == 1) v = (float)log1p((double)deg[j]);
  if (c == 2) v = (lb[j] == ub[j]) ? 1.f : 0.f;
  if (c == 3) v = (float)log(maxabs[j] + 1e-12);
  fc[idx] = v;
}

// ------------------------------------------------------------------------------ Hutchinson
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe_load(int n, const int8_t* __restrict__ z,
                                                       T* __restrict__ b) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) b[i] = (T)z[i];
}

// acc += z ∘ x (x = K⁻¹z from PCG)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe_acc(int n, const int8_t* __restrict__ z,
                                                      const T* __restrict__ x,
                                                      double* __restrict__ acc) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    acc[i] += (double)z[i] * (double)x[i];
}

}  // namespace qpg
