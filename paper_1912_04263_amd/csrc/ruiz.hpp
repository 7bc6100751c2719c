// Modified Ruiz equilibration (Algorithm 2) on the device, on the CSR arrays of Ā (m rows) and
// B = [P̄ | Āᵀ] (n rows: row j holds row j of P̄, then column j of Ā). Row j of B is column j of
// M = [P̄ Āᵀ; Ā 0] and row i of Ā is column n + i of M, so every norm the algorithm needs is a
// row norm of one of the two CSR matrices (Section 6.4: column norms as row norms of the stored
// transpose, as segmented reductions over RowPointer).
//
// One wavefront per row (rows grid-strided over the wavefronts of the launch): the lanes read
// the row's entries with a stride of 64 (coalesced), and a fixed shuffle tree combines them, so
// every result is deterministic. Pre- and post-multiplication (Section 6.4) happen in the same
// row loop, where the row index is known, so no RowIndex array is needed.
//
// Per pass: (1) row ∞-norms of B and Ā, after applying the cost factor γ of the previous pass to
// P̄; (2) δ = 1/√(norms), D ← δD, E ← δE, q̄ ← δγq̄, ‖1 − δ‖∞ and ‖q̄‖∞; (3) P̄ ← D P̄ D,
// Āᵀ ← D Āᵀ E (in B), Ā ← E Ā D, and the row ∞-norms of the new P̄; (4) γ = 1/max(mean, ‖q̄‖∞),
// c ← γc. Scalars live in DevState::norms during setup: [0] ‖1 − δ‖∞, [1] ‖q̄‖∞, [2] the γ not
// yet applied to P̄ and q̄, [3] c.
#pragma once

#include "kernels.hpp"

namespace qpg {

constexpr int kRuizDev = 0, kRuizQmax = 1, kRuizGamma = 2, kRuizC = 3;

// A vanishing norm (empty row or column of M) leaves its factor at 1; large norms are capped.
__device__ __forceinline__ double ruiz_guard(double v) {
  if (!(v >= 1e-4)) return 1.0;
  return v < 1e4 ? v : 1e4;
}

__device__ __forceinline__ double wave_max64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = nmax(x, __shfl_xor(x, off, 64));
  return x;
}

__device__ __forceinline__ double wave_sum64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

#define QPG_ROW_LOOP(rows)                                                                  \
  const int lane = threadIdx.x & 63;                                                        \
  const int nwaves = gridDim.x * (blockDim.x >> 6);                                         \
  for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < (rows); r += nwaves)

__global__ void k_ruiz_init(DevState* st) {
  if (threadIdx.x == 0) {
    st->norms[kRuizGamma] = 1.0;
    st->norms[kRuizC] = 1.0;
  }
}

// (1) for B: the pending γ applied to the P̄ part, then ‖B_r‖∞ → rmax[r]
__global__ __launch_bounds__(kBlock) void k_ruiz_norms_B(int n, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ split,
                                                         double* __restrict__ val,
                                                         const DevState* __restrict__ st,
                                                         double* __restrict__ rmax) {
  const double g = st->norms[kRuizGamma];
  QPG_ROW_LOOP(n) {
    const int k1 = ptr[r + 1], ks = split[r];
    double mx = 0.0;
    for (int k = ptr[r] + lane; k < k1; k += 64) {
      double v = val[k];
      if (k < ks && g != 1.0) {
        v *= g;
        val[k] = v;
      }
      mx = nmax(mx, fabs(v));
    }
    mx = wave_max64(mx);
    if (lane == 0) rmax[r] = mx;
  }
}

// (1) for Ā: ‖Ā_i‖∞ → rmax[i]
__global__ __launch_bounds__(kBlock) void k_ruiz_norms_A(int m, const int32_t* __restrict__ ptr,
                                                         const double* __restrict__ val,
                                                         double* __restrict__ rmax) {
  QPG_ROW_LOOP(m) {
    const int k1 = ptr[r + 1];
    double mx = 0.0;
    for (int k = ptr[r] + lane; k < k1; k += 64) mx = nmax(mx, fabs(val[k]));
    mx = wave_max64(mx);
    if (lane == 0) rmax[r] = mx;
  }
}

// (2) δ for the n + m columns of M; D, E, q̄ updated; partials ‖1 − δ‖∞ and ‖q̄‖∞.
__global__ __launch_bounds__(kBlock) void k_ruiz_delta(int n, int m, const double* __restrict__ rmaxB,
                                                       const double* __restrict__ rmaxA,
                                                       double* __restrict__ D, double* __restrict__ E,
                                                       double* __restrict__ dD, double* __restrict__ dE,
                                                       double* __restrict__ qb,
                                                       const DevState* __restrict__ st,
                                                       double* __restrict__ partials) {
  const double g = st->norms[kRuizGamma];
  double red[2] = {0.0, 0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n + m; i += gridDim.x * kBlock) {
    if (i < n) {
      const double d = 1.0 / sqrt(ruiz_guard(rmaxB[i]));
      dD[i] = d;
      D[i] *= d;
      const double q = (qb[i] * g) * d;
      qb[i] = q;
      red[0] = nmax(red[0], fabs(1.0 - d));
      red[1] = nmax(red[1], fabs(q));
    } else {
      const int j = i - n;
      const double e = 1.0 / sqrt(ruiz_guard(rmaxA[j]));
      dE[j] = e;
      E[j] *= e;
      red[0] = nmax(red[0], fabs(1.0 - e));
    }
  }
  publish<2, 3u>(red, partials);
}

struct FinRuizDelta {
  DevState* st;
  __device__ void operator()(const double* t) const {
    st->norms[kRuizDev] = t[0];
    st->norms[kRuizQmax] = t[1];
    st->norms[kRuizGamma] = 1.0;  // consumed by the norms of B and by q̄ above
  }
};

// (3) B ← [D P̄ D | D Āᵀ E] row by row, and ‖P̄_r‖∞ of the result → pmax[r]
__global__ __launch_bounds__(kBlock) void k_ruiz_scale_B(int n, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ split,
                                                         const int32_t* __restrict__ col,
                                                         double* __restrict__ val,
                                                         const double* __restrict__ dD,
                                                         const double* __restrict__ dE,
                                                         double* __restrict__ pmax) {
  QPG_ROW_LOOP(n) {
    const int k1 = ptr[r + 1], ks = split[r];
    const double dr = dD[r];
    double mx = 0.0;
    for (int k = ptr[r] + lane; k < k1; k += 64) {
      const int c = col[k];
      double v = val[k];
      if (k < ks) {
        v = (v * dr) * dD[c];
        mx = nmax(mx, fabs(v));
      } else {
        v = (v * dE[c - n]) * dr;
      }
      val[k] = v;
    }
    mx = wave_max64(mx);
    if (lane == 0) pmax[r] = mx;
  }
}

// (3) Ā ← E Ā D
__global__ __launch_bounds__(kBlock) void k_ruiz_scale_A(int m, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         double* __restrict__ val,
                                                         const double* __restrict__ dD,
                                                         const double* __restrict__ dE) {
  QPG_ROW_LOOP(m) {
    const int k1 = ptr[r + 1];
    const double er = dE[r];
    for (int k = ptr[r] + lane; k < k1; k += 64) val[k] = (val[k] * er) * dD[col[k]];
  }
}

// (4) Σ_r ‖P̄_r‖∞ (partials, then FinRuizGamma)
__global__ __launch_bounds__(kBlock) void k_ruiz_pmean(int n, const double* __restrict__ pmax,
                                                       double* __restrict__ partials) {
  double red[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) red[0] += pmax[i];
  publish<1, 0u>(red, partials);
}

struct FinRuizGamma {
  DevState* st;
  int n;
  __device__ void operator()(const double* t) const {
    const double mean = t[0] / (double)n;
    const double q = st->norms[kRuizQmax];
    const double g = 1.0 / ruiz_guard(mean > q ? mean : q);
    st->norms[kRuizGamma] = g;
    st->norms[kRuizC] *= g;
  }
};

// After the last pass: the pending γ applied to P̄; diag(P̄), ‖Ā_r‖² = Σ of the squared Āᵀ part
// of row r (Section 6.3.1) and, with equality-row flags, its equality rows' share.
__global__ __launch_bounds__(kBlock) void k_ruiz_final_B(int n, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ split,
                                                         const int32_t* __restrict__ col,
                                                         double* __restrict__ val,
                                                         const DevState* __restrict__ st,
                                                         const uint8_t* __restrict__ eq,
                                                         double* __restrict__ diagP,
                                                         double* __restrict__ colsq,
                                                         double* __restrict__ colsq_eq) {
  const double g = st->norms[kRuizGamma];
  QPG_ROW_LOOP(n) {
    const int k1 = ptr[r + 1], ks = split[r];
    double dg = 0.0, sq = 0.0, sqe = 0.0;
    for (int k = ptr[r] + lane; k < k1; k += 64) {
      double v = val[k];
      const int c = col[k];
      if (k < ks) {
        if (g != 1.0) {
          v *= g;
          val[k] = v;
        }
        if (c == r) dg = v;
      } else {
        const double v2 = v * v;
        sq += v2;
        if (eq && eq[c - n]) sqe += v2;
      }
    }
    dg = wave_sum64(dg);  // at most one lane holds the diagonal
    sq = wave_sum64(sq);
    sqe = wave_sum64(sqe);
    if (lane == 0) {
      diagP[r] = dg;
      colsq[r] = sq;
      if (colsq_eq) colsq_eq[r] = sqe;
    }
  }
}

// After the last pass: q̄ ← γq̄; l̄ = El, ū = Eu (bounds already clamped); D⁻¹, E⁻¹; ‖q̄‖∞.
__global__ __launch_bounds__(kBlock) void k_ruiz_final_vec(int n, int m, double* __restrict__ qb,
                                                           double* __restrict__ lb, double* __restrict__ ub,
                                                           const double* __restrict__ D,
                                                           const double* __restrict__ E,
                                                           double* __restrict__ dinv,
                                                           double* __restrict__ einv,
                                                           const DevState* __restrict__ st,
                                                           double* __restrict__ partials) {
  const double g = st->norms[kRuizGamma];
  double red[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n + m; i += gridDim.x * kBlock) {
    if (i < n) {
      const double q = qb[i] * g;
      qb[i] = q;
      dinv[i] = 1.0 / D[i];
      red[0] = nmax(red[0], fabs(q));
    } else {
      const int j = i - n;
      lb[j] = E[j] * lb[j];
      ub[j] = E[j] * ub[j];
      einv[j] = 1.0 / E[j];
    }
  }
  publish<1, 1u>(red, partials);
}

struct FinRuizFinal {
  DevState* st;
  __device__ void operator()(const double* t) const {
    st->norms[kRuizQmax] = t[0];  // ‖q̄‖∞ of the final q̄
    st->norms[kRuizGamma] = 1.0;
  }
};

// SELL-ordered values from CSR values: out[k] = val[src[k]], 0 where src[k] < 0 (padding).
__global__ __launch_bounds__(kBlock) void k_gather_values(int64_t count, const int32_t* __restrict__ src,
                                                          const double* __restrict__ val,
                                                          double* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < count; k += (int64_t)gridDim.x * kBlock) {
    const int32_t s = src[k];
    out[k] = s >= 0 ? val[s] : 0.0;
  }
}

// The entries of a work list in SELL order, from its lanes (see TilePlan): one workgroup per
// tile, one wavefront per chunk, a lane per lane. At step q, lane j of a chunk holds the CSR index
// start + q while q < len, else −1 (padding), and the column of that entry (of the segment's last
// entry in the padding; the window's first column, or 0 without a window, for an empty lane),
// stored as an offset from the window's first column in a windowed tile. The arguments are the
// planner's own arrays, whose bounds it guarantees; the indices are checked again here so that a
// malformed list cannot make this kernel read or write outside them.
__global__ __launch_bounds__(kBlock) void k_sell_build(const Tile* __restrict__ tiles, int32_t ntiles,
                                                       const Chunk* __restrict__ chunks, int64_t nchunk,
                                                       const int32_t* __restrict__ lstart,
                                                       const int32_t* __restrict__ llen,
                                                       const int32_t* __restrict__ col, int64_t nnz,
                                                       int32_t* __restrict__ src, int64_t n_src,
                                                       uint16_t* __restrict__ col16, int64_t n_c16,
                                                       int32_t* __restrict__ col32, int64_t n_c32) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kBlock >> 6;
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    const bool win = T.wlen > 0;
    if (T.chunk0 < 0) continue;
    for (int64_t ci = (int64_t)T.chunk0 + wave; ci < (int64_t)T.chunk0 + T.nchunk && ci < nchunk; ci += nwave) {
      const Chunk ch = chunks[ci];
      const int64_t steps = ch.steps, base = ch.base, cbase = ch.cbase;
      if (base < 0 || cbase < 0 || steps < 0 || base + steps * 64 > n_src ||
          cbase + steps * 64 > (win ? n_c16 : n_c32) || ch.seg0 < 0 || (int64_t)ch.seg0 + 64 > nchunk * 64)
        continue;
      const int32_t s0 = lstart[(int64_t)ch.seg0 + lane];
      int32_t len = llen[(int64_t)ch.seg0 + lane];
      if (s0 < 0 || (int64_t)s0 + len > nnz) len = -1;
      for (int64_t q = 0; q < steps; ++q) {
        const int32_t k = q < len ? s0 + (int32_t)q : -1;
        const int32_t c = len > 0 ? col[q < len ? k : s0 + len - 1] : (win ? T.wlo : 0);
        src[base + q * 64 + lane] = k;
        if (win)
          col16[cbase + q * 64 + lane] = (uint16_t)(c - T.wlo);
        else
          col32[cbase + q * 64 + lane] = c;
      }
    }
  }
}

// Values of B = [P | Aᵀ] in CSR (unscaled): row i is row i of the full P (p_val from p_ptr[i]),
// then column i of A (A's CSC values from a_colptr[i]), both contiguous; one wavefront per row.
__global__ __launch_bounds__(kBlock) void k_assemble_b(int n, const int32_t* __restrict__ b_ptr,
                                                       const int32_t* __restrict__ b_split,
                                                       const int32_t* __restrict__ p_ptr,
                                                       const double* __restrict__ p_val,
                                                       const int32_t* __restrict__ a_colptr,
                                                       const double* __restrict__ a_csc_val,
                                                       double* __restrict__ b_val) {
  const int lane = threadIdx.x & 63;
  for (int i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < n; i += (gridDim.x * kBlock) >> 6) {
    const int32_t o = b_ptr[i], sp = b_split[i], p0 = p_ptr[i], a0 = a_colptr[i];
    for (int32_t k = lane; k < sp - o; k += 64) b_val[o + k] = p_val[p0 + k];
    for (int32_t k = lane; k < b_ptr[i + 1] - sp; k += 64) b_val[sp + k] = a_csc_val[a0 + k];
  }
}

#undef QPG_ROW_LOOP

}  // namespace qpg
