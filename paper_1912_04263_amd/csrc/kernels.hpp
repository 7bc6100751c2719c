// Device kernels of the ADMM / reduced-KKT PCG path for gfx950 (wavefront 64, 256-thread
// workgroups). Included by solver.hip only.
//
// Every SpMV runs in two launches of one kernel pair: k_spmv streams the matrix in SELL chunks
// (one lane per row segment, 64 consecutive entries per load instruction, no barrier), gathering
// from a window of the multiplied vector staged in LDS where one is planned, and writes segment
// sums to slots; k_combine adds each row's slots in a fixed order and runs an operation-specific
// epilogue (the fused vector work of the ADMM / PCG step). Reduction contributions (FP64 sums and
// ∞-norms) are combined deterministically: per-workgroup partials, reduced in a fixed order by
// k_finalize, which also runs the scalar finalisation (α, β, stopping flags) on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "qpg_internal.hpp"

namespace qpg {

constexpr int kMaxSlots = 8;

// R = diag(ρ_i) with ρ_i = 10³ρ̄ on the equality rows (eq. rho_vec) when a row flag array is
// given; ρ̄ everywhere otherwise.
constexpr double kRhoEq = 1e3;
template <typename T>
__device__ __forceinline__ T row_rho(const uint8_t* eq, int i, T rho) {
  return (eq && eq[i]) ? T(kRhoEq) * rho : rho;
}

// Scalars of the iteration that live on the device.
struct DevState {
  double rzp[2];  // rᵀM⁻¹r of the current PCG iterate, indexed by the iteration's parity
  double alpha;   // PCG step length
  double beta;    // PCG direction update
  double kappa;   // pᵀKp
  double bnorm;   // ‖b‖∞
  double rnorm;   // ‖r‖∞
  double thresh;  // PCG stopping threshold on ‖r‖∞
  int32_t iter;       // PCG iterations of the current solve
  int32_t done;       // PCG finished (converged, capped or broken down)
  int32_t breakdown;  // pᵀKp ≤ 0 / NaN or rᵀM⁻¹r NaN seen
  int32_t maxit;      // PCG iteration cap
  // speculative ADMM iterations (launched without a host read between them)
  int32_t abort;         // set when one of them needs the host: everything after it is skipped
  int32_t abort_k;       // the ADMM iteration that set it
  int32_t abort_reason;  // 1 PCG not finished within the launched iterations, 2 breakdown, 3 capped
  int32_t pcg_sum;       // PCG iterations of the completed speculative ADMM iterations
  int32_t pcg_max;       // and their largest count
  double norms[24];   // residual-check outputs (OpUpdate<CHECK> or OpRPrim / OpRDual: 0..13, OpInfeasA/B: 16..22)
};

struct RedBuf {
  double* partials;   // [slot][workgroups] (kMaxSlots × grid), read by the next k_finalize or vector kernel
  double* vpartials;  // the same for k_pcg_update, which reads `partials` of the B pass meanwhile
};

// NaN-propagating max (a NaN residual must not disappear inside a norm).
__device__ __forceinline__ double nmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

template <unsigned MAXMASK>
__device__ __forceinline__ double comb(int s, double a, double b) {
  return ((MAXMASK >> s) & 1u) ? nmax(a, b) : a + b;
}

// Matrix-stream load. Plain loads: on gfx950 the non-temporal variant measured ~30% slower for
// this access pattern (coalesced value/index streams interleaved with random gathers).
template <typename T>
__device__ __forceinline__ T ldm(const T* p) {
  return *p;
}

// 256-thread reduction of NS slots; result valid in thread 0. Fixed order: deterministic.
template <int NS, unsigned MAXMASK>
__device__ __forceinline__ void block_reduce(double (&v)[NS], double* lds) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double x = v[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = comb<MAXMASK>(s, x, __shfl_xor(x, off, 64));
    v[s] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) lds[s * 4 + wid] = v[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      v[s] = comb<MAXMASK>(s, comb<MAXMASK>(s, lds[s * 4 + 0], lds[s * 4 + 1]),
                           comb<MAXMASK>(s, lds[s * 4 + 2], lds[s * 4 + 3]));
  }
}

// Publish this workgroup's partials (thread 0 after block_reduce). They are combined by
// k_finalize, launched next on the same stream: no cross-workgroup synchronisation inside a
// kernel, and the combination order is fixed (workgroup order), so results are reproducible.
// Slot-major layout, partials[s · grid + workgroup]: the readers take consecutive workgroups
// in consecutive lanes, so each wavefront load touches a few cache lines instead of 64.
template <int NS, unsigned MAXMASK>
__device__ __forceinline__ void publish(double (&v)[NS], double* partials) {
  __shared__ double lds[kMaxSlots * 4];
  block_reduce<NS, MAXMASK>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) partials[(size_t)s * gridDim.x + blockIdx.x] = v[s];
  }
}

// Thread t of a BLOCK-thread workgroup folds partials t, t + BLOCK, t + 2·BLOCK, … into acc, in
// that order. The loads of U consecutive steps are issued before any of them is folded (clamped
// to a valid index instead of branched around, so nothing serialises them): the partials were
// just written by other XCDs and each round trip costs a full memory latency.
template <int NS, unsigned MAXMASK, int BLOCK, int U>
__device__ __forceinline__ void gather_rounds(const double* __restrict__ partials, int count,
                                              double (&acc)[NS]) {
  for (int b0 = threadIdx.x; b0 < count; b0 += U * BLOCK) {
    double v[U][NS];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + u * BLOCK, count - 1);
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = partials[(size_t)s * count + b];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b0 + u * BLOCK < count) {
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = comb<MAXMASK>(s, acc[s], v[u][s]);
      }
  }
}

// U = the steps per thread (1, 2, 4), else the largest that keeps v within 48 doubles.
template <int NS, unsigned MAXMASK, int BLOCK>
__device__ __forceinline__ void gather_partials(const double* __restrict__ partials, int count,
                                                double (&acc)[NS]) {
  constexpr int kMaxU = 48 / NS < 8 ? (48 / NS > 4 ? 48 / NS : 4) : 8;
  if (count <= 0) return;
  if (count <= BLOCK)
    gather_rounds<NS, MAXMASK, BLOCK, 1>(partials, count, acc);
  else if (count <= 2 * BLOCK)
    gather_rounds<NS, MAXMASK, BLOCK, 2>(partials, count, acc);
  else if (count <= 4 * BLOCK)
    gather_rounds<NS, MAXMASK, BLOCK, 4>(partials, count, acc);
  else
    gather_rounds<NS, MAXMASK, BLOCK, kMaxU>(partials, count, acc);
}

// One 1024-thread workgroup: combine `count` partials in a fixed order (thread t takes
// workgroups t, t + 1024, …; then a fixed tree) and run the scalar finalisation, unless the gate
// is set; then, when `mirror` is given (only before a host read: the write crosses PCIe), copy the
// device scalars into host-visible memory, gate or not.
constexpr int kFinBlock = 1024;

template <int NS, unsigned MAXMASK, class Fin>
__global__ __launch_bounds__(kFinBlock) void k_finalize(const double* __restrict__ partials, int count,
                                                        Fin fin, const int32_t* __restrict__ gate,
                                                        const DevState* st, DevState* mirror) {
  if (gate && *gate) {
    if (mirror && threadIdx.x == 0) *mirror = *st;
    return;
  }
  __shared__ double lds[kMaxSlots][kFinBlock / 64];
  double acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.0;
  gather_partials<NS, MAXMASK, kFinBlock>(partials, count, acc);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double x = acc[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = comb<MAXMASK>(s, x, __shfl_xor(x, off, 64));
    if ((threadIdx.x & 63) == 0) lds[s][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double x = lds[s][0];
      for (int w = 1; w < kFinBlock / 64; ++w) x = comb<MAXMASK>(s, x, lds[s][w]);
      acc[s] = x;
    }
    fin(acc);
    if (mirror) *mirror = *st;
  }
}

template <class S>
__global__ void k_mirror(const S* st, S* mirror) {
  if (threadIdx.x == 0) *mirror = *st;
}

// After the PCG iterations launched for speculative ADMM iteration k: when the solve has not
// finished, broke down or hit the cap, set the abort flag (which gates every later kernel of the
// speculation) and `done` (which gates the PCG kernels), so that the host takes over from
// iteration k; otherwise count the iterations. It runs in a launch of its own, after the last
// k_pcg_dir of the iteration has completed: that kernel is itself gated on `done`, so a write of
// `done` from inside it could make its later workgroups skip their share of the direction update
// that the resumed solve still needs.
template <class S>
__device__ __forceinline__ void after_pcg(S* st, int k) {
  if (st->abort) return;
  const int it = st->iter;
  int reason = 0;
  if (st->breakdown)
    reason = 2;
  else if (!st->done)
    reason = 1;
  else if (it >= st->maxit && st->rnorm > st->thresh)
    reason = 3;
  if (reason) {
    st->abort = 1;
    st->abort_k = k;
    st->abort_reason = reason;
    st->done = 1;
  } else {
    st->pcg_sum += it;
    if (it > st->pcg_max) st->pcg_max = it;
  }
}

template <class S>
__global__ void k_after_pcg(S* st, int k) {
  if (threadIdx.x == 0) after_pcg(st, k);
}

// The host resumes after an abort: clear it, and reopen the PCG solve when it was cut short.
template <class S>
__global__ void k_resume(S* st, int reopen) {
  if (threadIdx.x != 0) return;
  st->abort = 0;
  if (reopen) st->done = 0;
}

template <class S>
__global__ void k_spec_reset(S* st) {
  if (threadIdx.x != 0) return;
  st->abort = 0;
  st->abort_k = 0;
  st->abort_reason = 0;
  st->pcg_sum = 0;
  st->pcg_max = 0;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, width);
  return x;
}

// ----------------------------------------------------------------------------------------------
// CSR SpMV with fused epilogue, in two launches: k_spmv sums the segments of a Tile work list
// (SELL chunks, one lane per segment, no barrier after the window is staged) into slots, and
// k_combine adds each row's slots in order and runs the epilogue. Op supplies:
//   static constexpr int NS;            reduction slots (0: none)
//   static constexpr unsigned MAXMASK;  bit s set: slot s is an ∞-norm (max), else a sum
//   T gather(int col) const;            the multiplied value of column col
//   void epilogue(int row, T s1, T s2, double* red) const;
//        s1 / s2: the products summed over the entries with column < nsplit / ≥ nsplit
//   void side() const;                  extra elementwise work (grid-stride, in k_spmv)
//   void operator()(const double* totals) const;  scalar finalisation (run by k_finalize)
// ----------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void accumulate(T v, T x, bool first, T& s1, T& s2) {
  const T pr = v * x;
  s1 += first ? pr : T(0);
  s2 += first ? T(0) : pr;
}

constexpr int kSpmvUnroll = 8;  // SELL steps in flight per lane

template <typename T, class Op>
__global__ __launch_bounds__(kSpmvBlock) void k_spmv(const Tile* __restrict__ tiles,
                                                 const Chunk* __restrict__ chunks,
                                                 const int32_t* __restrict__ segslot,
                                                 const uint16_t* __restrict__ col16,
                                                 const int32_t* __restrict__ col32,
                                                 const T* __restrict__ val, int nsplit, Op op,
                                                 T* __restrict__ slots, int64_t pstride, int planes,
                                                 const int32_t* __restrict__ gate) {
  if (gate && *gate) return;  // uniform across the grid: set before the launch
  extern __shared__ __align__(16) unsigned char smem[];
  T* win = reinterpret_cast<T*>(smem);
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (t.wlen > 0) {
#pragma unroll 8
    for (int i = threadIdx.x; i < t.wlen; i += kSpmvBlock) win[i] = op.gather(t.wlo + i);
    __syncthreads();
  }
  for (int ci = t.chunk0 + wave; ci < t.chunk0 + t.nchunk; ci += kSpmvBlock / 64) {
    const Chunk ch = chunks[ci];
    const int slot = segslot[ch.seg0 + lane];
    const T* vp = val + ch.base + lane;
    T s1 = T(0), s2 = T(0);
    if (t.wlen > 0) {
      const uint16_t* cp = col16 + ch.cbase + lane;
      const int lim = nsplit - t.wlo;  // window offsets below lim belong to the first part
#pragma unroll kSpmvUnroll
      for (int s = 0; s < ch.steps; ++s) {
        const int o = cp[64 * s];
        accumulate(vp[64 * s], win[o], o < lim, s1, s2);
      }
    } else {
      const int32_t* cp = col32 + ch.cbase + lane;
#pragma unroll kSpmvUnroll
      for (int s = 0; s < ch.steps; ++s) {
        const int c = cp[64 * s];
        accumulate(vp[64 * s], op.gather(c), c < nsplit, s1, s2);
      }
    }
    if (slot >= 0) {
      slots[slot] = s1;
      if (planes > 1) slots[pstride + slot] = s2;
    }
  }
  op.side();
}

// Two gathered vectors at once (an operation with NV = 2 and gather2(c) returning both values):
// one read of the matrix gives the segment sums of both products, written to slot planes 0–1
// (first vector: columns < nsplit, ≥ nsplit) and 2–3 (second vector). The window holds pairs,
// so it needs twice the LDS of k_spmv's.
template <typename T>
struct Pair {
  T a, b;
};

template <typename T, class Op>
__global__ __launch_bounds__(kSpmvBlock) void k_spmv2(const Tile* __restrict__ tiles,
                                                  const Chunk* __restrict__ chunks,
                                                  const int32_t* __restrict__ segslot,
                                                  const uint16_t* __restrict__ col16,
                                                  const int32_t* __restrict__ col32,
                                                  const T* __restrict__ val, int nsplit, Op op,
                                                  T* __restrict__ slots, int64_t pstride,
                                                  const int32_t* __restrict__ gate) {
  if (gate && *gate) return;
  extern __shared__ __align__(16) unsigned char smem[];
  Pair<T>* win = reinterpret_cast<Pair<T>*>(smem);
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (t.wlen > 0) {
#pragma unroll 8
    for (int i = threadIdx.x; i < t.wlen; i += kSpmvBlock) win[i] = op.gather2(t.wlo + i);
    __syncthreads();
  }
  for (int ci = t.chunk0 + wave; ci < t.chunk0 + t.nchunk; ci += kSpmvBlock / 64) {
    const Chunk ch = chunks[ci];
    const int slot = segslot[ch.seg0 + lane];
    const T* vp = val + ch.base + lane;
    T s1 = T(0), s2 = T(0), u1 = T(0), u2 = T(0);
    if (t.wlen > 0) {
      const uint16_t* cp = col16 + ch.cbase + lane;
      const int lim = nsplit - t.wlo;
#pragma unroll kSpmvUnroll
      for (int s = 0; s < ch.steps; ++s) {
        const int o = cp[64 * s];
        const Pair<T> x = win[o];
        const T v = vp[64 * s];
        accumulate(v, x.a, o < lim, s1, s2);
        accumulate(v, x.b, o < lim, u1, u2);
      }
    } else {
      const int32_t* cp = col32 + ch.cbase + lane;
#pragma unroll kSpmvUnroll
      for (int s = 0; s < ch.steps; ++s) {
        const int c = cp[64 * s];
        const Pair<T> x = op.gather2(c);
        const T v = vp[64 * s];
        accumulate(v, x.a, c < nsplit, s1, s2);
        accumulate(v, x.b, c < nsplit, u1, u2);
      }
    }
    if (slot >= 0) {
      slots[slot] = s1;
      slots[pstride + slot] = s2;
      slots[2 * pstride + slot] = u1;
      slots[3 * pstride + slot] = u2;
    }
  }
  op.side();
}

// Gathered vectors of an operation: 1, or NV when it declares it (2: k_spmv2, epilogue2).
template <class Op, class = void>
struct NumVec {
  static constexpr int v = 1;
};
template <class Op>
struct NumVec<Op, std::void_t<decltype(Op::NV)>> {
  static constexpr int v = Op::NV;
};

// Row sums from the slots, then the epilogue. 2^lg lanes per row: lane l adds the row's slots
// l, l + L, … (in column order, through slotidx) in order, then a fixed shuffle tree combines the
// lanes (deterministic). A grid item (lg < 0) gives each row one lane, which adds the row's K
// slots tbase[t0 + j] + row in order: consecutive lanes read consecutive slots. Reduction
// partials per workgroup for k_finalize.
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_combine(const CombItem* __restrict__ items,
                                                    const int32_t* __restrict__ rowslot,
                                                    const int32_t* __restrict__ slotidx,
                                                    const int32_t* __restrict__ tbase,
                                                    const T* __restrict__ slots, int64_t pstride,
                                                    int planes, Op op, double* __restrict__ partials,
                                                    const int32_t* __restrict__ gate) {
  if (gate && *gate) return;
  constexpr int NS = Op::NS > 0 ? Op::NS : 1;
  constexpr int NV = NumVec<Op>::v;  // 2: planes 2–3 hold the second vector's sums
  double red[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) red[s] = 0.0;
  const CombItem c = items[blockIdx.x];
  if (c.lg < 0) {
    const int r = c.r0 + threadIdx.x;
    if (r < c.r1) {
      T s1 = T(0), s2 = T(0), u1 = T(0), u2 = T(0);
      const int32_t* tb = tbase + c.t0;
#pragma unroll 8
      for (int j = 0; j < -c.lg; ++j) {
        const int64_t q = (int64_t)tb[j] + r;
        s1 += slots[q];
        if (planes > 1) s2 += slots[pstride + q];
        if constexpr (NV == 2) {
          u1 += slots[2 * pstride + q];
          u2 += slots[3 * pstride + q];
        }
      }
      if constexpr (NV == 2)
        op.epilogue2(r, s1, s2, u1, u2, red);
      else
        op.epilogue(r, s1, s2, red);
    }
    if constexpr (Op::NS > 0) publish<Op::NS, Op::MAXMASK>(red, partials);
    return;
  }
  const int lg = c.lg, L = 1 << lg, groups = kBlock >> lg;
  const int g = threadIdx.x >> lg, lane = threadIdx.x & (L - 1);
  for (int r = c.r0 + g; r < c.r1; r += groups) {
    T s1 = T(0), s2 = T(0), u1 = T(0), u2 = T(0);
    const int q1 = rowslot[r + 1];
#pragma unroll 4
    for (int q = rowslot[r] + lane; q < q1; q += L) {
      const int sq = slotidx[q];
      s1 += slots[sq];
      if (planes > 1) s2 += slots[pstride + sq];
      if constexpr (NV == 2) {
        u1 += slots[2 * pstride + sq];
        u2 += slots[3 * pstride + sq];
      }
    }
    if (L > 1) {
      s1 = wave_sum(s1, L);
      if (planes > 1) s2 = wave_sum(s2, L);
      if constexpr (NV == 2) {
        u1 = wave_sum(u1, L);
        u2 = wave_sum(u2, L);
      }
    }
    if (lane == 0) {
      if constexpr (NV == 2)
        op.epilogue2(r, s1, s2, u1, u2, red);
      else
        op.epilogue(r, s1, s2, red);
    }
  }
  if constexpr (Op::NS > 0) publish<Op::NS, Op::MAXMASK>(red, partials);
}

// ------------------------------------------------------------------------------- SpMV epilogues

#define QPG_NO_SIDE \
  __device__ void side() const {}
#define QPG_NO_FIN \
  __device__ void operator()(const double*) const {}

// out = scale · (M v)   (M = Ā, or the whole of B with v = [vp; vat]); with eq set (rows of Ā),
// out_r = ρ_r/ρ̄ · scale · (M v)_r, i.e. w = RĀv for scale = ρ̄.
template <typename T>
struct OpScaled {
  QPG_NO_SIDE
  QPG_NO_FIN
  static constexpr int NS = 0;
  static constexpr unsigned MAXMASK = 0;
  const T* v;
  T* out;
  T scale;
  const uint8_t* eq = nullptr;
  __device__ T gather(int c) const { return v[c]; }
  __device__ void epilogue(int r, T s1, T s2, double*) const {
    out[r] = row_rho(eq, r, scale) * (s1 + s2);
  }
};

// B-part products: P̄ vp + Āᵀ vat (either pointer may be null: that part contributes 0)
template <typename T>
struct OpB {
  QPG_NO_SIDE
  QPG_NO_FIN
  static constexpr int NS = 0;
  static constexpr unsigned MAXMASK = 0;
  const T* vp;
  const T* vat;
  T* out;
  int n;
  __device__ T gather(int c) const {
    if (c < n) return vp ? vp[c] : T(0);
    return vat ? vat[c - n] : T(0);
  }
  __device__ void epilogue(int r, T s1, T s2, double*) const { out[r] = s1 + s2; }
};

// Scalars of a right-hand-side pass: ‖b‖∞, the PCG threshold, r⁰ᵀM⁻¹r⁰, ‖r⁰‖∞ and the stopping
// flag of Algorithm 3's initialisation (the test ‖r‖∞ ≤ ε‖b‖∞, or ≤ ε when rel is 0).
__device__ inline void rhs_scalars(DevState* st, const double* t, int maxit, int rel, double eps) {
  st->bnorm = t[0];
  st->thresh = rel ? eps * t[0] : eps;
  st->rzp[0] = t[1];
  st->rnorm = t[2];
  st->iter = 0;
  st->maxit = maxit;
  st->breakdown = (t[1] != t[1]) ? 1 : 0;
  st->done = (t[2] <= st->thresh || st->breakdown || maxit <= 0) ? 1 : 0;
}

// Right-hand side of the reduced KKT system (eq. kkt_red_sc) and the warm-started PCG residual
// (Algorithm 3 initialisation), directly, in two passes over B = [P̄ | Āᵀ]:
//   b  = σx − q̄ + Āᵀ(ρ̄z − y)
//   r⁰ = Kx̃ − b = P̄x̃ + σ(x̃ − x) + q̄ + Āᵀ(ρ̄(z̃ − z) + y),  z̃ = Āx̃
//   p⁰ = −M⁻¹r⁰;  rᵀM⁻¹r;  ‖r‖∞.
// The gathered vectors are two planes of n + m entries in one allocation g (written by k_pairs):
// plane 0 holds x̃ for the P̄ columns, then ρ̄(z̃ − z) + y for the Āᵀ columns; plane 1 holds 0,
// then ρ̄z − y. The first pass (OpRhsAt) leaves Āᵀ(ρ̄z − y) in bk, the second (OpRhsR0) gathers
// plane 0 and completes b, which stays in bk for the next right-hand side (OpRhsRec).
template <typename T>
struct OpRhsAt {
  QPG_NO_SIDE
  QPG_NO_FIN
  static constexpr int NS = 0;
  static constexpr unsigned MAXMASK = 0;
  const T* g1;  // plane 1 of g
  T* bk;
  __device__ T gather(int c) const { return g1[c]; }
  // plane 1 is 0 on the P̄ columns: only the Āᵀ part (s2) contributes
  __device__ void epilogue(int i, T, T s2, double*) const { bk[i] = s2; }
};

template <typename T>
struct OpRhsR0 {
  QPG_NO_SIDE
  static constexpr int NS = 3;
  static constexpr unsigned MAXMASK = 0x5u;  // ‖b‖∞, rᵀM⁻¹r, ‖r‖∞
  const T* x;
  const T* xt;
  const T* qb;
  const T* g;  // plane 0 of g
  const T* dinv;
  T* r;
  T* p;
  T* bk;  // in: Āᵀ(ρ̄z − y) from OpRhsAt; out: b
  T sigma;
  int maxit, rel;
  double eps;
  DevState* st;
  __device__ T gather(int c) const { return g[c]; }
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const T xi = x[i];
    const T bi = sigma * xi - qb[i] + bk[i];
    const T ri = ((s1 + sigma * (xt[i] - xi)) + qb[i]) + s2;
    const T yi = ri * dinv[i];
    r[i] = ri;
    p[i] = -yi;
    bk[i] = bi;
    red[0] = nmax(red[0], fabs((double)bi));
    red[1] += (double)ri * (double)yi;
    red[2] = nmax(red[2], fabs((double)ri));
  }
  __device__ void operator()(const double* t) const { rhs_scalars(st, t, maxit, rel, eps); }
};

// The same right-hand side and warm-started residual in one pass over B instead of two,
// from the previous PCG solve (Algorithm 3) of K'x̃ = b' that left x̃ and its residual r' in place,
// K' = P̄ + σI + ρ̄'ĀᵀĀ. Since r' + b' = K'x̃ and z̃ = Āx̃,
//   ρ̄Āᵀz̃ = γ(r' + b' − P̄x̃ − σx̃),  γ = ρ̄/ρ̄'   (R = diag(ρ_i) scales by the same γ),
// and b = σx − q̄ + ρ̄Āᵀz̃ − Āᵀ(ρ̄(z̃ − z) + y). With s1 = P̄x̃ and s2 = Āᵀ(ρ̄(z̃ − z) + y), the
// sums of plane 0 of g over the two parts of B:
//   b = σx − q̄ + γ(r' + b' − s1 − σx̃) − s2,   r⁰ = s1 + σ(x̃ − x) + q̄ + s2 (as in OpRhsR0).
// r⁰ is computed exactly as in OpRhsR0. b differs from the direct value by rounding, by the gap
// between the recursively updated r' and K'x̃ − b', and by the error b' itself carried; it enters
// only the stopping threshold ε‖b‖∞ and the next pass (the caller recomputes it directly from time
// to time).
template <typename T>
struct OpRhsRec {
  QPG_NO_SIDE
  static constexpr int NS = 3;
  static constexpr unsigned MAXMASK = 0x5u;  // ‖b‖∞, rᵀM⁻¹r, ‖r‖∞
  const T* x;
  const T* xt;
  const T* qb;
  const T* g;  // plane 0 of the right-hand-side vectors (n + m)
  const T* dinv;
  T* r;   // in: r' (n); out: r⁰
  T* p;
  T* bk;  // in: b' (n); out: b
  T sigma, gamma;
  int maxit, rel;
  double eps;
  DevState* st;
  __device__ T gather(int c) const { return g[c]; }
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const T xi = x[i], xti = xt[i];
    const T bi = (sigma * xi - qb[i]) + gamma * (((r[i] + bk[i]) - s1) - sigma * xti) - s2;
    const T ri = ((s1 + sigma * (xti - xi)) + qb[i]) + s2;
    const T yi = ri * dinv[i];
    r[i] = ri;
    p[i] = -yi;
    bk[i] = bi;
    red[0] = nmax(red[0], fabs((double)bi));
    red[1] += (double)ri * (double)yi;
    red[2] = nmax(red[2], fabs((double)ri));
  }
  __device__ void operator()(const double* t) const { rhs_scalars(st, t, maxit, rel, eps); }
};

// PCG initialisation for a given right-hand side b (Algorithm 3): r = Kx̃ − b with
// Kx̃ = P̄x̃ + σx̃ + Āᵀw, w = ρ̄Āx̃ computed before; p = −M⁻¹r; rᵀM⁻¹r; ‖r‖∞.
template <typename T>
struct OpR0 {
  QPG_NO_SIDE
  static constexpr int NS = 2;
  static constexpr unsigned MAXMASK = 2u;
  const T* xt;
  const T* w;
  const T* b;
  const T* dinv;
  T* r;
  T* p;
  T sigma;
  int n;
  int maxit;
  DevState* st;
  __device__ T gather(int c) const { return c < n ? xt[c] : w[c - n]; }
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const T ri = (s1 + s2 + sigma * xt[i]) - b[i];
    const T yi = ri * dinv[i];
    r[i] = ri;
    p[i] = -yi;
    red[0] += (double)ri * (double)yi;
    red[1] = nmax(red[1], fabs((double)ri));
  }
  __device__ void operator()(const double* t) const {
    st->rzp[0] = t[0];
    st->rnorm = t[1];
    st->iter = 0;
    st->maxit = maxit;
    st->breakdown = (t[0] != t[0]) ? 1 : 0;
    st->done = (t[1] <= st->thresh || st->breakdown || maxit <= 0) ? 1 : 0;
  }
};

// PCG K-matvec, second half: Kp = P̄p + σp + Āᵀw (w = ρ̄Āp) and the partials of κ = pᵀKp, which
// k_pcg_update combines.
// p and w are the two parts of one allocation (w = p + n), so column c of B gathers p[c].
template <typename T>
struct OpKp {
  QPG_NO_SIDE
  QPG_NO_FIN
  static constexpr int NS = 1;
  static constexpr unsigned MAXMASK = 0u;
  const T* p;
  const T* w;
  T* kp;
  T sigma;
  int n;
  DevState* st;
  __device__ T gather(int c) const { return p[c]; }
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const T pi = p[i];
    const T k = s1 + s2 + sigma * pi;
    kp[i] = k;
    red[0] += (double)pi * (double)k;
  }
};

// ADMM update (Algorithm 1, relaxation, projection and dual steps) fused with z̃ = Āx̃
// (Section 4) over the rows of Ā:
//   v = αz̃ + (1−α)z;  z⁺ = Π_[l̄,ū](v + y/ρ̄);  y ← y + ρ̄(v − z⁺);  z̃ kept, and
//   ρ̄(z̃ − z⁺) + y⁺ written to plane 0 of the right-hand-side vectors (after the n entries x̃);
//   Āx ← αz̃ + (1−α)Āx when `ax` is tracked (x ← αx̃ + (1−α)x makes this exact);
//   side task: x ← αx̃ + (1−α)x, and x̃ into plane 0.
// With CHECK, the primal residual r̄_p = Āx − z⁺ and its norms are reduced as well:
// slots ‖r̄_p‖, ‖E⁻¹r̄_p‖, ‖Āx‖, ‖E⁻¹Āx‖, ‖z‖, ‖E⁻¹z‖ → norms[0..5].
// With dxy set, the iterate differences of this step, δx̄ = x⁺ − x (n) and δȳ = y⁺ − y (m), are
// written to it for the infeasibility tests (Section 3).
template <typename T, bool CHECK>
struct OpUpdate {
  static constexpr int NS = CHECK ? 6 : 0;
  static constexpr unsigned MAXMASK = 0x3Fu;
  const T* xt;
  T* x;
  T* z;
  T* y;
  T* zt;       // z̃ = s1 is stored here (null: not stored)
  double* ax;  // null, or Āx̄ tracked by its recurrence (FP64 in both precisions)
  T* g;  // plane 0 of the right-hand-side vectors (n + m), read by the next OpRhsRec / OpRhsR0
  const T* lb;
  const T* ub;
  const double* einv;
  T alpha, rho, rho_inv;
  int n;
  DevState* st;
  T* dxy;              // null, or n + m differences (δx̄, δȳ)
  const uint8_t* eq;   // null (R = ρ̄I), or the equality-row flags of R = diag(ρ_i)
  __device__ T gather(int c) const { return xt[c]; }
  __device__ void epilogue(int i, T s1, T, double* red) const {
    const bool e = eq && eq[i];
    const T ri = e ? T(kRhoEq) * rho : rho, ri_inv = e ? rho_inv / T(kRhoEq) : rho_inv;
    const T zi = z[i], yi = y[i];
    const T v = alpha * s1 + (T(1) - alpha) * zi;
    T zn = v + yi * ri_inv;
    zn = zn < lb[i] ? lb[i] : zn;
    zn = zn > ub[i] ? ub[i] : zn;
    const T yn = yi + ri * (v - zn);
    if (dxy) dxy[n + i] = yn - yi;
    y[i] = yn;
    z[i] = zn;
    if (zt) zt[i] = s1;  // null where s1 was read from z̃ itself (k_rows)
    g[n + i] = ri * (s1 - zn) + yn;
    if (ax) {
      const double al = (double)alpha;
      const double ad = al * (double)s1 + (1.0 - al) * ax[i];
      ax[i] = ad;
      if constexpr (CHECK) {
        const double e = einv[i], zd = (double)zn;
        const double rp = ad - zd;
        red[0] = nmax(red[0], fabs(rp));
        red[1] = nmax(red[1], fabs(rp * e));
        red[2] = nmax(red[2], fabs(ad));
        red[3] = nmax(red[3], fabs(ad * e));
        red[4] = nmax(red[4], fabs(zd));
        red[5] = nmax(red[5], fabs(zd * e));
      }
    }
  }
  __device__ void side() const {  // any workgroup size
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const T xti = xt[i], xi = x[i];
      const T xn = alpha * xti + (T(1) - alpha) * xi;
      x[i] = xn;
      if (dxy) dxy[i] = xn - xi;
      g[i] = xti;
    }
  }
  __device__ void operator()(const double* t) const {
    for (int s = 0; s < 6; ++s) st->norms[s] = t[s];
  }
};

// Primal residual check with Āx recomputed (Section 3.1): r̄_p = Āx̄ − z̄; norms[0..5] as above.
template <typename T>
struct OpRPrim {
  QPG_NO_SIDE
  static constexpr int NS = 6;
  static constexpr unsigned MAXMASK = 0x3Fu;
  const T* x;
  const T* z;
  const double* einv;
  DevState* st;
  __device__ T gather(int c) const { return x[c]; }
  __device__ void epilogue(int i, T s1, T, double* red) const {
    const double ax = (double)s1, zi = (double)z[i], e = einv[i];
    const double rp = ax - zi;
    red[0] = nmax(red[0], fabs(rp));
    red[1] = nmax(red[1], fabs(rp * e));
    red[2] = nmax(red[2], fabs(ax));
    red[3] = nmax(red[3], fabs(ax * e));
    red[4] = nmax(red[4], fabs(zi));
    red[5] = nmax(red[5], fabs(zi * e));
  }
  __device__ void operator()(const double* t) const {
    for (int s = 0; s < 6; ++s) st->norms[s] = t[s];
  }
};

// Dual residual check: r̄_d = P̄x̄ + q̄ + Āᵀȳ with both parts of B in one pass;
// norms[6..11] = ‖r̄_d‖, ‖D⁻¹r̄_d‖, ‖P̄x̄‖, ‖D⁻¹P̄x̄‖, ‖Āᵀȳ‖, ‖D⁻¹Āᵀȳ‖ (c⁻¹ applied on the host),
// norms[12] = x̄ᵀP̄x̄, norms[13] = q̄ᵀx̄ (objective = (½·[12] + [13]) / c).
template <typename T>
struct OpRDual {
  QPG_NO_SIDE
  static constexpr int NS = 8;
  static constexpr unsigned MAXMASK = 0x3Fu;
  const T* x;
  const T* y;
  const T* qb;
  const double* dinv_scale;
  int n;
  DevState* st;
  __device__ T gather(int c) const { return x[c]; }  // y = x + n (one allocation)
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const double px = (double)s1, aty = (double)s2, d = dinv_scale[i];
    const double rd = px + (double)qb[i] + aty;
    red[0] = nmax(red[0], fabs(rd));
    red[1] = nmax(red[1], fabs(rd * d));
    red[2] = nmax(red[2], fabs(px));
    red[3] = nmax(red[3], fabs(px * d));
    red[4] = nmax(red[4], fabs(aty));
    red[5] = nmax(red[5], fabs(aty * d));
    red[6] += (double)x[i] * px;
    red[7] += (double)qb[i] * (double)x[i];
  }
  __device__ void operator()(const double* t) const {
    for (int s = 0; s < 8; ++s) st->norms[6 + s] = t[s];
  }
};

// The dual residual check and, from the same read of B, the product B·g that the next ADMM
// iteration's right-hand side needs (g = plane 0 of the right-hand-side vectors, as written by
// this iteration's update): bg = [P̄x̃; Āᵀ(ρ̄(z̃ − z) + y); Āᵀy] (n each), for k_rows with
// OpRhsRec, or with OpRhsRescaled when ρ̄ has changed at this check.
template <typename T>
struct OpRDualRhs {
  QPG_NO_SIDE
  static constexpr int NV = 2;
  static constexpr int NS = OpRDual<T>::NS;
  static constexpr unsigned MAXMASK = OpRDual<T>::MAXMASK;
  OpRDual<T> rd;
  const T* g;
  T* bg;
  __device__ Pair<T> gather2(int c) const { return Pair<T>{rd.gather(c), g[c]}; }
  __device__ void epilogue2(int i, T s1, T s2, T u1, T u2, double* red) const {
    rd.epilogue(i, s1, s2, red);
    bg[i] = u1;
    bg[rd.n + i] = u2;
    bg[2 * rd.n + i] = s2;
  }
  __device__ void operator()(const double* t) const { rd(t); }
};

// OpRhsRec from a B·g formed with ρ̄_g before a ρ̄ update: g's second part scales with ρ̄
// (ρ_i = c_i·ρ̄ on every row), so Āᵀ(ρ̄(z̃ − z) + y) = Āᵀy + (ρ̄/ρ̄_g)·(Āᵀg_m − Āᵀy).
template <typename T>
struct OpRhsRescaled {
  QPG_NO_SIDE
  static constexpr int NS = OpRhsRec<T>::NS;
  static constexpr unsigned MAXMASK = OpRhsRec<T>::MAXMASK;
  OpRhsRec<T> rc;
  const T* aty;  // Āᵀy (n)
  T ratio;       // ρ̄ / ρ̄_g
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const T a = aty[i];
    rc.epilogue(i, s1, a + ratio * (s2 - a), red);
  }
  __device__ void operator()(const double* t) const { rc(t); }
};

// Infeasibility tests (Section 3.1) on the differences δx̄, δȳ of the last ADMM step, in two
// passes. Bounds with |l_i|, |u_i| ≥ kInf/2 (unscaled) are infinite.
// Pass 1 over the rows of Ā, gathering δx̄: with v = E⁻¹(Āδx̄) = Aδx,
//   norms[16] = max_i of v's violation of the sign pattern: |v_i| where l_i and u_i are finite,
//               max(−v_i, 0) where only u_i = +∞, max(v_i, 0) where only l_i = −∞, 0 where both;
// and δȳ is projected so that the support function has no infinite term (δȳ_i ≤ 0 where
// u_i = +∞, ≥ 0 where l_i = −∞) and written back, then
//   norms[17] = ‖Eδȳ‖∞,  norms[18] = ūᵀ(δȳ)₊ + l̄ᵀ(δȳ)₋ (the infinite terms being zero).
// With δy = Eδȳ/c the unscaled tests read ‖Aᵀδy‖ ≤ ε‖δy‖ and uᵀδy₊ + lᵀδy₋ < −ε‖δy‖; c cancels.
template <typename T>
struct OpInfeasA {
  QPG_NO_SIDE
  static constexpr int NS = 3;
  static constexpr unsigned MAXMASK = 0x3u;
  T* dxy;
  const T* lb;
  const T* ub;
  const double* einv;
  int n;
  DevState* st;
  __device__ T gather(int c) const { return dxy[c]; }
  __device__ void epilogue(int i, T s1, T, double* red) const {
    const double e = einv[i];
    const double lo = (double)lb[i], up = (double)ub[i];
    const bool linf = lo * e <= -0.5 * kInf, uinf = up * e >= 0.5 * kInf;
    const double v = (double)s1 * e;
    const double viol = linf ? (uinf ? 0.0 : nmax(v, 0.0)) : (uinf ? nmax(-v, 0.0) : fabs(v));
    T d = dxy[n + i];
    if (uinf) d = d < T(0) ? d : T(0);
    if (linf) d = d > T(0) ? d : T(0);
    dxy[n + i] = d;
    const double dd = (double)d;
    red[0] = nmax(red[0], viol);
    red[1] = nmax(red[1], fabs(dd / e));
    red[2] += (dd > 0.0 ? up * dd : 0.0) + (dd < 0.0 ? lo * dd : 0.0);
  }
  __device__ void operator()(const double* t) const {
    for (int s = 0; s < 3; ++s) st->norms[16 + s] = t[s];
  }
};

// Pass 2 over B = [P̄ | Āᵀ], gathering [δx̄; projected δȳ]:
//   norms[19] = ‖D⁻¹P̄δx̄‖∞ = c‖Pδx‖∞,  norms[20] = ‖D⁻¹Āᵀδȳ‖∞ = ‖Aᵀ(Eδȳ)‖∞,
//   norms[21] = ‖Dδx̄‖∞ = ‖δx‖∞,        norms[22] = q̄ᵀδx̄ = c·qᵀδx.
template <typename T>
struct OpInfeasB {
  QPG_NO_SIDE
  static constexpr int NS = 4;
  static constexpr unsigned MAXMASK = 0x7u;
  const T* dxy;
  const T* qb;
  const double* dinv_scale;
  DevState* st;
  __device__ T gather(int c) const { return dxy[c]; }
  __device__ void epilogue(int i, T s1, T s2, double* red) const {
    const double d = dinv_scale[i], dx = (double)dxy[i];
    red[0] = nmax(red[0], fabs((double)s1 * d));
    red[1] = nmax(red[1], fabs((double)s2 * d));
    red[2] = nmax(red[2], fabs(dx / d));
    red[3] += (double)qb[i] * dx;
  }
  __device__ void operator()(const double* t) const {
    for (int s = 0; s < 4; ++s) st->norms[19 + s] = t[s];
  }
};

// -------------------------------------------------------------------------------- vector kernels

// Every workgroup combines the same `count` published partials in the same fixed order (thread
// t takes workgroups t, t + 256, …, then a fixed tree), so all of them hold identical totals:
// the scalar step that a separate finalize kernel would take runs redundantly in each.
template <int NS, unsigned MAXMASK>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int count, double (&tot)[NS]) {
  __shared__ double lds[kMaxSlots * 4];
  __shared__ double res[kMaxSlots];
  double v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = 0.0;
  gather_partials<NS, MAXMASK, kBlock>(partials, count, v);
  block_reduce<NS, MAXMASK>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) res[s] = v[s];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NS; ++s) tot[s] = res[s];
}

// PCG update (Algorithm 3), iteration `it` of the solve: κ = pᵀKp from the B pass's partials,
// α = rᵀM⁻¹r / κ; x̃ += αp; r += αKp; y = M⁻¹r (not stored); partials of rᵀy and ‖r‖∞ for
// k_pcg_dir. With M⁻¹ positive, κ ≤ 0 means r = 0 (an exact solve) or a breakdown; α = 0 then,
// and k_pcg_dir ends the solve.
// With zt set, z̃ = Āx̃ follows x̃: z̃ += α·Āp, with Āp = w/ρ̄ from this iteration's Ā pass, so the
// ADMM update after PCG needs no SpMV of its own.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, T* __restrict__ xt,
                                                       T* __restrict__ r,
                                                       const T* __restrict__ p,
                                                       const T* __restrict__ kp,
                                                       const T* __restrict__ dinv,
                                                       DevState* st, const double* __restrict__ kp_partials,
                                                       int kp_count, double* __restrict__ partials,
                                                       const int32_t* __restrict__ gate, int m,
                                                       T* __restrict__ zt, const T* __restrict__ w,
                                                       T rho_inv, int it) {
  if (gate && *gate) return;
  double kap[1];
  reduce_partials<1, 0u>(kp_partials, kp_count, kap);
  const double kappa = kap[0];
  const double alpha = kappa > 0.0 ? st->rzp[it & 1] / kappa : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->kappa = kappa;
    st->alpha = alpha;
    if (!(kappa > 0.0) && !(kappa == 0.0 && st->rnorm == 0.0)) st->breakdown = 1;
  }
  const T a = (T)alpha;
  double red[2] = {0.0, 0.0};
  const int total = zt ? (n > m ? n : m) : n;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    if (i < n) {
      xt[i] += a * p[i];
      const T ri = r[i] + a * kp[i];
      r[i] = ri;
      red[0] += (double)ri * (double)(ri * dinv[i]);
      red[1] = nmax(red[1], fabs((double)ri));
    }
    if (zt && i < m) zt[i] += a * (w[i] * rho_inv);
  }
  publish<2, 2u>(red, partials);
}

// An SpMV operation's row epilogue and side task without the SpMV: the row values s1 (and s2, or
// zeros) are given (the ADMM update when z̃ = Āx̃ is already known; the right-hand side from B's
// product computed by the dual-residual pass). Reductions, if any, are published per workgroup
// like k_combine's.
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_rows(int rows, const T* __restrict__ s1,
                                                 const T* __restrict__ s2, Op op,
                                                 double* __restrict__ partials,
                                                 const int32_t* __restrict__ gate) {
  if (gate && *gate) return;
  constexpr int NS = Op::NS > 0 ? Op::NS : 1;
  double red[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) red[s] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < rows; i += gridDim.x * kBlock)
    op.epilogue(i, s1[i], s2 ? s2[i] : T(0), red);
  op.side();
  if constexpr (Op::NS > 0) publish<Op::NS, Op::MAXMASK>(red, partials);
}

// PCG direction (Algorithm 3), iteration `it`: β = r⁺ᵀy⁺ / rᵀy from k_pcg_update's partials;
// p = −M⁻¹r + βp. Workgroup 0 stores the new rᵀy under the next parity, β, ‖r‖∞, the iteration
// count and the stopping flag, and mirrors the scalars to the host when asked (also when the
// iteration is gated off). Other workgroups read only the previous parity's rᵀy, so no value is
// read while it is written. `done` is written here only when the solve has ended (converged,
// capped or broken down); a workgroup that sees it already set skips its share of p, which is
// not used once the solve has ended.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_dir(int n, T* __restrict__ p,
                                                    const T* __restrict__ r,
                                                    const T* __restrict__ dinv,
                                                    DevState* st, const double* __restrict__ partials,
                                                    int count, const int32_t* __restrict__ gate, int it,
                                                    DevState* mirror) {
  if (gate && *gate) {
    if (mirror && blockIdx.x == 0 && threadIdx.x == 0) *mirror = *st;
    return;
  }
  double t[2];
  reduce_partials<2, 2u>(partials, count, t);
  const double rz_new = t[0], beta = rz_new / st->rzp[it & 1];
  const T b = (T)beta;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    p[i] = -(r[i] * dinv[i]) + b * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rzp[(it + 1) & 1] = rz_new;
    st->beta = beta;
    st->rnorm = t[1];
    st->iter = it + 1;
    if (rz_new != rz_new) st->breakdown = 1;
    st->done = (t[1] <= st->thresh || it + 1 >= st->maxit || st->breakdown || !(st->kappa > 0.0)) ? 1 : 0;
    if (mirror) *mirror = *st;
  }
}

// Jacobi preconditioner (Section 6.3.1): M⁻¹_ii = 1 / (diag(P̄)_i + σ + ρ̄‖Ā_i‖²); with
// R = diag(ρ_i), (ĀᵀRĀ)_ii = ρ̄(‖Ā_i‖² + (10³ − 1)·Σ_{equality rows k} Ā_ki²).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi(int n, T* __restrict__ dinv,
                                                   const double* __restrict__ diagP,
                                                   const double* __restrict__ colsq, double sigma,
                                                   double rho, const double* __restrict__ colsq_eq) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double c = colsq_eq ? colsq[i] + (kRhoEq - 1.0) * colsq_eq[i] : colsq[i];
    dinv[i] = (T)(1.0 / (diagP[i] + sigma + rho * c));
  }
}

// The unscaled iterates of a solve (Section 3.3): x = D x̄, y = E ȳ / c, z = E⁻¹ z̄, in double,
// into out = [x; y; z]; de holds D (n) then E (m).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_unscale(int n, int m, const T* __restrict__ x, const T* __restrict__ y,
                                                    const T* __restrict__ z, const double* __restrict__ de,
                                                    double c, double* __restrict__ out) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n + m; i += gridDim.x * kBlock) {
    if (i < n) {
      out[i] = (double)x[i] * de[i];
    } else {
      const int j = i - n;
      const double e = de[i];
      out[i] = e * (double)y[j] / c;
      out[(size_t)n + m + j] = (double)z[j] / e;
    }
  }
}

// Both planes of the right-hand-side vectors read by OpRhsAt / OpRhsR0 (plane 0 also by OpRhsRec): x̃ and 0
// for the n P̄ columns, ρ̄(z̃ − z) + y and ρ̄z − y for the m Āᵀ columns. Run before every OpRhsR0
// pass: the update passes keep only plane 0 current.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pairs(int n, int m, T* __restrict__ g,
                                                  const T* __restrict__ xt, const T* __restrict__ zt,
                                                  const T* __restrict__ z, const T* __restrict__ y, T rho,
                                                  const uint8_t* __restrict__ eq) {
  const size_t ps = (size_t)n + m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n + m; i += gridDim.x * kBlock) {
    if (i < n) {
      g[i] = xt[i];
      g[ps + i] = T(0);
    } else {
      const int j = i - n;
      const T r = row_rho(eq, j, rho);
      g[i] = r * (zt[j] - z[j]) + y[j];
      g[ps + i] = r * z[j] - y[j];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int n, T* __restrict__ v, T val) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) v[i] = val;
}

template <typename D, typename S>
__global__ __launch_bounds__(kBlock) void k_cast(int n, D* __restrict__ d, const S* __restrict__ s) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[i] = (D)s[i];
}

// ‖b‖∞ for a caller-supplied right-hand side.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_absmax(int n, const T* __restrict__ b, double* partials) {
  double red[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    red[0] = nmax(red[0], fabs((double)b[i]));
  publish<1, 1u>(red, partials);
}

struct FinThresh {
  DevState* st;
  double eps;
  int rel;
  __device__ void operator()(const double* t) const {
    st->bnorm = t[0];
    st->thresh = rel ? eps * t[0] : eps;
  }
};

}  // namespace qpg
