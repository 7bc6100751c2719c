// Internal declarations shared by the host preparation code and the device solver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qpg.h"

namespace qpg {

constexpr double kInf = 1e20;       // |bound| ≥ kInf is infinite
constexpr int kBlock = 256;         // threads per workgroup (4 wavefronts of 64)
constexpr int kStreamCap = 2048;    // nnz staged through LDS by one workgroup (rows fully inside)
constexpr int kLongCap = 65536;     // a longer row is split into chunks of at most kChunk nnz
constexpr int kChunk = 32768;

// One workgroup's share of a CSR SpMV.
//   nchunk == 0: rows [r0, r1) entirely, entries [k0, k1) = [rowptr[r0], rowptr[r1]).
//                k1 − k0 ≤ kStreamCap unless r1 == r0 + 1 (a single long row).
//   nchunk  > 0: entries [k0, k1) of row r0 only; chunk `chunk` of `nchunk`; the row's chunk
//                partial sums live at partial slot `slot + chunk`, its ticket at `ticket`.
struct Item {
  int32_t r0, r1, k0, k1;
  int32_t nchunk, chunk, slot, ticket;
};

struct Plan {
  std::vector<Item> items;
  int32_t n_split_rows = 0;    // rows handled by chunks (tickets needed)
  int32_t n_chunk_slots = 0;   // chunk partial slots needed
};

// Build the work list of a CSR matrix with nrows rows (Section 5.1.4: SpMV row sums are a
// segmented reduction over the RowPointer segments; this balances it over workgroups).
Plan make_plan(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t cap = kStreamCap);

// The problem after validation, format conversion and Ruiz equilibration, all on the host.
struct HostProblem {
  int32_t n = 0, m = 0;
  // Ā in CSR (m rows, n columns)
  std::vector<int32_t> a_ptr, a_col;
  std::vector<double> a_val;
  // B = [P̄ | Āᵀ] in CSR (n rows, n + m columns): row i holds row i of the full P̄ (columns
  // 0..n−1) followed by row i of Āᵀ (columns n + j); b_split[i] is where the Āᵀ part starts.
  std::vector<int32_t> b_ptr, b_split, b_col;
  std::vector<double> b_val;
  std::vector<double> qb, lb, ub;      // q̄ = cDq, l̄ = El, ū = Eu (bounds clamped to ±kInf first)
  std::vector<double> D, E;            // Ruiz factors
  double c = 1.0;
  int32_t scaling_passes = 0;
  std::vector<double> diagP;           // diag(P̄)
  std::vector<double> colsq;           // ‖Ā_j‖₂² = (ĀᵀĀ)_jj  (Section 6.3.1)
  double q_norm_unscaled = 0.0;        // ‖q‖∞ of the original data
};

// Validate the inputs (returns QPG_OK or an error code with a message) and build HostProblem.
int prepare(const qpg_csc* P_triu, const double* q, const qpg_csc* A, const double* l,
            const double* u, const qpg_settings* s, HostProblem* out, std::string* msg);

int validate_settings(const qpg_settings* s, std::string* msg);

}  // namespace qpg
