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
constexpr int kTileNnz = 32768;    // SpMV entries per workgroup with an LDS gather window
constexpr int kPlainNnz = 8192;    // SpMV entries per workgroup without one
constexpr int kTileMaxRows = 4096; // rows per SpMV row block at most

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

// Build the row work list of a CSR matrix with nrows rows (used by the learned preconditioner's
// SpMM; Section 5.1.4: row sums are a segmented reduction over the RowPointer segments).
Plan make_plan(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t cap = kStreamCap);

// ---- SpMV work list (k_spmv / k_combine)
//
// The rows are cut into row blocks. A block is either single-range (each workgroup's row sums
// are complete and go straight to the operation's epilogue) or multi-range: its column space is
// cut into ranges, one workgroup per (block, range) computes partial row sums over the range,
// and k_combine adds them in range order before the epilogue. Each workgroup may stage one
// window of the gathered vector in LDS; gathers of columns inside it read LDS, the others read
// memory. A random gather from memory costs a whole cache line for one value, so a window that
// many of a workgroup's entries fall into turns most of the gather traffic into LDS reads.
// The kernel streams entries in the plan's order: CSR order, except that a multi-range block's
// entries are grouped range by range, so that each workgroup's entries are contiguous.

constexpr int kSubCap = 1920;  // entries loaded through LDS at a time by one workgroup
constexpr int kWinCols = 8192; // LDS gather window capacity in columns (at most)

// One workgroup: rows r0 .. r0 + nrow − 1, restricted to one column range of their block. Row i
// (local) has entries [trp[tr + i], trp[tr + i + 1]) in the plan's order; with a column split,
// those from tsp[tr + i] on belong to the second part. The rows are processed in sub-runs
// subs[sub0 .. sub0 + nsub). Columns in [wlo, wlo + wlen) are gathered from the LDS copy
// (wlen = 0: no window). part < 0: complete row sums, epilogue here; otherwise partial sums,
// stored at part + i.
struct Tile {
  int32_t r0, nrow, sub0, nsub, tr, wlo, wlen, part;
};

// Local rows [i0, i1) with entries [k0, k1): either whole rows with at most kSubCap entries in
// total, or one longer row.
struct Sub {
  int32_t i0, i1, k0, k1;
};

// Rows [r0, r1) (at most kBlock) of a multi-range block: the partial sum of range j for row r
// is at part + j·stride + (r − r0).
struct CombItem {
  int32_t r0, r1, nrange, part, stride, pad0, pad1, pad2;
};

struct TilePlan {
  std::vector<Tile> tiles;
  std::vector<Sub> subs;
  std::vector<int32_t> trp;   // row starts per workgroup (nrow + 1 each)
  std::vector<int32_t> tsp;   // first second-part entry per row (split matrices; same indexing)
  std::vector<int32_t> perm;  // plan order → CSR index (empty: CSR order throughout)
  std::vector<CombItem> comb;
  int64_t n_part = 0;    // partial-sum slots per component
  int32_t max_wlen = 0;  // largest staged window (gathered elements)
};

struct TileParams {
  int32_t wcap;       // window capacity in columns (a power of two)
  int32_t tile_nnz;   // target entries per workgroup when it stages a window
  int32_t plain_nnz;  // target entries per workgroup without a window
  int32_t max_rows;   // rows per block at most
};

// nrows × ncols CSR matrix with sorted column indices in each row; columns below nsplit form the
// first part of a row (nsplit = ncols: no split).
TilePlan make_tiles(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col, int32_t nrows,
                    int32_t ncols, int32_t nsplit, const TileParams& tp);

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
