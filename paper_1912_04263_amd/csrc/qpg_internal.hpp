// Internal declarations shared by the host preparation code and the device solver.
#pragma once

#include <sys/mman.h>

#include <cstdint>
#include <cstdlib>
#include <functional>
#include <new>
#include <memory>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/qpg.h"

namespace qpg {

// Allocator whose resize() leaves new elements default-initialised (for plain numbers: not
// written), so that nnz-sized host arrays are first touched by the threads that fill them rather
// than zeroed by one thread beforehand.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
  // Large arrays (the matrix in its several layouts) on transparent huge pages where the kernel
  // offers them: 2 MB-aligned, advised, so that their first touch takes 512× fewer page faults.
  static constexpr size_t kHuge = size_t(2) << 20;
  T* allocate(size_t count) {
    const size_t bytes = count * sizeof(T);
    if (bytes < 4 * kHuge) return std::allocator<T>::allocate(count);
    void* p = std::aligned_alloc(kHuge, (bytes + kHuge - 1) / kHuge * kHuge);
    if (!p) throw std::bad_alloc();
    (void)madvise(p, (bytes + kHuge - 1) / kHuge * kHuge, MADV_HUGEPAGE);
    return static_cast<T*>(p);
  }
  void deallocate(T* p, size_t count) {
    if (count * sizeof(T) < 4 * kHuge)
      std::allocator<T>::deallocate(p, count);
    else
      std::free(p);
  }
};
template <class T>
using hvec = std::vector<T, NoInit<T>>;

constexpr double kInf = 1e20;       // |bound| ≥ kInf is infinite
constexpr int kBlock = 256;         // threads per workgroup (4 wavefronts of 64)
constexpr int kStreamCap = 2048;    // nnz staged through LDS by one workgroup (rows fully inside)
constexpr int kLongCap = 65536;     // a longer row is split into chunks of at most kChunk nnz
constexpr int kChunk = 32768;
constexpr int kTileNnz = 65536;    // SpMV entries per workgroup with an LDS gather window
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
// Each row is cut into segments of at most kSegMax entries. One lane sums one segment; 64
// segments form a chunk, stored in SELL order (entry s of lane j at base + 64·s + j, so that
// every load instruction of a wavefront reads 64 consecutive entries), and a workgroup streams
// the chunks of one tile with no barrier. The segments of a tile are sorted by length so that
// the lanes of a chunk end together; the shorter ones are padded with zero values (and a column
// the lane reads anyway).
//
// A tile either gathers from a window of the vector staged in LDS (all its entries fall inside
// the window; their column indices are stored as 16-bit offsets into it), or from memory (32-bit
// column indices). A random gather from memory costs a whole cache line for one value; an LDS
// window that many entries fall into turns that traffic into LDS reads.
//
// Row blocks are single-range (all columns) or, where rows are wide, multi-range: the columns are
// cut at dense windows and each (block, range) gets its own windowed tile. Segment sums go to
// slots numbered tile by tile (the segments of one tile, in row order, get consecutive slots), so
// that every cache line of the slot array is written by one workgroup; a row's segments are
// listed in column order by slotidx, and k_combine adds each row's slots in that order and runs
// the operation's epilogue.

constexpr int kSegMax = 256;   // entries of one segment at most
constexpr int kSpmvBlock = 1024; // threads per SpMV workgroup (one chunk at a time per wavefront)
constexpr int kWinCols = 16384; // LDS gather window capacity in columns (at most; ≤ 65536)
constexpr int kMinSeg = 16;    // entries per row and range that make a multi-range layout
constexpr int kGridMinSeg = 2; // entries per row and window that make a grid layout (see tiles.cpp)
constexpr int kGridMaxRows = 16384;  // rows of a grid block at most
constexpr int kGridRound = 512;      // grid tiles that run at once (two 1024-thread workgroups per CU)
constexpr int kRunMinRows = 64;      // single-segment rows with consecutive slots that make a K = 1 combine item

struct Chunk {
  int32_t base;   // first value (SELL order)
  int32_t cbase;  // first column index, in the 16-bit array (windowed tile) or the 32-bit one
  int32_t steps;  // length of the longest segment
  int32_t seg0;   // index of the chunk's first segment slot
};

// chunks [chunk0, chunk0 + nchunk); wlen > 0: gathers read the LDS copy of [wlo, wlo + wlen).
struct Tile {
  int32_t chunk0, nchunk, wlo, wlen;
};

// k_combine work: rows [r0, r1), 2^lg lanes per row (rows with many slots share them out); or,
// with lg = −K < 0, rows of a grid block: one lane per row, whose K slots are tbase[t0 + j] + row
// (j = 0..K−1, column order), t0 = the block's first tile; or (K = 1) a run of single-segment
// rows whose slots are tbase[t0] + row, t0 past the tiles' entries.
struct CombItem {
  int32_t r0, r1, lg, t0;
};

struct TilePlan {
  std::vector<Tile> tiles;
  std::vector<CombItem> comb;
  std::vector<Chunk> chunks;
  std::vector<int32_t> segslot;  // per segment (64 per chunk, −1 for an empty lane): output slot
  std::vector<int32_t> rowslot;  // nrows + 1: row r has the segments [rowslot[r], rowslot[r + 1])
  std::vector<int32_t> slotidx;  // per segment in row order (column order within a row): its slot
  // per tile of a grid block: its first slot minus the block's first row; then one entry per run
  // of single-segment rows with consecutive slots (slot − row)
  std::vector<int32_t> tbase;
  // per lane (64 per chunk): the first CSR index of its segment and the segment's length (−1 for
  // an empty lane). Lane j of a chunk, at step q < steps, holds the entry lstart + q (CSR index
  // −1 and the lane's last column past the segment's end; the window's first column, or column 0
  // without a window, for a lane with no entries).
  hvec<int32_t> lstart, llen;
  hvec<int32_t> src;             // per SELL value position: CSR index, −1 for padding
  hvec<uint16_t> col16;          // column offsets of windowed tiles (SELL order)
  hvec<int32_t> col32;           // columns of the other tiles (SELL order)
  int64_t n_src = 0, n_c16 = 0, n_c32 = 0;  // their sizes (also when only the lanes are written)
  int64_t nslot = 0;
  int32_t max_wlen = 0;          // largest staged window (columns)
};

struct TileParams {
  int32_t wcap;       // window capacity in columns (a power of two, ≤ 65536)
  int32_t tile_nnz;   // target entries per windowed tile
  int32_t plain_nnz;  // target entries per tile without a window
  int32_t max_rows;   // rows per block at most
  int32_t min_seg = kMinSeg;  // entries per row and range (on average) for a multi-range layout
  bool grid = true;           // the grid layout may be used (see tiles.cpp)
  // write the entries in SELL order (src, col16, col32) on the host; without, only the lanes
  // (lstart, llen), from which the device writes them
  bool host_entries = true;
};

// nrows × ncols CSR matrix (row pointers rowptr[0..nrows], column indices col[rowptr[0] ..
// rowptr[nrows]), sorted within each row).
TilePlan make_tiles(const std::vector<int32_t>& rowptr, const int32_t* col, int32_t nrows, int32_t ncols,
                    const TileParams& tp);

// ---- host parallelism for setup
// f(c, lo, hi) for the chunks [c·chunk, min(n, (c+1)·chunk)) of [0, n), on up to 16 threads.
// The chunking does not depend on the thread count, so results that combine per-chunk partials
// in chunk order are the same on every machine.
void parallel_chunks(int64_t n, int64_t chunk, const std::function<void(int64_t, int64_t, int64_t)>& f);

// The problem after validation and format conversion on the host, values unscaled. The host
// converts the sparsity patterns; the values are placed on the device (qpg_solver::place_raw).
struct HostProblem {
  int32_t n = 0, m = 0;
  // A in CSR (m rows, n columns): pattern, and for each entry its index in A's CSC arrays
  std::vector<int32_t> a_ptr;
  hvec<int32_t> a_col;
  hvec<int32_t> a_src;
  // B = [P | Aᵀ] in CSR (n rows, n + m columns): row i holds row i of the full P (columns
  // 0..n−1) followed by row i of Aᵀ (columns n + j); b_split[i] is where the Aᵀ part starts.
  std::vector<int32_t> b_ptr, b_split;
  hvec<int32_t> b_col;
  // values: the full P in CSR (row i is the first part of B's row i); A's CSC values and column
  // pointers, the caller's arrays, read during setup (column i of A is the second part of B's
  // row i, in the same order)
  std::vector<int32_t> p_ptr;
  hvec<double> p_val;
  const double* a_csc_val = nullptr;
  const int32_t* a_colptr = nullptr;
  std::vector<double> qb, lb, ub;      // q, and l, u clamped to ±kInf
  std::vector<uint8_t> eqrow;          // l_i = u_i (eq. rho_vec); filled when settings.rho_vector
  double q_norm_unscaled = 0.0;        // ‖q‖∞ of the original data
};

// Validate the inputs (returns QPG_OK or an error code with a message) and build HostProblem.
// With with_a false, A's CSR pattern (a_ptr, a_col, a_src) is left to prepare_a, so that the
// caller can start on B's work list first.
int prepare(const qpg_csc* P_triu, const double* q, const qpg_csc* A, const double* l,
            const double* u, const qpg_settings* s, HostProblem* out, std::string* msg,
            bool with_a = true);
// A in CSR (after a successful prepare with with_a false).
void prepare_a(const qpg_csc* A, HostProblem* out);

int validate_settings(const qpg_settings* s, std::string* msg);

}  // namespace qpg
