// SpMV work-list construction (host): row blocks, column ranges, LDS gather windows, segments,
// and the SELL order of the entries that the SpMV kernel streams.
//
// Rows are grouped into runs of similar length. For each run, a histogram of its column indices
// over fixed windows of wcap columns decides the layout:
//   * multi-range, when at least two windows each hold ≥ min_seg entries per row on average and
//     together at least half of the run's entries: the columns are cut at those windows, and each
//     (row block, range) gets a tile that stages its window in LDS. Each range costs every row one
//     slot at least, hence the min_seg floor (TileParams);
//   * single-range otherwise: one windowed tile per row block, the window being either the block's
//     whole column span when it fits, or the run's densest wcap-wide window when that holds at
//     least half of the block's entries.
// A window is staged only if it holds at least one entry per 16 of its columns, so that staging
// never reads more than the gathers it replaces. Entries outside every staged window go to tiles
// without a window, of about plain_nnz entries each. Runs whose rows are too sparse for any
// window but spread over several 2^17-column ranges (≥ min_seg entries per row in each) are cut
// at those ranges too, and their tiles are issued range by range (L2 locality of the gathers).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "qpg_internal.hpp"

namespace qpg {

namespace {

constexpr int64_t kMinTiles = 512;  // workgroups a launch should have (two per compute unit)
constexpr int64_t kMinTileNnz = 1024;
constexpr int kLanes = 64;
// Column ranges of 2^17 entries (1 MB of FP64) for rows too sparse for LDS windows: their tiles
// are issued range by range, so that the workgroups in flight gather from one range that the L2
// caches hold, instead of from all of the vector.
constexpr int kL2Shift = 17;

int32_t log2_exact(int32_t v) {
  int32_t l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

struct Seg {
  int32_t start, len, slot;
};

// Column counts over eighth-windows (f), counted entry by entry, and from them over windows (w)
// and 2^kL2Shift ranges (l2), with the lists of the bins that are non-zero (so that clearing costs
// what was touched).
struct Hist {
  std::vector<int64_t> w, f, l2, tw, tf, t2;
  Hist(int64_t nw, int64_t nf, int64_t n2) : w(nw, 0), f(nf, 0), l2(n2, 0) {}
  static void bump(std::vector<int64_t>& cnt, std::vector<int64_t>& touched, int64_t b, int64_t by) {
    if (cnt[b] == 0) touched.push_back(b);
    cnt[b] += by;
  }
  void add(int32_t c, int32_t fsh) { bump(f, tf, c >> fsh, 1); }
  // adds o's fine counts and clears o
  void merge(Hist& o) {
    for (int64_t b : o.tf) bump(f, tf, b, o.f[b]), o.f[b] = 0;
    o.tf.clear();
  }
  // w and l2 from f: a window is 2^(sh − fsh) fine bins, an L2 range 2^(kL2Shift − fsh)
  // (fsh ≤ sh ≤ 16 < kL2Shift)
  void derive(int32_t sh, int32_t fsh) {
    for (int64_t b : tf) {
      bump(w, tw, b >> (sh - fsh), f[b]);
      bump(l2, t2, b >> (kL2Shift - fsh), f[b]);
    }
  }
};
constexpr int64_t kParHist = 1 << 20;  // runs with more entries are counted in parallel
constexpr int kHistParts = 16;

}  // namespace

TilePlan make_tiles(const std::vector<int32_t>& rowptr, const int32_t* col, int32_t nrows, int32_t ncols,
                    const TileParams& tp) {
  TilePlan plan;
  plan.rowslot.assign((size_t)std::max(nrows, 0) + 1, 0);
  if (nrows <= 0) return plan;
  // smaller tiles on small matrices, so that the launch still has ~kMinTiles of them
  const int64_t nnz_all = (int64_t)rowptr[nrows] - rowptr[0];
  const int32_t tile_nnz = (int32_t)std::max<int64_t>(kMinTileNnz, std::min<int64_t>(tp.tile_nnz, nnz_all / kMinTiles));
  // window capacity: at most half a windowed tile's entries, so that staging a full window costs
  // at most one column per two entries streamed (a power of two, at least 1024 columns)
  int32_t wcap = tp.wcap;
  while (wcap > 1024 && wcap > tile_nnz / 2) wcap >>= 1;
  const int32_t plain_nnz = (int32_t)std::max<int64_t>(kMinTileNnz, std::min<int64_t>(tp.plain_nnz, nnz_all / kMinTiles));
  // segment length: short segments on small matrices, so that a lane's serial chain stays short
  int32_t seg_max = kSegMax;
  while (seg_max > 16 && (int64_t)seg_max * kLanes * kMinTiles > nnz_all) seg_max >>= 1;
  // chunks per tile: up to one per wavefront of the workgroup, fewer when the matrix has too few
  // chunks for kMinTiles tiles of that size
  const double seg_est = std::min<double>(seg_max, std::max(1.0, (double)nnz_all / nrows));
  const int32_t tile_chunks = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>(kSpmvBlock / kLanes, (int64_t)(nnz_all / (kLanes * seg_est)) / kMinTiles));
  const int32_t sh = log2_exact(wcap);
  const int32_t fsh = std::max(0, sh - 3);  // eight fine bins per window
  const int64_t nwin = ((int64_t)ncols + wcap - 1) >> sh;
  const int64_t nfine = ((int64_t)ncols + (1 << fsh) - 1) >> fsh;
  Hist hist(std::max<int64_t>(nwin, 1), std::max<int64_t>(nfine, 1),
            std::max<int64_t>(((int64_t)ncols >> kL2Shift) + 1, 1));
  std::vector<int64_t>&cnt = hist.w, &fine = hist.f, &cnt2 = hist.l2;
  std::vector<int64_t>&touched_w = hist.tw, &touched_f = hist.tf, &touched_2 = hist.t2;
  std::vector<Hist> part;  // per-part histograms of long runs

  // first entry of row r at or after column c
  auto seek = [&](int32_t r, int64_t c) {
    const int32_t* first = col + rowptr[r];
    const int32_t* last = col + rowptr[r + 1];
    return (int32_t)(std::lower_bound(first, last, (int32_t)std::min<int64_t>(c, INT32_MAX)) - col);
  };
  // the same, by an exponential search outward from entry position h of the row (cheap when the
  // answer is near h, as for a row's bounds taken in column order)
  auto seek_near = [&](int32_t r, int64_t c, int32_t h) {
    const int32_t cc = (int32_t)std::min<int64_t>(c, INT32_MAX);
    int32_t lo = rowptr[r], hi = rowptr[r + 1];  // the answer lies in [lo, hi]
    h = std::min(std::max(h, lo), hi);
    int32_t step = 1;
    if (h < hi && col[h] < cc) {  // in (h, hi]: step right while col[p + step] < cc
      int32_t p = h;
      while (p + step < hi && col[p + step] < cc) p += step, step <<= 1;
      lo = p + 1;
      hi = (int32_t)std::min<int64_t>(hi, (int64_t)p + step);
    } else {  // in [lo, h]: step left while col[p − step] ≥ cc
      int32_t p = h;
      while (p - step >= lo && col[p - step] >= cc) p -= step, step <<= 1;
      lo = std::max(lo, p - step + 1);
      hi = p;
    }
    return (int32_t)(std::lower_bound(col + lo, col + hi, cc) - col);
  };

  // Tiles are listed first, in their final order, each with its segments in row order (grid
  // tiles with the first row of their block, b0 ≥ 0, and kept even when empty); they are built
  // afterwards, tile by tile in parallel: segments sorted by length, chunks of 64 lanes, entries.
  struct Pending {
    std::vector<Seg> segs;
    int32_t wlo, wlen, b0;
  };
  std::vector<Pending> pend;
  auto add_tile = [&](std::vector<Seg>&& segs, int32_t wlo, int32_t wlen, int32_t b0 = -1) {
    if (segs.empty() && b0 < 0) return;
    pend.push_back({std::move(segs), wlo, wlen, b0});
    if (wlen > 0) plan.max_wlen = std::max(plan.max_wlen, wlen);
  };

  std::vector<Seg> plain;  // segments waiting for a tile without a window
  int64_t plain_entries = 0;
  // all of them (at the end), or whole chunks' worth once there are enough entries
  auto flush_plain = [&](bool all) {
    if (!all && (plain_entries < plain_nnz || plain.size() < (size_t)(tile_chunks * kLanes))) return;
    const size_t take = all ? plain.size() : plain.size() / kLanes * kLanes;
    std::vector<Seg> t(plain.begin(), plain.begin() + take);
    plain.erase(plain.begin(), plain.begin() + take);
    add_tile(std::move(t), 0, 0);
    plain_entries = 0;
    for (const Seg& g : plain) plain_entries += g.len;
  };
  // segments of [a, e) with consecutive slots from *next
  auto cut_segs = [&](std::vector<Seg>& out, int32_t a, int32_t e, int32_t* next) {
    for (int32_t s = a; s < e; s += seg_max) out.push_back({s, std::min(seg_max, e - s), (*next)++});
  };
  auto pieces = [&](int32_t a, int32_t e) { return (e - a + seg_max - 1) / seg_max; };

  // Row block [b0, b1) with ranges cut at cut[0..K] and windows (wlen 0: none): for each row and
  // range, the entries left of the window, inside it, and right of it, in column order.
  struct Block {
    int32_t b0, b1;
    std::vector<int32_t> wlo, wlen;
    bool grid = false;  // asked for: one segment (possibly empty) per row and range
    bool grid_ok = false;  // granted: every row's entries lie in the windows, ≤ seg_max per range
  };
  // bounds of every row of a block (3K + 1 entry positions per row, searched in column order) and the
  // number of segments each row is cut into; reads the matrix only
  auto bounds = [&](Block& bl, int32_t K, int32_t* bnd, int32_t* np, const std::vector<int64_t>& cut) {
    const int32_t stride = 3 * K + 1;
    bool grid_ok = bl.grid;
    for (int32_t i = 0; i < bl.b1 - bl.b0; ++i) {
      const int32_t r = bl.b0 + i;
      int32_t* B = bnd + (size_t)i * stride;
      int32_t c = 0;
      int32_t a = rowptr[r];  // range j starts where range j − 1 ends
      for (int32_t j = 0; j < K; ++j) {
        int32_t ia = a, ie = a;  // window bounds, clamped to the range below
        if (bl.wlen[j] > 0) {
          ia = seek_near(r, bl.wlo[j], a);
          ie = seek_near(r, (int64_t)bl.wlo[j] + bl.wlen[j], ia);
        }
        const int32_t e = j == K - 1 ? rowptr[r + 1] : seek_near(r, cut[j + 1], ie);
        if (bl.wlen[j] > 0) {
          ia = std::max(a, ia);
          ie = std::min(e, ie);
        } else {
          ia = ie = e;
        }
        B[3 * j] = a;
        B[3 * j + 1] = ia;
        B[3 * j + 2] = ie;
        B[3 * j + 3] = e;
        c += pieces(a, ia) + pieces(ia, ie) + pieces(ie, e);
        if (grid_ok && (a != ia || ie != e || bl.wlen[j] == 0 || ie - ia > seg_max)) grid_ok = false;
        a = e;
      }
      np[i] = c;
    }
    bl.grid_ok = grid_ok;
    if (grid_ok)
      for (int32_t i = 0; i < bl.b1 - bl.b0; ++i) np[i] = K;
  };
  // segments of a block from its bounds, in row order, numbered from rowslot: per range, those
  // inside its window and those outside (one list, or one per range for by-range tiles)
  struct BlockSegs {
    std::vector<std::vector<Seg>> win, out;
  };
  auto cut_block = [&](const Block& bl, int32_t K, const int32_t* bnd, bool per_range, BlockSegs& o) {
    const int32_t stride = 3 * K + 1, Rb = bl.b1 - bl.b0;
    o.win.assign(K, {});
    o.out.assign(per_range ? K : 1, {});
    if (bl.grid_ok) {
      for (int32_t j = 0; j < K; ++j) o.win[j].reserve((size_t)Rb);
      for (int32_t i = 0; i < Rb; ++i) {
        const int32_t* B = bnd + (size_t)i * stride;
        int32_t next = plan.rowslot[bl.b0 + i];
        for (int32_t j = 0; j < K; ++j) o.win[j].push_back({B[3 * j + 1], B[3 * j + 2] - B[3 * j + 1], next++});
      }
      return;
    }
    for (int32_t i = 0; i < Rb; ++i) {
      const int32_t* B = bnd + (size_t)i * stride;
      int32_t next = plan.rowslot[bl.b0 + i];
      for (int32_t j = 0; j < K; ++j) {
        std::vector<Seg>& out = o.out[per_range ? j : 0];
        cut_segs(out, B[3 * j], B[3 * j + 1], &next);
        cut_segs(o.win[j], B[3 * j + 1], B[3 * j + 2], &next);
        cut_segs(out, B[3 * j + 2], B[3 * j + 3], &next);
      }
    }
  };
  // the tiles of a block, in block order: its windowed tiles, then (single list) a tile of the
  // segments outside windows once enough of them have gathered
  struct GridBlock {
    int32_t b0, b1, K, t0;
  };
  std::vector<GridBlock> grids;
  auto emit = [&](const Block& bl, int32_t K, BlockSegs& o, std::vector<std::vector<Seg>>* by_range) {
    if (bl.grid_ok) {
      const int32_t t0 = (int32_t)pend.size();
      for (int32_t j = 0; j < K; ++j) add_tile(std::move(o.win[j]), bl.wlo[j], bl.wlen[j], bl.b0);
      grids.push_back({bl.b0, bl.b1, K, t0});
      return;
    }
    if (by_range) {
      for (int32_t j = 0; j < K; ++j) (*by_range)[j].insert((*by_range)[j].end(), o.out[j].begin(), o.out[j].end());
    } else {
      for (const Seg& g : o.out[0]) plain_entries += g.len;
      plain.insert(plain.end(), o.out[0].begin(), o.out[0].end());
    }
    for (int32_t j = 0; j < K; ++j) add_tile(std::move(o.win[j]), bl.wlo[j], bl.wlen[j]);
    flush_plain(false);
  };
  // The blocks of one run, in batches of bounded size: the window decision (`decide`), the bounds
  // and the segments of the blocks of a batch are computed in parallel (the slot numbers of a
  // block's rows from the counts, in order, in between), then the blocks' tiles are listed in
  // order, so the work list does not depend on the number of threads.
  std::vector<int32_t> bbuf, npbuf;
  std::vector<BlockSegs> bsegs;
  auto run_blocks = [&](std::vector<Block>& blocks, const std::vector<int64_t>& cut,
                        std::vector<std::vector<Seg>>* by_range, const auto& decide) {
    const int32_t K = (int32_t)cut.size() - 1, stride = 3 * K + 1;
    constexpr int64_t kBatchInts = int64_t(1) << 24;
    size_t j0 = 0;
    while (j0 < blocks.size()) {
      std::vector<int64_t> off(1, 0), roff(1, 0);
      size_t j1 = j0;
      while (j1 < blocks.size()) {
        const int64_t rb = blocks[j1].b1 - blocks[j1].b0;
        if (j1 > j0 && off.back() + rb * stride > kBatchInts) break;
        off.push_back(off.back() + rb * stride);
        roff.push_back(roff.back() + rb);
        ++j1;
      }
      bbuf.resize((size_t)off.back());
      npbuf.resize((size_t)roff.back());
      parallel_chunks((int64_t)(j1 - j0), 1, [&](int64_t q, int64_t, int64_t) {
        Block& bl = blocks[j0 + q];
        decide(bl);
        bounds(bl, K, bbuf.data() + off[q], npbuf.data() + roff[q], cut);
      });
      for (size_t q = 0; q < j1 - j0; ++q) {
        const Block& bl = blocks[j0 + q];
        const int32_t* np = npbuf.data() + roff[q];
        for (int32_t i = 0; i < bl.b1 - bl.b0; ++i) plan.rowslot[bl.b0 + i + 1] = plan.rowslot[bl.b0 + i] + np[i];
      }
      bsegs.resize(j1 - j0);
      parallel_chunks((int64_t)(j1 - j0), 1, [&](int64_t q, int64_t, int64_t) {
        cut_block(blocks[j0 + q], K, bbuf.data() + off[q], by_range != nullptr, bsegs[q]);
      });
      for (size_t q = 0; q < j1 - j0; ++q) emit(blocks[j0 + q], K, bsegs[q], by_range);
      j0 = j1;
    }
  };
  const auto keep = [](Block&) {};

  // rows per block: about `target` entries, and at least one full chunk of segments
  auto block_rows = [&](int64_t target, double seg_entries) {
    const int64_t spr = std::max<int64_t>(1, (int64_t)std::ceil(seg_entries / seg_max));  // segments per row
    int64_t R = std::max<int64_t>((int64_t)(target / std::max(seg_entries, 1.0)), tile_chunks * kLanes / spr);
    R = (R * spr + kLanes - 1) / kLanes * kLanes / spr;  // whole chunks
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(tp.max_rows, R));
  };
  auto len = [&](int32_t r) { return rowptr[r + 1] - rowptr[r]; };
  int32_t g0 = 0;
  while (g0 < nrows) {
    // ---- run of rows of similar length (within a factor 4 of its first row)
    const int32_t l0 = len(g0);
    const int32_t lo = l0 / 4, hi = std::max(4, 4 * l0);
    int32_t g1 = g0 + 1;
    while (g1 < nrows && len(g1) >= lo && len(g1) <= hi) ++g1;
    const int64_t rows_g = g1 - g0;
    const int64_t nnz_g = (int64_t)rowptr[g1] - rowptr[g0];
    const double avg = (double)nnz_g / (double)rows_g;

    // ---- column histogram of the run (a long run in parts, counted in parallel and merged)
    if (nnz_g < kParHist) {
      for (int64_t k = rowptr[g0]; k < rowptr[g1]; ++k) hist.add(col[k], fsh);
    } else {
      if (part.empty()) part.assign(kHistParts, Hist(0, fine.size(), 0));
      parallel_chunks(kHistParts, 1, [&](int64_t t, int64_t, int64_t) {
        const int64_t k0 = rowptr[g0] + nnz_g * t / kHistParts, k1 = rowptr[g0] + nnz_g * (t + 1) / kHistParts;
        for (int64_t k = k0; k < k1; ++k) part[t].add(col[k], fsh);
      });
      for (Hist& h : part) hist.merge(h);
    }
    hist.derive(sh, fsh);
    std::vector<int64_t> S2;  // L2-sized column ranges holding min_seg entries per row
    int64_t covS2 = 0;
    for (int64_t w : touched_2)
      if (cnt2[w] >= (int64_t)tp.min_seg * rows_g) {
        S2.push_back(w);
        covS2 += cnt2[w];
      }
    std::sort(S2.begin(), S2.end());
    for (int64_t w : touched_2) cnt2[w] = 0;
    touched_2.clear();
    std::vector<int64_t> S;  // qualifying windows (sorted)
    int64_t covS = 0;
    for (int64_t w : touched_w)
      if (cnt[w] >= (int64_t)tp.min_seg * rows_g) {
        S.push_back(w);
        covS += cnt[w];
      }
    std::sort(S.begin(), S.end());

    // densest wcap-wide window on the fine grid
    std::sort(touched_f.begin(), touched_f.end());
    int64_t best = 0, best_lo = 0, best_hi = 0;
    {
      int64_t run = 0;
      size_t tail = 0, bt = 0, bh = 0;
      for (size_t h = 0; h < touched_f.size(); ++h) {
        run += fine[touched_f[h]];
        while (touched_f[h] - touched_f[tail] >= 8) run -= fine[touched_f[tail++]];
        if (run > best) {
          best = run;
          bt = tail;
          bh = h;
        }
      }
      // trim sparse fine bins off both ends (they keep at most 1% of the window's entries)
      int64_t drop = 0;
      while (bt < bh && drop + fine[touched_f[bt]] <= best / 100) drop += fine[touched_f[bt++]];
      while (bh > bt && drop + fine[touched_f[bh]] <= best / 100) drop += fine[touched_f[bh--]];
      if (!touched_f.empty()) {
        best_lo = touched_f[bt] << fsh;
        best_hi = std::min<int64_t>((touched_f[bh] + 1) << fsh, ncols);
      }
    }
    // grid windows (sparse rows spread over all columns): the run's column span, in fine bins,
    // cut into K ≤ wcap wide windows of near-equal width (window j: bins ⌊j·nf/K⌋ to
    // ⌊(j+1)·nf/K⌋), each holding kGridMinSeg entries per row or more
    std::vector<int64_t> gcut, cntG;
    bool grid_run = false;
    if (tp.grid && !touched_f.empty()) {
      const int64_t fb = int64_t(1) << fsh, f0 = touched_f.front(), f1 = touched_f.back() + 1;
      const int64_t nf = f1 - f0, K = (nf * fb + wcap - 1) / wcap;
      if (K >= 2 && (nf + K - 1) / K * fb <= wcap) {
        for (int64_t j = 0; j <= K; ++j) gcut.push_back(std::min<int64_t>((f0 + j * nf / K) * fb, ncols));
        cntG.assign((size_t)K, 0);
        size_t j = 0;
        for (int64_t f : touched_f) {
          while ((f0 + (int64_t)(j + 1) * nf / K) <= f) ++j;
          cntG[j] += fine[f];
        }
        grid_run = true;
        for (int64_t c : cntG) grid_run = grid_run && c >= (int64_t)kGridMinSeg * rows_g;
      }
    }
    std::vector<int64_t> cntS(S.size());
    for (size_t j = 0; j < S.size(); ++j) cntS[j] = cnt[S[j]];
    for (int64_t w : touched_w) cnt[w] = 0;
    for (int64_t f : touched_f) fine[f] = 0;
    touched_w.clear();
    touched_f.clear();

    if (!(S.size() >= 2 && 2 * covS >= nnz_g) && grid_run) {
      // ---- grid blocks: ranges are the windows, one segment per row and window (empty ones
      // included, so that row r's slot in the block's tile j is that tile's first slot + r − b0);
      // a block whose rows do not all fit falls back to the multi-range emission
      const int32_t K = (int32_t)cntG.size();
      std::vector<int64_t> cut(gcut);
      cut[K] = ncols;
      const double aseg = (double)nnz_g / (double)(rows_g * K);
      // blocks of equal size (whole chunks): about tile_nnz entries per tile, but no more tiles than
      // one round of two workgroups per compute unit when that keeps blocks within kGridMaxRows
      const int64_t Rmax = std::max<int64_t>(
          kLanes, std::min<int64_t>(kGridMaxRows, (int64_t)(tile_nnz / std::max(aseg, 1.0)) / kLanes * kLanes));
      int64_t nb = (rows_g + Rmax - 1) / Rmax;
      const int64_t nb_round = std::max<int64_t>(1, kGridRound / K);
      if (nb * K > kGridRound && (rows_g + nb_round - 1) / nb_round <= kGridMaxRows) nb = nb_round;
      const int32_t R = (int32_t)(((rows_g + nb - 1) / nb + kLanes - 1) / kLanes * kLanes);
      std::vector<Block> blocks;
      for (int32_t b0 = g0; b0 < g1; b0 += R) {
        const int32_t b1 = std::min(g1, b0 + R), Rb = b1 - b0;
        Block bl{b0, b1, std::vector<int32_t>(K, 0), std::vector<int32_t>(K, 0), true};
        for (int32_t j = 0; j < K; ++j) {
          const int32_t w0 = (int32_t)gcut[j];
          const int32_t wl = (int32_t)(gcut[j + 1] - gcut[j]);
          if (cntG[j] * Rb / rows_g * 16 >= wl) {
            bl.wlo[j] = w0;
            bl.wlen[j] = wl;
          }
        }
        blocks.push_back(std::move(bl));
      }
      run_blocks(blocks, cut, nullptr, keep);
    } else if (S.size() >= 2 && 2 * covS >= nnz_g) {
      // ---- multi-range blocks
      const int32_t K = (int32_t)S.size();
      std::vector<int64_t> cut(K + 1);
      cut[0] = 0;
      for (int32_t j = 1; j < K; ++j) cut[j] = S[j] << sh;
      cut[K] = ncols;
      const double aseg = (double)covS / (double)(rows_g * K);
      const int32_t R = block_rows(tile_nnz, aseg);
      std::vector<Block> blocks;
      for (int32_t b0 = g0; b0 < g1; b0 += R) {
        const int32_t b1 = std::min(g1, b0 + R), Rb = b1 - b0;
        Block bl{b0, b1, std::vector<int32_t>(K, 0), std::vector<int32_t>(K, 0)};
        for (int32_t j = 0; j < K; ++j) {
          const int32_t w0 = (int32_t)(S[j] << sh);
          const int32_t wl = (int32_t)std::min<int64_t>(wcap, (int64_t)ncols - w0);
          // entries of this block in the window ≈ its share of the run's count
          if (cntS[j] * Rb / rows_g * 16 >= wl) {
            bl.wlo[j] = w0;
            bl.wlen[j] = wl;
          }
        }
        blocks.push_back(std::move(bl));
      }
      run_blocks(blocks, cut, nullptr, keep);
    } else if (S2.size() >= 2 && 2 * covS2 >= nnz_g && 2 * best < nnz_g) {
      // ---- multi-range blocks without windows, tiles issued range by range
      const int32_t K = (int32_t)S2.size();
      std::vector<int64_t> cut(K + 1);
      cut[0] = 0;
      for (int32_t j = 1; j < K; ++j) cut[j] = S2[j] << kL2Shift;
      cut[K] = ncols;
      const int32_t R = block_rows(plain_nnz, (double)covS2 / (double)(rows_g * K));
      std::vector<std::vector<Seg>> by_range(K);
      std::vector<Block> blocks;
      for (int32_t b0 = g0; b0 < g1; b0 += R)
        blocks.push_back(Block{b0, std::min(g1, b0 + R), std::vector<int32_t>(K, 0), std::vector<int32_t>(K, 0)});
      run_blocks(blocks, cut, &by_range, keep);
      for (int32_t j = 0; j < K; ++j) {
        std::vector<Seg>& v = by_range[j];
        size_t i = 0;
        while (i < v.size()) {
          // about plain_nnz entries, in whole chunks
          size_t e = i;
          int64_t ent = 0;
          while (e < v.size() && (ent < plain_nnz || (e - i) % kLanes != 0)) ent += v[e++].len;
          add_tile(std::vector<Seg>(v.begin() + i, v.begin() + e), 0, 0);
          i = e;
        }
      }
    } else {
      // ---- single-range blocks
      const bool window_run = 2 * best >= nnz_g;
      const int32_t target = window_run ? tile_nnz : plain_nnz;
      const int32_t R = block_rows(target, avg);
      const int64_t run_lo = best_lo, run_hi = best_hi;
      const std::vector<int64_t> cut = {0, (int64_t)ncols};
      // the block's whole column span as its window when it fits, else the run's densest window
      // when that holds half of the block's entries
      auto decide = [&](Block& bl) {
        const int64_t nb = (int64_t)rowptr[bl.b1] - rowptr[bl.b0];
        int32_t cmin = ncols, cmax = -1;
        int64_t in_run = 0;
        for (int32_t r = bl.b0; r < bl.b1; ++r) {
          const int32_t a = rowptr[r], e = rowptr[r + 1];
          if (a == e) continue;
          cmin = std::min(cmin, col[a]);
          cmax = std::max(cmax, col[e - 1]);
          if (window_run) in_run += seek(r, run_hi) - seek(r, run_lo);
        }
        if (cmax >= 0 && (int64_t)cmax - cmin + 1 <= wcap) {
          if (nb * 16 >= (int64_t)cmax - cmin + 1) {
            bl.wlo[0] = cmin;
            bl.wlen[0] = cmax - cmin + 1;
          }
        } else if (window_run && 2 * in_run >= nb) {
          const int32_t a = (int32_t)std::max<int64_t>(run_lo, cmin);
          const int32_t e = (int32_t)std::min<int64_t>(run_hi, (int64_t)cmax + 1);
          if (e > a && in_run * 16 >= e - a) {
            bl.wlo[0] = a;
            bl.wlen[0] = e - a;
          }
        }
      };
      std::vector<Block> blocks;
      for (int32_t b0 = g0; b0 < g1; b0 += R)
        blocks.push_back(Block{b0, std::min(g1, b0 + R), std::vector<int32_t>(1, 0), std::vector<int32_t>(1, 0)});
      run_blocks(blocks, cut, nullptr, decide);
    }
    g0 = g1;
  }
  flush_plain(true);
  plan.nslot = plan.rowslot[nrows];
  // ---- the tiles. Pass 1, per tile: the slots (a tile's segments get consecutive slots in the
  // order they were listed, which is row order, and slotidx maps a segment's row-order id to its
  // slot), then the segments sorted by length, longest first (a stable counting sort, so ties stay
  // in row order), and the tile's count of entries in SELL order.
  const size_t nt = pend.size();
  std::vector<int64_t> first(nt + 1, 0), nent(nt, 0);
  for (size_t ti = 0; ti < nt; ++ti) first[ti + 1] = first[ti] + (int64_t)pend[ti].segs.size();
  plan.slotidx.assign((size_t)plan.nslot, -1);
  parallel_chunks((int64_t)nt, 8, [&](int64_t, int64_t t0, int64_t t1) {
    std::vector<int32_t> pos;
    std::vector<Seg> sorted;
    for (int64_t ti = t0; ti < t1; ++ti) {
      std::vector<Seg>& segs = pend[ti].segs;
      for (size_t k = 0; k < segs.size(); ++k) plan.slotidx[segs[k].slot] = (int32_t)(first[ti] + (int64_t)k);
      pos.assign((size_t)seg_max + 2, 0);  // lengths are 0..seg_max
      for (const Seg& g : segs) pos[(size_t)(seg_max - g.len) + 1]++;
      for (size_t b = 1; b < pos.size(); ++b) pos[b] += pos[b - 1];
      sorted.resize(segs.size());
      for (const Seg& g : segs) sorted[(size_t)pos[(size_t)(seg_max - g.len)]++] = g;
      segs.swap(sorted);
      int64_t e = 0;
      for (size_t c0 = 0; c0 < segs.size(); c0 += kLanes) e += (int64_t)segs[c0].len * kLanes;
      nent[ti] = e;
    }
  });
  // offsets, in tile order: chunks, entries, and column indices (16-bit for windowed tiles)
  plan.tiles.resize(nt);
  std::vector<int64_t> sbase(nt), cbase(nt);
  int64_t n_chunk = 0, n_src = 0, n_c16 = 0, n_c32 = 0;
  for (size_t ti = 0; ti < nt; ++ti) {
    const Pending& pt = pend[ti];
    const int32_t nch = (int32_t)((pt.segs.size() + kLanes - 1) / kLanes);
    plan.tiles[ti] = Tile{(int32_t)n_chunk, nch, pt.wlo, pt.wlen};
    int64_t& nc = pt.wlen > 0 ? n_c16 : n_c32;
    sbase[ti] = n_src;
    cbase[ti] = nc;
    n_chunk += nch;
    n_src += nent[ti];
    nc += nent[ti];
  }
  // ---- pass 2, per tile: chunks of 64 lanes in SELL order (a chunk takes as many steps as its
  // longest segment), each lane's slot, and the entries. Padding repeats the lane's last column
  // with a zero value.
  plan.chunks.resize((size_t)n_chunk);
  plan.segslot.resize((size_t)n_chunk * kLanes);
  plan.lstart.resize((size_t)n_chunk * kLanes);
  plan.llen.resize((size_t)n_chunk * kLanes);
  plan.n_src = n_src;
  plan.n_c16 = n_c16;
  plan.n_c32 = n_c32;
  if (tp.host_entries) {
    plan.src.resize((size_t)n_src);
    plan.col16.resize((size_t)n_c16);
    plan.col32.resize((size_t)n_c32);
  }
  parallel_chunks((int64_t)nt, 8, [&](int64_t, int64_t t0, int64_t t1) {
    Seg g[kLanes];
    for (int64_t ti = t0; ti < t1; ++ti) {
      const Tile& t = plan.tiles[ti];
      const std::vector<Seg>& segs = pend[ti].segs;
      const bool win = t.wlen > 0;
      int64_t base = sbase[ti], cb = cbase[ti];
      for (int32_t c = 0; c < t.nchunk; ++c) {
        const size_t c0 = (size_t)c * kLanes;
        const size_t nseg = std::min<size_t>(kLanes, segs.size() - c0);
        for (size_t j = 0; j < (size_t)kLanes; ++j) g[j] = j < nseg ? segs[c0 + j] : Seg{0, -1, -1};
        Chunk& ch = plan.chunks[(size_t)t.chunk0 + c];
        ch.base = (int32_t)base;
        ch.cbase = (int32_t)cb;
        ch.steps = g[0].len;
        ch.seg0 = (t.chunk0 + c) * kLanes;
        for (int32_t j = 0; j < kLanes; ++j) {
          plan.segslot[(size_t)ch.seg0 + j] = g[j].slot >= 0 ? plan.slotidx[g[j].slot] : -1;
          plan.lstart[(size_t)ch.seg0 + j] = g[j].start;
          plan.llen[(size_t)ch.seg0 + j] = g[j].len;
        }
        base += (int64_t)ch.steps * kLanes;
        cb += (int64_t)ch.steps * kLanes;
        if (!tp.host_entries) continue;
        int32_t* src = &plan.src[(size_t)ch.base];
        for (int32_t q = 0; q < ch.steps; ++q) {
          for (int32_t j = 0; j < kLanes; ++j) {
            const int32_t len = g[j].len;
            const int32_t k = q < len ? g[j].start + q : -1;
            const int32_t c1 = len > 0 ? col[q < len ? g[j].start + q : g[j].start + len - 1] : (win ? t.wlo : 0);
            src[(size_t)q * kLanes + j] = k;
            if (win)
              plan.col16[(size_t)ch.cbase + (size_t)q * kLanes + j] = (uint16_t)(c1 - t.wlo);
            else
              plan.col32[(size_t)ch.cbase + (size_t)q * kLanes + j] = c1;
          }
        }
      }
    }
  });
  // grid tiles: row r of the block has its slot at first + (r − b0)
  plan.tbase.assign(std::max<size_t>(nt, 1), 0);
  for (size_t ti = 0; ti < nt; ++ti)
    if (pend[ti].b0 >= 0) plan.tbase[ti] = (int32_t)(first[ti] - pend[ti].b0);
  std::vector<Pending>().swap(pend);
  // combine work: lanes per row ≈ a quarter of the row's slots (1..64), the largest over the
  // rows of one workgroup; a workgroup of kBlock threads takes one pass of consecutive rows
  auto lg_of = [&](int32_t q) {
    const int32_t ns = plan.rowslot[q + 1] - plan.rowslot[q];
    int32_t lg = 0;
    while (lg < 6 && (4 << lg) < ns) ++lg;
    return lg;
  };
  // Runs of rows with one segment each whose slots are consecutive (slot = D + row, as within
  // one tile of single-segment rows) are combined like a grid block with K = 1: the item reads
  // D from tbase (entries appended after the tiles') and each lane its slot D + row, without
  // the rowslot and slotidx lookups. run[r] = length of such a run starting at row r.
  std::vector<int32_t> run((size_t)nrows + 1, 0);
  auto delta = [&](int32_t q) { return (int64_t)plan.slotidx[plan.rowslot[q]] - q; };
  for (int32_t q = nrows - 1; q >= 0; --q)
    if (plan.rowslot[q + 1] - plan.rowslot[q] == 1)
      run[q] = (run[q + 1] > 0 && delta(q + 1) == delta(q)) ? run[q + 1] + 1 : 1;
  int32_t r = 0;
  size_t gi = 0;  // next grid block (in row order)
  while (r < nrows) {
    if (gi < grids.size() && grids[gi].b0 == r) {
      const GridBlock& gb = grids[gi++];
      for (int32_t a = gb.b0; a < gb.b1; a += kBlock) plan.comb.push_back({a, std::min(gb.b1, a + kBlock), -gb.K, gb.t0});
      r = gb.b1;
      continue;
    }
    const int32_t stop = gi < grids.size() ? grids[gi].b0 : nrows;
    if (run[r] >= kRunMinRows) {
      const int32_t e = std::min(stop, r + run[r]);
      const int32_t t0 = (int32_t)plan.tbase.size();
      plan.tbase.push_back((int32_t)delta(r));
      for (int32_t a = r; a < e; a += kBlock) plan.comb.push_back({a, std::min(e, a + kBlock), -1, t0});
      r = e;
      continue;
    }
    int32_t lg = lg_of(r), r1 = r + 1;
    while (r1 < stop && run[r1] < kRunMinRows) {
      const int32_t l2 = std::max(lg, lg_of(r1));
      if (r1 + 1 - r > (kBlock >> l2)) break;
      lg = l2;
      ++r1;
    }
    plan.comb.push_back({r, r1, lg, 0});
    r = r1;
  }
  return plan;
}

}  // namespace qpg
