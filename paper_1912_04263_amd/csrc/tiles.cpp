// SpMV work-list construction (host): row blocks, column ranges, LDS gather windows, and the
// entry order the SpMV kernel streams.
//
// Rows are grouped into runs of similar length. For each run, a histogram of its column indices
// over fixed windows of wcap columns decides the layout:
//   * multi-range, when at least two windows each hold ≥ kMinSeg entries per row on average and
//     together at least half of the run's entries: the columns are cut at those windows, and each
//     (row block, range) workgroup stages its window in LDS. The block's entries are reordered
//     range by range (rows in order inside each range), so that every workgroup streams one
//     contiguous run of entries. Partial sums per (row, range) cost one value per row and range,
//     hence the kMinSeg floor;
//   * single-range otherwise: consecutive rows in CSR order with one optional window, either the
//     block's whole column span when it fits, or the run's densest wcap-wide window when that
//     holds at least half of the block's entries.
// A window is staged only if it holds at least one entry per 16 of its elements, so that staging
// never reads more than the gathers it replaces. Each workgroup's rows are then packed into
// sub-runs of at most kSubCap entries (a longer row is a sub-run of its own), the unit that the
// kernel loads through LDS.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "qpg_internal.hpp"

namespace qpg {

namespace {

constexpr int kMinSeg = 16;         // entries per row and range for a multi-range layout
constexpr int64_t kMinTiles = 512;  // workgroups a launch should have (two per compute unit)
constexpr int64_t kMinTileNnz = 1024;

int32_t log2_exact(int32_t v) {
  int32_t l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Append the row structure of one workgroup: rows r0.. with the given (start, end, split)
// entry positions in the plan's order, and its sub-runs.
void add_tile(TilePlan& plan, int32_t r0, const std::vector<int32_t>& st, const std::vector<int32_t>& en,
              const std::vector<int32_t>& sp, bool has_split, int32_t wlo, int32_t wlen, int32_t part) {
  const int32_t R = (int32_t)st.size();
  Tile t{};
  t.r0 = r0;
  t.nrow = R;
  t.tr = (int32_t)plan.trp.size();
  t.wlo = wlo;
  t.wlen = wlen;
  t.part = part;
  t.sub0 = (int32_t)plan.subs.size();
  for (int32_t i = 0; i < R; ++i) plan.trp.push_back(st[i]);
  plan.trp.push_back(R > 0 ? en[R - 1] : 0);
  if (has_split) {
    for (int32_t i = 0; i < R; ++i) plan.tsp.push_back(sp[i]);
    plan.tsp.push_back(0);
  }
  int32_t i = 0;
  while (i < R) {
    const int32_t len = en[i] - st[i];
    if (len > kSubCap) {
      plan.subs.push_back({i, i + 1, st[i], en[i]});
      ++i;
      continue;
    }
    int32_t i1 = i, acc = 0;
    while (i1 < R && en[i1] - st[i1] <= kSubCap && acc + (en[i1] - st[i1]) <= kSubCap && i1 - i < kSubCap) {
      acc += en[i1] - st[i1];
      ++i1;
    }
    plan.subs.push_back({i, i1, st[i], en[i1 - 1]});
    i = i1;
  }
  t.nsub = (int32_t)plan.subs.size() - t.sub0;
  plan.tiles.push_back(t);
  if (wlen > 0) plan.max_wlen = std::max(plan.max_wlen, wlen);
}

}  // namespace

TilePlan make_tiles(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col, int32_t nrows,
                    int32_t ncols, int32_t nsplit, const TileParams& tp) {
  TilePlan plan;
  if (nrows <= 0) return plan;
  const bool has_split = nsplit < ncols;
  const int32_t wcap = tp.wcap;
  // smaller workgroups on small matrices, so that the launch still has ~kMinTiles of them
  const int64_t nnz_all = (int64_t)rowptr[nrows] - rowptr[0];
  const int32_t tile_nnz = (int32_t)std::max<int64_t>(kMinTileNnz, std::min<int64_t>(tp.tile_nnz, nnz_all / kMinTiles));
  const int32_t plain_nnz = (int32_t)std::max<int64_t>(kMinTileNnz, std::min<int64_t>(tp.plain_nnz, nnz_all / kMinTiles));
  const int32_t sh = log2_exact(wcap);
  const int32_t fsh = std::max(0, sh - 3);  // eight fine bins per window
  const int64_t nwin = ((int64_t)ncols + wcap - 1) >> sh;
  const int64_t nfine = ((int64_t)ncols + (1 << fsh) - 1) >> fsh;
  std::vector<int64_t> cnt(std::max<int64_t>(nwin, 1), 0), fine(std::max<int64_t>(nfine, 1), 0);
  std::vector<int64_t> touched_w, touched_f;
  std::vector<int32_t> st, en, sp;
  // first entry of row r at or after column c
  auto seek = [&](int32_t r, int64_t c) {
    const int32_t* first = col.data() + rowptr[r];
    const int32_t* last = col.data() + rowptr[r + 1];
    return (int32_t)(std::lower_bound(first, last, (int32_t)std::min<int64_t>(c, INT32_MAX)) - col.data());
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

    // ---- column histogram of the run
    for (int64_t k = rowptr[g0]; k < rowptr[g1]; ++k) {
      const int32_t c = col[k];
      if (cnt[c >> sh]++ == 0) touched_w.push_back(c >> sh);
      if (fine[c >> fsh]++ == 0) touched_f.push_back(c >> fsh);
    }
    std::vector<int64_t> S;  // qualifying windows (sorted)
    int64_t covS = 0;
    for (int64_t w : touched_w)
      if (cnt[w] >= kMinSeg * rows_g) {
        S.push_back(w);
        covS += cnt[w];
      }
    std::sort(S.begin(), S.end());
    // densest wcap-wide window on the fine grid
    std::sort(touched_f.begin(), touched_f.end());
    int64_t best = 0, best_lo = 0;
    {
      int64_t run = 0;
      size_t tail = 0;
      for (size_t h = 0; h < touched_f.size(); ++h) {
        run += fine[touched_f[h]];
        while (touched_f[h] - touched_f[tail] >= 8) run -= fine[touched_f[tail++]];
        if (run > best) {
          best = run;
          best_lo = touched_f[tail] << fsh;
        }
      }
    }
    std::vector<int64_t> cntS(S.size());
    for (size_t j = 0; j < S.size(); ++j) cntS[j] = cnt[S[j]];
    for (int64_t w : touched_w) cnt[w] = 0;
    for (int64_t f : touched_f) fine[f] = 0;
    touched_w.clear();
    touched_f.clear();

    const bool fits32 = plan.n_part + (int64_t)S.size() * rows_g < INT32_MAX;
    if (S.size() >= 2 && 2 * covS >= nnz_g && fits32) {
      // ---- multi-range blocks, entries reordered range by range
      if (plan.perm.empty()) {
        plan.perm.resize(nnz_all);
        for (int64_t k = 0; k < nnz_all; ++k) plan.perm[k] = (int32_t)(rowptr[0] + k);
      }
      const int32_t K = (int32_t)S.size();
      std::vector<int64_t> cut(K + 1);
      cut[0] = 0;
      for (int32_t j = 1; j < K; ++j) cut[j] = S[j] << sh;
      cut[K] = ncols;
      const double aseg = (double)covS / (double)(rows_g * K);
      const int32_t R = (int32_t)std::max<int64_t>(
          1, std::min<int64_t>(tp.max_rows, (int64_t)(tile_nnz / std::max(aseg, 1.0))));
      for (int32_t b0 = g0; b0 < g1; b0 += R) {
        const int32_t b1 = std::min(g1, b0 + R), Rb = b1 - b0;
        const int64_t part_base = plan.n_part;
        int32_t pos = rowptr[b0];  // next position in the plan's order
        for (int32_t j = 0; j < K; ++j) {
          st.clear();
          en.clear();
          sp.clear();
          for (int32_t r = b0; r < b1; ++r) {
            const int32_t a = j == 0 ? rowptr[r] : seek(r, cut[j]);
            const int32_t e = j == K - 1 ? rowptr[r + 1] : seek(r, cut[j + 1]);
            const int32_t s = has_split ? std::min(std::max(seek(r, nsplit), a), e) : e;
            st.push_back(pos);
            sp.push_back(pos + (s - a));
            for (int32_t k = a; k < e; ++k) plan.perm[pos++ - rowptr[0]] = k;
            en.push_back(pos);
          }
          const int32_t wlo = (int32_t)(S[j] << sh);
          const int32_t wlen = (int32_t)std::min<int64_t>(wcap, (int64_t)ncols - wlo);
          // entries of this block in the window ≈ its share of the run's count
          const bool stage = cntS[j] * Rb / rows_g * 16 >= wlen;
          add_tile(plan, b0, st, en, sp, has_split, stage ? wlo : 0, stage ? wlen : 0,
                   (int32_t)(part_base + (int64_t)j * Rb));
        }
        for (int32_t r = b0; r < b1; r += kBlock)
          plan.comb.push_back({r, std::min(b1, r + kBlock), K, (int32_t)(part_base + (r - b0)), Rb, 0, 0, 0});
        plan.n_part += (int64_t)K * Rb;
      }
    } else {
      // ---- single-range blocks (CSR order)
      const bool window_run = 2 * best >= nnz_g;
      const int32_t target = window_run ? tile_nnz : plain_nnz;
      const int32_t R = (int32_t)std::max<int64_t>(
          1, std::min<int64_t>(tp.max_rows, (int64_t)(target / std::max(avg, 1.0))));
      const int64_t run_lo = best_lo, run_hi = std::min<int64_t>(best_lo + wcap, ncols);
      for (int32_t b0 = g0; b0 < g1; b0 += R) {
        const int32_t b1 = std::min(g1, b0 + R);
        const int64_t nb = (int64_t)rowptr[b1] - rowptr[b0];
        int32_t cmin = ncols, cmax = -1;
        int64_t in_run = 0;
        st.clear();
        en.clear();
        sp.clear();
        for (int32_t r = b0; r < b1; ++r) {
          const int32_t a = rowptr[r], e = rowptr[r + 1];
          st.push_back(a);
          en.push_back(e);
          if (has_split) sp.push_back(seek(r, nsplit));
          if (a == e) continue;
          cmin = std::min(cmin, col[a]);
          cmax = std::max(cmax, col[e - 1]);
          if (window_run) in_run += seek(r, run_hi) - seek(r, run_lo);
        }
        int32_t wlo = 0, wlen = 0;
        if (cmax >= 0 && (int64_t)cmax - cmin + 1 <= wcap) {
          if (nb * 16 >= (int64_t)cmax - cmin + 1) {
            wlo = cmin;
            wlen = cmax - cmin + 1;
          }
        } else if (window_run && 2 * in_run >= nb) {
          const int32_t a = (int32_t)std::max<int64_t>(run_lo, cmin);
          const int32_t e = (int32_t)std::min<int64_t>(run_hi, (int64_t)cmax + 1);
          if (e > a && in_run * 16 >= e - a) {
            wlo = a;
            wlen = e - a;
          }
        }
        add_tile(plan, b0, st, en, sp, has_split, wlo, wlen, -1);
      }
    }
    g0 = g1;
  }
  return plan;
}

}  // namespace qpg
