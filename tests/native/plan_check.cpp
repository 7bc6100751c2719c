// Host check of the SpMV work lists built by make_tiles (csrc/tiles.cpp): every bound the
// kernels rely on, exact coverage of the entries, and the row sums the kernels would form
// (products summed per row, per column part, through the partial slots) against a plain CSR
// SpMV. Reads <prefix>_ptr.bin / <prefix>_col.bin (int32) and prints one line per window size.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "qpg_internal.hpp"

using namespace qpg;

template <typename T>
static std::vector<T> read_all(const std::string& f) {
  std::ifstream in(f, std::ios::binary | std::ios::ate);
  const size_t n = (size_t)in.tellg();
  in.seekg(0);
  std::vector<T> v(n / sizeof(T));
  in.read(reinterpret_cast<char*>(v.data()), (std::streamsize)n);
  return v;
}

#define FAIL(...)                 \
  do {                            \
    std::printf("FAIL: ");        \
    std::printf(__VA_ARGS__);     \
    std::printf("\n");            \
    return 1;                     \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 7) return 2;
  const std::string pre = argv[1];
  const int ncols = std::atoi(argv[2]), nsplit = std::atoi(argv[3]);
  const int tile_nnz = std::atoi(argv[4]), plain_nnz = std::atoi(argv[5]), wcap0 = std::atoi(argv[6]);
  const auto rp = read_all<int32_t>(pre + "_ptr.bin");
  const auto col = read_all<int32_t>(pre + "_col.bin");
  const int nrows = (int)rp.size() - 1;
  const long nnz = (long)col.size();
  std::vector<double> x(ncols), val(nnz), ref1(nrows, 0.0), ref2(nrows, 0.0);
  for (int j = 0; j < ncols; ++j) x[j] = std::sin(0.37 * j) + 1.5;
  for (long k = 0; k < nnz; ++k) val[k] = std::cos(0.11 * k);
  for (int r = 0; r < nrows; ++r)
    for (int k = rp[r]; k < rp[r + 1]; ++k) (col[k] < nsplit ? ref1 : ref2)[r] += val[k] * x[col[k]];
  for (int wcap = wcap0; wcap <= 2 * wcap0; wcap *= 2) {
    TilePlan p = make_tiles(rp, col, nrows, ncols, nsplit, TileParams{wcap, tile_nnz, plain_nnz, kTileMaxRows});
    const bool split = nsplit < ncols;
    if (split == p.tsp.empty()) FAIL("split positions present iff the matrix has a split");
    if (!p.perm.empty() && (long)p.perm.size() != nnz) FAIL("order size");
    std::vector<int> seen(nnz, 0);
    for (long k = 0; k < (long)p.perm.size(); ++k)
      if (p.perm[k] < 0 || p.perm[k] >= nnz || seen[p.perm[k]]++) FAIL("order is not a permutation");
    auto src = [&](long k) { return p.perm.empty() ? k : (long)p.perm[k]; };
    std::vector<int> covered(nnz, 0), done(nrows, 0);
    const size_t np = (size_t)std::max<int64_t>(p.n_part, 1);
    std::vector<double> part1(np, NAN), part2(np, NAN), y1(nrows, NAN), y2(nrows, NAN);
    std::vector<int> partset(np, 0);
    long multi = 0, staged = 0, longsubs = 0;
    for (const Tile& t : p.tiles) {
      if (t.r0 < 0 || t.nrow < 0 || t.r0 + t.nrow > nrows) FAIL("tile rows");
      if (t.wlen < 0 || t.wlo < 0 || (long)t.wlo + t.wlen > ncols || t.wlen > p.max_wlen || t.wlen > wcap)
        FAIL("window [%d, +%d)", t.wlo, t.wlen);
      if (t.tr < 0 || (size_t)t.tr + t.nrow >= p.trp.size()) FAIL("row-start index");
      if (split && (size_t)t.tr + t.nrow >= p.tsp.size()) FAIL("split index");
      multi += t.part >= 0;
      staged += t.wlen > 0;
      std::vector<int> rowseen(t.nrow, 0);
      for (int s = 0; s < t.nsub; ++s) {
        if (t.sub0 < 0 || (size_t)t.sub0 + s >= p.subs.size()) FAIL("sub-run index");
        const Sub u = p.subs[t.sub0 + s];
        if (u.i0 < 0 || u.i1 > t.nrow || u.i0 >= u.i1) FAIL("sub-run rows");
        if (u.k0 < 0 || u.k1 > nnz || u.k0 > u.k1) FAIL("sub-run entries");
        if (p.trp[t.tr + u.i0] != u.k0 || p.trp[t.tr + u.i1] != u.k1) FAIL("sub-run bounds");
        if (u.k1 - u.k0 > kSubCap) {
          ++longsubs;
          if (u.i1 != u.i0 + 1) FAIL("long sub-run with several rows");
        }
        if (u.i1 - u.i0 > kSubCap) FAIL("sub-run row count");
        for (int i = u.i0; i < u.i1; ++i) {
          if (rowseen[i]++) FAIL("row twice in a tile");
          const int a = p.trp[t.tr + i], b = p.trp[t.tr + i + 1], sp = split ? p.tsp[t.tr + i] : b;
          if (a > b || sp < a || sp > b) FAIL("row bounds");
          double s1 = 0, s2 = 0;
          for (int k = a; k < b; ++k) {
            const long o = src(k);
            covered[o]++;
            const double pr = val[o] * x[col[o]];
            if (k < sp) {
              if (col[o] >= nsplit) FAIL("entry of the second part before the split");
              s1 += pr;
            } else {
              if (col[o] < nsplit) FAIL("entry of the first part after the split");
              s2 += pr;
            }
          }
          const int r = t.r0 + i;
          if (t.part < 0) {
            if (done[r]++) FAIL("row finished twice");
            y1[r] = s1;
            y2[r] = s2;
          } else {
            const long q = (long)t.part + i;
            if (q >= p.n_part || partset[q]++) FAIL("partial slot");
            part1[q] = s1;
            part2[q] = s2;
          }
        }
      }
      for (int i = 0; i < t.nrow; ++i)
        if (rowseen[i] != 1) FAIL("tile row %d not in a sub-run", i);
    }
    for (const CombItem& c : p.comb) {
      if (c.r1 - c.r0 > kBlock || c.r0 < 0 || c.r1 > nrows || c.r0 > c.r1) FAIL("combine rows");
      for (int r = c.r0; r < c.r1; ++r) {
        double s1 = 0, s2 = 0;
        for (int j = 0; j < c.nrange; ++j) {
          const long q = (long)c.part + (long)j * c.stride + (r - c.r0);
          if (q < 0 || q >= p.n_part || !partset[q]) FAIL("combine slot");
          s1 += part1[q];
          s2 += part2[q];
        }
        if (done[r]++) FAIL("row finished twice (combine)");
        y1[r] = s1;
        y2[r] = s2;
      }
    }
    for (long k = 0; k < nnz; ++k)
      if (covered[k] != 1) FAIL("entry %ld covered %d times", k, covered[k]);
    double err = 0, scale = 0;
    for (int r = 0; r < nrows; ++r) {
      if (done[r] != 1) FAIL("row %d finished %d times", r, done[r]);
      err = std::max(err, std::fabs(y1[r] - ref1[r]) + std::fabs(y2[r] - ref2[r]));
      scale = std::max(scale, std::fabs(ref1[r]) + std::fabs(ref2[r]));
    }
    if (err > 1e-12 * std::max(scale, 1.0)) FAIL("row sums off by %g", err);
    std::printf("wcap %d tiles %zu multi %ld staged %ld long %ld comb %zu reordered %d\n", wcap, p.tiles.size(),
                multi, staged, longsubs, p.comb.size(), (int)!p.perm.empty());
  }
  return 0;
}
