// Host check of the SpMV work lists built by make_tiles (csrc/tiles.cpp): every bound the
// kernels rely on, exact coverage of the entries, and the row sums the kernels would form
// (segment sums split at column nsplit, added per row in slot order) against a plain CSR SpMV.
// Reads <prefix>_ptr.bin / <prefix>_col.bin (int32); prints one line per window size.
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

// FNV-1a over the bytes of an array (the work list's fingerprint, to compare builds)
template <class V>
static unsigned long long fnv(const V& v, unsigned long long x = 1469598103934665603ull) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(v.data());
  for (size_t i = 0; i < v.size() * sizeof(v[0]); ++i) x = (x ^ p[i]) * 1099511628211ull;
  return x;
}

#define FAIL(...)             \
  do {                        \
    std::printf("FAIL: ");    \
    std::printf(__VA_ARGS__); \
    std::printf("\n");        \
    return 1;                 \
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
    const TilePlan p = make_tiles(rp, col.data(), nrows, ncols, TileParams{wcap, tile_nnz, plain_nnz, kTileMaxRows});
    if ((int)p.rowslot.size() != nrows + 1 || p.rowslot[0] != 0 || p.rowslot[nrows] != p.nslot) FAIL("row slots");
    for (int r = 0; r < nrows; ++r)
      if (p.rowslot[r + 1] < p.rowslot[r]) FAIL("row slots decrease");
    if (p.col16.size() + p.col32.size() != p.src.size()) FAIL("column arrays");
    std::vector<int> covered(nnz, 0), slotset(std::max<int64_t>(p.nslot, 1), 0);
    std::vector<double> part1(std::max<int64_t>(p.nslot, 1), 0.0), part2(part1);
    long windowed = 0, padding = 0, in_win = 0, empty_segs = 0;
    for (const Tile& t : p.tiles) {
      if (t.chunk0 < 0 || t.nchunk < 1 || (size_t)t.chunk0 + t.nchunk > p.chunks.size()) FAIL("tile chunks");
      const bool win = t.wlen > 0;
      if (t.wlen < 0 || t.wlo < 0 || (long)t.wlo + t.wlen > ncols || t.wlen > wcap || t.wlen > 65536 ||
          t.wlen > p.max_wlen)
        FAIL("window [%d, +%d)", t.wlo, t.wlen);
      windowed += win;
      for (int ci = t.chunk0; ci < t.chunk0 + t.nchunk; ++ci) {
        const Chunk& ch = p.chunks[ci];
        if (ch.steps < 0 || ch.steps > kSegMax) FAIL("chunk steps %d", ch.steps);
        if (ch.base < 0 || (size_t)ch.base + 64 * (size_t)ch.steps > p.src.size()) FAIL("chunk values");
        const size_t csz = win ? p.col16.size() : p.col32.size();
        if (ch.cbase < 0 || (size_t)ch.cbase + 64 * (size_t)ch.steps > csz) FAIL("chunk columns");
        if (ch.seg0 < 0 || (size_t)ch.seg0 + 64 > p.segslot.size()) FAIL("chunk slots");
        for (int j = 0; j < 64; ++j) {
          const int slot = p.segslot[ch.seg0 + j];
          double s1 = 0, s2 = 0;
          bool any = false;
          for (int s = 0; s < ch.steps; ++s) {
            const long k = p.src[ch.base + 64 * s + j];
            const long cpos = ch.cbase + 64L * s + j;
            const long c = win ? (long)t.wlo + p.col16[cpos] : (long)p.col32[cpos];
            if (c < 0 || c >= ncols) FAIL("column out of range");
            if (win && c >= (long)t.wlo + t.wlen) FAIL("column outside the window");
            if (k < 0) {
              ++padding;
              continue;
            }
            if (k >= nnz || c != col[k]) FAIL("column mismatch");
            if (slot < 0) FAIL("entry in an empty lane");
            covered[k]++;
            in_win += win;
            any = true;
            (c < nsplit ? s1 : s2) += val[k] * x[c];
          }
          if (slot >= 0) {
            if (slot >= p.nslot || slotset[slot]++) FAIL("slot %d", slot);
            if (!any) ++empty_segs;  // grid blocks keep one (possibly empty) segment per window
            part1[slot] = s1;
            part2[slot] = s2;
          }
        }
      }
    }
    for (long k = 0; k < nnz; ++k)
      if (covered[k] != 1) FAIL("entry %ld covered %d times", k, covered[k]);
    for (long q = 0; q < p.nslot; ++q)
      if (!slotset[q]) FAIL("slot %ld never written", q);
    // slotidx is a permutation of the slots, and every tile writes one contiguous range of them
    if ((long)p.slotidx.size() != p.nslot) FAIL("slotidx size");
    std::vector<int> seen(std::max<int64_t>(p.nslot, 1), 0);
    for (long q = 0; q < p.nslot; ++q) {
      if (p.slotidx[q] < 0 || p.slotidx[q] >= p.nslot || seen[p.slotidx[q]]++) FAIL("slotidx not a permutation");
    }
    for (const Tile& t : p.tiles) {
      long lo = p.nslot, hi = -1, cnt = 0;
      for (int ci = t.chunk0; ci < t.chunk0 + t.nchunk; ++ci)
        for (int j = 0; j < 64; ++j) {
          const int sl = p.segslot[p.chunks[ci].seg0 + j];
          if (sl < 0) continue;
          lo = std::min<long>(lo, sl);
          hi = std::max<long>(hi, sl);
          ++cnt;
        }
      if (cnt && hi - lo + 1 != cnt) FAIL("tile slots not contiguous");
    }
    std::vector<int> combined(nrows, 0);
    long grid_rows = 0, run_rows = 0;
    for (const CombItem& c : p.comb) {
      if (c.lg > 6 || c.r0 < 0 || c.r1 > nrows || c.r0 >= c.r1) FAIL("combine item");
      if (c.lg < 0) {
        // grid item: K slots per row at tbase[t0 + j] + row, the row's slots in column order
        const int K = -c.lg;
        if (c.r1 - c.r0 > 256 || c.t0 < 0 || (size_t)c.t0 + K > p.tbase.size()) FAIL("grid item");
        if ((size_t)c.t0 >= p.tiles.size()) run_rows += c.r1 - c.r0;  // a run of single-segment rows
        for (int r = c.r0; r < c.r1; ++r) {
          if (p.rowslot[r + 1] - p.rowslot[r] != K) FAIL("grid row %d has %d slots", r, p.rowslot[r + 1] - p.rowslot[r]);
          for (int j = 0; j < K; ++j)
            if ((long)p.tbase[c.t0 + j] + r != p.slotidx[p.rowslot[r] + j]) FAIL("grid slot of row %d", r);
        }
        grid_rows += c.r1 - c.r0;
      }
      for (int r = c.r0; r < c.r1; ++r) combined[r]++;
    }
    for (int r = 0; r < nrows; ++r)
      if (combined[r] != 1) FAIL("row %d combined %d times", r, combined[r]);
    double err = 0, scale = 0;
    for (int r = 0; r < nrows; ++r) {
      double s1 = 0, s2 = 0;
      for (int q = p.rowslot[r]; q < p.rowslot[r + 1]; ++q) {
        s1 += part1[p.slotidx[q]];
        s2 += part2[p.slotidx[q]];
      }
      err = std::max(err, std::fabs(s1 - ref1[r]) + std::fabs(s2 - ref2[r]));
      scale = std::max(scale, std::fabs(ref1[r]) + std::fabs(ref2[r]));
    }
    if (err > 1e-12 * std::max(scale, 1.0)) FAIL("row sums off by %g", err);
    // the lanes alone give the same entries (the device writes them from the lanes): lane j of a
    // chunk at step q holds CSR index lstart + q while q < llen, else −1, and the column of that
    // entry, or of the segment's last entry past its end, or the window's first column (0 without
    // a window) for a lane with no entries
    if (p.lstart.size() != p.segslot.size() || p.llen.size() != p.segslot.size() || (long)p.src.size() != p.n_src ||
        (long)p.col16.size() != p.n_c16 || (long)p.col32.size() != p.n_c32)
      FAIL("lane arrays");
    for (const Tile& t : p.tiles) {
      const bool win = t.wlen > 0;
      for (int ci = t.chunk0; ci < t.chunk0 + t.nchunk; ++ci) {
        const Chunk& ch = p.chunks[ci];
        for (int j = 0; j < 64; ++j) {
          const long s0 = p.lstart[ch.seg0 + j], len = p.llen[ch.seg0 + j];
          if (len > ch.steps || (len > 0 && (s0 < 0 || s0 + len > nnz))) FAIL("lane %d of chunk %d", j, ci);
          for (int q = 0; q < ch.steps; ++q) {
            const long k = q < len ? s0 + q : -1;
            const long c = len > 0 ? col[q < len ? k : s0 + len - 1] : (win ? t.wlo : 0);
            const size_t o = (size_t)q * 64 + j;
            const long c2 = win ? (long)t.wlo + p.col16[ch.cbase + o] : (long)p.col32[ch.cbase + o];
            if (p.src[ch.base + o] != k || c2 != c) FAIL("lane %d of chunk %d at step %d", j, ci, q);
          }
        }
      }
    }
    std::printf("wcap %d tiles %zu windowed %ld chunks %zu padding %.1f%% in-window %.1f%% slots %ld maxwin %d grid_rows %ld empty %ld run_rows %ld\n", wcap,
                p.tiles.size(), windowed, p.chunks.size(), 100.0 * padding / std::max<size_t>(p.src.size(), 1),
                100.0 * in_win / std::max<long>(nnz, 1), (long)p.nslot, p.max_wlen, grid_rows, empty_segs, run_rows);
    unsigned long long hsh = fnv(p.tiles);
    hsh = fnv(p.chunks, hsh);
    hsh = fnv(p.comb, hsh);
    hsh = fnv(p.segslot, hsh);
    hsh = fnv(p.rowslot, hsh);
    hsh = fnv(p.slotidx, hsh);
    hsh = fnv(p.tbase, hsh);
    hsh = fnv(p.lstart, hsh);
    hsh = fnv(p.llen, hsh);
    hsh = fnv(p.src, hsh);
    hsh = fnv(p.col16, hsh);
    hsh = fnv(p.col32, hsh);
    std::printf("fingerprint wcap %d %016llx\n", wcap, hsh);
  }
  return 0;
}
