// Host-side preparation: input validation and the CSC → CSR conversions (full P from its upper
// triangle, A, and B = [P | Aᵀ]); the values stay unscaled (equilibration runs on the device).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <thread>

#include "qpg_internal.hpp"

namespace qpg {

namespace {

// The first structural error of column j of a CSC matrix (0 if none); `upper` additionally
// requires row ≤ column.
int column_error(const qpg_csc* M, int32_t j, int32_t nrows, bool upper, const char* name, std::string* msg) {
  char buf[256];
  const int32_t a = M->colptr[j], b = M->colptr[j + 1];
  if (b < a) {
    *msg = std::string(name) + ": colptr not monotone";
    return QPG_ERR_ARG;
  }
  for (int32_t k = a; k < b; ++k) {
    const int32_t i = M->rowidx[k];
    if (i < 0 || i >= nrows) {
      std::snprintf(buf, sizeof(buf), "%s: row index %d out of range in column %d", name, (int)i, (int)j);
      *msg = buf;
      return QPG_ERR_ARG;
    }
    if (k > a && i <= M->rowidx[k - 1]) {
      std::snprintf(buf, sizeof(buf), "%s: row indices of column %d not strictly increasing", name, (int)j);
      *msg = buf;
      return QPG_ERR_ARG;
    }
    if (upper && i > j) {
      std::snprintf(buf, sizeof(buf), "%s: entry (%d,%d) below the diagonal", name, (int)i, (int)j);
      *msg = buf;
      return QPG_ERR_ARG;
    }
  }
  return QPG_OK;
}

void atomic_min(std::atomic<int64_t>& a, int64_t v) {
  int64_t cur = a.load();
  while (v < cur && !a.compare_exchange_weak(cur, v)) {
  }
}

// Structural checks of a CSC matrix (columns checked in parallel; the first failing column is
// reported, as a serial scan would).
// [0, n) cut into `parts` ranges of about equal work, item i costing ptr[i + 1] − ptr[i] entries
// plus one (ptr non-decreasing): a few long columns or rows then no longer fall to one thread
template <typename I>
std::vector<int64_t> work_cuts(const I* ptr, int64_t n, int64_t parts) {
  std::vector<int64_t> cut((size_t)parts + 1, n);
  const int64_t total = (int64_t)(ptr[n] - ptr[0]) + n;
  cut[0] = 0;
  for (int64_t t = 1; t < parts; ++t) {
    const int64_t target = total * t / parts;
    int64_t lo = cut[(size_t)t - 1], hi = n;  // first i with (ptr[i] − ptr[0]) + i ≥ target
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if ((int64_t)(ptr[mid] - ptr[0]) + mid < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    cut[(size_t)t] = lo;
  }
  return cut;
}
constexpr int64_t kWorkParts = 256;

int check_csc(const qpg_csc* M, int32_t nrows, int32_t ncols, bool upper, const char* name,
              std::string* msg) {
  char buf[256];
  if (!M || M->nrows != nrows || M->ncols != ncols || M->nnz < 0) {
    std::snprintf(buf, sizeof(buf), "%s: null or dimension mismatch (expected %d x %d)", name,
                  (int)nrows, (int)ncols);
    *msg = buf;
    return QPG_ERR_ARG;
  }
  if (!M->colptr || (M->nnz > 0 && (!M->rowidx || !M->val))) {
    *msg = std::string(name) + ": null array";
    return QPG_ERR_ARG;
  }
  if (M->colptr[0] != 0 || M->colptr[ncols] != M->nnz) {
    *msg = std::string(name) + ": colptr must start at 0 and end at nnz";
    return QPG_ERR_ARG;
  }
  // monotone colptr first, so that every column range below is inside [0, nnz]
  for (int32_t j = 0; j < ncols; ++j)
    if (M->colptr[j + 1] < M->colptr[j]) {
      *msg = std::string(name) + ": colptr not monotone";
      return QPG_ERR_ARG;
    }
  std::atomic<int64_t> bad{INT64_MAX};
  const std::vector<int64_t> cols = work_cuts(M->colptr, ncols, kWorkParts);
  parallel_chunks(kWorkParts, 1, [&](int64_t t, int64_t, int64_t) {
    std::string m2;
    for (int64_t j = cols[(size_t)t]; j < cols[(size_t)t + 1]; ++j)
      if (column_error(M, (int32_t)j, nrows, upper, name, &m2)) {
        atomic_min(bad, j);
        return;
      }
  });
  if (bad.load() != INT64_MAX) return column_error(M, (int32_t)bad.load(), nrows, upper, name, msg);
  std::atomic<int64_t> nonfinite{INT64_MAX};
  parallel_chunks(M->nnz, 1 << 20, [&](int64_t, int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k)
      if (!std::isfinite(M->val[k])) {
        atomic_min(nonfinite, k);
        return;
      }
  });
  if (nonfinite.load() != INT64_MAX) {
    *msg = std::string(name) + ": non-finite value";
    return QPG_ERR_DATA;
  }
  return QPG_OK;
}

// Builds a CSR matrix (nrows rows) from entries produced column by column: emit(j, put) calls
// put(row, column, payload) for the entries of column j in order (the payload is the entry's value,
// or its index in the source arrays). Rows come out in the order a serial pass over the columns
// would produce. The columns are cut into parts of about equal work (work[j] = number of entries
// column j emits, as a prefix array). A direct scatter into the rows would write every entry to
// a random place in the output; instead the entries are first distributed into buckets of 4096
// consecutive rows (sequential appends: one write stream per bucket and part), bucket by bucket
// and, within a bucket, part by part, so that each bucket holds its entries in serial column
// order; then every bucket places its entries into its own rows, a range that stays in cache.
// The result does not depend on the number of parts.
template <class Emit, typename V>
void columns_to_rows(int32_t ncols, int32_t nrows, const std::vector<int64_t>& work, Emit emit,
                     std::vector<int32_t>& ptr, hvec<int32_t>& col, hvec<V>& val) {
  constexpr int kBucketShift = 12;
  const int64_t total = work[ncols];
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int T = total < (1 << 18) ? 1 : std::min(16, hw);
  std::vector<int32_t> cut(T + 1);
  for (int t = 0; t <= T; ++t)
    cut[t] = (int32_t)(std::lower_bound(work.begin(), work.end(), total * t / T) - work.begin());
  cut[0] = 0;
  cut[T] = ncols;
  const int64_t nb = ((int64_t)nrows >> kBucketShift) + 1;
  // entries per (part, bucket), then each (part, bucket)'s first position: bucket-major, parts in
  // order within a bucket
  std::vector<std::vector<int64_t>> pos(T);
  parallel_chunks(T, 1, [&](int64_t t, int64_t, int64_t) {
    auto& c = pos[t];
    c.assign((size_t)nb, 0);
    for (int32_t j = cut[t]; j < cut[t + 1]; ++j) emit(j, [&](int32_t r, int32_t, V) { c[r >> kBucketShift]++; });
  });
  std::vector<int64_t> bstart((size_t)nb + 1, 0);
  int64_t o = 0;
  for (int64_t b = 0; b < nb; ++b) {
    bstart[b] = o;
    for (int t = 0; t < T; ++t) {
      const int64_t c = pos[t][b];
      pos[t][b] = o;
      o += c;
    }
  }
  bstart[nb] = o;
  hvec<int32_t> trow((size_t)o), tcol((size_t)o);
  hvec<V> tval((size_t)o);
  parallel_chunks(T, 1, [&](int64_t t, int64_t, int64_t) {
    auto& q = pos[t];
    for (int32_t j = cut[t]; j < cut[t + 1]; ++j)
      emit(j, [&](int32_t r, int32_t c, V v) {
        const int64_t d = q[r >> kBucketShift]++;
        trow[d] = r;
        tcol[d] = c;
        tval[d] = v;
      });
  });
  // each bucket: its rows' lengths (hence ptr: a bucket's rows start where its entries start),
  // then its entries into their rows in bucket order
  ptr.assign((size_t)nrows + 1, 0);
  col.resize((size_t)o);
  val.resize((size_t)o);
  parallel_chunks(nb, 1, [&](int64_t b, int64_t, int64_t) {
    const int32_t r0 = (int32_t)(b << kBucketShift);
    const int32_t r1 = (int32_t)std::min<int64_t>(nrows, (b + 1) << kBucketShift);
    if (r0 >= r1) return;
    std::vector<int64_t> at((size_t)(r1 - r0) + 1, 0);
    for (int64_t d = bstart[b]; d < bstart[b + 1]; ++d) at[(size_t)(trow[d] - r0) + 1]++;
    for (int32_t i = 0; i < r1 - r0; ++i) at[i + 1] += at[i];
    for (int32_t i = 0; i < r1 - r0; ++i) ptr[(size_t)r0 + i + 1] = (int32_t)(bstart[b] + at[i + 1]);
    for (int64_t d = bstart[b]; d < bstart[b + 1]; ++d) {
      const int64_t e = bstart[b] + at[(size_t)(trow[d] - r0)]++;
      col[e] = tcol[d];
      val[e] = tval[d];
    }
  });
}

}  // namespace

int validate_settings(const qpg_settings* s, std::string* msg) {
  if (!s) {
    *msg = "settings: null";
    return QPG_ERR_ARG;
  }
  bool ok = s->rho > 0 && std::isfinite(s->rho) && s->sigma > 0 && std::isfinite(s->sigma) &&
            s->alpha > 0 && s->alpha < 2 && s->eps_abs >= 0 && s->eps_rel >= 0 &&
            std::isfinite(s->eps_abs) && std::isfinite(s->eps_rel) && s->max_iter >= 0 &&
            s->check_every >= 1 && s->rho_update_every >= 0 && s->rho_update_gate >= 1.0 &&
            s->pcg_lambda > 0 && s->pcg_eps_min >= 0 && s->pcg_eps_fixed >= 0 &&
            s->pcg_max_iter >= 1 && (s->pcg_rel_test == 0 || s->pcg_rel_test == 1) &&
            s->scaling_iters >= 0 && s->scaling_iters <= 100 &&
            (s->precision == QPG_FP64 || s->precision == QPG_MIXED) &&
            (s->precond == QPG_PRECOND_JACOBI ||
             (s->precond == QPG_PRECOND_LEARNED && s->precond_weights != nullptr)) &&
            (s->precond_trial == 0 || s->precond_trial == 1) && s->device >= 0 &&
            s->spmv_tile_nnz >= 0 && s->spmv_plain_nnz >= 0 && s->eps_prim_inf >= 0 &&
            s->eps_dual_inf >= 0 && std::isfinite(s->eps_prim_inf) && std::isfinite(s->eps_dual_inf) &&
            (s->rho_vector == 0 || (s->rho_vector == 1 && s->precond == QPG_PRECOND_JACOBI)) &&
            (s->pcg_eps_schedule == 0 || s->pcg_eps_schedule == 1) &&
            (s->speculate == 0 || s->speculate == 1) &&
            (s->spmv_window_cols == 0 ||
             (s->spmv_window_cols >= 1024 && s->spmv_window_cols <= 65536 &&
              (s->spmv_window_cols & (s->spmv_window_cols - 1)) == 0)) &&
            s->spmv_min_seg >= 0 && s->spmv_min_seg <= 256;
  if (!ok) {
    *msg = "settings: value out of range";
    return QPG_ERR_ARG;
  }
  return QPG_OK;
}

Plan make_plan(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t cap) {
  Plan p;
  int32_t r = 0;
  while (r < nrows) {
    int32_t len = rowptr[r + 1] - rowptr[r];
    if (len > cap) {
      if (len <= kLongCap) {
        p.items.push_back({r, r + 1, rowptr[r], rowptr[r + 1], 0, 0, 0, 0});
      } else {
        int32_t nch = (len + kChunk - 1) / kChunk;
        int32_t base = p.n_chunk_slots;
        int32_t ticket = p.n_split_rows++;
        p.n_chunk_slots += nch;
        // near-equal chunks
        for (int32_t c = 0; c < nch; ++c) {
          int32_t a = rowptr[r] + (int32_t)((int64_t)len * c / nch);
          int32_t b = rowptr[r] + (int32_t)((int64_t)len * (c + 1) / nch);
          p.items.push_back({r, r + 1, a, b, nch, c, base, ticket});
        }
      }
      ++r;
      continue;
    }
    int32_t r0 = r;
    int32_t acc = 0;
    while (r < nrows) {
      int32_t l2 = rowptr[r + 1] - rowptr[r];
      if (l2 > cap || acc + l2 > cap || (r - r0) >= cap) break;
      acc += l2;
      ++r;
    }
    p.items.push_back({r0, r, rowptr[r0], rowptr[r], 0, 0, 0, 0});
  }
  return p;
}

void prepare_a(const qpg_csc* A, HostProblem* out) {
  // A in CSR: the pattern, and each entry's index in the CSC arrays (visiting the CSC columns in
  // order keeps each row's columns sorted); the values follow on the device
  HostProblem& H = *out;
  std::vector<int64_t> a_work((size_t)H.n + 1);
  for (int32_t j = 0; j <= H.n; ++j) a_work[j] = A->colptr[j];
  columns_to_rows(
      H.n, H.m, a_work,
      [&](int32_t j, auto&& put) {
        for (int32_t k = A->colptr[j]; k < A->colptr[j + 1]; ++k) put(A->rowidx[k], j, (int32_t)k);
      },
      H.a_ptr, H.a_col, H.a_src);
}

int prepare(const qpg_csc* Pt, const double* q, const qpg_csc* A, const double* l,
            const double* u, const qpg_settings* s, HostProblem* out, std::string* msg, bool with_a) {
  int rc = validate_settings(s, msg);
  if (rc) return rc;
  if (!Pt || !A) {
    *msg = "P or A: null";
    return QPG_ERR_ARG;
  }
  const int32_t n = A->ncols, m = A->nrows;
  if (n < 1 || m < 0) {
    *msg = "dimensions: need n >= 1 and m >= 0";
    return QPG_ERR_ARG;
  }
  if ((int64_t)n + (int64_t)m > std::numeric_limits<int32_t>::max()) {
    *msg = "dimensions: n + m overflows int32";
    return QPG_ERR_SIZE;
  }
  if ((rc = check_csc(Pt, n, n, true, "P_triu", msg))) return rc;
  if ((rc = check_csc(A, m, n, false, "A", msg))) return rc;
  if (!q || (m > 0 && (!l || !u))) {
    *msg = "q, l or u: null";
    return QPG_ERR_ARG;
  }
  for (int32_t i = 0; i < n; ++i)
    if (!std::isfinite(q[i])) {
      *msg = "q: non-finite value";
      return QPG_ERR_DATA;
    }
  for (int32_t i = 0; i < m; ++i) {
    if (std::isnan(l[i]) || std::isnan(u[i])) {
      *msg = "l or u: NaN";
      return QPG_ERR_DATA;
    }
    if (l[i] > u[i]) {
      *msg = "l > u";
      return QPG_ERR_DATA;
    }
  }
  // full P has at most 2·nnz(triu) entries; B holds full P and Aᵀ
  std::vector<int64_t> p_work((size_t)n + 1, 0);
  parallel_chunks(n, 1 << 14, [&](int64_t, int64_t lo, int64_t hi) {
    for (int64_t j = lo; j < hi; ++j) {
      int64_t e = 0;
      for (int32_t k = Pt->colptr[j]; k < Pt->colptr[j + 1]; ++k) e += (Pt->rowidx[k] == j) ? 1 : 2;
      p_work[j + 1] = e;
    }
  });
  for (int32_t j = 0; j < n; ++j) p_work[j + 1] += p_work[j];
  if (p_work[n] + (int64_t)A->nnz > std::numeric_limits<int32_t>::max()) {
    *msg = "nnz(P) + nnz(A) overflows int32";
    return QPG_ERR_SIZE;
  }

  HostProblem& H = *out;
  H.n = n;
  H.m = m;

  // ---- full P in CSR from its upper triangle in CSC (Section 6.2). Visiting the triangle's
  // columns in order emits, for row i, first the entries (i, k < i) and the diagonal (from
  // column i), then (i, j > i) from later columns: each row comes out sorted.
  hvec<int32_t> p_col;
  columns_to_rows(
      n, n, p_work,
      [&](int32_t j, auto&& put) {
        for (int32_t k = Pt->colptr[j]; k < Pt->colptr[j + 1]; ++k) {
          const int32_t i = Pt->rowidx[k];
          const double v = Pt->val[k];
          if (i != j) put(j, i, v);  // (j, i), i < j: lower part of row j
          put(i, j, v);              // (i, j), i ≤ j
        }
      },
      H.p_ptr, p_col, H.p_val);
  H.a_csc_val = A->val;
  H.a_colptr = A->colptr;
  // ---- B = [P | Aᵀ]: row i is row i of the full P, then column i of A (CSC of A = CSR of Aᵀ)
  H.b_ptr.assign(n + 1, 0);
  H.b_split.resize(n);
  for (int32_t i = 0; i < n; ++i)
    H.b_ptr[i + 1] = H.b_ptr[i] + (H.p_ptr[i + 1] - H.p_ptr[i]) + (A->colptr[i + 1] - A->colptr[i]);
  H.b_col.resize(H.b_ptr[n]);
  const std::vector<int64_t> rows = work_cuts(H.b_ptr.data(), n, kWorkParts);
  parallel_chunks(kWorkParts, 1, [&](int64_t t, int64_t, int64_t) {
    for (int64_t i = rows[(size_t)t]; i < rows[(size_t)t + 1]; ++i) {
      int32_t o = H.b_ptr[i];
      for (int32_t k = H.p_ptr[i]; k < H.p_ptr[i + 1]; ++k, ++o) H.b_col[o] = p_col[k];
      H.b_split[i] = o;
      for (int32_t k = A->colptr[i]; k < A->colptr[i + 1]; ++k, ++o) H.b_col[o] = n + A->rowidx[k];
    }
  });

  // ---- q, and the bounds with infinities clamped to ±kInf (Ruiz equilibration, Algorithm 2,
  // runs on the device on these raw values)
  H.qb.assign(q, q + n);
  H.lb.resize(m);
  H.ub.resize(m);
  for (int32_t i = 0; i < m; ++i) {
    H.lb[i] = std::max(l[i], -kInf);
    H.ub[i] = std::min(u[i], kInf);
  }
  // equality rows, for R = diag(ρ_i) (eq. rho_vec)
  if (s->rho_vector) {
    H.eqrow.assign(m, 0);
    for (int32_t i = 0; i < m; ++i) H.eqrow[i] = (l[i] == u[i]) ? 1 : 0;
  }
  double qn = 0.0;
  for (int32_t i = 0; i < n; ++i) qn = std::max(qn, std::fabs(q[i]));
  H.q_norm_unscaled = qn;
  if (with_a) prepare_a(A, out);
  return QPG_OK;
}

}  // namespace qpg

// Defaults of the settings (include/qpg.h lists them with their sources in the paper).
extern "C" int qpg_default_settings(qpg_settings* s) {
  if (!s) return QPG_ERR_ARG;
  std::memset(s, 0, sizeof(*s));
  s->rho = 0.1;
  s->sigma = 1e-6;
  s->alpha = 1.6;
  s->eps_abs = 1e-3;
  s->eps_rel = 1e-3;
  s->max_iter = 100000;
  s->check_every = 5;
  s->rho_update_every = 10;
  s->rho_update_gate = 1.0;
  s->pcg_lambda = 0.15;
  s->pcg_eps_min = 1e-7;
  s->pcg_eps_fixed = 0.0;
  s->pcg_max_iter = 100;
  s->pcg_rel_test = 1;
  s->scaling_iters = 10;
  s->precision = QPG_FP64;
  s->precond = QPG_PRECOND_JACOBI;
  s->device = 0;
  s->stream = nullptr;
  s->verbose = 0;
  s->precond_weights = nullptr;
  s->precond_trial = 1;
  s->spmv_tile_nnz = qpg::kTileNnz;
  s->spmv_plain_nnz = qpg::kPlainNnz;
  s->eps_prim_inf = 1e-4;
  s->eps_dual_inf = 1e-4;
  s->rho_vector = 0;
  s->pcg_eps_schedule = 0;
  s->speculate = 1;
  s->spmv_window_cols = qpg::kWinCols;
  s->spmv_min_seg = qpg::kMinSeg;
  return QPG_OK;
}
