// Host-side preparation: input validation, CSC → CSR conversions, modified Ruiz
// equilibration (Algorithm 2) and the SpMV work schedule.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>

#include "qpg_internal.hpp"

namespace qpg {

namespace {

// Structural checks of a CSC matrix; `upper` additionally requires row ≤ column.
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
  for (int32_t j = 0; j < ncols; ++j) {
    int32_t a = M->colptr[j], b = M->colptr[j + 1];
    if (b < a) {
      *msg = std::string(name) + ": colptr not monotone";
      return QPG_ERR_ARG;
    }
    for (int32_t k = a; k < b; ++k) {
      int32_t i = M->rowidx[k];
      if (i < 0 || i >= nrows) {
        std::snprintf(buf, sizeof(buf), "%s: row index %d out of range in column %d", name, (int)i,
                      (int)j);
        *msg = buf;
        return QPG_ERR_ARG;
      }
      if (k > a && i <= M->rowidx[k - 1]) {
        std::snprintf(buf, sizeof(buf), "%s: row indices of column %d not strictly increasing",
                      name, (int)j);
        *msg = buf;
        return QPG_ERR_ARG;
      }
      if (upper && i > j) {
        std::snprintf(buf, sizeof(buf), "%s: entry (%d,%d) below the diagonal", name, (int)i,
                      (int)j);
        *msg = buf;
        return QPG_ERR_ARG;
      }
    }
  }
  for (int32_t k = 0; k < M->nnz; ++k) {
    if (!std::isfinite(M->val[k])) {
      *msg = std::string(name) + ": non-finite value";
      return QPG_ERR_DATA;
    }
  }
  return QPG_OK;
}

double guard_norm(double v) {
  // A vanishing norm (empty column or row) leaves its scaling at 1; large norms are capped.
  if (!(v >= 1e-4)) return 1.0;
  return std::min(v, 1e4);
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
            s->spmv_tile_nnz >= 0 && s->spmv_plain_nnz >= 0;
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

int prepare(const qpg_csc* Pt, const double* q, const qpg_csc* A, const double* l,
            const double* u, const qpg_settings* s, HostProblem* out, std::string* msg) {
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
  int64_t nnzP_full = 0;
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = Pt->colptr[j]; k < Pt->colptr[j + 1]; ++k)
      nnzP_full += (Pt->rowidx[k] == j) ? 1 : 2;
  if (nnzP_full + (int64_t)A->nnz > std::numeric_limits<int32_t>::max()) {
    *msg = "nnz(P) + nnz(A) overflows int32";
    return QPG_ERR_SIZE;
  }

  HostProblem& H = *out;
  H.n = n;
  H.m = m;

  // ---- full P in CSR from its upper triangle in CSC (Section 6.2). Visiting the triangle's
  // columns in order emits, for row i, first the entries (i, k < i) and the diagonal (from
  // column i), then (i, j > i) from later columns: each row comes out sorted.
  std::vector<int32_t> p_ptr(n + 1, 0);
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = Pt->colptr[j]; k < Pt->colptr[j + 1]; ++k) {
      int32_t i = Pt->rowidx[k];
      p_ptr[i + 1]++;
      if (i != j) p_ptr[j + 1]++;
    }
  for (int32_t i = 0; i < n; ++i) p_ptr[i + 1] += p_ptr[i];
  std::vector<int32_t> p_col(p_ptr[n]);
  std::vector<double> p_val(p_ptr[n]);
  {
    std::vector<int32_t> next(p_ptr.begin(), p_ptr.end() - 1);
    for (int32_t j = 0; j < n; ++j)
      for (int32_t k = Pt->colptr[j]; k < Pt->colptr[j + 1]; ++k) {
        int32_t i = Pt->rowidx[k];
        double v = Pt->val[k];
        if (i != j) {
          p_col[next[j]] = i;
          p_val[next[j]++] = v;  // (j, i), i < j: lower part of row j
        }
        p_col[next[i]] = j;
        p_val[next[i]++] = v;  // (i, j), i ≤ j
      }
  }
  // ---- A in CSR (counting sort over the CSC columns keeps each row's columns sorted)
  H.a_ptr.assign(m + 1, 0);
  for (int32_t k = 0; k < A->nnz; ++k) H.a_ptr[A->rowidx[k] + 1]++;
  for (int32_t i = 0; i < m; ++i) H.a_ptr[i + 1] += H.a_ptr[i];
  H.a_col.resize(A->nnz);
  std::vector<double> a_raw(A->nnz);
  {
    std::vector<int32_t> next(H.a_ptr.begin(), H.a_ptr.end() - 1);
    for (int32_t j = 0; j < n; ++j)
      for (int32_t k = A->colptr[j]; k < A->colptr[j + 1]; ++k) {
        int32_t i = A->rowidx[k];
        H.a_col[next[i]] = j;
        a_raw[next[i]++] = A->val[k];
      }
  }
  std::vector<double> at_raw(A->val, A->val + A->nnz);  // CSC of A = CSR of Aᵀ

  // ---- modified Ruiz equilibration (Algorithm 2), applied incrementally to the working copies.
  // Readings: P̄ ← c·DPD (so that P̄ = cDPD holds after every pass); stop after a pass whose δ
  // satisfies ‖1 − δ‖∞ ≤ 1e-3, at most scaling_iters passes; norms below 1e-4 count as 1 and
  // are capped at 1e4 (also for the denominator of γ).
  std::vector<double>& D = H.D;
  std::vector<double>& E = H.E;
  D.assign(n, 1.0);
  E.assign(m, 1.0);
  H.qb.assign(q, q + n);
  double c = 1.0;
  H.scaling_passes = 0;
  std::vector<double> dD(n), dE(m), nx(n), nz(m);
  for (int32_t pass = 0; pass < s->scaling_iters; ++pass) {
    H.scaling_passes++;
    // column ∞-norms of M = [P̄ Āᵀ; Ā 0]: column j ≤ n is column j of P̄ (= row j) and of Ā
    for (int32_t j = 0; j < n; ++j) {
      double mx = 0.0;
      for (int32_t k = p_ptr[j]; k < p_ptr[j + 1]; ++k) mx = std::max(mx, std::fabs(p_val[k]));
      for (int32_t k = A->colptr[j]; k < A->colptr[j + 1]; ++k)
        mx = std::max(mx, std::fabs(at_raw[k]));
      nx[j] = mx;
    }
    for (int32_t i = 0; i < m; ++i) {
      double mx = 0.0;
      for (int32_t k = H.a_ptr[i]; k < H.a_ptr[i + 1]; ++k) mx = std::max(mx, std::fabs(a_raw[k]));
      nz[i] = mx;
    }
    double dev = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      dD[j] = 1.0 / std::sqrt(guard_norm(nx[j]));
      dev = std::max(dev, std::fabs(1.0 - dD[j]));
      D[j] *= dD[j];
    }
    for (int32_t i = 0; i < m; ++i) {
      dE[i] = 1.0 / std::sqrt(guard_norm(nz[i]));
      dev = std::max(dev, std::fabs(1.0 - dE[i]));
      E[i] *= dE[i];
    }
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = p_ptr[i]; k < p_ptr[i + 1]; ++k) p_val[k] = (p_val[k] * dD[i]) * dD[p_col[k]];
    for (int32_t i = 0; i < m; ++i)
      for (int32_t k = H.a_ptr[i]; k < H.a_ptr[i + 1]; ++k)
        a_raw[k] = (a_raw[k] * dE[i]) * dD[H.a_col[k]];
    for (int32_t j = 0; j < n; ++j)
      for (int32_t k = A->colptr[j]; k < A->colptr[j + 1]; ++k)
        at_raw[k] = (at_raw[k] * dE[A->rowidx[k]]) * dD[j];
    double qmax = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      H.qb[j] *= dD[j];
      qmax = std::max(qmax, std::fabs(H.qb[j]));
    }
    // cost scaling γ = 1 / max(mean_j ‖P̄_j‖∞, ‖q̄‖∞)
    double mean = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      double mx = 0.0;
      for (int32_t k = p_ptr[j]; k < p_ptr[j + 1]; ++k) mx = std::max(mx, std::fabs(p_val[k]));
      mean += mx;
    }
    mean /= (double)n;
    double gamma = 1.0 / guard_norm(std::max(mean, qmax));
    for (auto& v : p_val) v *= gamma;
    for (auto& v : H.qb) v *= gamma;
    c *= gamma;
    if (dev <= 1e-3) break;
  }
  H.c = c;

  // ---- bounds: clamp infinities, then scale l̄ = El, ū = Eu
  H.lb.resize(m);
  H.ub.resize(m);
  for (int32_t i = 0; i < m; ++i) {
    double li = std::max(l[i], -kInf), ui = std::min(u[i], kInf);
    H.lb[i] = E[i] * li;
    H.ub[i] = E[i] * ui;
  }

  // ---- B = [P̄ | Āᵀ]
  H.b_ptr.assign(n + 1, 0);
  H.b_split.resize(n);
  for (int32_t i = 0; i < n; ++i)
    H.b_ptr[i + 1] = H.b_ptr[i] + (p_ptr[i + 1] - p_ptr[i]) + (A->colptr[i + 1] - A->colptr[i]);
  H.b_col.resize(H.b_ptr[n]);
  H.b_val.resize(H.b_ptr[n]);
  H.diagP.assign(n, 0.0);
  H.colsq.assign(n, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    int32_t o = H.b_ptr[i];
    for (int32_t k = p_ptr[i]; k < p_ptr[i + 1]; ++k, ++o) {
      H.b_col[o] = p_col[k];
      H.b_val[o] = p_val[k];
      if (p_col[k] == i) H.diagP[i] = p_val[k];
    }
    H.b_split[i] = o;
    double sq = 0.0;
    for (int32_t k = A->colptr[i]; k < A->colptr[i + 1]; ++k, ++o) {
      H.b_col[o] = n + A->rowidx[k];
      H.b_val[o] = at_raw[k];
      sq += at_raw[k] * at_raw[k];
    }
    H.colsq[i] = sq;
  }
  H.a_val = std::move(a_raw);
  double qn = 0.0;
  for (int32_t i = 0; i < n; ++i) qn = std::max(qn, std::fabs(q[i]));
  H.q_norm_unscaled = qn;
  return QPG_OK;
}

}  // namespace qpg
