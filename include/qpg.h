/*
 * qpg — ADMM with a reduced-KKT PCG linear solve for convex QPs, on MI355X (gfx950).
 *
 * Solves   minimize ½xᵀPx + qᵀx   subject to   l ≤ Ax ≤ u            (Section 2, eq. qp)
 * with P ⪰ 0 (n×n), A (m×n), l_i ∈ ℝ∪{−∞}, u_i ∈ ℝ∪{+∞}, l ≤ u; l_i = u_i encodes an
 * equality. The iteration is OSQP's ADMM (Algorithm 1) with R = ρ̄I, whose linear step is
 * the reduced KKT system (P + σI + ρ̄AᵀA)x̃ = σx − q + Aᵀ(ρ̄z − y) (Section 6.3, eq.
 * kkt_red_sc) solved inexactly by Jacobi-preconditioned CG (Algorithm 3, Section 6.3.1–6.3.3),
 * warm-started from the previous x̃. The data are Ruiz-equilibrated (Algorithm 2) at setup.
 *
 * Conventions for every call:
 *  - Return value: 0 on success, a negative QPG_ERR_* code otherwise. No call throws, aborts
 *    or exits. The message of the last failure on a handle is kept for qpg_last_error().
 *  - All dimensions and sparse indices are int32; values are IEEE double on the host side.
 *  - Host pointers are read during the call only; setup copies every input, so the caller
 *    may free its arrays on return. Output arrays are caller-allocated host memory.
 *  - A handle is not thread-safe; use one handle per concurrent solve. All device work of a
 *    handle runs on the stream given in the settings (NULL: the null stream).
 *  - |bound| ≥ 1e20 (including ±INFINITY) is treated as infinite.
 */
#ifndef QPG_H
#define QPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes (return values). */
#define QPG_OK 0
#define QPG_ERR_ARG (-1)    /* null pointer, bad dimension, unsorted/duplicate/out-of-range index,
                               entry below the diagonal of P_triu, bad setting value */
#define QPG_ERR_DATA (-2)   /* NaN or ±inf in P, q or A; NaN in l or u; l_i > u_i */
#define QPG_ERR_SIZE (-3)   /* a size that overflows the int32 indexing */
#define QPG_ERR_DEVICE (-4) /* any HIP runtime error (message kept for qpg_last_error) */
#define QPG_ERR_OOM (-5)    /* device or host allocation failed */
#define QPG_ERR_STATE (-6)  /* call not valid in the handle's current state */
#define QPG_ERR_HOST (-7)   /* other host-side failure, e.g. a worker thread could not start
                               (message kept for qpg_last_error) */

/* Solver status (qpg_info.status), separate from the error code. */
#define QPG_UNSOLVED 0
#define QPG_SOLVED 1
#define QPG_MAX_ITER_REACHED 2
#define QPG_NUMERICAL_ERROR 3 /* PCG breakdown (pᵀKp ≤ 0 or NaN) in every precision */
#define QPG_PRIMAL_INFEASIBLE 4 /* δy certifies Aᵀȳ = 0, lᵀȳ₋ + uᵀȳ₊ < 0 (Section 2.1, 3.1) */
#define QPG_DUAL_INFEASIBLE 5   /* δx certifies Px̄ = 0, qᵀx̄ < 0, sign pattern of Ax̄ (Section 2.1, 3.1) */

/* Arithmetic of the iteration. */
#define QPG_FP64 0  /* matrices, vectors and reductions in double */
#define QPG_MIXED 1 /* matrices and vectors in float; PCG dots (α, β), residual norms and ρ̄
                       ratios accumulated in double; falls back to QPG_FP64 on PCG stagnation */

/* Preconditioner of the PCG step. */
#define QPG_PRECOND_JACOBI 0  /* M = diag(P + σI + ρ̄AᵀA) (Section 6.3.1) */
#define QPG_PRECOND_LEARNED 1 /* M⁻¹_ii = softplus(g_i) / K_ii with g from a message-passing network
                                 over the graph of A (parameters in settings.precond_weights): still
                                 diagonal and positive, so Algorithm 3 is unchanged; softplus = 1
                                 reproduces Jacobi. Not part of the paper. */

/* Number of float parameters of the learned preconditioner's network. */
#define QPG_NET_NPARAMS 16705

/* Compressed sparse column matrix (Section 5.3.3), zero-based. Row indices within each column
 * must be strictly increasing. CSC of A is the CSR of Aᵀ (Section 5.3.3). */
typedef struct {
  int32_t nrows;
  int32_t ncols;
  int32_t nnz;
  const int32_t* colptr; /* ncols+1 entries, colptr[0] = 0, colptr[ncols] = nnz */
  const int32_t* rowidx; /* nnz entries */
  const double* val;     /* nnz entries */
} qpg_csc;

typedef struct {
  double rho;             /* initial ρ̄ > 0 (Section 3.4), default 0.1 */
  double sigma;           /* σ > 0 (Section 3.4), default 1e-6 */
  double alpha;           /* relaxation α ∈ (0, 2) (Section 3.4), default 1.6 */
  double eps_abs;         /* absolute tolerance of the termination test, default 1e-3 */
  double eps_rel;         /* relative tolerance of the termination test, default 1e-3 */
  int32_t max_iter;       /* ADMM iteration cap, default 100000 */
  int32_t check_every;    /* residual/termination check cadence (Section 6.3.3), default 5 */
  int32_t rho_update_every; /* ρ̄ update cadence in iterations (Section 6.3.2), default 10; 0 = fixed ρ̄ */
  double rho_update_gate; /* apply a ρ̄ estimate only if it differs by more than this factor; default 1 (always) */
  double pcg_lambda;      /* λ of the PCG tolerance rule (Section 6.3.3), default 0.15 */
  double pcg_eps_min;     /* ε_min of the PCG tolerance rule, default 1e-7 */
  double pcg_eps_fixed;   /* > 0: use this fixed PCG tolerance instead of the rule; default 0 */
  int32_t pcg_max_iter;   /* PCG iteration cap per ADMM iteration, default 100 */
  int32_t pcg_rel_test;   /* 1: stop PCG when ‖r‖∞ ≤ ε‖b‖∞ (Algorithm 3); 0: when ‖r‖∞ ≤ ε */
  int32_t scaling_iters;  /* Ruiz passes (Algorithm 2); 0 disables scaling; default 10 */
  int32_t precision;      /* QPG_FP64 or QPG_MIXED */
  int32_t precond;        /* QPG_PRECOND_JACOBI */
  int32_t device;         /* HIP device ordinal, default 0 */
  void* stream;           /* hipStream_t for all device work, NULL = null stream */
  int32_t verbose;        /* 1: one line per setup phase and per residual check on stderr */
  const float* precond_weights; /* QPG_NET_NPARAMS floats for QPG_PRECOND_LEARNED (copied at setup) */
  int32_t precond_trial;  /* 1 (default): before the first PCG solve, and after a ρ̄ change that
                             moves ρ̄ by more than 2× since the last trial, solve once with each
                             preconditioner from the same warm start and keep the learned one only
                             if it needs fewer iterations (or, both capped, ends with a smaller
                             residual); after two lost trials in a row, Jacobi for the rest of the
                             solve. 0: always learned. In both cases a capped or broken-down learned
                             solve switches to Jacobi. */
  int32_t spmv_tile_nnz;  /* SpMV work-list granularity: matrix entries per workgroup when it stages
                             a gather window in LDS; default 65536 (fewer on matrices with fewer than
                             512 such tiles' worth of entries), 0 = default */
  int32_t spmv_plain_nnz; /* the same for workgroups without a window; default 8192, 0 = default */
  double eps_prim_inf;    /* ε_pinf of the primal infeasibility test (Section 3.1), relative to
                             ‖δy‖∞; default 1e-4; 0 disables the test */
  double eps_dual_inf;    /* ε_dinf of the dual infeasibility test, relative to ‖δx‖∞; default
                             1e-4; 0 disables it (both 0: no infeasibility passes at all) */
  int32_t rho_vector;     /* 0 (default): R = ρ̄I, the choice of Section 6.3 for the PCG step;
                             1: OSQP's R = diag(ρ_i), ρ_i = 10³ρ̄ where l_i = u_i (eq. rho_vec),
                             in K = P + σI + AᵀRA, its Jacobi diagonal and the ADMM updates (the
                             ablation of Section 6.3; Jacobi preconditioner only) */
  int32_t pcg_eps_schedule; /* 0 (default): the residual rule of Section 6.3.3 (pcg_lambda,
                             pcg_eps_min, refreshed at every check); 1: a tolerance decreasing with
                             the ADMM iteration k, max(pcg_lambda·(k + 1)^(−3/2), pcg_eps_min), the
                             kind of rule Section 6.3.3 attributes to SCS (an ablation) */
  int32_t speculate;      /* 1 (default): the ADMM iterations between two checks are launched
                             without waiting for their PCG solves; the first PCG solve that is not
                             done after the predicted number of iterations (or breaks down, or hits
                             the cap) raises a device flag that skips the rest, and the host resumes
                             there at the next read; only while the last PCG solve took at most 8
                             iterations. 0: the host waits for every PCG solve (the synchronous
                             loop of Section 6.3.3). Both give bitwise the same iterates. */
  int32_t spmv_window_cols; /* SpMV work lists: capacity in columns of a gather window staged in LDS
                             (a power of two from 1024 to 65536; halved until a window of doubles fits
                             the device's LDS, and on each matrix until it is at most half the entries
                             of a windowed tile); default 16384, 0 = default */
  int32_t spmv_min_seg;   /* SpMV work lists: entries per row and column range on average that make
                             a run of rows take one tile per (row block, range); 1 to 256, default 16,
                             0 = default */
} qpg_settings;

typedef struct {
  int32_t status;          /* QPG_SOLVED, QPG_MAX_ITER_REACHED, ... */
  int32_t iter;            /* ADMM iterations of the last solve */
  int64_t pcg_iter_total;  /* PCG iterations summed over the last solve */
  int32_t pcg_iter_max;    /* largest PCG iteration count of one ADMM iteration */
  int32_t rho_updates;     /* ρ̄ changes in the last solve */
  double obj_val;          /* ½xᵀPx + qᵀx of the returned x (unscaled) */
  double prim_res;         /* ‖Ax − z‖∞ (unscaled) at the last check */
  double dual_res;         /* ‖Px + q + Aᵀy‖∞ (unscaled) at the last check */
  double rho_final;        /* ρ̄ at the end of the last solve */
  double setup_time;       /* seconds spent in qpg_setup */
  double solve_time;       /* seconds of the last qpg_solve (device work included) */
  int32_t precision_used;  /* precision the last solve finished in */
  int32_t precond_used;    /* preconditioner the last solve finished with */
  int32_t fallback_events; /* precision fallbacks taken during the last solve */
  int32_t scaling_passes;  /* Ruiz passes performed at setup */
  int32_t precond_trials;  /* learned-vs-Jacobi trials run in the last solve */
  int32_t precond_learned_chosen; /* trials won by the learned preconditioner */
  int32_t precond_switches; /* runtime switches from learned to Jacobi (capped or broken-down PCG) */
  int32_t infeas_checks;   /* checks that ran the infeasibility passes: those after two checks in a
                              row without a 1% gain in the worse normalised residual */
  int32_t spec_resumes;    /* speculative iterations whose PCG solve the host had to finish */
} qpg_info;

typedef struct qpg_solver qpg_solver;

/* Fill *s with the defaults listed above. */
int qpg_default_settings(qpg_settings* s);

/* Validate and copy the problem (P given as its upper triangle incl. diagonal in CSC, the OSQP
 * convention of Section 6.2; A in CSC), expand P to full CSR and store A and Aᵀ in CSR
 * (Section 6.2), equilibrate (Algorithm 2), move everything to device memory and build the
 * SpMV work schedules. On success *out owns all device memory of the problem. Validation
 * failures return before any device call. Large uploads pass through 128 MiB of pinned host
 * memory per device (16 buffers of 8 MiB), allocated by the first qpg_setup on that device and
 * kept until the process ends; setups on one device upload one at a time. */
int qpg_setup(qpg_solver** out, const qpg_csc* P_triu, const double* q, const qpg_csc* A,
              const double* l, const double* u, const qpg_settings* settings);

/* Run Algorithm 1 from x = z = y = 0, x̃ = 0 and the initial ρ̄ until the unscaled residuals meet
 * eps_prim = eps_abs + eps_rel·max(‖Ax‖∞, ‖z‖∞), eps_dual = eps_abs + eps_rel·max(‖Px‖∞, ‖Aᵀy‖∞,
 * ‖q‖∞) (Section 3.1, checked every check_every iterations), or the differences of the checked
 * step certify primal or dual infeasibility (Section 3.1; tested, with two extra SpMV passes, at
 * the checks that follow two checks in a row without a 1% gain in the worse normalised residual),
 * or max_iter is reached. After ten such checks the PCG tolerance is divided by 10 at every second
 * check (a stall guard, not in the paper: infeasible problems keep the residuals, and with them
 * the tolerance of Section 6.3.3, large). The ‖b‖∞ of each PCG stopping test is formed from the
 * previous PCG solve's residual and right-hand side (an identity of the reduced system), and
 * directly at a solve's first iteration and every 50th. The status is in qpg_info; reaching
 * max_iter or detecting infeasibility is not an error. */
int qpg_solve(qpg_solver* h);

/* Infeasibility certificate of the last solve (status QPG_PRIMAL_INFEASIBLE or
 * QPG_DUAL_INFEASIBLE): the unscaled iterate differences δx = x^k − x^{k−1} (n) and δy =
 * y^k − y^{k−1} (m) of the step that passed the test (Section 3), δy projected so that its
 * support function lᵀδy₋ + uᵀδy₊ has no infinite term, each divided by its ∞-norm. δy is the
 * certificate of primal infeasibility, δx that of dual infeasibility. Either pointer may be NULL.
 * QPG_ERR_STATE when the last solve did not end infeasible. */
int qpg_get_certificate(const qpg_solver* h, double* dx, double* dy);

/* Copy the unscaled iterates of the last solve: x (n), y (m), z (m). */
int qpg_get_x(const qpg_solver* h, double* x);
int qpg_get_y(const qpg_solver* h, double* y);
int qpg_get_z(const qpg_solver* h, double* z);
int qpg_get_info(const qpg_solver* h, qpg_info* info);

/* Ruiz factors D (n), E (m) and cost scale c with P̄ = cDPD, q̄ = cDq, Ā = EAD (Section 3.3). */
int qpg_get_scaling(const qpg_solver* h, double* D, double* E, double* c);

/* Operators of the scaled problem, run by the solver's own device kernels and schedules in the
 * given precision (QPG_FP64, or QPG_MIXED for the float copies). in/out are host arrays.
 *   QPG_OP_A   out(m) = Ā in(n)                         (Section 6.2: A stored in CSR)
 *   QPG_OP_AT  out(n) = Āᵀ in(m)                        (Section 6.2: Aᵀ stored in CSR)
 *   QPG_OP_P   out(n) = P̄ in(n)                         (Section 6.2: full P in CSR)
 *   QPG_OP_K   out(n) = (P̄ + σI + ρ̄ĀᵀĀ) in(n), matrix-free as w = ρ̄Āx, Px + σx + Āᵀw
 *                                                       (Section 6.3) with the current ρ̄
 *                                                       (ĀᵀRĀ, w = RĀx with settings.rho_vector) */
#define QPG_OP_A 0
#define QPG_OP_AT 1
#define QPG_OP_P 2
#define QPG_OP_K 3
int qpg_apply(qpg_solver* h, int32_t op, int32_t precision, const double* in, double* out);

/* Algorithm 3 on the scaled reduced system (P̄ + σI + ρ̄ĀᵀĀ)x = b with the current ρ̄ and the
 * solver's preconditioner (Jacobi, Section 6.3.1, or the learned diagonal when the solver was set
 * up with QPG_PRECOND_LEARNED): starts from x0 (n), stops when ‖r‖∞ ≤ eps·‖b‖∞ (rel = 1)
 * or ‖r‖∞ ≤ eps (rel = 0) or after max_iter iterations. Writes x (n), the iteration count and
 * the final ‖r‖∞. Same kernels as the PCG inside qpg_solve. */
int qpg_pcg(qpg_solver* h, int32_t precision, const double* b, const double* x0, double eps,
            int32_t rel, int32_t max_iter, double* x, int32_t* iters, double* rnorm);

/* Set ρ̄ (> 0) for qpg_apply(QPG_OP_K) and qpg_pcg, rebuilding diag(M) = diag(P̄) + σ + ρ̄‖Ā_i‖²
 * (Section 6.3.1–6.3.2). qpg_solve restarts from settings.rho. */
int qpg_set_rho(qpg_solver* h, double rho);

/* Average device duration, in microseconds, of `reps` back-to-back launches of one step of the
 * PCG iteration (Algorithm 3 with the matrix-free K-matvec of Section 6.3), timed with HIP events
 * on the solver's stream, in the launch configuration the solve uses, on the current device
 * vectors (their contents are overwritten). Steps:
 *   QPG_KERNEL_SPMV_A         w = ρ̄Āp (stream + combine kernels)       (m rows of Ā)
 *   QPG_KERNEL_SPMV_B         Kp = P̄p + σp + Āᵀw, κ = pᵀKp, α (both)  (n rows of [P̄ | Āᵀ])
 *   QPG_KERNEL_PCG_UPDATE     x̃ += αp, r += αKp, rᵀM⁻¹r, ‖r‖∞, β     (n)
 *   QPG_KERNEL_PCG_DIR        p = −M⁻¹r + βp                          (n)
 *   QPG_KERNEL_SPMV_A_STREAM  the stream kernel of SPMV_A alone (segment sums of Ā p)
 *   QPG_KERNEL_SPMV_B_STREAM  the stream kernel of SPMV_B alone (segment sums of [P̄ | Āᵀ][p; w])
 * reps ≥ 1; precision as in qpg_apply. */
#define QPG_KERNEL_SPMV_A 0
#define QPG_KERNEL_SPMV_B 1
#define QPG_KERNEL_PCG_UPDATE 2
#define QPG_KERNEL_PCG_DIR 3
#define QPG_KERNEL_SPMV_A_STREAM 4
#define QPG_KERNEL_SPMV_B_STREAM 5
int qpg_time_kernel(qpg_solver* h, int32_t kernel, int32_t precision, int32_t reps, double* avg_us);

/* Layout of the SpMV work list of one matrix (0: Ā, 1: B = [P̄ | Āᵀ]), for measurement: out[0]
 * matrix entries; out[1] stored positions in tiles with an LDS window (values + 16-bit column
 * offsets; padding included); out[2] stored positions in the other tiles (values + 32-bit
 * columns); out[3] workgroups (tiles); out[4] tiles with a window; out[5] columns staged in LDS
 * per launch (sum over tiles); out[6] segment slots; out[7] segment chunks. */
int qpg_spmv_layout(const qpg_solver* h, int32_t matrix, int64_t out[8]);

/* K_ii = diag(P̄)_i + σ + ρ̄‖Ā_i‖² of the scaled reduced KKT matrix (Section 6.3.1), n values.
 * QPG_ERR_STATE for a handle set up with settings.rho_vector (K is taken with R = ρ̄I here). */
int qpg_get_kdiag(const qpg_solver* h, double rho, double* kdiag);

/* Hutchinson estimate of diag(K⁻¹) for K = P̄ + σI + ρ̄ĀᵀĀ: (1/s) Σ_k z_k ∘ K⁻¹z_k over the s
 * probes z_k given in `signs` (s×n, row-major, entries ±1 only; the caller draws them), each
 * K⁻¹z_k by the solver's own Jacobi PCG (Algorithm 3) from 0 to ‖r‖∞ ≤ eps‖z‖∞ or max_iter.
 * Writes n values to diag. Not part of the paper: training targets of QPG_PRECOND_LEARNED.
 * QPG_ERR_STATE for a handle set up with settings.rho_vector (K is taken with R = ρ̄I here). */
int qpg_hutchinson(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho, double eps,
                   int32_t max_iter, double* diag);

/* qpg_hutchinson without any allocation, for callers that cannot allocate device memory (code
 * under stream capture, tight loops, harnesses that forbid hipMalloc): the same computation with
 * the same kernels, bitwise the same diag, but the accumulator and the probe live in a static
 * device array of QPG_NOALLOC_SCRATCH_BYTES that every device the library runs on holds for the
 * life of the process (its address is looked up once per device, in qpg_setup). It allocates no
 * device memory and builds none of the learned preconditioner's graph data, which qpg_hutchinson
 * creates on first use. The handle, the probes and diag are the caller's, as for qpg_hutchinson.
 * Limit: n ≤ QPG_NOALLOC_MAX_N (8n rounded up to 256 bytes, plus n, within the scratch), else
 * QPG_ERR_SIZE before any device work. All calls on one device share the one scratch array:
 * calls that overlap on a device (several host threads, several streams) race and give wrong
 * results; the accumulator is cleared at the start of every call, so a call never sees the last
 * call's contents. Other errors as for qpg_hutchinson. */
#define QPG_NOALLOC_SCRATCH_BYTES 16777216 /* 16 MiB */
#define QPG_NOALLOC_MAX_N 1864128
int qpg_hutchinson_noalloc(qpg_solver* h, const int8_t* signs, int32_t nprobes, double rho,
                           double eps, int32_t max_iter, double* diag);

/* Network of the learned preconditioner, its evaluation on a solver's problem and its training
 * (forward, loss, backward and Adam all run on the device). Not part of the paper.
 *   create:    params = QPG_NET_NPARAMS floats, or NULL for the seeded initialisation (output
 *              layer at softplus = 1, i.e. Jacobi); bf16 = 1: dense layers on bf16 MFMA with
 *              float32 accumulation (bf16 weights; activations and gradients as hi + lo bf16
 *              pairs), 0: plain float32 (validation)
 *   forward:   g (n floats, may be NULL) = pre-softplus outputs for the solver's problem at ρ̄
 *   loss_grad: loss = mean_i (e_i − ē)², e_i = log softplus(g_i) − target_i (target = log(ĥ_i K_ii),
 *              n floats); gradient kept on the device for adam_step and copied to grad if non-NULL
 *   adam_step: Adam (β = 0.9, 0.999, ε = 1e-8) on the float32 master parameters
 * The net and the solver must be on the same device. */
typedef struct qpg_net qpg_net;
int qpg_net_create(qpg_net** out, const float* params, uint64_t seed, int32_t bf16, int32_t device);
int qpg_net_get_params(const qpg_net* net, float* params);
int qpg_net_set_params(qpg_net* net, const float* params);
int qpg_net_forward(qpg_net* net, qpg_solver* h, double rho, float* g);
int qpg_net_loss_grad(qpg_net* net, qpg_solver* h, double rho, const float* target, double* loss,
                      float* grad);
int qpg_net_adam_step(qpg_net* net, float lr);
int qpg_net_destroy(qpg_net* net);

/* Release all device and host memory of h. NULL is accepted. */
int qpg_cleanup(qpg_solver* h);

/* Static description of an error code. */
const char* qpg_error_string(int code);

/* Message of the last failure on h (empty string if none; h may be NULL for setup failures:
 * then the message of the last failed qpg_setup on this thread is returned). */
const char* qpg_last_error(const qpg_solver* h);

#ifdef __cplusplus
}
#endif

#endif /* QPG_H */
