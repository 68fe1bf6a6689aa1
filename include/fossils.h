/*
 * fossils.h -- C ABI of the MI355X (gfx950) FOSSILS / SPIR least-squares library.
 *
 * Solves the overdetermined least-squares problem  x = argmin_x ||b - A x||_2  with A m x n,
 * m >= n (Epperly, Meier, Nakatsukasa, "Fast randomized least-squares solvers can be just as
 * accurate and stable as classical direct solvers", Section 1, eq:ls), with the two backward
 * stable randomized solvers of that paper:
 *   FOSSILS  -- Algorithm 1 with the Polyak heavy-ball inner solver (Algorithms 2, 4 and 5);
 *   SPIR     -- Algorithm 1 with conjugate gradient on the preconditioned normal equations
 *               (Algorithm 3).
 * Both sketch [A b] with a sparse sign embedding (Section 4.2), factor the sketch, start from the
 * sketch-and-solve solution (eq:sketch-and-solve-2.3) and run exactly two refinement steps
 * (eq:precond-normal-RHSc) with the adaptive stopping rules of Section 4.2 (first step: size of
 * the update; second step: the sketched Karlson-Walden backward-error estimate, eq:sketched-kw).
 *
 * Conventions for every entry point
 *   - Matrices are column-major with a leading dimension (lda >= rows).  Arrays named A, b, x, Y,
 *     R, V, z, v, g are DEVICE pointers (HIP device memory of the context's device) unless the
 *     name ends in _host.  The caller owns them; they must stay valid until the call returns.
 *     The library never writes A or b (column scaling is applied to vectors, not to A).
 *   - Work is enqueued on the context's HIP stream; every call below is synchronous with respect
 *     to that stream on return (results are in place when the call returns).
 *   - Return codes: FS_OK (0), positive warnings (the result is valid), negative errors (nothing
 *     was written to the outputs).  Argument validation happens before any device work.
 *   - A context is used by one host thread at a time.
 */
#ifndef FOSSILS_H
#define FOSSILS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fs_status {
  FS_OK = 0,
  FS_WARN_RANK_DEFICIENT = 1,  /* condest > 1/(30u): truncated SVD preconditioner used (Alg 4) */
  FS_WARN_NOT_CONVERGED = 2,   /* second-step rule not met within max_inner iterations */
  FS_ERR_INVALID_ARG = -1,     /* null pointer or invalid option value */
  FS_ERR_SHAPE = -2,           /* m < n, n < 1, d < n, zeta < 1, zeta > d, zeta > 64, lda < m, ... */
  FS_ERR_NOMEM = -3,           /* device allocation failed */
  FS_ERR_DEVICE = -4,          /* a HIP call failed (see fs_last_error_detail) */
  FS_ERR_NONFINITE = -5,       /* A or b holds NaN or Inf */
  FS_ERR_TOO_LARGE = -6,       /* size beyond what the library supports (n > 15000, d > 65536, a server's
                                  budget, the no-alloc array), or finite entries of A or b so large that
                                  their column norms overflow FP64 (column scaling impossible) */
  FS_ERR_UNKNOWN_TICKET = -7,  /* batched_poll / fs_server_ticket_times: no such ticket */
  FS_ERR_UNSUPPORTED = -8,
  /* not statuses: they make every 32-bit value a valid fs_status (fs_status_string of any int) */
  FS_STATUS_RANGE_MIN_ = -2147483647 - 1,
  FS_STATUS_RANGE_MAX_ = 2147483647
} fs_status;

typedef struct fs_context_s* fs_context;
typedef struct fs_sketch_s* fs_sketch;
typedef struct fs_server_s* fs_server;

enum { FS_PRECOND_QR = 0, FS_PRECOND_SVD = 1 };
enum { FS_FP64 = 0, FS_MIXED = 1 };
enum { FS_INIT_SKETCH = 0, FS_INIT_ZERO = 1 };
/* bits of fs_info.flags */
enum {
  FS_FLAG_RANK_DEFICIENT = 1,
  FS_FLAG_NOT_CONVERGED = 2,
  FS_FLAG_FP64_SKETCH = 4,        /* mixed form: the sketch was redone in FP64 */
  FS_FLAG_EARLY_SECOND_STEP = 8,  /* overlap_svd: the second step started before the SVD of R finished */
  FS_FLAG_SVD_ABANDONED = 16      /* ... and met its rule through ||R^{-T} g|| before the SVD was needed:
                                     the SVD was stopped, normest and condest are lower bounds */
};

/* Solver options (Section 4.2 and Algorithm 4).  Fill with fs_options_default. */
typedef struct fs_options {
  int32_t d;              /* sketch rows; Alg 4 uses 12 n */
  int32_t zeta;           /* nonzeros per column of S; Alg 4 uses 8 (1..64 supported) */
  uint64_t seed;          /* seed of the sketch's counter-based generator */
  double eta;             /* distortion estimate; <= 0 means sqrt(n/d) (Section 4.2) */
  double eta_factor;      /* multiplies eta; 1.1 is the paper's conservative choice */
  double gamma, rho;      /* first-step rule constants; Alg 4 uses 10 and 0.4 */
  int32_t kw_every;       /* second-step sketched-KW cadence; 5 in Section 4.2 */
  int32_t max_inner;      /* iteration cap per refinement step; 100 in Alg 4 */
  double tau_factor;      /* rank truncation at tau = tau_factor * u; 30 in Alg 4 */
  int32_t column_scaling; /* 1: unit-norm columns (Alg 4, first statement) */
  int32_t precond;        /* FS_PRECOND_QR: P = R^{-1} by substitution; FS_PRECOND_SVD: P = V Sigma^{-1} */
  int32_t fixed_q;        /* 0: adaptive stopping; q > 0: Algorithm 2 with q heavy-ball steps;
                             -1: q_0 of Theorem 7.1 (eq:iterations) with kappa = condest */
  int32_t steps;          /* refinement steps: 2 (the method) or 1 ("one step" variant) */
  int32_t precision;      /* FS_FP64, or FS_MIXED: FP32 sketch (see fossils_solve_mixed) */
  int32_t max_sweeps;     /* Jacobi sweep cap of the SVD of R */
  int32_t init;           /* FS_INIT_SKETCH: x_0 = sketch-and-solve (Alg 4); FS_INIT_ZERO: x_0 = 0 (the
                             zero start of plain sketch-and-precondition, for the Section 5.1 comparisons) */
  int32_t overlap_svd;    /* 1 (P = V Sigma^{-1}, adaptive FOSSILS or CG-SPIR): the SVD of R runs on a
                             second stream while the refinement iterates with P = R^{-1} (the same
                             preconditioned system up to an orthogonal change of variables; R^{-1} is
                             formed once after the QR, see fs_triangular_inverse, and applied as a
                             product; the workspace holds 2 n^2 doubles more for it).  Until the
                             SVD is done the first-step rule uses lower bounds of normest and condest
                             (diag(R), power and inverse iteration): if the SVD arrives first, the step is
                             cut back to the iteration where the true rule stops; if the step stops on
                             the bounds first, the second step starts at once with P = R^{-1}, its KW
                             checkpoints recorded and evaluated in order once Sigma and V exist (flag
                             FS_FLAG_EARLY_SECOND_STEP); a checkpoint where even the upper bound
                             theta ||R^{-T} g|| / sqrt(1 + theta^2 ||x||^2) of the sketched KW estimate
                             meets the rule (times 1.25, where n u condest <= 0.1) ends the step at once
                             and stops the SVD (FS_FLAG_SVD_ABANDONED).  Falls back to the serial order when R turns out
                             numerically rank deficient; not used when the SVD's work-groups would hold
                             more than half of the compute units (n above ~1500 on 256 compute units). */
  int32_t graph_sweeps;   /* 1: the inner iterations run as a captured HIP graph of kw_every iterations,
                             replayed until the device-side stop flag is set (one launch and one
                             host poll per kw_every iterations); 0: kernel-by-kernel launches */
  int32_t overlap_pass_groups; /* work-groups of each pass over A in the first step while the SVD runs
                             beside it (overlap_svd); 0: the compute units the SVD's work-groups leave
                             free (rounded down to a multiple of 8), so that every pass work-group is
                             resident at once; other passes take one per compute unit */
} fs_options;

/* Per-solve report. */
typedef struct fs_info {
  int32_t iters[2];       /* inner iterations of the two refinement steps */
  int32_t flags;          /* FS_FLAG_*: rank deficient, not converged, FP64 sketch (mixed form), early
                             second step (overlap_svd) */
  int32_t rank;           /* rank of the preconditioner (n unless truncated) */
  double be_sk;           /* last sketched KW estimate of the scaled problem (absolute) */
  double normest;         /* sigma_max of the sketch */
  double condest;         /* sigma_max / sigma_min of the sketch */
  double cnorm[2];        /* ||c_i|| at the start of each refinement step */
  int32_t svd_sweeps;     /* Jacobi sweeps used */
  int32_t kw_evals;       /* sketched-KW evaluations */
  double phase_ms[6];     /* sketch, QR, SVD, init (x0 + first residual), step 0, step 1 */
} fs_info;

/* Human-readable name of a status code; detail of the last failing HIP call of this thread. */
const char* fs_status_string(fs_status s);
const char* fs_last_error_detail(void);

/* Context: a device and a HIP stream (hip_stream may be NULL for the null stream); owns the
 * workspace, which grows to the largest problem seen and is freed by fs_context_destroy. */
fs_status fs_context_create(int device, void* hip_stream, fs_context* out);
fs_status fs_context_destroy(fs_context ctx);

/* Defaults of Algorithm 4 for an m x n problem (d = 12 n, zeta = 8, gamma = 10, rho = 0.4,
 * kw_every = 5, max_inner = 100, tau_factor = 30, column scaling on, SVD preconditioner
 * P = V Sigma^{-1} as in Algorithm 4). */
fs_status fs_options_default(int64_t m, int32_t n, fs_options* opts);

/* FOSSILS (Algorithm 4 with Polyak inner solves; Algorithm 2 when opts->fixed_q != 0).
 * A: m x n (lda >= m), b: m, x: n output.  opts may be NULL (defaults).  info may be NULL.
 * Returns FS_OK, a warning, or an error; FS_ERR_NONFINITE when A or b holds NaN/Inf.  b = 0 gives
 * x = 0. */
fs_status fossils_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                        double* x, const fs_options* opts, fs_info* info);

/* SPIR (Algorithm 3: conjugate gradient on the preconditioned normal equations) with the same
 * sketch, preconditioner, initialization and stopping rules as fossils_solve. */
fs_status spir_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                     double* x, const fs_options* opts, fs_info* info);

/* SPIR with LSQR as the Krylov method (Section 4.3: LSQR on the preconditioned least-squares
 * problem of each refinement step instead of CG on its normal equations; the paper reports the two
 * similarly stable).  Each step runs Paige and Saunders' bidiagonalization on A_s P from
 * beta_1 u_1 = b - A_s x_i; one read of A per iteration (the residual pass that also stores the
 * m-vector alpha u - A_s P v), plus 16 m bytes of workspace.  Same sketch, preconditioner, start
 * and stopping rules as spir_solve (Delta = the update of the correction). */
fs_status spir_lsqr_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                          double* x, const fs_options* opts, fs_info* info);

/* Complex least squares, min ||A x - b|| with A in C^{m x n} (m >= n), b in C^m: the Prony problems
 * of Section 5.2 (Appendix B, the first least-squares solve of Prony's method).  A (lda >= m), b and
 * x are complex128 column-major device arrays of interleaved (re, im) doubles, 16-byte aligned.
 * Solved by FOSSILS on the realification A_R = [Re A, -Im A; Im A, Re A] (2m x 2n), b_R = [Re b;
 * Im b], x = x_R[0:n] + i x_R[n:2n]: the map is an isometry of the residual and A_R has A's
 * singular values, each twice, so the backward-error estimate and the stopping rules carry over.
 * opts, if not NULL, describe the realified problem (fs_options_default(2m, 2n): d = 24 n); info
 * reports the realified solve.  Workspace: the realified copy, 32 m n + 16 (m + n) bytes. */
fs_status fossils_solve_complex(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                                double* x, const fs_options* opts, fs_info* info);
/* The same with SPIR (conjugate gradient) as the inner solver. */
fs_status spir_solve_complex(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                             double* x, const fs_options* opts, fs_info* info);

/* FOSSILS for k (1..64) right-hand sides sharing A: column j of X (n x k, ldx >= n) solves the
 * least-squares problem with column j of B (m x k, ldb >= m), both column-major device arrays.
 * One sketch S [A B], one QR and one SVD serve every column (x_0 = R^{-1} t_j); the inner
 * heavy-ball iterations of all columns run together, each pass A^T (A Z) over the k columns on the
 * FP64 matrix cores, and every column keeps Algorithm 4's stopping rules of its own (a column
 * that has stopped is frozen).  Adaptive mode from the sketch-and-solve start only (opts->fixed_q 0,
 * FP64, FS_INIT_SKETCH; otherwise FS_ERR_UNSUPPORTED); P = V Sigma^{-1}.
 * info, if not NULL, points to k fs_info records (per right-hand side).  Returns
 * FS_WARN_NOT_CONVERGED if any column hit the iteration cap in the second step. */
fs_status fossils_solve_multi(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, int32_t k,
                              const double* B, int64_t ldb, double* X, int64_t ldx, const fs_options* opts,
                              fs_info* info);

/* One problem of a batch: A (m x n, lda >= m), b (m) and x (n, output), device arrays; method: the inner
 * solver, FS_METHOD_FOSSILS (0: heavy ball, Algorithm 4) or FS_METHOD_SPIR (1: CG, Algorithm 3). */
typedef struct fs_problem {
  int64_t m;
  int32_t n;
  const double* A;
  int64_t lda;
  const double* b;
  double* x;
  int32_t method;
} fs_problem;

/* FOSSILS (Algorithm 4, P = V Sigma^{-1}) or SPIR (Algorithm 3 with the same preconditioner), as each
 * problem's method says, for count (1..65535) independent problems of any shapes, each with the result
 * fossils_solve (spir_solve) gives it in the serial order (opts->overlap_svd = 0), up to the order of
 * floating-point sums: the same iterations, stopping rules and d = 12 n.  opts, if not NULL,
 * applies to every problem except d, which is 12 n_i for each (zeta <= d), and the form: FP64,
 * sketch-and-solve start, adaptive steps.  The sketch, QR, SVD and x_0 of the problems run in problem
 * order on up to 32 internal streams of the context (their grid-synchronizing kernels reserve
 * compute units so that concurrent grids fit).  The two refinement steps run in lockstep on the
 * context's stream for waves of consecutive problems (a quarter of the batch, 8 to 64 problems) as soon
 * as their setup is done, beside the setup of the next waves: each phase of an inner iteration is one
 * launch for the whole wave (the passes over A as one grid whose work-groups are shared out among the
 * problems in proportion to their m n), and a problem that has met its stopping rule skips the rest.
 * Problems with n > 1024 (or 16 lda (512 / H) >= 2^32 bytes, H the pass tile height), a numerically
 * rank-deficient sketch, or b = 0, are solved by fossils_solve (spir_solve) after the batch, with the
 * caller's options (overlap_svd as given, default on).  A method other than FOSSILS or SPIR gives that
 * problem FS_ERR_UNSUPPORTED.
 * statuses[i] receives problem i's status; infos (if not NULL) count records, where phase_ms[0] is
 * that problem's setup time on its stream and phase_ms[4] its wave's refinement time (other phases
 * 0).  Inputs must be complete on the context's stream (the call waits for it); on return every x is
 * written.  Returns FS_OK, the largest warning of the problems, or the first error among them.
 * Workspace: about 8 n_i^2 + 8 G_i n_i bytes per problem kept for the batch, plus 32 per-stream
 * workspaces sized like fossils_solve's for the largest problem.  The context's thread only. */
fs_status fossils_solve_batched(fs_context ctx, int32_t count, const fs_problem* problems, const fs_options* opts,
                                fs_info* infos, fs_status* statuses);

/* Mixed-precision form: the sketch S [A_s b] is taken of the single-precision copy of A (A32 =
 * fl32(A), column-major lda32 >= m, when A32 is not NULL, else A rounded to FP32 as it is read), with
 * FP64 sums; QR, SVD and the whole refinement (every pass over A) stay FP64 on A.  The FP32 copy
 * perturbs S A by about u32 ||A||, which keeps A_s R^{-1} well conditioned only while condest * u32
 * is small; above the threshold (u32 condest > 2, condest > ~3.4e7) the sketch is redone in FP64 and
 * info->flags gets FS_FLAG_FP64_SKETCH.  The result meets the same backward-error bar as
 * fossils_solve. */
fs_status fossils_solve_mixed(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const float* A32,
                              int64_t lda32, const double* b, double* x, const fs_options* opts, fs_info* info);
/* A32 = fl32(A) on the context's stream (for callers that keep an FP32 copy resident). */
fs_status fs_to_fp32(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, float* A32, int64_t lda32);

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): fossils_solve with the same arguments and results, whose every
 * device buffer is a slice of one array of 256 MiB that the library holds on each GPU it runs on until
 * the process ends (its device address is looked up on the first call on a device).  Nothing is
 * allocated or freed; the solve runs in the serial order (opts->overlap_svd and opts->graph_sweeps are
 * treated as 0).  FS_ERR_TOO_LARGE, before any device work, when the solve's workspace (about
 * m (2 zeta + 8) + 8 d (n + 1) + 40 n^2 bytes plus the QR and SVD exchange buffers) exceeds the array:
 * with n = 1000, d = 12000 it fits m up to about 2.9e6.  All calls on one GPU share the array, so calls
 * that overlap in time on one GPU (two threads, or two streams in flight) race: the caller serializes
 * them.  Nothing carries over between calls: every buffer is initialized by the call's own kernels. */
fs_status fossils_solve_noalloc(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                                double* x, const fs_options* opts, fs_info* info);

/* ---------------- sparse sign embedding (Section 4.2, "Choice of embedding") ---------------- */

/* Sketch handle for S (d x m, zeta nonzeros per column).  The index stream is generated on the
 * device from (seed, column) with a Philox4x32-10 counter-based generator and kept by the handle. */
fs_status sketch_create(fs_context ctx, int64_t m, int32_t d, int32_t zeta, uint64_t seed, fs_sketch* out);
fs_status sketch_destroy(fs_sketch sk);

/* Copy the row positions and signs of columns [col0, col0+ncols) of S to host arrays
 * rows_host[ncols*zeta] (int32, positions in [0,d)) and signs_host[ncols*zeta] (+1/-1). */
fs_status sketch_indices(fs_sketch sk, int64_t col0, int64_t ncols, int32_t* rows_host, int8_t* signs_host);

/* Y = S [A b] (d x (n+1), ldy >= d; the last column is S b; b may be NULL, then Y is d x n).
 * With scale_columns, column j < n is divided by ||a_j|| (zero columns by 1), i.e. Y = S [A D^{-1} b]
 * (Alg 4's column scaling).  colnorm2 (n, device, may be NULL) receives ||a_j||^2 from the same
 * read of A. */
fs_status sketch_apply(fs_sketch sk, int32_t n, const double* A, int64_t lda, const double* b, double* Y,
                       int64_t ldy, double* colnorm2, int32_t scale_columns);

/* ---------------- step-level entry points (the parts of the hot path) ---------------- */

/* In-place Householder QR of the d x k matrix Y (ldy >= d, d >= k) (eq:sketch_qr).  On return the
 * upper triangle of Y[0:k, 0:k] holds R with a non-negative diagonal; entries below the diagonal
 * are overwritten with reflector data. */
fs_status fs_sketch_qr(fs_context ctx, int32_t d, int32_t k, double* Y, int64_t ldy);

/* SVD of an n x n upper-triangular R (upper triangle of R, ldr >= n) by one-sided Jacobi:
 * sigma (n, decreasing), V (n x n, ldv >= n) right singular vectors, so R^T R = V diag(sigma)^2 V^T
 * (Alg 4: normest = sigma[0], condest = sigma[0]/sigma[n-1]).  sweeps_host (may be NULL) receives
 * the number of Jacobi sweeps. */
fs_status fs_svd_triangular(fs_context ctx, int32_t n, const double* R, int64_t ldr, double* sigma, double* V,
                            int64_t ldv, int32_t* sweeps_host);

/* v = A^T (A z): the operator of the preconditioned normal equations (eq:precond-normal) in one
 * read of A.  z, v: n. */
fs_status fs_normal_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z,
                         double* v);

/* g = A^T (b - A x) and ||b - A x||^2 (the right-hand side of a refinement step, Algorithm 1) in
 * one read of A.  rnorm2_host may be NULL. */
fs_status fs_residual_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                           const double* x, double* g, double* rnorm2_host);

/* Measurement helper: run fs_normal_pass `repeats` times back to back on the context stream,
 * bracketed by HIP events; *ms_per_pass_host = average time of one pass (fused kernel + its
 * fixed-order partial reduction), *ms_kernel_host (may be NULL) = average of the fused kernel
 * alone.  v receives A^T (A z). */
fs_status fs_time_normal_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z,
                              double* v, int32_t repeats, double* ms_per_pass_host, double* ms_kernel_host);

/* Autotuning of the fused pass over A (the refinement loop's kernel, the operator of
 * eq:precond-normal).  Its two knobs are the tile height H (rows per work-group tile, held in
 * registers between the products A z and A^T w; 64, 32, 16, 8 or 4, as far as the kernel is built
 * for ceil(n H / 1024) column slots per lane) and the work-group count G (the schedule: a multiple of
 * 8, the rows banded across the 8 XCDs, at most 2 x the compute units).  fs_tune_pass times every
 * admissible (H, G) on the caller's A (m x n column-major, lda >= m; z and v device n-vectors) with
 * `repeats` back-to-back passes each and keeps the fastest in the context, keyed by (n, floor(log2 m)):
 * every later pass of that key on this context uses it (solves included).  v receives A^T (A z)
 * from the kept configuration; *H_out, *G_out, *ms_out (each may be NULL) the kept pair and its time
 * per pass.  FS_ERR_SHAPE when no fused configuration fits (n > 4096, or lda too large).
 * fs_set_pass_tuning stores a pair directly (for instance from a saved cache), FS_ERR_INVALID_ARG
 * when it is not admissible; fs_clear_pass_tuning drops all.  Results are the same up to the
 * rounding of the partial sums, whatever the pair. */
fs_status fs_tune_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z, double* v,
                       int32_t repeats, int32_t* H_out, int32_t* G_out, double* ms_out);
fs_status fs_set_pass_tuning(fs_context ctx, int64_t m, int32_t n, int32_t H, int32_t G);
fs_status fs_clear_pass_tuning(fs_context ctx);

/* x = R^{-1} y (transpose = 0, back substitution) or x = R^{-T} y (transpose = 1, forward
 * substitution) for upper-triangular R (ldr >= n); x may equal y.  n <= 15000. */
fs_status fs_trsv(fs_context ctx, int32_t n, const double* R, int64_t ldr, int32_t transpose, const double* y,
                  double* x);

/* X = R^{-1} for upper-triangular R (ldr >= n): X is n x n, ld n, zeros below the diagonal; formed
 * by blocks of 64 (diagonal blocks by back substitution, then the recursive 2 x 2 block form
 * X12 = -X11 R12 X22).  This is P = R^{-1} of the QR preconditioner (Section 2.3) in explicit form,
 * the form in which the refinement steps beside the SVD of R apply it.  Synchronous; uses the
 * context's workspace (n^2 doubles of scratch).  n <= 15000; FS_ERR_SHAPE for n < 1 or ldr < n. */
fs_status fs_triangular_inverse(fs_context ctx, int32_t n, const double* R, int64_t ldr, double* X);

/* ---------------- serving: many independent solves on one GPU ---------------- */

/* A solve request.  A (m x n, lda >= m), b (m) and x (n) are device arrays owned by the caller;
 * they must stay valid (and A, b unchanged) until batched_poll reports the ticket done.  method:
 * FS_METHOD_FOSSILS, FS_METHOD_SPIR or FS_METHOD_SPIR_LSQR.  opts may be NULL (defaults); it is
 * copied at submission (opts->precision = FS_MIXED gives the mixed-precision form with A rounded to
 * FP32 as it is read).  stream: the HIP stream on which the caller produced A and b (NULL: the null
 * stream); batched_submit records an event on it, and the solve's kernels wait for that event, so
 * work the caller enqueued there before the submission is complete before the solve reads A or b.
 * When the ticket is done, x has been written and the solve's stream has drained. */
enum { FS_METHOD_FOSSILS = 0, FS_METHOD_SPIR = 1, FS_METHOD_SPIR_LSQR = 2 };
typedef struct {
  int32_t method;
  int64_t m;
  int32_t n;
  const double* A;
  int64_t lda;
  const double* b;
  double* x;
  const fs_options* opts;
  void* stream;
} fs_request;

/* A server on the device of ctx (continuous batching, the serving form of the solvers): max_slots
 * worker slots (1..16), each a host thread with its own stream and workspace, take requests from
 * one FIFO queue as they free up, so the passes of different solves overlap on the GPU; the
 * cooperative QR/SVD grids of different slots reserve their work-groups from one device-wide
 * budget (a cooperative grid must be fully resident).
 * Admission is against a device-wide ledger of hbm_budget workspace bytes: it charges each slot the
 * workspace it holds between requests plus, while a request runs, the further growth that
 * request's footprint allows.  The head of the queue starts on a free slot once its growth fits
 * the ledger; until then slots give their idle workspace back (fs_context_trim) and the request
 * waits, so requests are admitted in arrival order as memory frees up.  A request whose footprint
 * alone exceeds hbm_budget is refused at submission with FS_ERR_TOO_LARGE.  With more than one slot
 * the solves run in the serial order (opts->overlap_svd is treated as 0): the slots already share
 * the GPU. */
fs_status fs_server_create(fs_context ctx, size_t hbm_budget, int32_t max_slots, fs_server* out);
/* Finishes every queued request, then frees the slots. */
fs_status fs_server_destroy(fs_server srv);
/* Non-blocking: validate and enqueue; *ticket identifies the request. */
fs_status batched_submit(fs_server srv, const fs_request* req, uint64_t* ticket);
/* Non-blocking: *done = 1 once the solve has finished; then *result is its status (as returned by
 * fossils_solve / spir_solve) and *info (if not NULL) its record. */
fs_status batched_poll(fs_server srv, uint64_t ticket, int32_t* done, fs_status* result, fs_info* info);
/* Blocks until the ticket is done. */
fs_status fs_server_wait(fs_server srv, uint64_t ticket);
/* Seconds on the server's steady clock at submission, start on a slot and completion (-1 if not
 * yet reached). */
fs_status fs_server_ticket_times(fs_server srv, uint64_t ticket, double* submit_s, double* start_s, double* finish_s);
/* Ledger of a server: bytes charged now, the most charged at any time, and hbm_budget (each
 * pointer may be NULL).  The charge never exceeds hbm_budget. */
fs_status fs_server_memory(fs_server srv, size_t* used, size_t* peak, size_t* budget);
/* Footprint the server charges for an m x n request with options opts (NULL: defaults). */
fs_status fs_server_request_footprint(fs_server srv, int64_t m, int32_t n, const fs_options* opts, size_t* bytes);
/* Upper bound of the workspace bytes one single-right-hand-side solve (fossils_solve, spir_solve,
 * spir_lsqr_solve, fossils_solve_mixed) of an m x n problem with options opts (NULL: defaults)
 * grows a context to, on a GPU with 256 compute units. */
size_t fs_solve_footprint(int64_t m, int32_t n, const fs_options* opts);
/* Device bytes of workspace a context holds now (it grows to the largest problem seen). */
fs_status fs_context_workspace(fs_context ctx, size_t* bytes);
/* Frees a context's workspace (after draining its stream); the next solve allocates again. */
fs_status fs_context_trim(fs_context ctx);

#ifdef __cplusplus
}
#endif

#endif /* FOSSILS_H */
