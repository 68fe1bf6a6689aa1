// Device-resident control block of one solve and the vector-kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct DevState {
  double alpha, beta;    // heavy-ball coefficients (eq:optimal-coeffs)
  double thr_first;      // first-step threshold (gamma normest ||x0|| + rho condest ||r0||) u
  double fro2;           // ||A_s||_F^2
  double fro_u;          // ||A_s||_F u  (second-step threshold)
  double theta2;         // theta^2 = ||A_s||_F^2 / ||b||^2
  double r2;             // ||r||^2 of the last residual pass
  double x2;             // ||x_hat||^2 at the last KW check
  double rho_cg;         // CG: res^T res
  double be_sk;          // last sketched KW estimate (absolute)
  double dnorm2;         // ||Delta||^2 of the last inner update
  double cnorm2;         // ||c||^2 at the start of the step
  double normest, condest;
  double x0norm, r0norm;
  double b2;             // ||b||^2
  double l_alpha, l_beta;       // LSQR: alpha_i, beta_i of the Golub-Kahan bidiagonalization
  double l_phibar, l_rhobar;    // LSQR: the rotated right-hand side and diagonal
  double smin_ub;        // upper bound of sigma_min(R) (inverse iteration), for the condest bound
  int stop;              // inner-loop stop flag
  int iters;             // inner iterations in the current step
  int converged;         // the current step stopped by its rule (not by the cap)
  int max_inner;         // iteration cap per step
  int rank_trunc;        // #{sigma_i > tau normest}
  int kw_evals;          // sketched-KW evaluations
  int kw_pending;        // second step beside the SVD: KW checkpoints recorded, not yet evaluated
  int svd_abort;         // the SVD beside the refinement is no longer needed (its sweeps stop)
};

hipError_t fs_vec_gemv_v(const double* V, int64_t ldv, int n, int k, const double* y, const double* ydiv,
                         const double* oscale, const double* addv, double* out, double* part, const int* stop,
                         hipStream_t s);
hipError_t fs_vec_gemv_vt(const double* V, int64_t ldv, int n, int k, const double* v, const double* div, double* out,
                          const int* stop, hipStream_t s);
hipError_t fs_vec_polyak(int n, const double* c, const double* u, double* dy, double* dy_old, DevState* st,
                         bool first_step, hipStream_t s);
// First step overlapped with the SVD of R: per-iteration record of dy and ||Delta||^2, and the
// rollback to the first recorded iteration that meets the first-step rule once thr_first is known.
hipError_t fs_vec_diag_bounds(int n, const double* R, int64_t ldr, DevState* st, hipStream_t s);
// Sharper bounds for the same purpose (after fs_vec_diag_bounds): `iters` steps of power iteration
// on R^T R (normest from below) and of inverse iteration (sigma_min from above, condest from below).
// work: 6 n doubles; part: the partials of a product with an n x n matrix.  Rinv (may be null): R^{-1}
// (ld n), whose products then replace the substitutions; trsv_ws: the workspace of the triangular
// solves across work-groups.
hipError_t fs_vec_spectral_bounds(int n, const double* R, int64_t ldr, const double* Rinv, int iters, double* work,
                                  double* part, void* trsv_ws, DevState* st, hipStream_t s);
hipError_t fs_vec_record_iter(int j, int n, const double* dy, double* hist_dy, double* hist_dn, const DevState* st,
                              hipStream_t s);
hipError_t fs_vec_rollback(int n, const double* hist_dy, const double* hist_dn, double* dy, DevState* st,
                           hipStream_t s);
// Second step beside the SVD of R: a KW checkpoint (Alg 4's second-step rule) cannot be evaluated
// before Sigma and V exist, so it is recorded (dy, g = A_s^T r_hat, ||r_hat||^2, ||x_hat||^2, j) into
// slot c; once they exist, the recorded checkpoints are evaluated in order (W: slot c holds
// V^T g_c) and the first that meets the rule ends the step there (dy and the count rolled back).
hipError_t fs_vec_kw_record(int c, int j, int n, const double* dy, const double* g, double* kdy, double* kg,
                            double* ks, DevState* st, hipStream_t s);
hipError_t fs_vec_kw_replay(int n, int ncheck, const double* W, const double* sigma, const double* kdy,
                            const double* ks, double* dy, DevState* st, hipStream_t s);
// LSQR form of SPIR: start of a step (needs st->r2 = ||r||^2 and c = P^T A_s^T r), one bidiagonalization
// and rotation step (h = P^T A_s^T (alpha u - A_s P v), st->r2 its squared residual), and the
// m-vector ubar = alpha u from the stored residual r (sign -1 inside the iteration).
hipError_t fs_vec_lsqr_init(int n, const double* c, double* v, double* w, double* dy, DevState* st, hipStream_t s);
hipError_t fs_vec_lsqr_step(int n, const double* h, double* v, double* w, double* dy, DevState* st, bool first_step,
                            hipStream_t s);
hipError_t fs_vec_lsqr_ubar(int64_t m, const double* r, double* ubar, double sign, const DevState* st,
                            hipStream_t s);
hipError_t fs_vec_cg(int n, double* p, const double* q, double* res, double* dy, DevState* st, bool first_step,
                     hipStream_t s);
hipError_t fs_vec_step_init(int n, const double* c, double* a, double* b, double* dy, bool spir, DevState* st,
                            hipStream_t s);
hipError_t fs_vec_add_norm(int n, const double* x, const double* z, double* out, double* norm2, const int* stop,
                           hipStream_t s);
hipError_t fs_vec_mul(int n, const double* a, const double* b, double* out, const int* stop, hipStream_t s);
hipError_t fs_vec_scaling(int n, const double* colnorm2, bool use_scaling, double* dinv, DevState* st, hipStream_t s);
hipError_t fs_vec_sigma_stats(int n, const double* sigma, double tau_factor, DevState* st, hipStream_t s);
// The second step beside the SVD: an upper bound of the sketched KW estimate from R alone,
// ||(Sigma^2 + lambda I)^{-1/2} V^T g|| <= ||Sigma^{-1} V^T g|| = ||R^{-T} g|| (h = R^{-T} g given).  When
// `margin` times the bound meets the second-step rule, the rule is met: the step stops there and the
// SVD is told to stop (st->svd_abort).
hipError_t fs_vec_kw_upper(int n, const double* h, double margin, DevState* st, hipStream_t s);
hipError_t fs_vec_first_threshold(int n, const double* x0, double gamma, double rho, DevState* st, hipStream_t s);
hipError_t fs_vec_kw(int n, const double* w, const double* sigma, DevState* st, hipStream_t s);
hipError_t fs_vec_set_int(int* p, int v, hipStream_t s);
hipError_t fs_vec_set_double(double* p, double v, hipStream_t s);
hipError_t fs_vec_state_init(DevState* st, double alpha, double beta, int max_inner, hipStream_t s);
hipError_t fs_vec_trmv_t(const double* R, int64_t ldr, int n, const double* t, double* out, hipStream_t s);

// Per-right-hand-side control block of a multi-RHS solve (k <= FS_MULTI_MAX columns).
constexpr int FS_MULTI_MAX = 64;
struct MultiState {
  double thr[FS_MULTI_MAX];     // first-step thresholds
  double be_sk[FS_MULTI_MAX];   // last sketched KW estimates
  double r2[FS_MULTI_MAX];      // ||r_j||^2 of the last residual pass
  double x2[FS_MULTI_MAX];      // ||x_hat_j||^2 at the last KW check
  double b2[FS_MULTI_MAX];      // ||b_j||^2
  double cnorm2[FS_MULTI_MAX];  // ||c_j||^2 at the start of the step
  int active[FS_MULTI_MAX];     // column still iterating in the current step
  int iters[FS_MULTI_MAX];      // inner iterations of the current step
  int converged[FS_MULTI_MAX];  // stopped by its rule in the current step
  int kw_evals[FS_MULTI_MAX];
  int zero[FS_MULTI_MAX];       // b_j = 0: x_j = 0, never iterated
  int stop;                     // no active column left
  int pad[15];
};

hipError_t fs_m_step_init(int nr, int k, const double* C, double* DY, double* DY_old, MultiState* ms, hipStream_t s);
hipError_t fs_m_polyak(int nr, int k, const double* C, const double* U, double* DY, double* DY_old, MultiState* ms,
                       double alpha, double beta, bool first_step, hipStream_t s);
hipError_t fs_m_update_stop(int k, MultiState* ms, hipStream_t s);
hipError_t fs_m_first_threshold(int n, int k, const double* X0, MultiState* ms, double gamma, double rho,
                                double normest, double condest, hipStream_t s);
hipError_t fs_m_kw(int n, int k, const double* Wv, const double* sigma, MultiState* ms, double fro2, double fro_u,
                   hipStream_t s);
hipError_t fs_m_add_norm(int n, int k, const double* X, const double* Z, double* out, MultiState* ms, hipStream_t s);
// Zs[c * kp + j] = scale[c] X[c + j ldxin] (zero for j >= k)
hipError_t fs_m_to_panel(int n, int k, const double* X, int64_t ldxin, const double* scale, double* Zs,
                         const int* stop, hipStream_t s);
hipError_t fs_m_init_columns(int n, int k, const double* colnorm2, MultiState* ms, hipStream_t s);
hipError_t fs_m_unscale(int n, int k, const double* X, const double* dinv, double* Xout, int64_t ldx, hipStream_t s);
// out(c, j) = oscale[c] * (sum_{i < nr} V[c, i] Y[i, j] / sigma[i] + addX[c, j]);  Y: nr x k (ld nr),
// addX: n x k (ld n, may be null), out: n x k (ld n) or, if panel, n x kp row-major.
hipError_t fs_m_gemm_P(const double* V, int64_t ldv, int n, int nr, int k, const double* sigma, const double* Y,
                       const double* addX, const double* oscale, double* out, bool panel, const int* stop,
                       hipStream_t s);
// U[i, j] = (sum_c V[c, i] G(c, j)) / sigma[i] (sigma may be null);  G: n x kp row-major panel;
// U: nr x k (ld nr).
hipError_t fs_m_gemm_PT(const double* V, int64_t ldv, int n, int nr, int k, const double* sigma, const double* G,
                        double* U, const int* stop, hipStream_t s);

// One problem of a batched refinement (fossils_solve_batched): its n-vectors, V and Sigma of its
// sketch, the column scaling, the slices of its V products and its control block.
struct BatchVec {
  int n;
  int done;  // finished before the refinement (nothing to iterate)
  const double* V;
  const double* sigma;
  const double* dinv;
  double *x, *x0, *c, *dy, *dy_old, *zs, *v, *u, *g, *xh, *w;
  double* gpart;  // ceil(n / 64) x n
  double* x_out;  // the caller's x
  DevState* st;
  int spir;           // CG inner solver (SPIR) instead of heavy ball
  double *res, *p;    // CG residual and direction (SPIR)
};
enum class BatchOp { SCALE, FIRST_THRESHOLD, STEP_INIT, UPDATE, XH_NORM, KW, FINAL };
// P y for every problem (mode 0: zs = D^{-1} P y with y = dy, or the CG direction p for SPIR; 1: xh =
// x + P dy; 2: x = x + P dy) and P^T
// (mode 0: c = P^T g; 1: u = P^T v; 2: w = V^T g), P = V Sigma^{-1}; max_n: the largest n.
hipError_t fs_b_gemv_P(const BatchVec* list, int count, int max_n, int mode, hipStream_t s);
hipError_t fs_b_gemv_PT(const BatchVec* list, int count, int max_n, int mode, hipStream_t s);
// One-work-group-per-problem steps: SCALE (arg 0: zs = D^{-1} x, 1: zs = D^{-1} xh), FIRST_THRESHOLD
// (gamma, rho), STEP_INIT, UPDATE (heavy ball or CG by each problem's method; arg: first step), XH_NORM, KW,
// FINAL (x_out = D^{-1} x).
hipError_t fs_b_vec(const BatchVec* list, int count, BatchOp op, int arg, double gamma, double rho, hipStream_t s);
// Everything the host reads back after one problem's setup, gathered on the device for one copy.
struct BatchReport {
  DevState st;
  int sweeps;   // Jacobi sweeps of the SVD
  int err;      // a grid barrier (QR, SVD) or a block flag (substitution) gave up waiting
  int nan;      // a column norm (or ||b||^2) is NaN: A or b holds NaN or Inf
  int inf;      // a column norm is +Inf: finite entries whose squares overflow
  double b2;    // ||b||^2
};
hipError_t fs_b_report(const DevState* st, const int* sweeps, const int* qr_err, const int* svd_err,
                       const int* trsv_err, const double* colnorm2, int n, BatchReport* out, hipStream_t s);
// out[k] = *list[k].st for the count problems
hipError_t fs_b_gather(const BatchVec* list, int count, DevState* out, hipStream_t s);
// theta^2 and ||b||^2 of one problem from the sketch's column norms (colnorm2[n] = ||b||^2).
hipError_t fs_b_prep(const double* colnorm2, int n, DevState* st, hipStream_t s);
