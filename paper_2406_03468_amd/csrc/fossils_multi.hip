// fossils_solve_multi: FOSSILS (Alg 4) for k <= 64 right-hand sides sharing A.
//
// The sketch, its QR factorization and the SVD of R depend on A only and are done once: the k
// right-hand sides are sketched with A (Y = S [A_s B], one read of A and B), so the QR of Y also
// yields T = (Q^T S B)[0:n] and every x_0 = R^{-1} t_j (eq:sketch-and-solve-2.3).  Each refinement
// step (Alg 1) runs the k heavy-ball iterations (eq:polyak_iteration) in lockstep, the per-
// iteration products A^T (A Z) for all k columns in one MFMA pass over A; every column keeps its
// own stopping rule (first step: ||Delta_j|| threshold; second step: sketched KW every kw_every
// iterations, Alg 4) and is frozen once it meets it; the step ends when all columns have stopped
// or at the iteration cap.  Preconditioner: P = V Sigma^{-1} (truncated if rank deficient).
#include <math.h>
#include <string.h>

#include <memory>
#include <vector>

#include "common.hpp"
#include "context.hpp"
#include "internal.hpp"
#include "state.hpp"

hipError_t fs_launch_svd_full(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                              double* Uout, int64_t ldu, void* work, int num_cu, int max_sweeps, int* sweeps_out_dev,
                              hipStream_t s);

extern "C" fs_status fossils_solve_multi(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda,
                                         int32_t k, const double* B, int64_t ldb, double* X_out, int64_t ldx,
                                         const fs_options* opts_in, fs_info* info) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  FS_TRY(fs_validate_problem(m, n, A, lda, B, X_out));
  if (k < 1 || k > FS_MULTI_MAX) return FS_ERR_SHAPE;
  if (ldb < m || ldx < n) return FS_ERR_SHAPE;
  fs_options o;
  if (opts_in) o = *opts_in;
  else FS_TRY(fs_options_default(m, n, &o));
  FS_TRY(fs_validate_options(m, n, o));
  if (o.fixed_q != 0 || o.precision != FS_FP64 || o.init != FS_INIT_SKETCH) return FS_ERR_UNSUPPORTED;  // adaptive FP64 only
  FS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  FS_HIP(hipStreamSynchronize(s));
  Workspace& W = ctx->ws;
  const int d = o.d, zeta = o.zeta, kc = n + k;
  const bool i16 = fs_idx16_ok(d);
  const int kp = 16 * fs_multi_blocks(k);

  // ---- workspace
  int64_t rc = 0;
  const size_t mwd = fs_multi_work_doubles(m, n, k, &rc);
  FS_TRY(fs_grow(W.idx, (size_t)m * zeta * (i16 ? 2 : 4)));
  FS_TRY(fs_grow(W.Y, sizeof(double) * (size_t)d * kc));
  FS_TRY(fs_grow(W.colnorm2, sizeof(double) * (size_t)kc));
  FS_TRY(fs_grow(W.dinv, sizeof(double) * (size_t)n));
  FS_TRY(fs_grow(W.qrwork, fs_qr_work_bytes(d, kc, ctx->num_cu)));
  FS_TRY(fs_grow(W.svdwork, fs_svd_work_bytes(n)));
  FS_TRY(fs_grow(W.sigma, sizeof(double) * (size_t)n));
  FS_TRY(fs_grow(W.V, sizeof(double) * (size_t)n * n));
  FS_TRY(fs_grow(W.UR, sizeof(double) * (size_t)n * n));
  FS_TRY(fs_grow(W.state, sizeof(DevState) + 64));
  FS_TRY(fs_grow(W.mwork, sizeof(double) * mwd));
  const size_t nk = (size_t)n * k, npan = (size_t)n * kp;
  const int NBLK = 9;  // X, C, DY, DY_old, U, Xh, Wv, T(x0 scratch), Zs/Vout panels (2)
  FS_TRY(fs_grow(W.mvecs, sizeof(double) * (NBLK * nk + 2 * npan)));
  FS_TRY(fs_grow(W.mstate, sizeof(MultiState)));
  double* mv = (double*)W.mvecs.p;
  double *Xs = mv, *Cm = mv + nk, *DY = mv + 2 * nk, *DYo = mv + 3 * nk, *Um = mv + 4 * nk, *Xh = mv + 5 * nk,
         *Wv = mv + 6 * nk;
  double* Zs = mv + NBLK * nk;
  double* Vout = Zs + npan;
  double* mw = (double*)W.mwork.p;
  const int64_t nchunk = (m + rc - 1) / rc;
  double* Wbuf = mw;
  double* Vpart = Wbuf + (size_t)m * kp;
  double* r2part = Vpart + (size_t)nchunk * n * kp;
  DevState* st = (DevState*)W.state.p;
  int* svd_sweeps_dev = (int*)((char*)W.state.p + sizeof(DevState));
  MultiState* ms = (MultiState*)W.mstate.p;
  const int* mstop = &ms->stop;
  double* Y = (double*)W.Y.p;
  double* cn2 = (double*)W.colnorm2.p;
  double* dinv = (double*)W.dinv.p;
  double* sigma = (double*)W.sigma.p;
  double* V = (double*)W.V.p;
  double* UR = (double*)W.UR.p;
  const double* R = Y;
  const int64_t ldr = d;
  const double* T = Y + (int64_t)n * d;  // column j of (Q^T S B)[0:n] at T + j d

  const double eta = ((o.eta > 0) ? o.eta : sqrt((double)n / d)) * o.eta_factor;
  const double beta = eta * eta, alpha = (1.0 - beta) * (1.0 - beta);  // eq:optimal-coeffs
  FS_K(fs_vec_state_init(st, alpha, beta, o.max_inner, s));
  FS_HIP(hipMemsetAsync(ms, 0, sizeof(MultiState), s));

  hipEvent_t* ev = ctx->ev;
  FS_HIP(hipEventRecord(ev[0], s));
  FS_K(fs_launch_sketch_indices(m, d, zeta, o.seed, 0, m, W.idx.p, i16, s));
  FS_K(fs_launch_sketch_apply(A, lda, m, n, B, ldb, k, W.idx.p, i16, d, zeta, Y, d, cn2, o.column_scaling != 0,
                              true, ctx->lds_bytes, s));
  FS_K(fs_vec_scaling(n, cn2, o.column_scaling != 0, dinv, st, s));
  FS_HIP(hipEventRecord(ev[1], s));
  std::unique_ptr<CoopSection> coop(new CoopSection(
      ctx, std::max(fs_qr_grid_size(d, ctx->num_cu), fs_svd_grid_size(n, ctx->num_cu, false))));
  FS_K(fs_launch_qr(Y, d, d, kc, W.qrwork.p, ctx->num_cu, s));
  FS_HIP(hipEventRecord(ev[2], s));
  FS_K(fs_launch_svd_full(R, ldr, n, sigma, V, n, nullptr, n, W.svdwork.p, ctx->num_cu, o.max_sweeps, svd_sweeps_dev,
                          s));
  FS_K(fs_vec_sigma_stats(n, sigma, o.tau_factor, st, s));
  FS_HIP(hipEventRecord(ev[3], s));
  FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  std::vector<double> cnh(kc);
  FS_HIP(hipMemcpyAsync(cnh.data(), cn2, sizeof(double) * kc, hipMemcpyDeviceToHost, s));
  int svd_sweeps = 0, bar_err[2] = {0, 0};
  FS_HIP(hipMemcpyAsync(&svd_sweeps, svd_sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  FS_HIP(hipMemcpyAsync(&bar_err[0], fs_qr_err_word(W.qrwork.p, d, kc, ctx->num_cu), sizeof(int),
                        hipMemcpyDeviceToHost, s));
  FS_HIP(hipMemcpyAsync(&bar_err[1], fs_svd_err_word(W.svdwork.p, n), sizeof(int), hipMemcpyDeviceToHost, s));
  FS_HIP(hipStreamSynchronize(s));
  coop.reset();
  if (bar_err[0] || bar_err[1]) {
    fs_set_last_hip_error(hipErrorLaunchTimeOut, "grid barrier of the QR/SVD kernels gave up waiting", __FILE__,
                          __LINE__);
    return FS_ERR_DEVICE;
  }
  // NaN norm: the column holds NaN or Inf; +Inf: finite entries whose squares overflow FP64
  for (int j = 0; j < kc; ++j)
    if (std::isnan(cnh[j])) return FS_ERR_NONFINITE;
  for (int j = 0; j < kc; ++j)
    if (!std::isfinite(cnh[j])) return FS_ERR_TOO_LARGE;
  const DevState hs = *ctx->st_host;
  const double fro2 = hs.fro2, fro_u = sqrt(hs.fro2) * FS_U_ROUND;
  // per-column ||b_j||^2; b_j = 0 columns are never iterated (x_j = 0)
  FS_K(fs_m_init_columns(n, k, cn2, ms, s));
  int flags = 0, nr = n;
  if (!(hs.condest <= 1.0 / (o.tau_factor * FS_U_ROUND))) {  // Alg 4: numerically rank deficient
    flags |= 1;
    nr = hs.rank_trunc > 0 ? hs.rank_trunc : 1;
    CoopSection cs(ctx, fs_svd_grid_size(n, ctx->num_cu, true));
    FS_K(fs_launch_svd_full(R, ldr, n, sigma, V, n, UR, n, W.svdwork.p, ctx->num_cu, o.max_sweeps, svd_sweeps_dev,
                            s));
    // x_0 = V_r Sigma_r^{-1} U_r^T t_j: U_r^T T (as P^T with sigma = 1), then V_r Sigma_r^{-1}
    FS_K(fs_m_to_panel(n, k, T, d, nullptr, Zs, nullptr, s));
    FS_K(fs_m_gemm_PT(UR, n, n, nr, k, nullptr, Zs, Um, nullptr, s));
    FS_K(fs_m_gemm_P(V, n, n, nr, k, sigma, Um, nullptr, nullptr, Xs, false, nullptr, s));
  } else {
    FS_K(fs_launch_trsv_batched(R, ldr, n, false, T, d, Xs, n, k, s));  // x_0 = R^{-1} t_j
  }

  std::vector<int> iters0(k, 0), iters1(k, 0), conv(k, 0);
  std::vector<double> cnorm0(k, 0.0), cnorm1(k, 0.0);
  MultiPassArgs pa{A, lda, m, n, k, Zs, nullptr, ldb, Wbuf, Vpart, r2part, rc, dinv, Vout, ms->r2, mstop};
  for (int step = 0; step < o.steps; ++step) {
    // residual pass: Vout = D^{-1} A^T (B - A D^{-1} X), r2_j
    FS_K(fs_m_to_panel(n, k, Xs, n, dinv, Zs, nullptr, s));
    MultiPassArgs rp = pa;
    rp.B = B;
    rp.stop = nullptr;
    FS_K(fs_launch_multi_pass(rp, s));
    if (step == 0) {
      FS_K(fs_m_first_threshold(n, k, Xs, ms, o.gamma, o.rho, hs.normest, hs.condest, s));
      FS_HIP(hipEventRecord(ev[5], s));
    }
    FS_K(fs_m_gemm_PT(V, n, n, nr, k, sigma, Vout, Cm, nullptr, s));  // c_j = P^T g_j
    FS_K(fs_m_step_init(nr, k, Cm, DY, DYo, ms, s));
    const bool first = (step == 0);
    bool stopped = false;
    for (int j = 0; j < o.max_inner && !stopped; ++j) {
      FS_K(fs_m_gemm_P(V, n, n, nr, k, sigma, DY, nullptr, dinv, Zs, true, mstop, s));  // Zs = D^{-1} P dy
      FS_K(fs_launch_multi_pass(pa, s));                                                 // Vout = D^{-1} A^T A Zs
      FS_K(fs_m_gemm_PT(V, n, n, nr, k, sigma, Vout, Um, mstop, s));                     // u = P^T v
      FS_K(fs_m_polyak(nr, k, Cm, Um, DY, DYo, ms, alpha, beta, first, s));
      FS_K(fs_m_update_stop(k, ms, s));
      if (step == 1 && (j % o.kw_every) == 0) {  // Alg 4 second-step rule at x_hat = x + P dy
        FS_K(fs_m_gemm_P(V, n, n, nr, k, sigma, DY, Xs, nullptr, Xh, false, mstop, s));
        FS_K(fs_m_add_norm(n, k, Xh, nullptr, Xh, ms, s));
        FS_K(fs_m_to_panel(n, k, Xh, n, dinv, Zs, mstop, s));
        MultiPassArgs kp2 = pa;
        kp2.B = B;
        FS_K(fs_launch_multi_pass(kp2, s));
        FS_K(fs_m_gemm_PT(V, n, n, n, k, nullptr, Vout, Wv, mstop, s));  // V^T g (all n)
        FS_K(fs_m_kw(n, k, Wv, sigma, ms, fro2, fro_u, s));
        FS_K(fs_m_update_stop(k, ms, s));
      }
      if (((j + 1) % o.kw_every) == 0 || j == o.max_inner - 1) {
        int stp = 0;
        FS_HIP(hipMemcpyAsync(&stp, mstop, sizeof(int), hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        stopped = stp != 0;
      }
    }
    // x_j <- x_j + P dy_j
    FS_K(fs_m_gemm_P(V, n, n, nr, k, sigma, DY, Xs, nullptr, Xs, false, nullptr, s));
    MultiState hm;
    FS_HIP(hipMemcpyAsync(&hm, ms, sizeof(MultiState), hipMemcpyDeviceToHost, s));
    FS_HIP(hipEventRecord(ev[6 + (step > 0 ? 1 : 0)], s));
    FS_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) {
      (step == 0 ? iters0 : iters1)[j] = hm.iters[j];
      (step == 0 ? cnorm0 : cnorm1)[j] = sqrt(hm.cnorm2[j]);
      conv[j] = hm.converged[j];
    }
  }
  FS_K(fs_m_unscale(n, k, Xs, dinv, X_out, ldx, s));
  MultiState hm;
  FS_HIP(hipMemcpyAsync(&hm, ms, sizeof(MultiState), hipMemcpyDeviceToHost, s));
  FS_HIP(hipStreamSynchronize(s));
  bool any_nc = false;
  if (info) {
    auto el = [&](int a, int bb) -> double {
      float t = 0;
      return (hipEventElapsedTime(&t, ev[a], ev[bb]) == hipSuccess) ? (double)t : -1.0;
    };
    for (int j = 0; j < k; ++j) {
      fs_info f{};
      f.iters[0] = iters0[j];
      f.iters[1] = iters1[j];
      f.flags = flags;
      if (o.steps == 2 && !conv[j] && !hm.zero[j]) f.flags |= 2;
      f.rank = nr;
      f.be_sk = hm.be_sk[j];
      f.normest = hs.normest;
      f.condest = hs.condest;
      f.cnorm[0] = cnorm0[j];
      f.cnorm[1] = cnorm1[j];
      f.svd_sweeps = svd_sweeps;
      f.kw_evals = hm.kw_evals[j];
      f.phase_ms[0] = el(0, 1);
      f.phase_ms[1] = el(1, 2);
      f.phase_ms[2] = el(2, 3);
      f.phase_ms[3] = el(3, 5);
      f.phase_ms[4] = el(5, 6);
      f.phase_ms[5] = (o.steps > 1) ? el(6, 7) : 0.0;
      info[j] = f;
    }
  }
  for (int j = 0; j < k; ++j) any_nc |= (o.steps == 2 && !conv[j] && !hm.zero[j]);
  if (flags & 1) return FS_WARN_RANK_DEFICIENT;
  if (any_nc) return FS_WARN_NOT_CONVERGED;
  return FS_OK;
}
