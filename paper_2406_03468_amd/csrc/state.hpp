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
  int stop;              // inner-loop stop flag
  int iters;             // inner iterations in the current step
  int converged;         // the current step stopped by its rule (not by the cap)
  int max_inner;         // iteration cap per step
  int rank_trunc;        // #{sigma_i > tau normest}
  int kw_evals;          // sketched-KW evaluations
  int pad[2];
};

hipError_t fs_vec_gemv_v(const double* V, int64_t ldv, int n, int k, const double* y, const double* ydiv,
                         const double* oscale, const double* addv, double* out, double* part, const int* stop,
                         hipStream_t s);
hipError_t fs_vec_gemv_vt(const double* V, int64_t ldv, int n, int k, const double* v, const double* div, double* out,
                          const int* stop, hipStream_t s);
hipError_t fs_vec_polyak(int n, const double* c, const double* u, double* dy, double* dy_old, DevState* st,
                         bool first_step, hipStream_t s);
hipError_t fs_vec_cg(int n, double* p, const double* q, double* res, double* dy, DevState* st, bool first_step,
                     hipStream_t s);
hipError_t fs_vec_step_init(int n, const double* c, double* a, double* b, double* dy, bool spir, DevState* st,
                            hipStream_t s);
hipError_t fs_vec_add_norm(int n, const double* x, const double* z, double* out, double* norm2, const int* stop,
                           hipStream_t s);
hipError_t fs_vec_mul(int n, const double* a, const double* b, double* out, const int* stop, hipStream_t s);
hipError_t fs_vec_scaling(int n, const double* colnorm2, bool use_scaling, double* dinv, DevState* st, hipStream_t s);
hipError_t fs_vec_sigma_stats(int n, const double* sigma, double tau_factor, DevState* st, hipStream_t s);
hipError_t fs_vec_first_threshold(int n, const double* x0, double gamma, double rho, DevState* st, hipStream_t s);
hipError_t fs_vec_kw(int n, const double* w, const double* sigma, DevState* st, hipStream_t s);
hipError_t fs_vec_set_int(int* p, int v, hipStream_t s);
hipError_t fs_vec_set_double(double* p, double v, hipStream_t s);
hipError_t fs_vec_state_init(DevState* st, double alpha, double beta, int max_inner, hipStream_t s);
hipError_t fs_vec_trmv_t(const double* R, int64_t ldr, int n, const double* t, double* out, hipStream_t s);
