// n-vector kernels of the batched refinement (fossils_solve_batched): the heavy-ball iteration of
// Algorithm 4 (FOSSILS) or the CG iteration of Algorithm 3 (SPIR), each problem's method, with
// P = V Sigma^{-1}, for many problems in lockstep.  Each launch covers every problem of the batch
// (blockIdx.y or blockIdx.x = problem); a problem whose stop flag is set skips the kernels of an inner
// iteration, as in the single-problem kernels.  The arithmetic of each problem is that of the
// single-problem kernels (k_gemv_v_part / k_sum_slices, k_gemv_vt, k_polyak, k_cg, k_kw, ...).
#include "common.hpp"
#include "internal.hpp"
#include "state.hpp"

namespace {

constexpr int BNT = 1024;
constexpr double U_ROUND = 2.220446049250313e-16;
constexpr int GEMV_CS = 64;  // columns per slice of the V products

__device__ __forceinline__ double bbsum(double v, double* sh) { return block_sum<BNT>(v, sh); }
__device__ __forceinline__ bool b_stopped(const BatchVec& p) { return p.st->stop != 0; }

// P y partial sums: part[slice][i] = sum_{j in slice} V[i, j] y[j] / sigma[j], y = dy (or p for SPIR in
// the iteration's product, stop_aware = 2); stop_aware 0: the final update, run for every problem
__global__ __launch_bounds__(256) void k_b_gemv_v_part(const BatchVec* __restrict__ list, int stop_aware) {
  const BatchVec& p = list[blockIdx.z];
  if (stop_aware && b_stopped(p)) return;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * GEMV_CS, j1 = min(n, j0 + GEMV_CS);
  if (i >= n || j0 >= n) return;
  const double* y = (stop_aware == 2 && p.spir) ? p.p : p.dy;  // the direction of the iteration (mode 0)
  double s = 0.0;
  for (int j = j0; j < j1; ++j) s = fma(p.V[(int64_t)j * n + i], y[j] / p.sigma[j], s);
  p.gpart[(int64_t)blockIdx.y * n + i] = s;
}

// mode 0: zs = dinv .* (P dy);  mode 1: xh = x + P dy;  mode 2: x = x + P dy
__global__ __launch_bounds__(256) void k_b_sum_slices(const BatchVec* __restrict__ list, int mode) {
  const BatchVec& p = list[blockIdx.y];
  if (mode != 2 && b_stopped(p)) return;
  const int n = p.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int ns = (n + GEMV_CS - 1) / GEMV_CS;
  double s = 0.0;
  for (int q = 0; q < ns; ++q) s += p.gpart[(int64_t)q * n + i];
  if (mode == 0) p.zs[i] = s * p.dinv[i];
  else if (mode == 1) p.xh[i] = p.x[i] + s;
  else p.x[i] = p.x[i] + s;
}

// mode 0: c = Sigma^{-1} V^T g;  mode 1: u = Sigma^{-1} V^T v (stop-aware);  mode 2: w = V^T g (stop-aware)
__global__ __launch_bounds__(256) void k_b_gemv_vt(const BatchVec* __restrict__ list, int mode) {
  const BatchVec& p = list[blockIdx.y];
  if (mode != 0 && b_stopped(p)) return;
  const int n = p.n;
  const int j = blockIdx.x;
  if (j >= n) return;
  __shared__ double sh[4];
  const double* in = (mode == 1) ? p.v : p.g;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s = fma(p.V[(int64_t)j * n + i], in[i], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) {
    if (mode == 0) p.c[j] = s / p.sigma[j];
    else if (mode == 1) p.u[j] = s / p.sigma[j];
    else p.w[j] = s;
  }
}

// zs = dinv .* x (mode 0, start of a step) or dinv .* xh (mode 1, KW check; stop-aware)
__global__ __launch_bounds__(BNT) void k_b_scale(const BatchVec* __restrict__ list, int mode) {
  const BatchVec& p = list[blockIdx.x];
  if (mode == 1 && b_stopped(p)) return;
  const double* src = mode ? p.xh : p.x;
  for (int i = threadIdx.x; i < p.n; i += BNT) p.zs[i] = src[i] * p.dinv[i];
}

// first-step threshold (gamma normest ||x_0|| + rho condest ||r_0||) u, as k_first_threshold
__global__ __launch_bounds__(BNT) void k_b_first_threshold(const BatchVec* __restrict__ list, double gamma,
                                                           double rho) {
  const BatchVec& p = list[blockIdx.x];
  __shared__ double sh[BNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < p.n; i += BNT) s = fma(p.x0[i], p.x0[i], s);
  s = bbsum(s, sh);
  if (threadIdx.x == 0) {
    DevState* st = p.st;
    st->x0norm = sqrt(s);
    st->r0norm = sqrt(st->r2);
    st->thr_first = (gamma * st->normest * st->x0norm + rho * st->condest * st->r0norm) * U_ROUND;
    st->fro_u = sqrt(st->fro2) * U_ROUND;
  }
}

// start of a step, as k_step_init: FOSSILS dy = dy_old = c; SPIR res = p = c, dy = 0
__global__ __launch_bounds__(BNT) void k_b_step_init(const BatchVec* __restrict__ list) {
  const BatchVec& p = list[blockIdx.x];
  __shared__ double sh[BNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < p.n; i += BNT) {
    const double v = p.c[i];
    if (p.spir) {
      p.res[i] = v;
      p.p[i] = v;
      p.dy[i] = 0.0;
    } else {
      p.dy[i] = v;
      p.dy_old[i] = v;
    }
    s = fma(v, v, s);
  }
  s = bbsum(s, sh);
  if (threadIdx.x == 0) {
    DevState* st = p.st;
    st->rho_cg = s;
    st->cnorm2 = s;
    st->stop = p.done ? 1 : 0;
    st->iters = 0;
    st->converged = p.done ? 1 : 0;
  }
}

// the heavy-ball update with the first-step rule, as k_polyak
__device__ __forceinline__ void polyak_one(const BatchVec& p, int first_step, double* sh) {
  DevState* st = p.st;
  const double al = st->alpha, be = st->beta;
  double s = 0.0;
  for (int i = threadIdx.x; i < p.n; i += BNT) {
    const double y = p.dy[i];
    const double D = al * (p.c[i] - p.u[i]) + be * (y - p.dy_old[i]);
    p.dy_old[i] = y;
    p.dy[i] = y + D;
    s = fma(D, D, s);
  }
  s = bbsum(s, sh);
  if (threadIdx.x == 0) {
    st->dnorm2 = s;
    st->iters += 1;
    if (first_step && sqrt(s) <= st->thr_first) {
      st->stop = 1;
      st->converged = 1;
    }
    if (st->iters >= st->max_inner) st->stop = 1;
  }
}

// CG on the preconditioned normal equations (SPIR), as k_cg: q = u = P^T A_s^T A_s P p given;
// a = rho / p^T q; Delta = a p; dy += Delta; res -= a q; p = res + (rho' / rho) p; the first-step rule
__device__ __forceinline__ void cg_one(const BatchVec& b, int first_step, double* sh) {
  DevState* st = b.st;
  double s = 0.0;
  for (int i = threadIdx.x; i < b.n; i += BNT) s = fma(b.p[i], b.u[i], s);
  const double pq = bbsum(s, sh);
  const double rho = st->rho_cg;
  if (!(pq > 0.0) || rho == 0.0) {
    if (threadIdx.x == 0) {
      st->stop = 1;
      if (rho == 0.0) st->converged = 1;
    }
    return;
  }
  const double a = rho / pq;
  double s2 = 0.0, sd = 0.0;
  for (int i = threadIdx.x; i < b.n; i += BNT) {
    const double D = a * b.p[i];
    b.dy[i] += D;
    const double r = b.res[i] - a * b.u[i];
    b.res[i] = r;
    s2 = fma(r, r, s2);
    sd = fma(D, D, sd);
  }
  const double rho2 = bbsum(s2, sh);
  const double dn2 = bbsum(sd, sh);
  const double bet = rho2 / rho;
  for (int i = threadIdx.x; i < b.n; i += BNT) b.p[i] = b.res[i] + bet * b.p[i];
  if (threadIdx.x == 0) {
    st->rho_cg = rho2;
    st->dnorm2 = dn2;
    st->iters += 1;
    if (first_step && sqrt(dn2) <= st->thr_first) {
      st->stop = 1;
      st->converged = 1;
    }
    if (st->iters >= st->max_inner) st->stop = 1;
  }
}

// one inner-iteration update per problem: heavy ball (FOSSILS) or CG (SPIR), uniform per work-group
__global__ __launch_bounds__(BNT) void k_b_update(const BatchVec* __restrict__ list, int first_step) {
  const BatchVec& p = list[blockIdx.x];
  if (p.st->stop) return;
  __shared__ double sh[BNT / 64];
  if (p.spir) cg_one(p, first_step, sh);
  else polyak_one(p, first_step, sh);
}

// ||x_hat||^2 (KW check)
__global__ __launch_bounds__(BNT) void k_b_xh_norm(const BatchVec* __restrict__ list) {
  const BatchVec& p = list[blockIdx.x];
  if (b_stopped(p)) return;
  __shared__ double sh[BNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < p.n; i += BNT) s = fma(p.xh[i], p.xh[i], s);
  s = bbsum(s, sh);
  if (threadIdx.x == 0) p.st->x2 = s;
}

// the sketched KW estimate and the second-step rule, as k_kw (w = V^T g given)
__global__ __launch_bounds__(BNT) void k_b_kw(const BatchVec* __restrict__ list) {
  const BatchVec& p = list[blockIdx.x];
  DevState* st = p.st;
  if (st->stop) return;
  __shared__ double sh[BNT / 64];
  const double th2 = st->theta2;
  const double x2 = st->x2, r2 = st->r2;
  const double lam = th2 * r2 / (1.0 + th2 * x2);
  double s = 0.0;
  for (int i = threadIdx.x; i < p.n; i += BNT) {
    const double si = p.sigma[i];
    s += p.w[i] * p.w[i] / (si * si + lam);
  }
  s = bbsum(s, sh);
  if (threadIdx.x == 0) {
    const double be = sqrt(th2 / (1.0 + th2 * x2)) * sqrt(s);
    st->be_sk = be;
    st->kw_evals += 1;
    if (be < st->fro_u) {
      st->stop = 1;
      st->converged = 1;
    }
  }
}

// x_out = dinv .* x
__global__ __launch_bounds__(BNT) void k_b_final(const BatchVec* __restrict__ list) {
  const BatchVec& p = list[blockIdx.x];
  if (p.done) return;
  for (int i = threadIdx.x; i < p.n; i += BNT) p.x_out[i] = p.x[i] * p.dinv[i];
}

// after the setup: theta^2 = ||A_s||_F^2 / ||b||^2, ||b||^2 from the sketch's read of b
__global__ void k_b_prep(const double* __restrict__ colnorm2, int n, DevState* __restrict__ st) {
  if (threadIdx.x == 0) {
    const double b2 = colnorm2[n];
    st->b2 = b2;
    st->theta2 = (b2 > 0.0) ? st->fro2 / b2 : 0.0;
  }
}

// out[k] = problem k's state (one read-back for the host's polls)
__global__ void k_b_gather(const BatchVec* __restrict__ list, int count, DevState* __restrict__ out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) out[k] = *list[k].st;
}

__global__ __launch_bounds__(256) void k_b_report(const DevState* __restrict__ st, const int* __restrict__ sweeps,
                                                  const int* __restrict__ qr_err, const int* __restrict__ svd_err,
                                                  const int* __restrict__ trsv_err,
                                                  const double* __restrict__ colnorm2, int n,
                                                  BatchReport* __restrict__ out) {
  int nan = 0, inf = 0;
  for (int j = threadIdx.x; j <= n; j += 256) {
    const double v = colnorm2[j];
    nan |= isnan(v) ? 1 : 0;
    inf |= isfinite(v) ? 0 : 1;
  }
  nan = __syncthreads_or(nan);
  inf = __syncthreads_or(inf);
  if (threadIdx.x == 0) {
    out->st = *st;
    out->sweeps = *sweeps;
    out->err = (*qr_err != 0 || *svd_err != 0 || *trsv_err != 0) ? 1 : 0;
    out->nan = nan;
    out->inf = inf;
    out->b2 = colnorm2[n];
  }
}

}  // namespace

hipError_t fs_b_report(const DevState* st, const int* sweeps, const int* qr_err, const int* svd_err,
                       const int* trsv_err, const double* colnorm2, int n, BatchReport* out, hipStream_t s) {
  hipLaunchKernelGGL(k_b_report, dim3(1), dim3(256), 0, s, st, sweeps, qr_err, svd_err, trsv_err, colnorm2, n, out);
  return hipGetLastError();
}

hipError_t fs_b_gather(const BatchVec* list, int count, DevState* out, hipStream_t s) {
  hipLaunchKernelGGL(k_b_gather, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, list, count, out);
  return hipGetLastError();
}

hipError_t fs_b_gemv_P(const BatchVec* list, int count, int max_n, int mode, hipStream_t s) {
  const int ns = (max_n + GEMV_CS - 1) / GEMV_CS;
  hipLaunchKernelGGL(k_b_gemv_v_part, dim3((unsigned)((max_n + 255) / 256), (unsigned)ns, (unsigned)count), dim3(256),
                     0, s, list, mode == 0 ? 2 : (mode == 1 ? 1 : 0));
  hipLaunchKernelGGL(k_b_sum_slices, dim3((unsigned)((max_n + 255) / 256), (unsigned)count), dim3(256), 0, s, list,
                     mode);
  return hipGetLastError();
}

hipError_t fs_b_gemv_PT(const BatchVec* list, int count, int max_n, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_b_gemv_vt, dim3((unsigned)max_n, (unsigned)count), dim3(256), 0, s, list, mode);
  return hipGetLastError();
}

hipError_t fs_b_vec(const BatchVec* list, int count, BatchOp op, int arg, double gamma, double rho, hipStream_t s) {
  const dim3 g((unsigned)count), b(BNT);
  switch (op) {
    case BatchOp::SCALE: hipLaunchKernelGGL(k_b_scale, g, b, 0, s, list, arg); break;
    case BatchOp::FIRST_THRESHOLD: hipLaunchKernelGGL(k_b_first_threshold, g, b, 0, s, list, gamma, rho); break;
    case BatchOp::STEP_INIT: hipLaunchKernelGGL(k_b_step_init, g, b, 0, s, list); break;
    case BatchOp::UPDATE: hipLaunchKernelGGL(k_b_update, g, b, 0, s, list, arg); break;
    case BatchOp::XH_NORM: hipLaunchKernelGGL(k_b_xh_norm, g, b, 0, s, list); break;
    case BatchOp::KW: hipLaunchKernelGGL(k_b_kw, g, b, 0, s, list); break;
    case BatchOp::FINAL: hipLaunchKernelGGL(k_b_final, g, b, 0, s, list); break;
  }
  return hipGetLastError();
}

hipError_t fs_b_prep(const double* colnorm2, int n, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_b_prep, dim3(1), dim3(64), 0, s, colnorm2, n, st);
  return hipGetLastError();
}
