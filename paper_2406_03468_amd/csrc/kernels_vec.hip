// n-vector work of the refinement loop: triangular solves with R, products with V Sigma^{-1},
// the heavy-ball and CG updates, the stopping rules and the sketched Karlson-Walden estimate.
// Every reduction is a fixed-order tree (deterministic).  Kernels of an inner iteration take the
// device stop flag and return at once when it is set.
#include "common.hpp"
#include "internal.hpp"
#include "state.hpp"

namespace {

constexpr int VNT = 1024;
constexpr double U_ROUND = 2.220446049250313e-16;

// ---------------------------------------------------------------- triangular solves (one work-group)
// Back substitution R x = y (upper) or forward substitution R^T x = y, blocked by 64: the diagonal
// block is solved by one wave row by row; the off-diagonal blocks are applied by all threads.
// x may alias y.  x_out = xscale .* x (optional); y is read as yscale .* y (optional).
__global__ __launch_bounds__(VNT) void k_trsv(const double* __restrict__ R, int64_t ldr, int n, int transpose,
                                              const double* y, double* x, const double* __restrict__ yscale,
                                              const double* __restrict__ xscale, const int* __restrict__ stop,
                                              int64_t ldy, int64_t ldx) {
  if (fs_stopped(stop)) return;
  y += (int64_t)blockIdx.x * ldy;  // batched: right-hand side blockIdx.x
  x += (int64_t)blockIdx.x * ldx;
  extern __shared__ double xs[];   // n
  __shared__ double dblk[64][65];  // current 64 x 64 diagonal block of R (padded)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < n; i += VNT) xs[i] = yscale ? y[i] * yscale[i] : y[i];
  const int nblk = (n + 63) / 64;
  auto load_diag = [&](int b0, int b1) {
    // dblk[r][c] = R[b0 + r, b0 + c] for r <= c (coalesced down each column)
    for (int q = tid; q < 64 * 64; q += VNT) {
      const int r = q & 63, c = q >> 6;
      dblk[r][c] = (b0 + r < b1 && b0 + c < b1 && r <= c) ? R[(int64_t)(b0 + c) * ldr + b0 + r] : 0.0;
    }
  };
  if (!transpose) {
    for (int kb = nblk - 1; kb >= 0; --kb) {
      const int b0 = kb * 64, b1 = min(n, b0 + 64);
      load_diag(b0, b1);
      __syncthreads();
      if (wv == 0) {  // rows b0..b1-1 held by lanes; solve bottom-up from LDS
        double xi = (b0 + lane < b1) ? xs[b0 + lane] : 0.0;
        for (int i = b1 - 1 - b0; i >= 0; --i) {
          const double xv = __shfl(xi, i, 64) / dblk[i][i];
          if (lane == i) xi = xv;
          if (lane < i) xi = fma(-dblk[lane][i], xv, xi);
        }
        if (b0 + lane < b1) xs[b0 + lane] = xi;
      }
      __syncthreads();
      // x[0:b0] -= R[0:b0, b0:b1] x[b0:b1]: eight independent sums per row, so that eight loads of R
      // are in flight at a time instead of one
      for (int i = tid; i < b0; i += VNT) {
        double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int j = b0;
        for (; j + 8 <= b1; j += 8) {
#pragma unroll
          for (int u = 0; u < 8; ++u) s8[u] = fma(R[(int64_t)(j + u) * ldr + i], xs[j + u], s8[u]);
        }
        for (; j < b1; ++j) s8[0] = fma(R[(int64_t)j * ldr + i], xs[j], s8[0]);
        xs[i] -= ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
      }
      __syncthreads();
    }
  } else {
    for (int kb = 0; kb < nblk; ++kb) {
      const int b0 = kb * 64, b1 = min(n, b0 + 64);
      load_diag(b0, b1);
      // x[b0:b1] -= R[0:b0, b0:b1]^T x[0:b0]: 16 threads per output
      {
        const int o = tid >> 4, sub = tid & 15;
        const int i = b0 + o;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};  // four loads of R in flight per thread
        if (i < b1) {
          const double* Ri = R + (int64_t)i * ldr;
          int j = sub;
          for (; j + 48 < b0; j += 64) {
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] = fma(Ri[j + 16 * u], xs[j + 16 * u], s4[u]);
          }
          for (; j < b0; j += 16) s4[0] = fma(Ri[j], xs[j], s4[0]);
        }
        double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
        __syncthreads();
        if (i < b1 && sub == 0) xs[i] -= s;
        __syncthreads();
      }
      if (wv == 0) {  // forward substitution with R^T (lower) from LDS
        double xi = (b0 + lane < b1) ? xs[b0 + lane] : 0.0;
        for (int i = 0; i < b1 - b0; ++i) {
          const double xv = __shfl(xi, i, 64) / dblk[i][i];
          if (lane == i) xi = xv;
          if (lane > i) xi = fma(-dblk[i][lane], xv, xi);  // (R^T)[lane][i] = R[i][lane]
        }
        if (b0 + lane < b1) xs[b0 + lane] = xi;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += VNT) x[i] = xscale ? xs[i] * xscale[i] : xs[i];
}

// ---------------------------------------------------------------- dense products with V (n x k, ld)
// out[i] = oscale[i] * sum_j V[i, j] (y[j] * yscale[j])  -- partial over column slices
__global__ __launch_bounds__(256) void k_gemv_v_part(const double* __restrict__ V, int64_t ldv, int n, int k,
                                                     const double* __restrict__ y, const double* __restrict__ ydiv,
                                                     double* __restrict__ part, int cs, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int slice = blockIdx.y;
  const int j0 = slice * cs, j1 = min(k, j0 + cs);
  if (i >= n) return;
  double s = 0.0;
  for (int j = j0; j < j1; ++j) s = fma(V[(int64_t)j * ldv + i], ydiv ? y[j] / ydiv[j] : y[j], s);
  part[(int64_t)slice * n + i] = s;
}

__global__ __launch_bounds__(256) void k_sum_slices(const double* __restrict__ part, int nslices, int n,
                                                    const double* __restrict__ oscale, const double* __restrict__ addv,
                                                    double* __restrict__ out, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < nslices; ++q) s += part[(int64_t)q * n + i];
  if (addv) s += addv[i];
  out[i] = oscale ? s * oscale[i] : s;
}

// out[j] = (sum_i V[i, j] v[i]) / div[j]  for j < k: one work-group per column
__global__ __launch_bounds__(256) void k_gemv_vt(const double* __restrict__ V, int64_t ldv, int n, int k,
                                                 const double* __restrict__ v, const double* __restrict__ div,
                                                 double* __restrict__ out, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s = fma(V[(int64_t)j * ldv + i], v[i], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) out[j] = div ? s / div[j] : s;
}

// out[j] = sum_{i <= j} R[i, j] t[i]  (R^T t for upper-triangular R): one work-group per output
__global__ __launch_bounds__(256) void k_trmv_t(const double* __restrict__ R, int64_t ldr, int n,
                                                const double* __restrict__ t, double* __restrict__ out) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i <= j; i += 256) s = fma(R[(int64_t)j * ldr + i], t[i], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// ---------------------------------------------------------------- small vector kernels (one work-group)
__device__ __forceinline__ double bsum(double v, double* sh) { return block_sum<VNT>(v, sh); }

// Alg 1/5 heavy-ball update with Alg 4's first-step rule:
//   Delta = alpha (c - u) + beta (dy - dy_old); dy_old <- dy; dy <- dy + Delta;
//   if first_step and ||Delta|| <= thr_first: stop.
__global__ __launch_bounds__(VNT) void k_polyak(int n, const double* __restrict__ c, const double* __restrict__ u,
                                                double* __restrict__ dy, double* __restrict__ dy_old,
                                                DevState* __restrict__ st, int first_step) {
  if (st->stop) return;
  __shared__ double sh[VNT / 64];
  const double al = st->alpha, be = st->beta;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double y = dy[i];
    const double D = al * (c[i] - u[i]) + be * (y - dy_old[i]);
    dy_old[i] = y;
    dy[i] = y + D;
    s = fma(D, D, s);
  }
  s = bsum(s, sh);
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

// CG on M dy = c (SPIR): q = M p given; a = rho / p^T q; Delta = a p; dy += Delta; res -= a q;
// rho' = res^T res; p = res + (rho'/rho) p.
__global__ __launch_bounds__(VNT) void k_cg(int n, double* __restrict__ p, const double* __restrict__ q,
                                            double* __restrict__ res, double* __restrict__ dy,
                                            DevState* __restrict__ st, int first_step) {
  if (st->stop) return;
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) s = fma(p[i], q[i], s);
  const double pq = bsum(s, sh);
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
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double D = a * p[i];
    dy[i] += D;
    const double r = res[i] - a * q[i];
    res[i] = r;
    s2 = fma(r, r, s2);
    sd = fma(D, D, sd);
  }
  const double rho2 = bsum(s2, sh);
  const double dn2 = bsum(sd, sh);
  const double bet = rho2 / rho;
  for (int i = threadIdx.x; i < n; i += VNT) p[i] = res[i] + bet * p[i];
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

// LSQR (Paige and Saunders) on min || r - (A_s P) dy ||, the LSQR form of SPIR (Section 4.3).
// Start: beta_1 u_1 = r (st->r2 = ||r||^2), alpha_1 v_1 = (A_s P)^T u_1 = c / beta_1, w = v_1,
// phibar = beta_1, rhobar = alpha_1, dy = 0.  A zero r or c ends the step at once (dy = 0 is exact).
__global__ __launch_bounds__(VNT) void k_lsqr_init(int n, const double* __restrict__ c, double* __restrict__ v,
                                                   double* __restrict__ w, double* __restrict__ dy,
                                                   DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) s = fma(c[i], c[i], s);
  const double cn2 = bsum(s, sh);
  const double cn = sqrt(cn2), bet = sqrt(st->r2);
  const bool zero = !(cn > 0.0) || !(bet > 0.0);
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double vi = zero ? 0.0 : c[i] / cn;
    v[i] = vi;
    w[i] = vi;
    dy[i] = 0.0;
  }
  if (threadIdx.x == 0) {
    st->cnorm2 = cn2;
    st->iters = 0;
    st->l_beta = bet;
    st->l_alpha = zero ? 0.0 : cn / bet;
    st->l_phibar = bet;
    st->l_rhobar = st->l_alpha;
    st->stop = zero ? 1 : 0;
    st->converged = zero ? 1 : 0;
  }
}

// One step.  Input h = P^T A_s^T (alpha u - A_s P v) = -beta P^T A_s^T u' (the pass ran on
// ubar = alpha u), st->r2 = beta^2.  Then
//   alpha' v' = -h / beta - beta v;  rho = hypot(rhobar, beta), c = rhobar / rho, s = beta / rho,
//   theta = s alpha', rhobar' = -c alpha', phi = c phibar, phibar' = s phibar,
//   Delta = (phi / rho) w, dy += Delta, w' = v' - (theta / rho) w,
// with SPIR's first-step rule on ||Delta||, the cap, and termination at beta = 0 or alpha' = 0.
__global__ __launch_bounds__(VNT) void k_lsqr_step(int n, const double* __restrict__ h, double* __restrict__ v,
                                                   double* __restrict__ w, double* __restrict__ dy,
                                                   DevState* __restrict__ st, int first_step) {
  if (st->stop) return;
  __shared__ double sh[VNT / 64];
  const double bet = sqrt(st->r2);
  const double ib = (bet > 0.0) ? 1.0 / bet : 0.0;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double si = -h[i] * ib - bet * v[i];
    v[i] = si;  // unnormalized until alpha' is known
    s = fma(si, si, s);
  }
  const double alf = sqrt(bsum(s, sh));
  const double ia = (alf > 0.0) ? 1.0 / alf : 0.0;
  const double rhobar = st->l_rhobar, phibar = st->l_phibar;
  const double rho = hypot(rhobar, bet);
  const double cs = rhobar / rho, sn = bet / rho;
  const double theta = sn * alf, phi = cs * phibar;
  const double fd = phi / rho, fw = theta / rho;
  double sd = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double vi = v[i] * ia;
    v[i] = vi;
    const double wi = w[i];
    const double D = fd * wi;
    dy[i] += D;
    w[i] = vi - fw * wi;
    sd = fma(D, D, sd);
  }
  const double dn2 = bsum(sd, sh);
  if (threadIdx.x == 0) {
    st->l_alpha = alf;
    st->l_beta = bet;
    st->l_rhobar = -cs * alf;
    st->l_phibar = sn * phibar;
    st->dnorm2 = dn2;
    st->iters += 1;
    if (!(bet > 0.0) || !(alf > 0.0)) {
      st->stop = 1;
      st->converged = 1;
    }
    if (first_step && sqrt(dn2) <= st->thr_first) {
      st->stop = 1;
      st->converged = 1;
    }
    if (st->iters >= st->max_inner) st->stop = 1;
  }
}

// ubar = sign (alpha / beta) r: alpha_1 u_1 = (alpha_1 / beta_1) r at the start of a step (sign +1);
// alpha' u' = -(alpha' / beta) r_out inside the iteration (sign -1, r_out = alpha u - A_s P v).
__global__ __launch_bounds__(256) void k_lsqr_ubar(int64_t m, const double* __restrict__ r, double* __restrict__ ubar,
                                                   double sign, const DevState* __restrict__ st) {
  if (st->stop) return;
  const double bet = st->l_beta;
  const double f = (bet > 0.0) ? sign * st->l_alpha / bet : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    ubar[i] = f * r[i];
}

// Lower bounds of normest and condest from the diagonal of R (|r_ii| lies between sigma_min and
// sigma_max), used for the first-step threshold until the SVD of R has produced the true values:
// the threshold they give is never above the true one.
__global__ __launch_bounds__(VNT) void k_diag_bounds(int n, const double* __restrict__ R, int64_t ldr,
                                                     DevState* __restrict__ st) {
  __shared__ double smax[VNT / 64], smin[VNT / 64];
  double mx = 0.0, mn = INFINITY;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double a = fabs(R[(int64_t)i * ldr + i]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    mn = fmin(mn, __shfl_xor(mn, off, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smax[w] = mx;
    smin[w] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < VNT / 64; ++i) {
      mx = fmax(mx, smax[i]);
      mn = fmin(mn, smin[i]);
    }
    mx = fmax(mx, smax[0]);
    mn = fmin(mn, smin[0]);
    st->normest = mx;
    st->condest = (mn > 0.0) ? mx / mn : 0.0;  // a zero diagonal: no usable bound
  }
}

// First-step history while the SVD of R is still running (its normest and condest, hence the
// first-step threshold, are not known yet): after inner iteration j (0-based) the iterate dy and
// ||Delta||^2 are recorded when the iteration ran (iters == j + 1).
__global__ __launch_bounds__(VNT) void k_record_iter(int j, int n, const double* __restrict__ dy,
                                                     double* __restrict__ hist_dy, double* __restrict__ hist_dn,
                                                     const DevState* __restrict__ st) {
  if (st->iters != j + 1) return;
  for (int i = threadIdx.x; i < n; i += VNT) hist_dy[(int64_t)j * n + i] = dy[i];
  if (threadIdx.x == 0) hist_dn[j] = st->dnorm2;
}

// Once the threshold is known: the first recorded iteration with ||Delta|| <= thr_first is where
// the first-step rule stops (Alg 4); its iterate becomes dy and the step ends there.
__global__ __launch_bounds__(VNT) void k_rollback(int n, const double* __restrict__ hist_dy,
                                                  const double* __restrict__ hist_dn, double* __restrict__ dy,
                                                  DevState* __restrict__ st) {
  __shared__ int sj;
  if (threadIdx.x == 0) {
    int jj = -1;
    const double thr = st->thr_first;
    for (int i = 0; i < st->iters; ++i)
      if (sqrt(hist_dn[i]) <= thr) {
        jj = i;
        break;
      }
    sj = jj;
  }
  __syncthreads();
  const int jj = sj;
  if (jj < 0) return;
  for (int i = threadIdx.x; i < n; i += VNT) dy[i] = hist_dy[(int64_t)jj * n + i];
  __syncthreads();
  if (threadIdx.x == 0) {
    st->iters = jj + 1;
    st->stop = 1;
    st->converged = 1;
  }
}

// Start of a refinement step: dy = dy_old = c (FOSSILS) or dy = 0, res = p = c (SPIR); rho = c^T c.
__global__ __launch_bounds__(VNT) void k_step_init(int n, const double* __restrict__ c, double* __restrict__ a,
                                                   double* __restrict__ b, double* __restrict__ dy, int spir,
                                                   DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double v = c[i];
    a[i] = v;
    b[i] = v;
    if (spir) dy[i] = 0.0;
    s = fma(v, v, s);
  }
  s = bsum(s, sh);
  if (threadIdx.x == 0) {
    st->rho_cg = s;
    st->cnorm2 = s;
    st->stop = 0;
    st->iters = 0;
    st->converged = 0;
  }
}

// x_hat = x + z (z = P dy already formed); ||x_hat||^2 into the state.
__global__ __launch_bounds__(VNT) void k_add_norm(int n, const double* __restrict__ x, const double* __restrict__ z,
                                                  double* __restrict__ out, double* __restrict__ norm2_out,
                                                  const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double v = z ? x[i] + z[i] : x[i];
    out[i] = v;
    s = fma(v, v, s);
  }
  s = bsum(s, sh);
  if (threadIdx.x == 0 && norm2_out) *norm2_out = s;
}

// out = a .* b (elementwise), or a copy when b is null
__global__ void k_mul(int n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                      const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = b ? a[i] * b[i] : a[i];
}

// Column scaling: dinv_j = 1/||a_j|| (1 for zero columns); ||A_s||_F^2 = sum_j ||a_j||^2 dinv_j^2.
__global__ __launch_bounds__(VNT) void k_scaling(int n, const double* __restrict__ colnorm2, int use_scaling,
                                                 double* __restrict__ dinv, DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double c2 = colnorm2[i];
    const double di = (use_scaling && c2 > 0.0) ? 1.0 / sqrt(c2) : 1.0;
    dinv[i] = di;
    s = fma(c2 * di, di, s);
  }
  s = bsum(s, sh);
  if (threadIdx.x == 0) st->fro2 = s;
}

// normest, condest from sigma (descending); rank for truncation (Alg 4).
__global__ void k_sigma_stats(int n, const double* __restrict__ sigma, double tau_factor, DevState* __restrict__ st) {
  if (threadIdx.x == 0) {
    const double s1 = sigma[0], sn = sigma[n - 1];
    st->normest = s1;
    st->condest = (sn > 0.0) ? s1 / sn : INFINITY;
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sigma[i] > tau_factor * U_ROUND * s1) ? 1 : 0;
    st->rank_trunc = r;
  }
}

// After the residual pass at x_0: keep ||x_0||, ||r_0|| and the first-step threshold (Alg 4).
__global__ __launch_bounds__(VNT) void k_first_threshold(int n, const double* __restrict__ x0, double gamma,
                                                         double rho, DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) s = fma(x0[i], x0[i], s);
  s = bsum(s, sh);
  if (threadIdx.x == 0) {
    st->x0norm = sqrt(s);
    st->r0norm = sqrt(st->r2);
    st->thr_first = (gamma * st->normest * st->x0norm + rho * st->condest * st->r0norm) * U_ROUND;
    st->fro_u = sqrt(st->fro2) * U_ROUND;
  }
}

// Sketched Karlson-Walden estimate (eq:sketched-kw, via the SVD of the sketch) and the
// second-step rule BE_sk < ||A||_F u.  w = V^T g is given (g = A_s^T r_hat); x2 = ||x_hat||^2,
// r2 = ||r_hat||^2 in the state; theta = ||A_s||_F / ||b||.
__global__ __launch_bounds__(VNT) void k_kw(int n, const double* __restrict__ w, const double* __restrict__ sigma,
                                            DevState* __restrict__ st) {
  if (st->stop) return;
  __shared__ double sh[VNT / 64];
  const double th2 = st->theta2;
  const double x2 = st->x2, r2 = st->r2;
  const double lam = th2 * r2 / (1.0 + th2 * x2);
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double si = sigma[i];
    s += w[i] * w[i] / (si * si + lam);
  }
  s = bsum(s, sh);
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

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_set_double(double* p, double v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_state_init(DevState* st, double alpha, double beta, int max_inner) {
  if (threadIdx.x == 0) {
    DevState z{};
    z.alpha = alpha;
    z.beta = beta;
    z.max_inner = max_inner;
    *st = z;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t fs_launch_trsv(const double* R, int64_t ldr, int n, bool transpose, const double* y, double* x,
                          const double* yscale, const double* xscale, const int* stop, hipStream_t s) {
  const size_t sh = (size_t)n * sizeof(double);
  if (sh > 120 * 1024) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_trsv, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL(k_trsv, dim3(1), dim3(VNT), sh, s, R, ldr, n, transpose ? 1 : 0, y, x, yscale, xscale, stop,
                     (int64_t)0, (int64_t)0);
  return hipGetLastError();
}

hipError_t fs_launch_trsv_batched(const double* R, int64_t ldr, int n, bool transpose, const double* Yb, int64_t ldy,
                                  double* Xb, int64_t ldx, int nrhs, hipStream_t s) {
  const size_t sh = (size_t)n * sizeof(double);
  if (sh > 120 * 1024 || nrhs < 1) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)k_trsv, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
  hipLaunchKernelGGL(k_trsv, dim3((unsigned)nrhs), dim3(VNT), sh, s, R, ldr, n, transpose ? 1 : 0, Yb, Xb,
                     (const double*)nullptr, (const double*)nullptr, (const int*)nullptr, ldy, ldx);
  return hipGetLastError();
}

hipError_t fs_vec_gemv_v(const double* V, int64_t ldv, int n, int k, const double* y, const double* ydiv,
                         const double* oscale, const double* addv, double* out, double* part, const int* stop,
                         hipStream_t s) {
  const int cs = 64;
  const int ns = (k + cs - 1) / cs;
  hipLaunchKernelGGL(k_gemv_v_part, dim3((n + 255) / 256, ns), dim3(256), 0, s, V, ldv, n, k, y, ydiv, part, cs,
                     stop);
  hipLaunchKernelGGL(k_sum_slices, dim3((n + 255) / 256), dim3(256), 0, s, part, ns, n, oscale, addv, out, stop);
  return hipGetLastError();
}

hipError_t fs_vec_gemv_vt(const double* V, int64_t ldv, int n, int k, const double* v, const double* div, double* out,
                          const int* stop, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_vt, dim3(k), dim3(256), 0, s, V, ldv, n, k, v, div, out, stop);
  return hipGetLastError();
}

hipError_t fs_vec_polyak(int n, const double* c, const double* u, double* dy, double* dy_old, DevState* st,
                         bool first_step, hipStream_t s) {
  hipLaunchKernelGGL(k_polyak, dim3(1), dim3(VNT), 0, s, n, c, u, dy, dy_old, st, first_step ? 1 : 0);
  return hipGetLastError();
}

hipError_t fs_vec_diag_bounds(int n, const double* R, int64_t ldr, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_bounds, dim3(1), dim3(VNT), 0, s, n, R, ldr, st);
  return hipGetLastError();
}
hipError_t fs_vec_record_iter(int j, int n, const double* dy, double* hist_dy, double* hist_dn, const DevState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_record_iter, dim3(1), dim3(VNT), 0, s, j, n, dy, hist_dy, hist_dn, st);
  return hipGetLastError();
}
hipError_t fs_vec_rollback(int n, const double* hist_dy, const double* hist_dn, double* dy, DevState* st,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rollback, dim3(1), dim3(VNT), 0, s, n, hist_dy, hist_dn, dy, st);
  return hipGetLastError();
}
hipError_t fs_vec_lsqr_init(int n, const double* c, double* v, double* w, double* dy, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_init, dim3(1), dim3(VNT), 0, s, n, c, v, w, dy, st);
  return hipGetLastError();
}
hipError_t fs_vec_lsqr_step(int n, const double* h, double* v, double* w, double* dy, DevState* st, bool first_step,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_step, dim3(1), dim3(VNT), 0, s, n, h, v, w, dy, st, first_step ? 1 : 0);
  return hipGetLastError();
}
hipError_t fs_vec_lsqr_ubar(int64_t m, const double* r, double* ubar, double sign, const DevState* st,
                            hipStream_t s) {
  const int64_t nb = (m + 255) / 256;
  hipLaunchKernelGGL(k_lsqr_ubar, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, s, m, r, ubar, sign, st);
  return hipGetLastError();
}

hipError_t fs_vec_cg(int n, double* p, const double* q, double* res, double* dy, DevState* st, bool first_step,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_cg, dim3(1), dim3(VNT), 0, s, n, p, q, res, dy, st, first_step ? 1 : 0);
  return hipGetLastError();
}

hipError_t fs_vec_step_init(int n, const double* c, double* a, double* b, double* dy, bool spir, DevState* st,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_step_init, dim3(1), dim3(VNT), 0, s, n, c, a, b, dy, spir ? 1 : 0, st);
  return hipGetLastError();
}

hipError_t fs_vec_add_norm(int n, const double* x, const double* z, double* out, double* norm2, const int* stop,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_add_norm, dim3(1), dim3(VNT), 0, s, n, x, z, out, norm2, stop);
  return hipGetLastError();
}

hipError_t fs_vec_mul(int n, const double* a, const double* b, double* out, const int* stop, hipStream_t s) {
  hipLaunchKernelGGL(k_mul, dim3((n + 255) / 256), dim3(256), 0, s, n, a, b, out, stop);
  return hipGetLastError();
}

hipError_t fs_vec_scaling(int n, const double* colnorm2, bool use_scaling, double* dinv, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_scaling, dim3(1), dim3(VNT), 0, s, n, colnorm2, use_scaling ? 1 : 0, dinv, st);
  return hipGetLastError();
}

hipError_t fs_vec_sigma_stats(int n, const double* sigma, double tau_factor, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_sigma_stats, dim3(1), dim3(64), 0, s, n, sigma, tau_factor, st);
  return hipGetLastError();
}

hipError_t fs_vec_first_threshold(int n, const double* x0, double gamma, double rho, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_first_threshold, dim3(1), dim3(VNT), 0, s, n, x0, gamma, rho, st);
  return hipGetLastError();
}

hipError_t fs_vec_kw(int n, const double* w, const double* sigma, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_kw, dim3(1), dim3(VNT), 0, s, n, w, sigma, st);
  return hipGetLastError();
}

hipError_t fs_vec_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t fs_vec_set_double(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t fs_vec_state_init(DevState* st, double alpha, double beta, int max_inner, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, alpha, beta, max_inner);
  return hipGetLastError();
}

hipError_t fs_vec_trmv_t(const double* R, int64_t ldr, int n, const double* t, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trmv_t, dim3(n), dim3(256), 0, s, R, ldr, n, t, out);
  return hipGetLastError();
}
