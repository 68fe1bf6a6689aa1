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

// ---------------------------------------------------------------- triangular solves across work-groups
// Back substitution R x = y (or forward substitution R^T x = y) with one work-group per block of 64
// rows.  Block I needs the solution of the blocks it depends on (J > I for R, J < I for R^T): it
// accumulates R_IJ x_J (R_JI^T x_J) as each x_J is published, then solves its 64 x 64 diagonal block
// with one wave (row by row, as the single-work-group solve does) and publishes x_I.  Publication:
// x_I goes to xbuf with device-coherent stores; after they complete, flag[I] is set to the launch's
// epoch.  Readers poll the flag, then load x_J with device-coherent loads.  The work-group of the
// block without dependencies gets blockIdx 0 and each block waits only for blocks with smaller
// blockIdx, which the GPU dispatches first, so the wait needs no co-residency.  The epoch is a device
// word: each launch targets its value + 1 and the last block (the one depending on all others, so
// every work-group has read it) advances it, which keeps captured graphs correct on replay.  Waits
// are bounded: on expiry the error word is set and the work-group proceeds.  The divisions by r_ii
// are multiplications by the reciprocal formed once per block (one rounding more per row).
constexpr int TF_NT = 512;
constexpr int TF_B = 64;
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// flags layout (ints): [0, nb) block flags | nb: epoch | nb + 1: error word
__global__ __launch_bounds__(TF_NT) void k_trsv_flow(const double* __restrict__ R, int64_t ldr, int n, int transpose,
                                                     const double* y, double* x, const double* __restrict__ yscale,
                                                     const double* __restrict__ xscale, const int* __restrict__ stop,
                                                     double* __restrict__ xbuf, int* __restrict__ flags) {
  if (fs_stopped(stop)) return;
  const int nb = (n + TF_B - 1) / TF_B;
  const int I = transpose ? (int)blockIdx.x : nb - 1 - (int)blockIdx.x;
  const int r0 = I * TF_B;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;  // 8 waves
  __shared__ double dblk[TF_B][TF_B + 1];
  __shared__ double red[TF_NT / 64][TF_B];
  int* epoch_w = flags + nb;
  int* err_w = flags + nb + 1;
  const int target = __hip_atomic_load(epoch_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
  // the diagonal block (rows past n: identity, so their x is 0) and the right-hand side
  for (int q = tid; q < TF_B * TF_B; q += TF_NT) {
    const int r = q & 63, c = q >> 6;
    const bool in = r0 + r < n && r0 + c < n;
    double v = 0.0;
    if (!transpose) {
      if (in && r <= c) v = R[(int64_t)(r0 + c) * ldr + r0 + r];
    } else {
      if (in && c <= r) v = R[(int64_t)(r0 + r) * ldr + r0 + c];  // (R^T)[r][c] = R[c][r]
    }
    if (r == c && !in) v = 1.0;
    dblk[r][c] = v;
  }
  double t = 0.0;
  if (wv == 0 && r0 + lane < n) t = yscale ? y[r0 + lane] * yscale[r0 + lane] : y[r0 + lane];
  // off-diagonal blocks in dependency order: thread (row lane, column group wv) sums 8 columns
  const int nj = transpose ? I : nb - 1 - I;  // number of blocks this one depends on
  double acc = 0.0;
  auto tile_ptr = [&](int J, int u) -> double {
    const int c = J * TF_B + wv * 8 + u;  // source index of x_J
    if (!transpose) {
      if (r0 + lane >= n || c >= n) return 0.0;
      return R[(int64_t)c * ldr + r0 + lane];  // R[r0 + lane][c]
    }
    if (r0 + lane >= n || c >= n) return 0.0;
    return R[(int64_t)(r0 + lane) * ldr + c];  // (R^T)[r0 + lane][c] = R[c][r0 + lane]
  };
  const __amdgpu_buffer_rsrc_t xr = co_rsrc(xbuf, (size_t)n * sizeof(double));  // reads past n give 0
  double cur[8];
  if (nj > 0) {
    const int J0 = transpose ? 0 : nb - 1;
#pragma unroll
    for (int u = 0; u < 8; ++u) cur[u] = tile_ptr(J0, u);
  }
  for (int q = 0; q < nj; ++q) {
    const int J = transpose ? q : nb - 1 - q;
    double nxt[8];
    if (q + 1 < nj) {
      const int Jn = transpose ? q + 1 : nb - 2 - q;
#pragma unroll
      for (int u = 0; u < 8; ++u) nxt[u] = tile_ptr(Jn, u);
    }
    if (tid == 0) {
      unsigned long long spins = 0;
      while (__hip_atomic_load(flags + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1ull << 24)) {
          __hip_atomic_store(err_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __syncthreads();
    double xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = ld_cob(xr, (size_t)(J * TF_B + wv * 8 + u) * sizeof(double));
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(cur[u], xv[u], acc);
    if (q + 1 < nj) {
#pragma unroll
      for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
    }
  }
  red[wv][lane] = acc;
  __syncthreads();
  if (wv == 0) {
    double sred = 0.0;
#pragma unroll
    for (int g = 0; g < TF_NT / 64; ++g) sred += red[g][lane];
    t -= sred;
    const double rinv = 1.0 / dblk[lane][lane];
    double xl = 0.0;
    if (!transpose) {
#pragma unroll 8
      for (int i = TF_B - 1; i >= 0; --i) {
        const double xi = readlane_d(t, i) * readlane_d(rinv, i);
        if (lane == i) xl = xi;
        if (lane < i) t = fma(-dblk[lane][i], xi, t);
      }
    } else {
#pragma unroll 8
      for (int i = 0; i < TF_B; ++i) {
        const double xi = readlane_d(t, i) * readlane_d(rinv, i);
        if (lane == i) xl = xi;
        if (lane > i) t = fma(-dblk[lane][i], xi, t);
      }
    }
    if (r0 + lane < n) {
      st_co(xbuf + r0 + lane, xl);
      x[r0 + lane] = xscale ? xl * xscale[r0 + lane] : xl;
    }
    stores_complete();
    if (lane == 0) {
      __hip_atomic_store(flags + I, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (nj == nb - 1) __hip_atomic_store(epoch_w, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------- dense products with V (n x k, ld)
// out[i] = oscale[i] * sum_j V[i, j] (y[j] / ydiv[j])  -- partials over column slices of cs columns:
// a work-group takes 64 rows of one slice, each of its four waves a quarter of the slice's columns
// (two accumulators), the quarters summed in LDS
__global__ __launch_bounds__(256) void k_gemv_v_part(const double* __restrict__ V, int64_t ldv, int n, int k,
                                                     const double* __restrict__ y, const double* __restrict__ ydiv,
                                                     double* __restrict__ part, int cs, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int slice = blockIdx.y;
  const int qc = cs / 4;
  const int j0 = slice * cs + w * qc, j1 = min(k, j0 + qc);
  double s0 = 0.0, s1 = 0.0;
  if (i < n) {
    int j = j0;
#pragma unroll 4
    for (; j + 1 < j1; j += 2) {
      s0 = fma(V[(int64_t)j * ldv + i], ydiv ? y[j] / ydiv[j] : y[j], s0);
      s1 = fma(V[(int64_t)(j + 1) * ldv + i], ydiv ? y[j + 1] / ydiv[j + 1] : y[j + 1], s1);
    }
    if (j < j1) s0 = fma(V[(int64_t)j * ldv + i], ydiv ? y[j] / ydiv[j] : y[j], s0);
  }
  red[w][lane] = s0 + s1;
  __syncthreads();
  if (w == 0 && i < n) part[(int64_t)slice * n + i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
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

// out partials: part[slice][i] = sum_{j in slice, j >= i} R[i, j] v[j]  (R v for upper-triangular R)
__global__ __launch_bounds__(256) void k_trmv_part(const double* __restrict__ R, int64_t ldr, int n,
                                                   const double* __restrict__ v, double* __restrict__ part, int cs) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * cs, j1 = min(n, j0 + cs);
  if (i >= n) return;
  double acc = 0.0;
  for (int j = max(i, j0); j < j1; ++j) acc = fma(R[(int64_t)j * ldr + i], v[j], acc);
  part[(int64_t)blockIdx.y * n + i] = acc;
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
    st->smin_ub = mn;
  }
}

// One step of each bound iteration (one work-group).  Power iteration: est = ||R v|| / ||v|| <= sigma_max
// (the running maximum goes to normest); v <- R^T R v / ||.||.  Inverse iteration: with w = R^{-T} x
// and y = R^{-1} w, x_new = y / ||y|| is a unit vector with ||R x_new|| = ||w|| / ||y|| >= sigma_min
// (the running minimum goes to smin_ub); condest = normest / smin_ub is then a lower bound.
__global__ __launch_bounds__(VNT) void k_bound_step(int n, const double* __restrict__ p, const double* v,
                                                    const double* __restrict__ q, const double* __restrict__ w,
                                                    const double* __restrict__ y, double* v_out, double* x_out,
                                                    DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  double p2 = 0.0, v2 = 0.0, q2 = 0.0, w2 = 0.0, y2 = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    p2 = fma(p[i], p[i], p2);
    v2 = fma(v[i], v[i], v2);
    q2 = fma(q[i], q[i], q2);
    w2 = fma(w[i], w[i], w2);
    y2 = fma(y[i], y[i], y2);
  }
  p2 = bsum(p2, sh);
  v2 = bsum(v2, sh);
  q2 = bsum(q2, sh);
  w2 = bsum(w2, sh);
  y2 = bsum(y2, sh);
  const bool qok = q2 > 0.0 && isfinite(q2), yok = y2 > 0.0 && isfinite(y2);
  const double sq = qok ? 1.0 / sqrt(q2) : 0.0, sy = yok ? 1.0 / sqrt(y2) : 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) {
    if (qok) v_out[i] = q[i] * sq;
    if (yok) x_out[i] = y[i] * sy;
  }
  if (threadIdx.x == 0) {
    if (v2 > 0.0 && isfinite(p2)) st->normest = fmax(st->normest, sqrt(p2 / v2));
    if (yok && isfinite(w2)) st->smin_ub = fmin(st->smin_ub, sqrt(w2 / y2));
    st->condest = (st->smin_ub > 0.0) ? st->normest / st->smin_ub : 0.0;
  }
}

// start vectors: v = x = (1, -2/3, 2/4, ...) (components in every singular direction); the diag(R)
// bounds (k_diag_bounds) seed the running maximum and minimum
__global__ __launch_bounds__(VNT) void k_bound_init(int n, double* __restrict__ v, double* __restrict__ x) {
  for (int i = threadIdx.x; i < n; i += VNT) {
    const double e = ((i & 1) ? -1.0 : 1.0) / (1.0 + 0.5 * i);
    v[i] = e;
    x[i] = e;
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

// A KW checkpoint of the second step recorded while the SVD of R is still running (skipped, like
// every kernel of an iteration, once the stop flag is set).
__global__ __launch_bounds__(VNT) void k_kw_record(int c, int j, int n, const double* __restrict__ dy,
                                                   const double* __restrict__ g, double* __restrict__ kdy,
                                                   double* __restrict__ kg, double* __restrict__ ks,
                                                   DevState* __restrict__ st) {
  if (st->stop) return;
  for (int i = threadIdx.x; i < n; i += VNT) {
    kdy[(int64_t)c * n + i] = dy[i];
    kg[(int64_t)c * n + i] = g[i];
  }
  if (threadIdx.x == 0) {
    ks[4 * c + 0] = st->r2;
    ks[4 * c + 1] = st->x2;
    ks[4 * c + 2] = (double)j;
    st->kw_pending = c + 1;
  }
}

// The recorded checkpoints in order, each with k_kw's formula; the first whose estimate meets the
// second-step rule ends the step at its iteration.  Runs whether or not the cap stopped the loop.
__global__ __launch_bounds__(VNT) void k_kw_replay(int n, int ncheck, const double* __restrict__ W,
                                                   const double* __restrict__ sigma, const double* __restrict__ kdy,
                                                   const double* __restrict__ ks, double* __restrict__ dy,
                                                   DevState* __restrict__ st) {
  __shared__ double sh[VNT / 64];
  __shared__ int hit;
  const int C = min(ncheck, st->kw_pending);
  const double th2 = st->theta2;
  if (threadIdx.x == 0) hit = -1;
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    const double r2 = ks[4 * c + 0], x2 = ks[4 * c + 1];
    const double lam = th2 * r2 / (1.0 + th2 * x2);
    const double* w = W + (int64_t)c * n;
    double sacc = 0.0;
    for (int i = threadIdx.x; i < n; i += VNT) {
      const double si = sigma[i];
      sacc += w[i] * w[i] / (si * si + lam);
    }
    sacc = bsum(sacc, sh);
    if (threadIdx.x == 0) {
      const double be = sqrt(th2 / (1.0 + th2 * x2)) * sqrt(sacc);
      st->be_sk = be;
      st->kw_evals += 1;
      st->x2 = x2;
      st->r2 = r2;
      if (be < st->fro_u) hit = c;
    }
    __syncthreads();
    if (hit >= 0) break;
  }
  if (hit >= 0) {
    for (int i = threadIdx.x; i < n; i += VNT) dy[i] = kdy[(int64_t)hit * n + i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (hit >= 0) {
      st->iters = (int)ks[4 * hit + 2] + 1;
      st->stop = 1;
      st->converged = 1;
    }
    st->kw_pending = 0;
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
__global__ __launch_bounds__(VNT) void k_kw_upper(int n, const double* __restrict__ h, double margin,
                                                  DevState* __restrict__ st) {
  if (st->stop) return;
  __shared__ double sh[VNT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += VNT) s = fma(h[i], h[i], s);
  s = bsum(s, sh);
  if (threadIdx.x == 0) {
    const double th2 = st->theta2, x2 = st->x2;
    const double bound = sqrt(th2 / (1.0 + th2 * x2)) * sqrt(s);
    if (margin * bound < st->fro_u) {
      st->be_sk = bound;
      st->kw_evals += 1;
      st->stop = 1;
      st->converged = 1;
      __hip_atomic_store(&st->svd_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void k_sigma_stats(int n, const double* __restrict__ sigma, double tau_factor, DevState* __restrict__ st) {
  // an SVD abandoned by the refinement (st->svd_abort) leaves the bounds in place
  if (__hip_atomic_load(&st->svd_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
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

__global__ void k_fill_ints(int* p, int count, int v) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = v;
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

size_t fs_trsv_flow_bytes(int n) {
  const int nb = (n + TF_B - 1) / TF_B;
  return sizeof(double) * (size_t)n + sizeof(int) * ((size_t)nb + 8) + 64;
}

// xbuf (n doubles) then the flag words: cleared by fs_trsv_flow_reset before the first launch
hipError_t fs_trsv_flow_reset(int n, void* ws, hipStream_t s) {
  const int nb = (n + TF_B - 1) / TF_B;
  int* flags = (int*)((double*)ws + n);
  hipLaunchKernelGGL(k_fill_ints, dim3(1), dim3(256), 0, s, flags, nb + 2, 0);
  return hipGetLastError();
}

int* fs_trsv_flow_err_word(int n, void* ws) {
  const int nb = (n + TF_B - 1) / TF_B;
  return (int*)((double*)ws + n) + nb + 1;
}

hipError_t fs_launch_trsv_flow(const double* R, int64_t ldr, int n, bool transpose, const double* y, double* x,
                               const double* yscale, const double* xscale, const int* stop, void* ws, hipStream_t s) {
  const int nb = (n + TF_B - 1) / TF_B;
  double* xbuf = (double*)ws;
  int* flags = (int*)(xbuf + n);
  hipLaunchKernelGGL(k_trsv_flow, dim3((unsigned)nb), dim3(TF_NT), 0, s, R, ldr, n, transpose ? 1 : 0, y, x, yscale,
                     xscale, stop, xbuf, flags);
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
  hipLaunchKernelGGL(k_gemv_v_part, dim3((n + 63) / 64, ns), dim3(256), 0, s, V, ldv, n, k, y, ydiv, part, cs,
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
hipError_t fs_vec_spectral_bounds(int n, const double* R, int64_t ldr, const double* Rinv, int iters, double* work,
                                  double* part, void* trsv_ws, DevState* st, hipStream_t s) {
  double* v = work;          // power-iteration vector
  double* x = work + n;      // inverse-iteration vector
  double* p = work + 2 * n;  // R v
  double* q = work + 3 * n;  // R^T R v
  double* w = work + 4 * n;  // R^{-T} x
  double* y = work + 5 * n;  // R^{-1} R^{-T} x
  hipLaunchKernelGGL(k_bound_init, dim3(1), dim3(VNT), 0, s, n, v, x);
  const int cs = 64, ns = (n + cs - 1) / cs;
  for (int k = 0; k < iters; ++k) {
    hipLaunchKernelGGL(k_trmv_part, dim3((n + 255) / 256, ns), dim3(256), 0, s, R, ldr, n, v, part, cs);
    hipLaunchKernelGGL(k_sum_slices, dim3((n + 255) / 256), dim3(256), 0, s, part, ns, n, (const double*)nullptr,
                       (const double*)nullptr, p, (const int*)nullptr);
    hipLaunchKernelGGL(k_trmv_t, dim3(n), dim3(256), 0, s, R, ldr, n, p, q);
    hipError_t e;
    if (Rinv) {  // products with the explicit inverse (ld n)
      e = fs_vec_gemv_vt(Rinv, n, n, n, x, nullptr, w, nullptr, s);
      if (e != hipSuccess) return e;
      e = fs_vec_gemv_v(Rinv, n, n, n, w, nullptr, nullptr, nullptr, y, part, nullptr, s);
    } else {
      e = fs_launch_trsv_flow(R, ldr, n, true, x, w, nullptr, nullptr, nullptr, trsv_ws, s);
      if (e != hipSuccess) return e;
      e = fs_launch_trsv_flow(R, ldr, n, false, w, y, nullptr, nullptr, nullptr, trsv_ws, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bound_step, dim3(1), dim3(VNT), 0, s, n, p, v, q, w, y, v, x, st);
  }
  return hipGetLastError();
}

hipError_t fs_vec_record_iter(int j, int n, const double* dy, double* hist_dy, double* hist_dn, const DevState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_record_iter, dim3(1), dim3(VNT), 0, s, j, n, dy, hist_dy, hist_dn, st);
  return hipGetLastError();
}
hipError_t fs_vec_kw_upper(int n, const double* h, double margin, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_kw_upper, dim3(1), dim3(VNT), 0, s, n, h, margin, st);
  return hipGetLastError();
}
hipError_t fs_vec_kw_record(int c, int j, int n, const double* dy, const double* g, double* kdy, double* kg,
                            double* ks, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_kw_record, dim3(1), dim3(VNT), 0, s, c, j, n, dy, g, kdy, kg, ks, st);
  return hipGetLastError();
}
hipError_t fs_vec_kw_replay(int n, int ncheck, const double* W, const double* sigma, const double* kdy,
                            const double* ks, double* dy, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_kw_replay, dim3(1), dim3(VNT), 0, s, n, ncheck, W, sigma, kdy, ks, dy, st);
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
