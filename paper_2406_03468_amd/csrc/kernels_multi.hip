// Passes over A for k <= 64 right-hand sides at once (the multi-RHS form of the refinement loop):
//
//   apply  : W = A Zs            or  W = B - A Zs  (and ||w_j||^2)   W: m x kp, row-major
//   gather : V = A^T W                                                V: n x kp, row-major
//
// With k right-hand sides the operator of eq:precond-normal costs 4 m n k flops per read of A
// (32 flop/byte at k = 64), above the FP64 ridge point, so both halves run on the matrix cores
// (v_mfma_f64_16x16x4f64; lane l supplies A_op[l%16][l/16] and B_op[l/16][l%16], and holds
// D[4r + l/16][l%16] in accumulator register r).  The intermediate W (m x kp doubles) is
// streamed through HBM once each way; at k = 64 that is 1 GB against 2 x 8 GB of A and the pass
// is bound by the FP64 MFMA rate, not by the extra traffic.
//
// apply : a work-group owns 256 rows (8 waves x 32 rows, two 16-row MFMA blocks per wave) and all
//         kp = 16*NB right-hand sides; Zs is staged through LDS in chunks of 32 rows of Zs
//         (shared by the 8 waves), A operands are loaded a chunk ahead (coalesced: 16 lanes read
//         16 consecutive rows of one column).
// gather: a work-group owns 128 columns of A (one 16-column block per wave) x kp and a chunk of
//         rows; the chunk partials are summed by a fixed-order reduction (deterministic).  Work-
//         groups sharing a row chunk are placed on the same XCD so W is fetched into one L2 once.
#include "common.hpp"
#include "internal.hpp"
#include "state.hpp"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int AP_WAVES = 8;
constexpr int AP_RW = 32;                    // rows per wave
constexpr int AP_TM = AP_WAVES * AP_RW;      // rows per work-group
constexpr int AP_KC = 32;                    // rows of Zs per LDS chunk (8 MFMA k-steps)

template <int NB, bool RESID>
__global__ __launch_bounds__(512) void k_mr_apply(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                  const double* __restrict__ Zs, const double* __restrict__ B,
                                                  int64_t ldb, int k, double* __restrict__ W,
                                                  double* __restrict__ r2part, const int* __restrict__ stop) {
  constexpr int KP = 16 * NB;
  constexpr int KS = AP_KC / 4;  // k-steps per chunk
  __shared__ double zsh[2][AP_KC][KP];
  __shared__ double rsh[AP_WAVES][KP];
  if (fs_stopped(stop)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rw = (int64_t)blockIdx.x * AP_TM + wv * AP_RW;  // first row of this wave
  int64_t ra0 = rw + li, ra1 = rw + 16 + li;                      // A-operand rows (clamped)
  if (ra0 >= m) ra0 = m - 1;
  if (ra1 >= m) ra1 = m - 1;
  const int nch = (n + AP_KC - 1) / AP_KC;

  // Zs staging: thread q covers entries q, q + 512, ... of the AP_KC x KP chunk
  constexpr int ZPT = (AP_KC * KP + 511) / 512;
  double zreg[ZPT];
  auto zload = [&](int c0) {
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      const int q = tid + u * 512;
      const int rr = q / KP, j = q % KP, c = c0 + rr;
      zreg[u] = (q < AP_KC * KP && c < n) ? Zs[(int64_t)c * KP + j] : 0.0;
    }
  };
  auto zstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      const int q = tid + u * 512;
      if (q < AP_KC * KP) zsh[buf][q / KP][q % KP] = zreg[u];
    }
  };
  // A operands two chunks ahead, in three register slots (chunk c in slot c % 3)
  double a0[3][KS], a1[3][KS];
  auto aload = [&](double (&p0)[KS], double (&p1)[KS], int c0) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      int c = c0 + 4 * s + lk;
      if (c >= n) c = n - 1;  // matching Zs rows are zero
      p0[s] = A[(int64_t)c * lda + ra0];
      p1[s] = A[(int64_t)c * lda + ra1];
    }
  };

  v4d acc0[NB], acc1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc0[b] = v4d{0.0, 0.0, 0.0, 0.0};
    acc1[b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // one chunk: x = its operands, p = the slot that receives chunk ch + 2
  auto chunk_step = [&](int ch, const double (&x0)[KS], const double (&x1)[KS], double (&p0)[KS], double (&p1)[KS]) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) zload((ch + 1) * AP_KC);
    if (ch + 2 < nch) aload(p0, p1, (ch + 2) * AP_KC);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double zb = zsh[buf][4 * s + lk][16 * b + li];
        acc0[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[s], zb, acc0[b], 0, 0, 0);
        acc1[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[s], zb, acc1[b], 0, 0, 0);
      }
    }
    if (more) zstore(buf ^ 1);  // buf^1 was last read in chunk ch-1 (synchronized below)
    __syncthreads();
  };
  zload(0);
  zstore(0);
  aload(a0[0], a1[0], 0);
  if (nch > 1) aload(a0[1], a1[1], AP_KC);
  __syncthreads();
  for (int ch = 0; ch < nch; ch += 3) {  // (the conditions are uniform over the work-group)
    chunk_step(ch, a0[0], a1[0], a0[2], a1[2]);
    if (ch + 1 < nch) chunk_step(ch + 1, a0[1], a1[1], a0[0], a1[0]);
    if (ch + 2 < nch) chunk_step(ch + 2, a0[2], a1[2], a0[1], a1[1]);
  }

  // epilogue: lane (li, lk), register r -> row 4r + lk of the 16-row block, column 16b + li
  double r2loc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) r2loc[b] = 0.0;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = 16 * b + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rw + 16 * blk + 4 * r + lk;
        if (row < m) {
          const double s = blk ? acc1[b][r] : acc0[b][r];
          double w;
          if (RESID) {
            w = (j < k) ? B[(int64_t)j * ldb + row] - s : 0.0;
            r2loc[b] = fma(w, w, r2loc[b]);
          } else {
            w = s;
          }
          W[row * KP + j] = w;
        }
      }
    }
  }
  if (RESID) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = r2loc[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lk == 0) rsh[wv][16 * b + li] = v;
    }
    __syncthreads();
    if (tid < KP) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < AP_WAVES; ++w) t += rsh[w][tid];
      r2part[(int64_t)blockIdx.x * KP + tid] = t;
    }
  }
}

constexpr int GA_WAVES = 8;
constexpr int GA_TN = GA_WAVES * 16;   // columns of A per work-group
constexpr int GA_GS = 8;               // k-steps per load group
constexpr int GA_FLUSH = 64;           // k-steps between flushes of the MFMA accumulators

template <int NB>
__global__ __launch_bounds__(512) void k_mr_gather(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                   const double* __restrict__ W, int64_t rc, int ncb,
                                                   double* __restrict__ Vpart, const int* __restrict__ stop) {
  constexpr int KP = 16 * NB;
  if (fs_stopped(stop)) return;
  // blockIdx -> (chunk, column block): the ncb blocks of one chunk are 8 apart in blockIdx, i.e.
  // on the same XCD (work-group g runs on XCD g % 8)
  const int g = blockIdx.x;
  const int xcd = g % 8, slot = g / 8;
  const int cb = slot % ncb;
  const int64_t chunk = (int64_t)(slot / ncb) * 8 + xcd;
  const int64_t nchunk = (m + rc - 1) / rc;
  if (chunk >= nchunk) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int c = cb * GA_TN + wv * 16 + li;
  const bool cvalid = c < n;
  if (!cvalid) c = n - 1;
  const int64_t r_lo = chunk * rc, r_hi = (r_lo + rc < m) ? r_lo + rc : m;
  const double* Ac = A + (int64_t)c * lda;

  v4d acc[NB], acc2[NB], tot[NB];  // acc: even k-steps, acc2: odd ones (two chains per block)
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
    acc2[b] = v4d{0.0, 0.0, 0.0, 0.0};
    tot[b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // W rows of a group (4 GA_GS rows x KP) are staged once per work-group in LDS (double-buffered)
  // instead of being loaded by each of the 8 waves; A operands and the next group's W are loaded
  // one group ahead.
  constexpr int GR = 4 * GA_GS;               // rows per group
  constexpr int WPT = (GR * KP + 511) / 512;  // W entries per thread per group
  __shared__ double wsh[2][GR][KP];
  double wreg[WPT], av[3][GA_GS];
  auto wload = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = tid + 512 * u;
      const int64_t row = r0 + q / KP;
      wreg[u] = (q < GR * KP && row < r_hi) ? W[row * KP + q % KP] : 0.0;
    }
  };
  auto wstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = tid + 512 * u;
      if (q < GR * KP) wsh[buf][q / KP][q % KP] = wreg[u];
    }
  };
  auto aload = [&](double (&p)[GA_GS], int64_t r0) {
#pragma unroll
    for (int s = 0; s < GA_GS; ++s) {
      const int64_t row = r0 + 4 * s + lk;
      p[s] = (row < r_hi) ? Ac[row] : 0.0;
    }
  };
  int since = 0;
  // one group of rows: x = its A operands (loaded two groups earlier), p = the slot that receives
  // the A operands of the group after next
  auto group_step = [&](int64_t r, int buf, const double (&x)[GA_GS], double (&p)[GA_GS]) {
    const bool more = r + GR < r_hi;
    if (more) wload(r + GR);
    if (r + 2 * GR < r_hi) aload(p, r + 2 * GR);
#pragma unroll
    for (int s = 0; s < GA_GS; s += 2) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], wsh[buf][4 * s + lk][16 * b + li], acc[b], 0, 0, 0);
        acc2[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s + 1], wsh[buf][4 * s + 4 + lk][16 * b + li], acc2[b],
                                                      0, 0, 0);
      }
    }
    if (more) wstore(buf ^ 1);  // buf ^ 1 was last read in the previous group (synchronized below)
    __syncthreads();
    since += GA_GS;
    if (since >= GA_FLUSH) {  // two-level summation: bounded accumulation chains
      since = 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        tot[b] += acc[b] + acc2[b];
        acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
        acc2[b] = v4d{0.0, 0.0, 0.0, 0.0};
      }
    }
  };
  wload(r_lo);
  wstore(0);
  aload(av[0], r_lo);
  if (r_lo + GR < r_hi) aload(av[1], r_lo + GR);
  __syncthreads();
  // groups g, g+1, g+2 use slots 0, 1, 2 and LDS buffers alternating (uniform conditions)
  int buf = 0;
  for (int64_t r = r_lo; r < r_hi; r += 3 * GR) {
    group_step(r, buf, av[0], av[2]);
    buf ^= 1;
    if (r + GR < r_hi) {
      group_step(r + GR, buf, av[1], av[0]);
      buf ^= 1;
    }
    if (r + 2 * GR < r_hi) {
      group_step(r + 2 * GR, buf, av[2], av[1]);
      buf ^= 1;
    }
  }
  // D layout: register r holds column (row of V) 4r + lk of the wave's 16-column block, RHS 16b + li
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    tot[b] += acc[b] + acc2[b];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = cb * GA_TN + wv * 16 + 4 * r + lk;
      if (cc < n) Vpart[(chunk * n + cc) * KP + 16 * b + li] = tot[b][r];
    }
  }
  (void)cvalid;
}

// V[c][j] = scale[c] * sum_chunk Vpart[chunk][c][j] (fixed order, compensated), one thread per entry
// in the first ceil(n kp / 256) work-groups; r2[j] = sum_g r2part[g][j] in one work-group per j after
// them (each thread a strided compensated sum, then the 256 partial sums in thread order).
__global__ __launch_bounds__(256) void k_mr_reduce(const double* __restrict__ Vpart, int64_t nchunk, int n, int kp,
                                                   const double* __restrict__ scale, double* __restrict__ V,
                                                   const double* __restrict__ r2part, int64_t nr2, double* __restrict__ r2,
                                                   const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int64_t tot = (int64_t)n * kp;
  const int64_t nbv = (tot + 255) / 256;
  if ((int64_t)blockIdx.x < nbv) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < tot) {
      double s = 0.0, e = 0.0;
      for (int64_t ch = 0; ch < nchunk; ++ch) {
        double t, d;
        two_sum(s, Vpart[ch * tot + q], t, d);
        s = t;
        e += d;
      }
      s += e;
      V[q] = scale ? s * scale[q / kp] : s;
    }
    return;
  }
  const int j = (int)((int64_t)blockIdx.x - nbv);  // r2 work-groups (launched only with r2part)
  if (!r2part || j >= kp) return;
  __shared__ double ss[256], se[256];
  double s = 0.0, e = 0.0;
  for (int64_t g = threadIdx.x; g < nr2; g += 256) {
    double t, d;
    two_sum(s, r2part[g * kp + j], t, d);
    s = t;
    e += d;
  }
  ss[threadIdx.x] = s;
  se[threadIdx.x] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, te = 0.0;
    for (int q = 0; q < 256; ++q) {
      double u, d;
      two_sum(t, ss[q], u, d);
      t = u;
      te += d + se[q];
    }
    r2[j] = t + te;
  }
}

template <int NB>
hipError_t launch_nb(const MultiPassArgs& a, hipStream_t s) {
  const int G1 = (int)((a.m + AP_TM - 1) / AP_TM);
  if (a.B)
    hipLaunchKernelGGL((k_mr_apply<NB, true>), dim3(G1), dim3(512), 0, s, a.A, a.lda, a.m, a.n, a.Zs, a.B, a.ldb,
                       a.k, a.W, a.r2part, a.stop);
  else
    hipLaunchKernelGGL((k_mr_apply<NB, false>), dim3(G1), dim3(512), 0, s, a.A, a.lda, a.m, a.n, a.Zs, a.B,
                       a.ldb, a.k, a.W, a.r2part, a.stop);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ncb = (a.n + GA_TN - 1) / GA_TN;
  const int64_t nchunk = (a.m + a.rc - 1) / a.rc;
  const int64_t slots = (nchunk + 7) / 8 * ncb;  // per XCD
  hipLaunchKernelGGL((k_mr_gather<NB>), dim3((unsigned)(slots * 8)), dim3(512), 0, s, a.A, a.lda, a.m, a.n, a.W,
                     a.rc, ncb, a.Vpart, a.stop);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nbv = ((int64_t)a.n * 16 * NB + 255) / 256;  // V work-groups, then one per r2 entry
  hipLaunchKernelGGL(k_mr_reduce, dim3((unsigned)(nbv + (a.B ? 16 * NB : 0))), dim3(256), 0, s, a.Vpart, nchunk, a.n,
                     16 * NB, a.scale, a.V, a.B ? a.r2part : (const double*)nullptr, (int64_t)G1, a.r2, a.stop);
  return hipGetLastError();
}

}  // namespace

int fs_multi_blocks(int k) { return (k + 15) / 16; }

size_t fs_multi_work_doubles(int64_t m, int n, int k, int64_t* rc_out) {
  const int kp = 16 * fs_multi_blocks(k);
  const int64_t rc = 8192;
  if (rc_out) *rc_out = rc;
  const int64_t nchunk = (m + rc - 1) / rc;
  const int64_t G1 = (m + AP_TM - 1) / AP_TM;
  // W | Vpart | r2part
  return (size_t)m * kp + (size_t)nchunk * n * kp + (size_t)G1 * kp;
}

hipError_t fs_launch_multi_pass(const MultiPassArgs& a, hipStream_t s) {
  switch (fs_multi_blocks(a.k)) {
    case 1: return launch_nb<1>(a, s);
    case 2: return launch_nb<2>(a, s);
    case 3: return launch_nb<3>(a, s);
    case 4: return launch_nb<4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- per-right-hand-side vector work
// Multi-RHS n-vectors are column-major n x k blocks (ld n); the MFMA passes read and write n x kp
// row-major panels.  Per-column reductions use one 256-thread work-group per column, in a fixed
// order (deterministic).
namespace {

constexpr int MV = 256;

__device__ __forceinline__ double blk_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(MV) void k_m_step_init(int nr, const double* __restrict__ C, double* __restrict__ DY,
                                                    double* __restrict__ DY_old, MultiState* __restrict__ ms) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  const double* c = C + (int64_t)j * nr;
  double s = 0.0;
  for (int i = threadIdx.x; i < nr; i += MV) {
    const double v = c[i];
    DY[(int64_t)j * nr + i] = v;
    DY_old[(int64_t)j * nr + i] = v;
    s = fma(v, v, s);
  }
  s = blk_sum256(s, sh);
  if (threadIdx.x == 0) {
    ms->cnorm2[j] = s;
    ms->active[j] = ms->zero[j] ? 0 : 1;
    ms->iters[j] = 0;
    ms->converged[j] = ms->zero[j] ? 1 : 0;
  }
}

__global__ __launch_bounds__(MV) void k_m_polyak(int nr, const double* __restrict__ C, const double* __restrict__ U,
                                                 double* __restrict__ DY, double* __restrict__ DY_old,
                                                 MultiState* __restrict__ ms, double alpha, double beta, int first) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  if (ms->stop || !ms->active[j]) return;
  const int64_t o = (int64_t)j * nr;
  double s = 0.0;
  for (int i = threadIdx.x; i < nr; i += MV) {
    const double dy = DY[o + i], dyo = DY_old[o + i];
    const double delta = alpha * (C[o + i] - U[o + i]) + beta * (dy - dyo);  // eq:polyak_iteration
    DY_old[o + i] = dy;
    DY[o + i] = dy + delta;
    s = fma(delta, delta, s);
  }
  s = blk_sum256(s, sh);
  if (threadIdx.x == 0) {
    ms->iters[j] += 1;
    if (first && sqrt(s) <= ms->thr[j]) {  // Alg 4, first step: ||Delta|| small
      ms->active[j] = 0;
      ms->converged[j] = 1;
    }
  }
}

__global__ void k_m_update_stop(int k, MultiState* __restrict__ ms) {
  const int j = threadIdx.x;
  int a = (j < k) ? ms->active[j] : 0;
  a = __any(a) ? 1 : 0;
  if (threadIdx.x == 0) ms->stop = a ? 0 : 1;
}

__global__ __launch_bounds__(MV) void k_m_first_threshold(int n, const double* __restrict__ X0,
                                                          MultiState* __restrict__ ms, double gamma, double rho,
                                                          double normest, double condest) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += MV) {
    const double v = X0[(int64_t)j * n + i];
    s = fma(v, v, s);
  }
  s = blk_sum256(s, sh);
  if (threadIdx.x == 0)
    ms->thr[j] = (gamma * normest * sqrt(s) + rho * condest * sqrt(ms->r2[j])) * 2.220446049250313e-16;
}

__global__ __launch_bounds__(MV) void k_m_kw(int n, const double* __restrict__ Wv, const double* __restrict__ sigma,
                                             MultiState* __restrict__ ms, double fro2, double fro_u) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  if (ms->stop || !ms->active[j]) return;
  const double th2 = fro2 / ms->b2[j];
  const double x2 = ms->x2[j], r2 = ms->r2[j];
  const double lam = th2 * r2 / (1.0 + th2 * x2);
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += MV) {
    const double w = Wv[(int64_t)j * n + i], si = sigma[i];
    s += w * w / (si * si + lam);
  }
  s = blk_sum256(s, sh);
  if (threadIdx.x == 0) {  // eq:sketched-kw; Alg 4 second-step rule
    const double be = sqrt(th2 / (1.0 + th2 * x2)) * sqrt(s);
    ms->be_sk[j] = be;
    ms->kw_evals[j] += 1;
    if (be < fro_u) {
      ms->active[j] = 0;
      ms->converged[j] = 1;
    }
  }
}

__global__ __launch_bounds__(MV) void k_m_add_norm(int n, const double* __restrict__ X, const double* __restrict__ Z,
                                                   double* __restrict__ out, MultiState* __restrict__ ms) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  if (ms->stop) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += MV) {
    const double v = X[(int64_t)j * n + i] + (Z ? Z[(int64_t)j * n + i] : 0.0);
    out[(int64_t)j * n + i] = v;
    s = fma(v, v, s);
  }
  s = blk_sum256(s, sh);
  if (threadIdx.x == 0) ms->x2[j] = s;
}

__global__ void k_m_to_panel(int n, int k, int kp, const double* __restrict__ X, int64_t ldxin,
                             const double* __restrict__ scale, double* __restrict__ Zs, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * kp) return;
  const int c = (int)(q / kp), j = (int)(q % kp);
  Zs[q] = (j < k) ? X[(int64_t)j * ldxin + c] * (scale ? scale[c] : 1.0) : 0.0;
}

__global__ void k_m_init_columns(int n, int k, const double* __restrict__ colnorm2, MultiState* __restrict__ ms) {
  const int j = threadIdx.x;
  if (j < k) {
    const double b2 = colnorm2[n + j];
    ms->b2[j] = b2;
    ms->zero[j] = (b2 == 0.0) ? 1 : 0;
  }
}

__global__ void k_m_unscale(int n, int k, const double* __restrict__ X, const double* __restrict__ dinv,
                            double* __restrict__ Xout, int64_t ldx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * k) return;
  const int c = (int)(q % n), j = (int)(q / n);
  Xout[(int64_t)j * ldx + c] = X[q] * dinv[c];
}

// Small products with V (n x n, ld ldv).  Output tile: 64 rows x 16 columns per 256-thread
// work-group (thread: one row, four columns); the inner dimension goes through LDS in steps of 32.
constexpr int GT_R = 64, GT_C = 16, GT_K = 32;

// out(c, j) = oscale[c] (sum_i V[c, i] Y[i, j] / sigma[i] + addX[c, j])
__global__ __launch_bounds__(256) void k_m_gemm_P(const double* __restrict__ V, int64_t ldv, int n, int nr, int k,
                                                  const double* __restrict__ sigma, const double* __restrict__ Y,
                                                  const double* __restrict__ addX, const double* __restrict__ oscale,
                                                  double* __restrict__ out, int panel, int kp,
                                                  const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sv[GT_K][GT_R + 1];
  __shared__ double sy[GT_K][GT_C];
  const int tid = threadIdx.x;
  const int rl = tid % GT_R, jg = tid / GT_R;  // 4 groups of 4 columns
  const int c = blockIdx.x * GT_R + rl;
  const int j0 = blockIdx.y * GT_C;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < nr; i0 += GT_K) {
    for (int q = tid; q < GT_K * GT_R; q += 256) {
      const int ii = q / GT_R, cc = q % GT_R;
      const int gi = i0 + ii, gc = blockIdx.x * GT_R + cc;
      sv[ii][cc] = (gi < nr && gc < n) ? V[(int64_t)gi * ldv + gc] : 0.0;
    }
    for (int q = tid; q < GT_K * GT_C; q += 256) {
      const int ii = q % GT_K, jj = q / GT_K;
      const int gi = i0 + ii, gj = j0 + jj;
      sy[ii][jj] = (gi < nr && gj < k) ? Y[(int64_t)gj * nr + gi] / sigma[gi] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < GT_K; ++ii) {
      const double v = sv[ii][rl];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(v, sy[ii][jg * 4 + u], acc[u]);
    }
    __syncthreads();
  }
  if (c >= n) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + jg * 4 + u;
    if (j >= k) continue;
    double r = acc[u] + (addX ? addX[(int64_t)j * n + c] : 0.0);
    if (oscale) r *= oscale[c];
    if (panel) out[(int64_t)c * kp + j] = r;
    else out[(int64_t)j * n + c] = r;
  }
}

// U[i, j] = (sum_c V[c, i] G[c * kp + j]) / sigma[i]
__global__ __launch_bounds__(256) void k_m_gemm_PT(const double* __restrict__ V, int64_t ldv, int n, int nr, int k,
                                                   const double* __restrict__ sigma, const double* __restrict__ G,
                                                   int kp, double* __restrict__ U, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sv[GT_K][GT_R + 1];  // [c][i]
  __shared__ double sg[GT_K][GT_C];
  const int tid = threadIdx.x;
  const int il = tid % GT_R, jg = tid / GT_R;
  const int i = blockIdx.x * GT_R + il;
  const int j0 = blockIdx.y * GT_C;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < n; c0 += GT_K) {
    for (int q = tid; q < GT_K * GT_R; q += 256) {
      const int cc = q % GT_K, ii = q / GT_K;  // consecutive threads: consecutive c (contiguous in V)
      const int gc = c0 + cc, gi = blockIdx.x * GT_R + ii;
      sv[cc][ii] = (gc < n && gi < nr) ? V[(int64_t)gi * ldv + gc] : 0.0;
    }
    for (int q = tid; q < GT_K * GT_C; q += 256) {
      const int cc = q / GT_C, jj = q % GT_C;
      const int gc = c0 + cc, gj = j0 + jj;
      sg[cc][jj] = (gc < n && gj < k) ? G[(int64_t)gc * kp + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int cc = 0; cc < GT_K; ++cc) {
      const double v = sv[cc][il];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(v, sg[cc][jg * 4 + u], acc[u]);
    }
    __syncthreads();
  }
  if (i >= nr) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + jg * 4 + u;
    if (j < k) U[(int64_t)j * nr + i] = sigma ? acc[u] / sigma[i] : acc[u];
  }
}

}  // namespace

hipError_t fs_m_step_init(int nr, int k, const double* C, double* DY, double* DY_old, MultiState* ms, hipStream_t s) {
  hipLaunchKernelGGL(k_m_step_init, dim3(k), dim3(MV), 0, s, nr, C, DY, DY_old, ms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return fs_m_update_stop(k, ms, s);
}
hipError_t fs_m_polyak(int nr, int k, const double* C, const double* U, double* DY, double* DY_old, MultiState* ms,
                       double alpha, double beta, bool first_step, hipStream_t s) {
  hipLaunchKernelGGL(k_m_polyak, dim3(k), dim3(MV), 0, s, nr, C, U, DY, DY_old, ms, alpha, beta, first_step ? 1 : 0);
  return hipGetLastError();
}
hipError_t fs_m_update_stop(int k, MultiState* ms, hipStream_t s) {
  hipLaunchKernelGGL(k_m_update_stop, dim3(1), dim3(64), 0, s, k, ms);
  return hipGetLastError();
}
hipError_t fs_m_first_threshold(int n, int k, const double* X0, MultiState* ms, double gamma, double rho,
                                double normest, double condest, hipStream_t s) {
  hipLaunchKernelGGL(k_m_first_threshold, dim3(k), dim3(MV), 0, s, n, X0, ms, gamma, rho, normest, condest);
  return hipGetLastError();
}
hipError_t fs_m_kw(int n, int k, const double* Wv, const double* sigma, MultiState* ms, double fro2, double fro_u,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_m_kw, dim3(k), dim3(MV), 0, s, n, Wv, sigma, ms, fro2, fro_u);
  return hipGetLastError();
}
hipError_t fs_m_add_norm(int n, int k, const double* X, const double* Z, double* out, MultiState* ms, hipStream_t s) {
  hipLaunchKernelGGL(k_m_add_norm, dim3(k), dim3(MV), 0, s, n, X, Z, out, ms);
  return hipGetLastError();
}
hipError_t fs_m_to_panel(int n, int k, const double* X, int64_t ldxin, const double* scale, double* Zs,
                         const int* stop, hipStream_t s) {
  const int kp = 16 * fs_multi_blocks(k);
  const int64_t tot = (int64_t)n * kp;
  hipLaunchKernelGGL(k_m_to_panel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, kp, X, ldxin, scale,
                     Zs, stop);
  return hipGetLastError();
}
hipError_t fs_m_init_columns(int n, int k, const double* colnorm2, MultiState* ms, hipStream_t s) {
  hipLaunchKernelGGL(k_m_init_columns, dim3(1), dim3(64), 0, s, n, k, colnorm2, ms);
  return hipGetLastError();
}
hipError_t fs_m_unscale(int n, int k, const double* X, const double* dinv, double* Xout, int64_t ldx, hipStream_t s) {
  const int64_t tot = (int64_t)n * k;
  hipLaunchKernelGGL(k_m_unscale, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, X, dinv, Xout, ldx);
  return hipGetLastError();
}
hipError_t fs_m_gemm_P(const double* V, int64_t ldv, int n, int nr, int k, const double* sigma, const double* Y,
                       const double* addX, const double* oscale, double* out, bool panel, const int* stop,
                       hipStream_t s) {
  const dim3 grid((unsigned)((n + GT_R - 1) / GT_R), (unsigned)((k + GT_C - 1) / GT_C));
  hipLaunchKernelGGL(k_m_gemm_P, grid, dim3(256), 0, s, V, ldv, n, nr, k, sigma, Y, addX, oscale, out, panel ? 1 : 0,
                     16 * fs_multi_blocks(k), stop);
  return hipGetLastError();
}
hipError_t fs_m_gemm_PT(const double* V, int64_t ldv, int n, int nr, int k, const double* sigma, const double* G,
                        double* U, const int* stop, hipStream_t s) {
  const dim3 grid((unsigned)((nr + GT_R - 1) / GT_R), (unsigned)((k + GT_C - 1) / GT_C));
  hipLaunchKernelGGL(k_m_gemm_PT, grid, dim3(256), 0, s, V, ldv, n, nr, k, sigma, G, 16 * fs_multi_blocks(k), U,
                     stop);
  return hipGetLastError();
}
