// Fused passes over A for the refinement loop (one HBM read of A per pass).
//
//   normal pass   : v  = A^T (A z)                      (operator of eq:precond-normal, Alg 1/5)
//   residual pass : g  = A^T (b - A x),  ||b - A x||^2  (right-hand side c_i of Alg 1, KW check)
//
// Column scaling (Alg 4, first statement) is folded into the vectors by the caller: the kernels
// see the unscaled A and a pre-scaled z' = D^{-1} z; the caller scales the result by D^{-1}.
//
// Design: A is column-major (lda >= m).  A work-group owns a tile of H consecutive rows across all
// n columns.  Each lane loads two consecutive rows of one column (16-byte loads; H/2 lanes cover
// the H*8-byte contiguous segment of a column), so a wave instruction reads whole cache lines.
// The tile stays in registers between the two products:
//   phase 1  w_r = sum_c A[r,c] z[c]      (lane-local FMAs, then a shuffle + LDS reduction
//                                          across the lanes/waves holding the same rows)
//   phase 2  acc[c] += sum_r A[r,c] w_r   (lane-local; the cross-lane sum for v is deferred to
//                                          the end of the persistent loop)
// The next tile's loads are issued before the current tile is processed (two register buffers).
// Tiles are banded by XCD (work-group g runs on XCD g % 8): each XCD streams one contiguous band
// of rows, so neighbouring tiles share that XCD's L2.  Each work-group writes one partial vector;
// a second kernel sums the partials in a fixed order (deterministic results).
#include "common.hpp"
#include "internal.hpp"

namespace {

typedef double fs_v2d __attribute__((ext_vector_type(2)));

// The pass of one problem by work-group g of the G work-groups that share it (the whole grid in the
// single-problem kernel; a slice of the grid in the batched one).
template <int H, int NT, int L, bool RESID, bool VEC, bool PF>
__device__ __forceinline__ void fused_pass_body(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                const double* __restrict__ zs, const double* __restrict__ b,
                                                double* __restrict__ partial, double* __restrict__ partial_r2,
                                                const int* __restrict__ stop, double* __restrict__ rout,
                                                const int g, const int G) {
  static_assert(H >= 2 && (H & (H - 1)) == 0 && H <= 128, "H must be a power of two in [2,128]");
  constexpr int RP = H / 2;           // row pairs per tile == lanes per column segment
  constexpr int CPR = NT / RP;        // columns per round
  constexpr int NW = NT / 64;
  constexpr int LOG2RP = __builtin_ctz(RP);
  static_assert(RP <= 64, "row pairs must fit in a wave");

  if (fs_stopped(stop)) return;

  __shared__ double sw[2][NW][H];
  __shared__ double sred[NW];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int rp = tid % RP;
  const int cb = tid / RP;

  // XCD banding of the full row tiles; a ragged last tile (m % H rows) is done at the end.
  const int64_t T = m / H;
  const int nb = (G >= 8 && (G % 8) == 0) ? 8 : 1;
  const int band = g % nb, step = G / nb, l0 = g / nb;
  const int64_t lo = (T * band) / nb, hi = (T * (band + 1)) / nb;

  // z lives in LDS (read once per tile and slot; keeps the registers for the two tile buffers)
  __shared__ double sz[L * CPR];
  for (int q = tid; q < L * CPR; q += NT) sz[q] = (q < n) ? zs[q] : 0.0;
  // Residual passes feed the step heads and the backward-error checks, whose noise floor is the
  // rounding error of A^T r: their accumulations are compensated (Dot2), the normal pass's plain.
  double acc[L], cmp[RESID ? L : 1];
#pragma unroll
  for (int k = 0; k < L; ++k) acc[k] = 0.0;
#pragma unroll
  for (int k = 0; k < (RESID ? L : 1); ++k) cmp[k] = 0.0;
  double r2 = 0.0;
  __syncthreads();

  // Lane byte offsets inside a column slot (32-bit, so loads use a scalar base + vector offset);
  // the host guarantees CPR * lda * 8 + H * 8 < 2^32 on this path.  L is exactly ceil(n / CPR)
  // (the launcher instantiates every value), so only the last slot holds columns >= n; its lanes
  // beyond n re-read the slot's first column (< n): their z entry is zero and their sums are never
  // written, so every load stays inside A and full tiles need no per-lane branch.
  const uint32_t voff = (uint32_t)(((int64_t)cb * lda + 2 * rp) * (int64_t)sizeof(double));
  const uint32_t boff = (uint32_t)(2 * rp * sizeof(double));
  const uint32_t voffL = (cb + (L - 1) * CPR < n) ? voff : boff;
  // Streaming loads carry the non-temporal hint: A is read once per pass and should not displace
  // the reused data (z, the partials) from the caches (a read-only stream measured 6.2 -> 6.9 TB/s
  // with it on this GPU).
  auto ld2 = [&](const char* p) -> double2 {
    if (VEC) {
      const fs_v2d t = __builtin_nontemporal_load(reinterpret_cast<const fs_v2d*>(p));
      return make_double2(t.x, t.y);
    }
    const double* q = reinterpret_cast<const double*>(p);
    return make_double2(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1));
  };
  auto load = [&](double2 (&a)[L + 1], int64_t t) {  // a full tile
    // The tile's byte offset goes through readfirstlane: it stays a scalar, and the compiler
    // does not turn the slot addresses into per-lane 64-bit induction pointers (which would cost
    // two registers per slot).
    const int64_t tb = fs_uniform64(t * H * (int64_t)sizeof(double));
    const char* A0 = reinterpret_cast<const char*>(A) + tb;
    if (RESID) a[L] = ld2(reinterpret_cast<const char*>(b) + tb + boff);
#pragma unroll
    for (int k = 0; k < L; ++k)
      a[k] = ld2(A0 + (int64_t)(k * CPR) * lda * (int64_t)sizeof(double) + (k == L - 1 ? voffL : voff));
  };
  auto load_tail = [&](double2 (&a)[L + 1], int64_t t) {  // rows t*H .. m-1, zero-padded
    const int64_t r0 = t * H + 2 * rp;
    if (RESID) {
      a[L].x = (r0 < m) ? b[r0] : 0.0;
      a[L].y = (r0 + 1 < m) ? b[r0 + 1] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int c = cb + k * CPR;
      const double* p = A + (int64_t)c * lda + r0;
      a[k].x = (c < n && r0 < m) ? p[0] : 0.0;
      a[k].y = (c < n && r0 + 1 < m) ? p[1] : 0.0;
    }
  };

  auto process = [&](const double2 (&a)[L + 1], int64_t t, int par) {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const double zk = sz[cb + k * CPR];
      p0 = fma(a[k].x, zk, p0);
      p1 = fma(a[k].y, zk, p1);
    }
    p0 = wave_sum_high<LOG2RP>(p0);
    p1 = wave_sum_high<LOG2RP>(p1);
    if (lane < RP) {
      sw[par][wv][2 * rp] = p0;
      sw[par][wv][2 * rp + 1] = p1;
    }
    __syncthreads();
    double w0 = 0.0, w1 = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      w0 += sw[par][i][2 * rp];
      w1 += sw[par][i][2 * rp + 1];
    }
    if (RESID) {
      const int64_t r0 = t * H + 2 * rp;  // rows past m carry zeros in a[L] and A
      w0 = (r0 < m) ? a[L].x - w0 : 0.0;
      w1 = (r0 + 1 < m) ? a[L].y - w1 : 0.0;
      if (cb == 0) {
        r2 = fma(w0, w0, fma(w1, w1, r2));
        if (rout) {  // the residual itself (LSQR keeps it as its left Lanczos vector)
          if (r0 < m) rout[r0] = w0;
          if (r0 + 1 < m) rout[r0 + 1] = w1;
        }
      }
    }
    if (RESID) {
#pragma unroll
      for (int k = 0; k < L; ++k) {
        acc_dot(acc[k], cmp[RESID ? k : 0], a[k].x, w0);
        acc_dot(acc[k], cmp[RESID ? k : 0], a[k].y, w1);
      }
    } else {
#pragma unroll
      for (int k = 0; k < L; ++k) acc[k] = fma(a[k].x, w0, fma(a[k].y, w1, acc[k]));
    }
  };

  double2 bufA[L + 1];
  int64_t t = lo + l0;
  if constexpr (PF) {
    double2 bufB[L + 1];
    if (t < hi) load(bufA, t);
    while (t < hi) {
      if (t + step < hi) load(bufB, t + step);
      process(bufA, t, 0);
      t += step;
      if (t >= hi) break;
      if (t + step < hi) load(bufA, t + step);
      process(bufB, t, 1);
      t += step;
    }
  } else {
    int par = 0;
    for (; t < hi; t += step, par ^= 1) {
      load(bufA, t);
      process(bufA, t, par);
    }
  }
  if (T * H < m && g == G - 1) {  // ragged last tile (uniform branch: whole work-group)
    __syncthreads();
    load_tail(bufA, T);
    process(bufA, T, 0);
  }

  // v partial: sum the RP lanes of each column segment, then one lane per column writes.
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const double s = RESID ? wave_sum_low_comp<LOG2RP>(acc[k], cmp[RESID ? k : 0]) : wave_sum_low<LOG2RP>(acc[k]);
    const int c = cb + k * CPR;
    if (rp == 0 && c < n) partial[(int64_t)g * n + c] = s;
  }
  if (RESID) {
    const double s = block_sum<NT>(r2, sred);
    if (tid == 0) partial_r2[g] = s;
  }
}

// PF: the next tile's loads are issued while the current tile is processed (a second register
// buffer).  32-row tiles with more than 8 column slots per lane (256 < n <= 1024) have no registers
// for it; their 256-byte column segments read HBM faster than 16-row tiles with the prefetch.
template <int H, int NT, int L, bool RESID, bool VEC, bool PF = !(H == 32 && L > 8)>
__global__ __launch_bounds__(NT, 1) void k_fused_pass(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                   const double* __restrict__ zs, const double* __restrict__ b,
                                                   double* __restrict__ partial, double* __restrict__ partial_r2,
                                                   const int* __restrict__ stop, double* __restrict__ rout) {
  fused_pass_body<H, NT, L, RESID, VEC, PF>(A, lda, m, n, zs, b, partial, partial_r2, stop, rout, (int)blockIdx.x,
                                            (int)gridDim.x);
}

// Many problems in one launch: a work-list of problems (all of this instantiation's H and L), each
// with G_k work-groups starting at wg0[k] (multiples of 8, so a problem's XCD bands stay whole).
// Work-group -> (problem, local index) by a scan of the list; each problem's partials as above.
template <int H, int NT, int L, bool RESID, bool VEC>
__global__ __launch_bounds__(NT, 1) void k_fused_pass_batched(const BatchPass* __restrict__ list, int count) {
  const int gw = (int)blockIdx.x;
  int k = 0;
  while (k + 1 < count && list[k + 1].wg0 <= gw) ++k;
  const BatchPass& p = list[k];
  fused_pass_body<H, NT, L, RESID, VEC, !(H == 32 && L > 8)>(p.A, p.lda, p.m, p.n, p.zs, RESID ? p.b : nullptr, p.partial,
                                               p.partial_r2, p.stop, nullptr, gw - p.wg0, p.G);
}

// out[c] = scale[c] * sum_g partial[g][c]; optionally r2 = sum_g partial_r2[g].  A work-group
// takes 64 columns; its 16 row groups each sum every 16th partial, then the 16 sums are added in a
// fixed order (deterministic, and 16 independent loads in flight per thread instead of G).
__global__ __launch_bounds__(1024) void k_reduce_partials(const double* __restrict__ partial, int G, int n,
                                                          const double* __restrict__ scale, double* __restrict__ out,
                                                          const double* __restrict__ partial_r2, double* __restrict__ r2,
                                                          const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sh[16][65], she[16][65];
  __shared__ double sr[16];
  const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  double s = 0.0, e = 0.0;  // compensated (Neumaier) sums: the partials can cancel
  if (c < n) {
#pragma unroll 8
    for (int gi = grp; gi < G; gi += 16) {
      double t, d;
      two_sum(s, partial[(int64_t)gi * n + c], t, d);
      s = t;
      e += d;
    }
  }
  sh[grp][cl] = s;
  she[grp][cl] = e;
  __syncthreads();
  if (grp == 0 && c < n) {
    double t = 0.0, te = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double u, d;
      two_sum(t, sh[q][cl], u, d);
      t = u;
      te += d + she[q][cl];
    }
    t += te;
    out[c] = scale ? t * scale[c] : t;
  }
  if (partial_r2 && blockIdx.x == 0) {
    double v = 0.0;
    for (int gi = threadIdx.x; gi < G; gi += 1024) v += partial_r2[gi];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += sr[q];
      *r2 = t;
    }
  }
}

// The reduction of k_reduce_partials for each problem of a batched pass (blockIdx.y = problem).
__global__ __launch_bounds__(1024) void k_reduce_partials_batched(const BatchPass* __restrict__ list) {
  const BatchPass& p = list[blockIdx.y];
  if (fs_stopped(p.stop)) return;
  const int n = p.n, G = p.G;
  if ((int)blockIdx.x * 64 >= n && blockIdx.x > 0) return;
  __shared__ double sh[16][65], she[16][65];
  __shared__ double sr[16];
  const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  double s = 0.0, e = 0.0;
  if (c < n) {
#pragma unroll 8
    for (int gi = grp; gi < G; gi += 16) {
      double t, d;
      two_sum(s, p.partial[(int64_t)gi * n + c], t, d);
      s = t;
      e += d;
    }
  }
  sh[grp][cl] = s;
  she[grp][cl] = e;
  __syncthreads();
  if (grp == 0 && c < n) {
    double t = 0.0, te = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double u, d;
      two_sum(t, sh[q][cl], u, d);
      t = u;
      te += d + she[q][cl];
    }
    t += te;
    p.out[c] = p.out_scale ? t * p.out_scale[c] : t;
  }
  if (p.r2_out && blockIdx.x == 0) {
    double v = 0.0;
    for (int gi = threadIdx.x; gi < G; gi += 1024) v += p.partial_r2[gi];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += sr[q];
      *p.r2_out = t;
    }
  }
}

// Unfused fallback for very wide A (n > 4096): w = A z (or b - A z) then v = A^T w.
__global__ __launch_bounds__(256) void k_gemv_n(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                const double* __restrict__ z, const double* __restrict__ b,
                                                double* __restrict__ w, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  double s = 0.0;
  for (int c = 0; c < n; ++c) s = fma(A[(int64_t)c * lda + r], z[c], s);
  w[r] = b ? b[r] - s : s;
}

__global__ __launch_bounds__(256) void k_gemv_t(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                const double* __restrict__ w, double* __restrict__ partial, int G,
                                                const int* __restrict__ stop) {
  // block (c, gslice): partial[gslice][c] = sum over a row slice of A[r,c] w[r]
  if (fs_stopped(stop)) return;
  __shared__ double sh[4];
  const int c = blockIdx.x;
  const int gs = blockIdx.y;
  const int64_t rows_per = (m + G - 1) / G;
  const int64_t r0 = gs * rows_per, r1 = (r0 + rows_per < m) ? r0 + rows_per : m;
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) s = fma(A[(int64_t)c * lda + r], w[r], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) partial[(int64_t)gs * n + c] = s;
}

__global__ __launch_bounds__(256) void k_sumsq_partials(const double* __restrict__ w, int64_t m, int G,
                                                        double* __restrict__ partial_r2, const int* __restrict__ stop) {
  if (fs_stopped(stop)) return;
  __shared__ double sh[4];
  const int64_t rows_per = (m + G - 1) / G;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = (r0 + rows_per < m) ? r0 + rows_per : m;
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) s = fma(w[r], w[r], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) partial_r2[blockIdx.x] = s;
}

template <int H, int NT, int L, bool RESID>
hipError_t launch_one(const PassArgs& a, int G, bool vec, hipStream_t s) {
  if (vec)
    hipLaunchKernelGGL((k_fused_pass<H, NT, L, RESID, true>), dim3(G), dim3(NT), 0, s, a.A, a.lda, a.m, a.n, a.zs,
                       a.b, a.partial, a.partial_r2, a.stop, a.rout);
  else
    hipLaunchKernelGGL((k_fused_pass<H, NT, L, RESID, false>), dim3(G), dim3(NT), 0, s, a.A, a.lda, a.m, a.n,
                       a.zs, a.b, a.partial, a.partial_r2, a.stop, a.rout);
  return hipGetLastError();
}

// L must equal ceil(n / CPR) exactly (see the kernel): dispatch over [LO, HI].
template <int H, int NT, bool RESID, int LO, int HI>
hipError_t launch_exact(const PassArgs& a, int G, bool vec, int L, hipStream_t s) {
  if constexpr (LO > HI) {
    return hipErrorInvalidValue;
  } else {
    if (L == LO) return launch_one<H, NT, LO, RESID>(a, G, vec, s);
    return launch_exact<H, NT, RESID, LO + 1, HI>(a, G, vec, L, s);
  }
}

template <int H, int NT, bool RESID>
hipError_t launch_L(const PassArgs& a, int G, bool vec, hipStream_t s) {
  constexpr int CPR = NT / (H / 2);
  const int L = (a.n + CPR - 1) / CPR;
  // ranges of L each tile height serves (fs_pass_config): 64: n <= 64; 32: 64 < n <= 1024 (the residual
  // pass: n <= 256); 16: 256 < n <= 1024; 8: 1024 < n <= 2048; 4: 2048 < n <= 4096 (direct calls may
  // go lower)
  if constexpr (H == 64) return launch_exact<H, NT, RESID, 1, 4>(a, G, vec, L, s);
  // 32-row tiles: the normal pass up to 32 slots (n <= 1024); the residual pass's compensated sums need
  // the registers of 16-row tiles above 8 slots (its launcher switches to H = 16 there)
  if constexpr (H == 32) return launch_exact<H, NT, RESID, 1, RESID ? 8 : 32>(a, G, vec, L, s);
  if constexpr (H == 16) return launch_exact<H, NT, RESID, 1, 16>(a, G, vec, L, s);
  return launch_exact<H, NT, RESID, 5, 16>(a, G, vec, L, s);
}

template <bool RESID>
hipError_t launch_fused(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
  const bool vec = ((a.lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.b) & 15) == 0);
  if (RESID && cfg.H == 32 && a.n > 256) return launch_L<16, 512, RESID>(a, cfg.G, vec, s);
  switch (cfg.H) {
    case 64: return launch_L<64, 512, RESID>(a, cfg.G, vec, s);
    case 32: return launch_L<32, 512, RESID>(a, cfg.G, vec, s);
    case 16: return launch_L<16, 512, RESID>(a, cfg.G, vec, s);
    case 8: return launch_L<8, 512, RESID>(a, cfg.G, vec, s);
    case 4: return launch_L<4, 512, RESID>(a, cfg.G, vec, s);
    default: return hipErrorInvalidValue;
  }
}

template <int H, bool RESID, bool VEC, int LO, int HI>
hipError_t launch_batched_exact(const BatchPass* list, int count, int L, int total, hipStream_t s) {
  if constexpr (LO > HI) {
    return hipErrorInvalidValue;
  } else {
    if (L == LO) {
      hipLaunchKernelGGL((k_fused_pass_batched<H, 512, LO, RESID, VEC>), dim3(total), dim3(512), 0, s, list, count);
      return hipGetLastError();
    }
    return launch_batched_exact<H, RESID, VEC, LO + 1, HI>(list, count, L, total, s);
  }
}

template <bool RESID, bool VEC>
hipError_t launch_batched(const BatchPass* list, int count, int H, int L, int total, hipStream_t s) {
  switch (H) {
    case 64: return launch_batched_exact<64, RESID, VEC, 1, 4>(list, count, L, total, s);
    case 32: return launch_batched_exact<32, RESID, VEC, 1, RESID ? 8 : 32>(list, count, L, total, s);
    case 16: return launch_batched_exact<16, RESID, VEC, 1, 16>(list, count, L, total, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

__global__ void k_barrier_reset(unsigned* words, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) words[i] = 0u;
}

// Pick the tile height from n: 64 rows up to 64 columns, 32 rows up to 1024 (the normal pass without
// the prefetch buffer above 256; the residual pass takes 16 rows there), then the widest tile whose L
// (column slots per lane) stays <= 16.  At 1e6 x 1000 the 32-row normal pass runs at 1.193 ms against
// 1.298 ms for 16 rows with the prefetch.
PassConfig fs_pass_config(int64_t m, int n, int num_cu) {
  PassConfig c{};
  if (n <= 64) c.H = 64;
  else if (n <= 1024) c.H = 32;
  else if (n <= 2048) c.H = 8;
  else if (n <= 4096) c.H = 4;
  else c.H = 0;  // unfused fallback
  const int64_t T = c.H ? (m + c.H - 1) / c.H : 0;
  int G = num_cu;  // one 512-thread work-group per CU (register-bound occupancy)
  if (c.H && T < G) G = (int)((T + 7) / 8 * 8);
  if (G < 1) G = 1;
  c.G = c.H ? G : 512;
  return c;
}

hipError_t fs_launch_pass(const PassArgs& a, const PassConfig& cfg, double* out, const double* out_scale,
                          double* r2_out, double* w_scratch, hipStream_t s) {
  hipError_t e;
  const bool resid = a.b != nullptr;
  if (cfg.H) {
    e = resid ? launch_fused<true>(a, cfg, s) : launch_fused<false>(a, cfg, s);
    if (e != hipSuccess) return e;
  } else {
    // unfused: two reads of A
    const int gb = (int)((a.m + 255) / 256);
    double* w = (resid && a.rout) ? a.rout : w_scratch;  // the residual goes straight to rout when asked
    hipLaunchKernelGGL(k_gemv_n, dim3(gb), dim3(256), 0, s, a.A, a.lda, a.m, a.n, a.zs, a.b, w, a.stop);
    hipLaunchKernelGGL(k_gemv_t, dim3(a.n, cfg.G), dim3(256), 0, s, a.A, a.lda, a.m, a.n, w, a.partial,
                       cfg.G, a.stop);
    if (resid)
      hipLaunchKernelGGL(k_sumsq_partials, dim3(cfg.G), dim3(256), 0, s, w, a.m, cfg.G, a.partial_r2, a.stop);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_partials, dim3((a.n + 63) / 64), dim3(1024), 0, s, a.partial, cfg.G, a.n, out_scale,
                     out, resid ? a.partial_r2 : nullptr, r2_out, a.stop);
  return hipGetLastError();
}

hipError_t fs_launch_pass_kernel_only(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
  if (!cfg.H) return hipErrorInvalidValue;
  return a.b ? launch_fused<true>(a, cfg, s) : launch_fused<false>(a, cfg, s);
}

hipError_t fs_launch_pass_batched(const BatchPass* list, int count, int H, int L, bool vec, bool resid,
                                  int total_wgs, int max_n, hipStream_t s) {
  if (count < 1 || total_wgs < 1) return hipSuccess;
  // the residual pass of a 32-row group above 8 column slots: 16-row tiles (ceil(L / 2) slots for every
  // problem of the group), the same work-groups and partials
  if (resid && H == 32 && L > 8) {
    H = 16;
    L = (L + 1) / 2;
  }
  hipError_t e = resid ? (vec ? launch_batched<true, true>(list, count, H, L, total_wgs, s)
                              : launch_batched<true, false>(list, count, H, L, total_wgs, s))
                       : (vec ? launch_batched<false, true>(list, count, H, L, total_wgs, s)
                              : launch_batched<false, false>(list, count, H, L, total_wgs, s));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_partials_batched, dim3((unsigned)((max_n + 63) / 64), (unsigned)count), dim3(1024), 0, s,
                     list);
  return hipGetLastError();
}
