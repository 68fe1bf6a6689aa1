// SVD of the n x n triangular factor R of the sketch (Alg 4 needs Sigma and V of S A; with
// S A = Q R, the SVD R = U_R Sigma V^T gives S A = (Q U_R) Sigma V^T).
//
// One-sided (Hestenes) Jacobi applied to the columns of G = R^T: plane rotations J orthogonalize
// the columns, R^T J = V Sigma, hence R = J Sigma V^T: sigma_i = ||g_i||, v_i = g_i / sigma_i and
// U_R = J (accumulated when requested).  Working on R^T instead of R converges in far fewer
// sweeps for the triangular factor of a sketch.
//
// Parallel order: the round-robin (circle) tournament, n'/2 disjoint pairs per round, n'-1
// rounds per sweep (n' = n rounded up to even).  One cooperative kernel runs all sweeps; rounds
// are separated by grid-wide barriers.  A pair is rotated when |g_i^T g_j| > tol ||g_i|| ||g_j||;
// the sweep loop ends after a sweep without rotations (or at max_sweeps).  A final kernel sorts
// the singular values in decreasing order and writes sigma, V (and U_R).
#include "common.hpp"
#include "internal.hpp"

namespace {

constexpr int SVD_NT = 256;

__device__ __forceinline__ int rr_player(int pos, int r, int npl) {
  return (pos == 0) ? 0 : 1 + (pos - 1 + r) % (npl - 1);
}

__global__ __launch_bounds__(SVD_NT) void k_jacobi_coop(double* __restrict__ Gm, double* __restrict__ U, int n,
                                                        int max_sweeps, double tol, int* __restrict__ rotcount,
                                                        int* __restrict__ sweeps_out, GridBarrier bar) {
  unsigned bgen = 0;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int npl = n + (n & 1);
  const int npairs = npl / 2;
  __shared__ double sh[3][SVD_NT / 64];
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int myrot = 0;
    for (int r = 0; r < npl - 1; ++r) {
      for (int p = g; p < npairs; p += G) {
        int a = rr_player(p, r, npl), b = rr_player(npl - 1 - p, r, npl);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        if (b >= n) continue;  // pair with the dummy player (odd n): uniform across the work-group
        double* gi = Gm + (int64_t)a * n;
        double* gj = Gm + (int64_t)b * n;
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int q = tid; q < n; q += SVD_NT) {
          const double x = gi[q], y = gj[q];
          sa = fma(x, x, sa);
          sb = fma(y, y, sb);
          sc = fma(x, y, sc);
        }
        sa = wave_sum(sa);
        sb = wave_sum(sb);
        sc = wave_sum(sc);
        if ((tid & 63) == 0) {
          sh[0][tid >> 6] = sa;
          sh[1][tid >> 6] = sb;
          sh[2][tid >> 6] = sc;
        }
        __syncthreads();
        double A2 = 0.0, B2 = 0.0, C = 0.0;
#pragma unroll
        for (int w = 0; w < SVD_NT / 64; ++w) {
          A2 += sh[0][w];
          B2 += sh[1][w];
          C += sh[2][w];
        }
        __syncthreads();
        if (A2 > 0.0 && B2 > 0.0 && fabs(C) > tol * sqrt(A2) * sqrt(B2)) {
          const double zeta = (B2 - A2) / (2.0 * C);
          double t;
          if (fabs(zeta) > 1e150) t = 0.5 / zeta;
          else t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int q = tid; q < n; q += SVD_NT) {
            const double x = gi[q], y = gj[q];
            gi[q] = cs * x - sn * y;
            gj[q] = sn * x + cs * y;
          }
          if (U) {
            double* ui = U + (int64_t)a * n;
            double* uj = U + (int64_t)b * n;
            for (int q = tid; q < n; q += SVD_NT) {
              const double x = ui[q], y = uj[q];
              ui[q] = cs * x - sn * y;
              uj[q] = sn * x + cs * y;
            }
          }
          ++myrot;
        }
      }
      grid_barrier(bar, (unsigned)G, bgen);
    }
    if (tid == 0 && myrot) atomicAdd(&rotcount[sweep], myrot);
    grid_barrier(bar, (unsigned)G, bgen);
    const int tot = __hip_atomic_load(&rotcount[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tot == 0) {
      ++sweep;
      break;
    }
  }
  if (g == 0 && tid == 0 && sweeps_out) *sweeps_out = sweep;
}

// ---------------------------------------------------------------- block (systolic) variant
// 8 waves: a round has at most b = 8 disjoint pairs at a time, and 512 threads leave each wave 256
// VGPRs for a register-resident column pair.
constexpr int SVD_BLOCK_NT = 512;
// Columns are grouped in NBLK blocks of b columns (padded to an even count with an empty block).
// Work-group p holds two blocks in LDS, at circle positions p ("top") and NBLK-1-p ("bottom").
// In a round it orthogonalizes every column of its top block against every column of its bottom
// block (b sub-rounds of b disjoint pairs, one wave per pair); the first round of a sweep also
// does the pairs inside each block.  Between rounds the blocks move one position around the
// circle (position 0 fixed): top blocks travel to work-group p+1, bottom blocks to p-1, through
// double-buffered mailboxes in global memory with point-to-point ready flags, so only the
// neighbours synchronize.  After NBLK-1 rounds every pair of columns has met once (one sweep) and
// the blocks are back where they started; a grid barrier then sums the sweep's rotation count.
__device__ __forceinline__ void jac_rotate_pair(double* __restrict__ x, double* __restrict__ y, int n, double tol,
                                                int lane, int& nrot, double& c2max) {
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int q = lane; q < n; q += 64) {
    const double a = x[q], bq = y[q];
    sa = fma(a, a, sa);
    sb = fma(bq, bq, sb);
    sc = fma(a, bq, sc);
  }
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  sc = wave_sum(sc);
  if (sa > 0.0 && sb > 0.0) c2max = fmax(c2max, (sc * sc) / (sa * sb));
  if (sa > 0.0 && sb > 0.0 && fabs(sc) > tol * sqrt(sa) * sqrt(sb)) {
    const double zeta = (sb - sa) / (2.0 * sc);
    double t;
    if (fabs(zeta) > 1e150) t = 0.5 / zeta;
    else t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
    for (int q = lane; q < n; q += 64) {
      const double a = x[q], bq = y[q];
      x[q] = cs * a - sn * bq;
      y[q] = sn * a + cs * bq;
    }
    ++nrot;
  }
}

// Full-wave sum with DPP lane moves (a few cycles each, instead of an LDS round trip per
// ds_bpermute step): quad butterflies, half-row and row mirrors, then the gfx9 row broadcasts
// gather the four row sums in lane 63, which is read back into every lane.  All 64 lanes active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_d<0x140, 0xf>(v);  // row_mirror: every lane holds its row's sum
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row (a pair handled by a 16-lane group); every lane of the row
// receives the row's sum.
__device__ __forceinline__ double row_sum_dpp(double v) {
  v += dpp_d<0xB1, 0xf>(v);
  v += dpp_d<0x4E, 0xf>(v);
  v += dpp_d<0x141, 0xf>(v);
  v += dpp_d<0x140, 0xf>(v);
  return v;
}
template <int LP>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(LP == 16 || LP == 64, "pairs are handled by 16-lane rows or whole waves");
  if constexpr (LP == 16) return row_sum_dpp(v);
  else return wave_sum_dpp(v);
}

// The same rotation with the column pair held in registers (NQ = ceil(n / 64) elements per lane):
// every LDS load is issued before the first use, so the dot products wait once for the whole column
// instead of once per 64-element step.  Same arithmetic in the same order as jac_rotate_pair.
template <int NQ, int LP>
__device__ __forceinline__ void jac_rotate_pair_r(double* __restrict__ x, double* __restrict__ y, int n, double tol,
                                                  int lane, int& nrot, double& c2max) {
  double xr[NQ], yr[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = lane + LP * k;
    xr[k] = (q < n) ? x[q] : 0.0;
    yr[k] = (q < n) ? y[q] : 0.0;
  }
  double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    sa = fma(xr[k], xr[k], sa);
    sb = fma(yr[k], yr[k], sb);
    sc = fma(xr[k], yr[k], sc);
  }
  sa = group_sum<LP>(sa);
  sb = group_sum<LP>(sb);
  sc = group_sum<LP>(sc);
  if (sa > 0.0 && sb > 0.0) c2max = fmax(c2max, (sc * sc) / (sa * sb));
  // |cos| > tol without square roots (column norms of R are O(1): no overflow or underflow here)
  if (sa > 0.0 && sb > 0.0 && sc * sc > (tol * tol) * (sa * sb)) {
    const double zeta = (sb - sa) / (2.0 * sc);
    double t;
    if (fabs(zeta) > 1e150) t = 0.5 / zeta;
    else t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int q = lane + LP * k;
      if (q < n) {
        x[q] = cs * xr[k] - sn * yr[k];
        y[q] = sn * xr[k] + cs * yr[k];
      }
    }
    ++nrot;
  }
}

// Rotation of a pair whose first column stays in registers (xr, NQ elements per lane) and whose
// second column is in LDS: a group keeps its top column through all sub-rounds of a round, so only
// the partner column moves through LDS.  The squared norms are carried between sub-rounds instead of
// summed again: the top column's in sa_x, each bottom column's in *ynorm (LDS, one per column);
// a rotation with tangent t maps them to sa - t c and sb + t c (c = x^T y), and a norm that falls
// below half its value (where that update cancels) is marked stale (-1) and summed at its next use.
// Only x^T y is summed on every call.
template <int NQ, int LP>
__device__ __forceinline__ void jac_rotate_xreg(double (&xr)[NQ], double& sa_x, double* __restrict__ y,
                                                double* __restrict__ ynorm, int n, double tol, int lane, int& nrot,
                                                double& c2max) {
  double yr[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = lane + LP * k;
    yr[k] = (q < n) ? y[q] : 0.0;
  }
  const double yn = *ynorm;
  // wave-uniform choices: the group sums below run in every active lane of the wave.  With 32
  // elements per lane the carried norms cost registers the kernel does not have (it would spill),
  // so that variant sums all three products every time.
  constexpr bool carry = NQ < 32;
  const bool need_a = !carry || __ballot(!(sa_x >= 0.0)) != 0ull;
  const bool need_b = !carry || __ballot(!(yn >= 0.0)) != 0ull;
  double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
  for (int k = 0; k < NQ; ++k) sc = fma(xr[k], yr[k], sc);
  if (need_a) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) sa = fma(xr[k], xr[k], sa);
  }
  if (need_b) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) sb = fma(yr[k], yr[k], sb);
  }
  sc = group_sum<LP>(sc);
  if (need_a) sa = group_sum<LP>(sa);
  else sa = sa_x;
  if (need_b) sb = group_sum<LP>(sb);
  else sb = yn;
  if (sa > 0.0 && sb > 0.0) c2max = fmax(c2max, (sc * sc) / (sa * sb));
  if (sa > 0.0 && sb > 0.0 && sc * sc > (tol * tol) * (sa * sb)) {
    const double zeta = (sb - sa) / (2.0 * sc);
    double t;
    if (fabs(zeta) > 1e150) t = 0.5 / zeta;
    else t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
    const double tc = t * sc, sa2 = sa - tc, sb2 = sb + tc;
    sa_x = (sa2 > 0.5 * sa) ? sa2 : -1.0;
    if (lane == 0) *ynorm = (sb2 > 0.5 * sb) ? sb2 : -1.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int q = lane + LP * k;
      const double xn = cs * xr[k] - sn * yr[k];
      if (q < n) y[q] = sn * xr[k] + cs * yr[k];
      xr[k] = (q < n) ? xn : 0.0;
    }
    ++nrot;
  } else {
    sa_x = sa;
    if (lane == 0) *ynorm = sb;
  }
}

template <int NQ, int LP>
__device__ __forceinline__ void jac_rotate(double* __restrict__ x, double* __restrict__ y, int n, double tol,
                                           int lane, int& nrot, double& c2max) {
  if constexpr (NQ > 0) jac_rotate_pair_r<NQ, LP>(x, y, n, tol, lane, nrot, c2max);
  else jac_rotate_pair(x, y, n, tol, lane, nrot, c2max);  // LP == 64
}

// 16-byte coherent mailbox traffic (two doubles per access; offsets are 16-byte aligned).
typedef unsigned int fs_u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned int))));
typedef double fs_f64x2 __attribute__((__vector_size__(2 * sizeof(double))));
__device__ __forceinline__ fs_f64x2 ld_cob2(__amdgpu_buffer_rsrc_t r, size_t byte_off) {
  return __builtin_bit_cast(fs_f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)(uint32_t)byte_off, 0, FS_CPOL_SC1));
}
__device__ __forceinline__ void st_cob2(__amdgpu_buffer_rsrc_t r, size_t byte_off, fs_f64x2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(fs_u32x4, v), r, (int)(uint32_t)byte_off, 0, FS_CPOL_SC1);
}

__device__ __forceinline__ int circle_player(int pos, int r, int nb) {
  return (pos == 0) ? 0 : 1 + (pos - 1 + r) % (nb - 1);
}

__device__ __forceinline__ void wait_flag(unsigned* f, unsigned target, int* err) {
  unsigned long long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > (1ull << 26)) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

// NQ: elements per lane of a register-resident column (0: loop over LDS); LP: lanes per pair (16 for
// n <= 256, so that a wave rotates four pairs at once, else 64); NT: threads per work-group; SINGLE:
// one work-group holds every column (two blocks, nothing is exchanged), so the exchange code and its
// registers are left out and the work-group can have 1024 threads (64 pair groups of 16 lanes).
template <int NQ, int LP, int NT = SVD_BLOCK_NT, bool SINGLE = false>
__global__ __launch_bounds__(NT) void k_jacobi_block(double* __restrict__ Gm, int n, int b, int NBLK, int max_sweeps,
                                                      double tol, double* __restrict__ mbox, unsigned* __restrict__ flags,
                                                      int* __restrict__ rotcount, int* __restrict__ sweeps_out,
                                                      GridBarrier bar, unsigned long long* __restrict__ maxcos2,
                                                      double stop_cos2, const int* __restrict__ abort_flag) {
  extern __shared__ double lds[];  // [2][b][n]
  const int P = gridDim.x, p = blockIdx.x, tid = threadIdx.x;
  const int gl = tid % LP, grp = tid / LP, ngrp = blockDim.x / LP;  // pair groups (rows or waves)
  const size_t blk = (size_t)b * n;
  double* slot[2] = {lds, lds + blk};
  unsigned bgen = 0;
  auto ncols = [&](int id) { const int c = n - id * b; return c < 0 ? 0 : (c > b ? b : c); };
  // initial arrangement: top = block p, bottom = block NBLK-1-p
  int id[2] = {p, NBLK - 1 - p};
  for (int s2 = 0; s2 < 2; ++s2) {
    const int nc = ncols(id[s2]);
    for (size_t q = tid; q < blk; q += blockDim.x) {
      const int c = (int)(q / n);
      slot[s2][q] = (c < nc) ? Gm[(size_t)(id[s2] * b + c) * n + (q % n)] : 0.0;
    }
  }
  __syncthreads();
  // mailbox layout: [P][2 slots][2 parities][b*n]
  auto mb = [&](int wg, int sl, int par) { return (((size_t)wg * 2 + sl) * 2 + par) * blk; };  // element offset
  const auto rmbox = co_rsrc(mbox, sizeof(double) * (size_t)P * 4 * blk);
  __shared__ int s_nrot[NT / 16];
  __shared__ double s_c2[NT / 16];
  __shared__ double s_ynorm[NT / 16];  // b <= groups <= NT / 16
  int sweep = 0;
  unsigned rr = 0;  // global round counter
  for (; sweep < max_sweeps; ++sweep) {
    int nrot = 0;
    double c2max = 0.0;  // largest cos^2 met this sweep (wave-uniform)
    for (int r = 0; r < NBLK - 1; ++r, ++rr) {
      const int nc0 = ncols(id[0]), nc1 = ncols(id[1]);
      if (r == 0) {
        // pairs inside each block: round-robin over b' = b rounded up to even
        const int be = b + (b & 1);
        for (int sr = 0; sr < be - 1; ++sr) {
          for (int pp = grp; pp < be; pp += ngrp) {  // be/2 pairs per block, two blocks
            const int s2 = pp / (be / 2), k = pp % (be / 2);
            int a = circle_player(k, sr, be), c2 = circle_player(be - 1 - k, sr, be);
            const int nc = s2 ? nc1 : nc0;
            if (a < nc && c2 < nc)
              jac_rotate<NQ, LP>(slot[s2] + (size_t)a * n, slot[s2] + (size_t)c2 * n, n, tol, gl, nrot, c2max);
          }
          __syncthreads();
        }
      }
      // pairs between the two blocks: sub-round s pairs top column t with bottom column (t+s) mod b
      if constexpr (NQ > 0) {
        if (b <= ngrp) {
          // group t holds top column t in registers for the whole round
          const int t = grp;
          const bool own = t < b && t < nc0;
          double xr[NQ];
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            const int q = gl + LP * k;
            xr[k] = (own && q < n) ? slot[0][(size_t)t * n + q] : 0.0;
          }
          double sa_x = -1.0;            // ||x_t||^2, summed at the first sub-round
          if (tid < b) s_ynorm[tid] = -1.0;  // ||y_c||^2 of the bottom columns, likewise
          __syncthreads();
          for (int sr = 0; sr < b; ++sr) {
            const int c2 = (t + sr) % b;
            if (own && c2 < nc1)
              jac_rotate_xreg<NQ, LP>(xr, sa_x, slot[1] + (size_t)c2 * n, &s_ynorm[c2], n, tol, gl, nrot, c2max);
            __syncthreads();
          }
          if (own) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
              const int q = gl + LP * k;
              if (q < n) slot[0][(size_t)t * n + q] = xr[k];
            }
          }
          __syncthreads();
        } else {
          for (int sr = 0; sr < b; ++sr) {
            for (int t = grp; t < b; t += ngrp) {
              const int c2 = (t + sr) % b;
              if (t < nc0 && c2 < nc1)
                jac_rotate<NQ, LP>(slot[0] + (size_t)t * n, slot[1] + (size_t)c2 * n, n, tol, gl, nrot, c2max);
            }
            __syncthreads();
          }
        }
      } else {
        for (int sr = 0; sr < b; ++sr) {
          for (int t = grp; t < b; t += ngrp) {
            const int c2 = (t + sr) % b;
            if (t < nc0 && c2 < nc1)
              jac_rotate<NQ, LP>(slot[0] + (size_t)t * n, slot[1] + (size_t)c2 * n, n, tol, gl, nrot, c2max);
          }
          __syncthreads();
        }
      }
      if (SINGLE || NBLK == 2) continue;  // a single work-group holds every column: nothing moves
      // ---- exchange.  In the next round position q >= 2 holds the block now at q + 1... i.e. blocks
      // move from position q to q - 1 (q >= 2), position 1 wraps to NBLK - 1, position 0 is fixed:
      //   top (position p):          p >= 2 -> top of p-1;  p == 1 -> bottom of 0
      //   bottom (position NBLK-1-p): p <= P-2 -> bottom of p+1;  p == P-1 -> own top (local)
      const int par = rr & 1;
      int dst_top = -1, dst_top_slot = 0, dst_bot = -1;
      if (p >= 2) { dst_top = p - 1; dst_top_slot = 0; }
      if (p == 1) { dst_top = 0; dst_top_slot = 1; }
      if (p <= P - 2) dst_bot = p + 1;
      // mailboxes are written and read with coherent accesses; the flag is raised once every
      // thread's stores have completed (no cache flush needed, see grid_barrier_co)
      auto send = [&](const double* src, size_t o) {
        if ((blk & 1) == 0) {  // pairs of doubles (the mailboxes and b n are even, so 16-byte aligned)
          for (size_t q = 2 * tid; q < blk; q += 2 * (size_t)blockDim.x)
            st_cob2(rmbox, 8 * (o + q), (fs_f64x2){src[q], src[q + 1]});
        } else {
          for (size_t q = tid; q < blk; q += blockDim.x) st_cob(rmbox, 8 * (o + q), src[q]);
        }
      };
      if (dst_top >= 0) send(slot[0], mb(dst_top, dst_top_slot, par));
      if (dst_bot >= 0) send(slot[1], mb(dst_bot, 1, par));
      stores_complete();
      __syncthreads();
      if (tid == 0) {
        if (dst_top >= 0)
          __hip_atomic_store(&flags[dst_top * 2 + dst_top_slot], rr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (dst_bot >= 0)
          __hip_atomic_store(&flags[dst_bot * 2 + 1], rr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // local move: the last work-group's bottom becomes its top (its old top was sent above)
      if (p == P - 1 && p >= 1) {
        for (size_t q = tid; q < blk; q += blockDim.x) slot[0][q] = slot[1][q];
      }
      // receives: top from p+1 (p <= P-2, p >= 1); bottom from p-1's bottom (p >= 1) or 1's top (p == 0)
      const bool recv_top = (p >= 1 && p <= P - 2);
      const bool recv_bot = true;
      if (tid == 0) {
        if (recv_top) wait_flag(&flags[p * 2 + 0], rr + 1, bar.err);
        if (recv_bot) wait_flag(&flags[p * 2 + 1], rr + 1, bar.err);
      }
      __syncthreads();
      // batches of 8 independent coherent loads per thread (offsets past the block read 0)
      auto recv = [&](double* dst, size_t src) {
        if ((blk & 1) == 0) {
          for (size_t q0 = 2 * tid; q0 < blk; q0 += 16 * (size_t)blockDim.x) {
            fs_f64x2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const size_t q = q0 + (size_t)u * 2 * blockDim.x;
              v[u] = ld_cob2(rmbox, q < blk ? 8 * (src + q) : (size_t)0xFFFFFFF0u);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const size_t q = q0 + (size_t)u * 2 * blockDim.x;
              if (q < blk) {
                dst[q] = v[u][0];
                dst[q + 1] = v[u][1];
              }
            }
          }
          return;
        }
        for (size_t q0 = tid; q0 < blk; q0 += 8 * (size_t)blockDim.x) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const size_t q = q0 + (size_t)u * blockDim.x;
            v[u] = ld_cob(rmbox, q < blk ? 8 * (src + q) : (size_t)0xFFFFFFF0u);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const size_t q = q0 + (size_t)u * blockDim.x;
            if (q < blk) dst[q] = v[u];
          }
        }
      };
      // (not in the 32-elements-per-lane variant: its registers are spent on the columns)
      if (NQ != 32 && (blk & 1) == 0 && blk <= 16 * (size_t)blockDim.x) {
        // both blocks in one batch of coherent loads (one round trip instead of two)
        const size_t s0 = mb(p, 0, par), s1 = mb(p, 1, par);
        fs_f64x2 v0[8], v1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const size_t q = 2 * tid + (size_t)u * 2 * blockDim.x;
          v0[u] = ld_cob2(rmbox, (recv_top && q < blk) ? 8 * (s0 + q) : (size_t)0xFFFFFFF0u);
          v1[u] = ld_cob2(rmbox, (recv_bot && q < blk) ? 8 * (s1 + q) : (size_t)0xFFFFFFF0u);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const size_t q = 2 * tid + (size_t)u * 2 * blockDim.x;
          if (q < blk) {
            if (recv_top) {
              slot[0][q] = v0[u][0];
              slot[0][q + 1] = v0[u][1];
            }
            if (recv_bot) {
              slot[1][q] = v1[u][0];
              slot[1][q + 1] = v1[u][1];
            }
          }
        }
      } else {
        if (recv_top) recv(slot[0], mb(p, 0, par));
        if (recv_bot) recv(slot[1], mb(p, 1, par));
      }
      __syncthreads();
      // block ids after the move (round r + 1 of this sweep)
      id[0] = circle_player(p, r + 1, NBLK);
      id[1] = circle_player(NBLK - 1 - p, r + 1, NBLK);
    }
    // sweep total and largest cosine (positive doubles order like their bit patterns)
    if (gl == 0) {
      s_nrot[grp] = nrot;
      s_c2[grp] = c2max;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      double c2 = 0.0;
      for (int w = 0; w < ngrp; ++w) {
        t += s_nrot[w];
        c2 = fmax(c2, s_c2[w]);
      }
      if (t) __hip_atomic_fetch_add(&rotcount[sweep], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // a caller that no longer needs the SVD raises abort_flag; any work-group that has seen it by
      // now marks the sweep (bit 30 of its count, far above any rotation count), so all agree after
      // the barrier and stop together
      if (abort_flag && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        __hip_atomic_fetch_or(&rotcount[sweep], 1 << 30, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_max(&maxcos2[sweep], (unsigned long long)__double_as_longlong(c2), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_barrier_co(bar, (unsigned)P, bgen);
    const int tot = __hip_atomic_load(&rotcount[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double c2s = __longlong_as_double(
        (long long)__hip_atomic_load(&maxcos2[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    // Converged, or in the quadratic phase: a sweep whose largest cosine was <= sqrt(stop_cos2)
    // leaves cosines of order n stop_cos2, which the orthogonality correction of V removes; the
    // sweep that would only confirm convergence is skipped.
    if (tot & (1 << 30)) {  // abandoned: the results are not used
      ++sweep;
      break;
    }
    if (tot == 0 || c2s <= stop_cos2) {
      ++sweep;
      break;
    }
  }
  // write the blocks back (after a full sweep they are at their starting positions)
  for (int s2 = 0; s2 < 2; ++s2) {
    const int nc = ncols(id[s2]);
    for (size_t q = tid; q < blk; q += blockDim.x) {
      const int c = (int)(q / n);
      if (c < nc) Gm[(size_t)(id[s2] * b + c) * n + (q % n)] = slot[s2][q];
    }
  }
  if (p == 0 && tid == 0 && sweeps_out) *sweeps_out = sweep;
}

// G0 = R^T (n x n, ld n) from the upper triangle of R (ldr); U = I.
__global__ void k_svd_init(const double* __restrict__ R, int64_t ldr, int n, double* __restrict__ Gm,
                           double* __restrict__ U) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * n) return;
  const int row = (int)(q % n), col = (int)(q / n);  // Gm[row, col] = R[col, row]
  Gm[q] = (row >= col) ? R[(int64_t)row * ldr + col] : 0.0;
  if (U) U[q] = (row == col) ? 1.0 : 0.0;
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

__global__ void k_svd_norms(const double* __restrict__ Gm, int n, double* __restrict__ norms, const int* __restrict__ skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int i = blockIdx.x;
  __shared__ double sh[4];
  const double* gi = Gm + (int64_t)i * n;
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) s = fma(gi[q], gi[q], s);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) norms[i] = sqrt(s);
}

__global__ void k_svd_sort_write(const double* __restrict__ Gm, const double* __restrict__ U, int n,
                                 const double* __restrict__ norms, double* __restrict__ sigma, double* __restrict__ V,
                                 int64_t ldv, double* __restrict__ Uout, int64_t ldu, const int* __restrict__ skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int i = blockIdx.x;
  __shared__ int srank;
  const double si = norms[i];
  if (threadIdx.x == 0) srank = 0;
  __syncthreads();
  int cnt = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double sj = norms[j];
    cnt += (sj > si || (sj == si && j < i)) ? 1 : 0;
  }
  atomicAdd(&srank, cnt);
  __syncthreads();
  const int rk = srank;
  if (threadIdx.x == 0) sigma[rk] = si;
  const double inv = (si > 0.0) ? 1.0 / si : 0.0;
  const double* gi = Gm + (int64_t)i * n;
  for (int q = threadIdx.x; q < n; q += 256) V[(int64_t)rk * ldv + q] = gi[q] * inv;
  if (Uout)
    for (int q = threadIdx.x; q < n; q += 256) Uout[(int64_t)rk * ldu + q] = U[(int64_t)i * n + q];
}

// ---------------------------------------------------------------- orthogonality correction of V
// The Jacobi sweeps stop once every pair satisfies |v_i^T v_j| <= tol (tol = n u), so the normalized
// columns are orthogonal only to n u.  The preconditioner V Sigma^{-1} turns that into
// R V Sigma^{-1} = J Sigma (V^T V) Sigma^{-1}, whose (i, j) entry carries sigma_i / sigma_j times the
// cosine: up to condest * n u, far above 1 at condest ~ 1e13 and n ~ 1000.  One first-order Cholesky
// step restores orthogonality to working precision: with C = V^T V - I and T = triu(C, 1) + diag(C) / 2
// (V^T V = (I + T)^T (I + T) + O(C^2)), V <- V (I + T)^{-1} ~= V - V T.  Columns are sorted by
// decreasing sigma, so the remaining lower-triangular coupling is damped (sigma_i / sigma_j <= 1).
//
// Both products run on the FP64 matrix cores: a 256-thread work-group owns a 64 x 64 output tile,
// each wave a 32 x 32 block (2 x 2 v_mfma_f64_16x16x4f64 accumulators); operands come straight from
// global memory (V is 8 MB at n = 1000 and stays in L2 / MALL).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int OC_T = 64;

// Tc[i, j] (ld n) = v_i^T v_j for i < j, (v_i^T v_i - 1) / 2 on the diagonal, 0 below (tiles on or
// above the diagonal only; tiles wholly below it are never read).
__global__ __launch_bounds__(256) void k_v_gram_upper(const double* __restrict__ V, int64_t ldv, int n,
                                                      double* __restrict__ Tc, const int* __restrict__ skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = I * OC_T + (w >> 1) * 32, j0 = J * OC_T + (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int ia[2] = {i0 + lr, i0 + 16 + lr};
  const int jb[2] = {j0 + lr, j0 + 16 + lr};
  for (int k = 0; k < n; k += 16) {
    double av[4][2], bv[4][2];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = k + 4 * s + lk;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[s][q] = (kk < n && ia[q] < n) ? V[(int64_t)ia[q] * ldv + kk] : 0.0;
        bv[s][q] = (kk < n && jb[q] < n) ? V[(int64_t)jb[q] * ldv + kk] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a], bv[s][b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + a * 16 + 4 * r + lk, j = j0 + b * 16 + lr;
        if (i >= n || j >= n) continue;
        const double c = acc[a][b][r];
        Tc[(int64_t)j * n + i] = (i < j) ? c : ((i == j) ? 0.5 * (c - 1.0) : 0.0);
      }
}

// Vout[:, j] (ld n) = V[:, j] - sum_{i <= j} V[:, i] Tc[i, j].
__global__ __launch_bounds__(256) void k_v_correct(const double* __restrict__ V, int64_t ldv, int n,
                                                   const double* __restrict__ Tc, double* __restrict__ Vout, const int* __restrict__ skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int I = blockIdx.y, J = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = I * OC_T + (w >> 1) * 32, j0 = J * OC_T + (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  const int kend = min(n, (J + 1) * OC_T);  // Tc is upper triangular
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int ra[2] = {r0 + lr, r0 + 16 + lr};
  const int jb[2] = {j0 + lr, j0 + 16 + lr};
  for (int k = 0; k < kend; k += 16) {
    double av[4][2], bv[4][2];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = k + 4 * s + lk;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[s][q] = (kk < kend && ra[q] < n) ? V[(int64_t)kk * ldv + ra[q]] : 0.0;
        bv[s][q] = (kk < kend && jb[q] < n) ? Tc[(int64_t)jb[q] * n + kk] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a], bv[s][b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + a * 16 + 4 * r + lk, j = j0 + b * 16 + lr;
        if (row >= n || j >= n) continue;
        Vout[(int64_t)j * n + row] = V[(int64_t)j * ldv + row] - acc[a][b][r];
      }
}

}  // namespace

namespace {
constexpr int SVD_LDS_BYTES = 144 * 1024;
// counters region (ints): rotation counts [0, 64) | fenced barrier [64, 67) | fence-free barrier
// [72, 72 + FS_BAR_WORDS) | per-sweep largest cos^2 (64 x 8 bytes, 8-byte aligned); in doubles
constexpr int SVD_MC_INT = (72 + FS_BAR_WORDS + 2) & ~1;
constexpr int SVD_CTR_DOUBLES = (SVD_MC_INT + 128) / 2 + 1;
// Block width for the systolic kernel: two blocks of b columns must fit in LDS.
int svd_block_width(int n) {
  const int bmax = SVD_LDS_BYTES / (2 * 8 * n);
  if (bmax < 1) return 0;                 // too large: pairwise fallback
  if (2 * bmax >= n) return (n + 1) / 2;  // everything in one work-group
  // a work-group rotates 8 pairs at once with whole-wave pairs, 32 with 16-lane pairs (n <= 256)
  const int bcap = (n <= 256) ? 32 : 8;
  return bmax < bcap ? bmax : bcap;
}
}  // namespace

int* fs_svd_err_word(void* work, int n) {
  double* norms = (double*)work + (size_t)2 * n * n;
  return (int*)(norms + n) + 66;
}

// Work-groups of the block (systolic) variant, or 0 when it does not apply: U_R wanted, columns too
// long for two blocks in LDS, or more block pairs than compute units (n above ~2170).
static int svd_block_grid(int n, int num_cu, bool with_u) {
  const int bw = svd_block_width(n);
  if (with_u || bw <= 0) return 0;
  const int nblk = (n + bw - 1) / bw;
  const int P = (nblk + (nblk & 1)) / 2;
  return (P <= num_cu) ? P : 0;
}

int fs_svd_grid_size(int n, int num_cu, bool with_u) {
  const int Pb = svd_block_grid(n, num_cu, with_u);
  if (Pb > 0) return Pb;
  const int G = (n + 1) / 2;
  return G < num_cu ? (G < 1 ? 1 : G) : num_cu;
}

size_t fs_svd_work_bytes(int n) {
  // Gm | Uacc | norms | counters | mailboxes [P][2][2][b*n] | flags [P][2]
  const int b = svd_block_width(n);
  size_t mbox = 0, nflags = 0;
  if (b > 0) {
    const int nblk = (n + b - 1) / b;
    const int NBLK = nblk + (nblk & 1);
    const int P = NBLK / 2;
    mbox = (size_t)P * 4 * b * n;
    nflags = (size_t)P * 2;
  }
  return sizeof(double) * ((size_t)2 * n * n + n + SVD_CTR_DOUBLES + mbox) + sizeof(int) * nflags + 1024;
}

// work layout: Gm (n*n) | Uacc (n*n) | norms (n) | rotcount (64 ints) | sweeps (int)
hipError_t fs_launch_svd_abortable(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                                   double* Uout, int64_t ldu, void* work, int num_cu, int max_sweeps,
                                   int* sweeps_out_dev, const int* abort_flag, hipStream_t s) {
  if (max_sweeps > 64) max_sweeps = 64;
  double* Gm = (double*)work;
  double* Uacc = Gm + (size_t)n * n;
  double* norms = Uacc + (size_t)n * n;
  int* rot = (int*)(norms + n);
  // rotation counts (64) | fenced-barrier words (count, gen, err) | fence-free barrier words
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, s, rot, 2 * SVD_CTR_DOUBLES, 0);
  GridBarrier bar{(unsigned*)(rot + 64), (unsigned*)(rot + 65), rot + 66};
  GridBarrier bar_co{(unsigned*)(rot + 72), nullptr, rot + 66};
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_svd_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, R, ldr, n, Gm,
                     Uout ? Uacc : (double*)nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double tol = (double)(n > 1 ? n : 1) * 2.220446049250313e-16;
  double* Uarg = Uout ? Uacc : nullptr;
  const int bw = svd_block_width(n);
  if (svd_block_grid(n, num_cu, Uout != nullptr) > 0) {
    // systolic block Jacobi (no accumulation of U_R)
    const int nblk = (n + bw - 1) / bw;
    const int NBLK = nblk + (nblk & 1);
    const int P = NBLK / 2;
    // after the counters, 16-byte aligned (the workspace has 1 KB of slack)
    double* mbox = (double*)(((uintptr_t)(norms + n + SVD_CTR_DOUBLES) + 15) & ~(uintptr_t)15);
    unsigned* flg = (unsigned*)(mbox + (size_t)P * 4 * bw * n);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, s, (int*)flg, 2 * P, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t shmem = (size_t)2 * bw * n * sizeof(double);
    // columns of up to 2048 rows are rotated from registers (NQ = elements per lane)
    // (65..128 columns: one work-group of 1024 threads holds them all, blocks of up to 64 columns)
    const bool single1k = (n > 64 && n <= 128 && P == 1);
    const void* kfn = (n <= 64)     ? (const void*)k_jacobi_block<4, 16>
                      : single1k    ? (const void*)k_jacobi_block<8, 16, 1024, true>
                      : (n <= 128)  ? (const void*)k_jacobi_block<8, 16>
                      : (n <= 256)  ? (const void*)k_jacobi_block<16, 16>
                      : (n <= 512)  ? (const void*)k_jacobi_block<8, 64>
                      : (n <= 1024) ? (const void*)k_jacobi_block<16, 64>
                      : (n <= 2048) ? (const void*)k_jacobi_block<32, 64>
                                    : (const void*)k_jacobi_block<0, 64>;
    (void)hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    int NB2 = NBLK;
    int bw2 = bw;
    unsigned long long* mc2 = (unsigned long long*)(rot + SVD_MC_INT);
    double stop_cos2 = 1e-10;  // a sweep whose cosines all stayed <= 1e-5 ends the iteration
    void* args[] = {&Gm, &n, &bw2, &NB2, &max_sweeps, &tol, &mbox, &flg, &rot, &sweeps_out_dev, &bar_co, &mc2,
                    &stop_cos2, &abort_flag};
    e = fs_launch_resident(kfn, dim3(P), dim3(single1k ? 1024 : SVD_BLOCK_NT), args, shmem, s);
    if (e != hipSuccess) return e;
  } else {
    int G = (n + 1) / 2;
    if (G > num_cu) G = num_cu;
    if (G < 1) G = 1;
    void* args[] = {&Gm, &Uarg, &n, &max_sweeps, &tol, &rot, &sweeps_out_dev, &bar};
    e = fs_launch_resident((const void*)k_jacobi_coop, dim3(G), dim3(SVD_NT), args, 0, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_svd_norms, dim3(n), dim3(256), 0, s, Gm, n, norms, abort_flag);
  hipLaunchKernelGGL(k_svd_sort_write, dim3(n), dim3(256), 0, s, Gm, Uarg, n, norms, sigma, V, ldv, Uout, ldu,
                     abort_flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // orthogonality correction of V (Gm and Uacc are free once sorted and written): Tc in Gm, the
  // corrected V in Uacc, copied back to V
  // Two passes: the Jacobi stop leaves cosines up to ~n 1e-10; each pass squares the remainder.
  const unsigned T = (unsigned)((n + OC_T - 1) / OC_T);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_v_gram_upper, dim3(T, T), dim3(256), 0, s, V, ldv, n, Gm, abort_flag);
    hipLaunchKernelGGL(k_v_correct, dim3(T, T), dim3(256), 0, s, V, ldv, n, Gm, Uacc, abort_flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipMemcpy2DAsync(V, sizeof(double) * ldv, Uacc, sizeof(double) * n, sizeof(double) * n, n,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fs_launch_svd_full(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv, double* Uout,
                              int64_t ldu, void* work, int num_cu, int max_sweeps, int* sweeps_out_dev,
                              hipStream_t s) {
  return fs_launch_svd_abortable(R, ldr, n, sigma, V, ldv, Uout, ldu, work, num_cu, max_sweeps, sweeps_out_dev,
                                 nullptr, s);
}

hipError_t fs_launch_svd(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv, void* work,
                         int num_cu, int max_sweeps, int* sweeps_out_dev, hipStream_t s) {
  return fs_launch_svd_full(R, ldr, n, sigma, V, ldv, nullptr, 0, work, num_cu, max_sweeps, sweeps_out_dev, s);
}
