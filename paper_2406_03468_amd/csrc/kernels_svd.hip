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

__global__ void k_svd_norms(const double* __restrict__ Gm, int n, double* __restrict__ norms) {
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
                                 int64_t ldv, double* __restrict__ Uout, int64_t ldu) {
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

}  // namespace

size_t fs_svd_work_bytes(int n) { return sizeof(double) * ((size_t)2 * n * n + n) + sizeof(int) * 160 + 512; }

// work layout: Gm (n*n) | Uacc (n*n) | norms (n) | rotcount (64 ints) | sweeps (int)
hipError_t fs_launch_svd_full(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv, double* Uout,
                              int64_t ldu, void* work, int num_cu, int max_sweeps, int* sweeps_out_dev,
                              hipStream_t s) {
  if (max_sweeps > 64) max_sweeps = 64;
  double* Gm = (double*)work;
  double* Uacc = Gm + (size_t)n * n;
  double* norms = Uacc + (size_t)n * n;
  int* rot = (int*)(norms + n);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, rot, 80, 0);  // rotation counts + barrier words
  GridBarrier bar{(unsigned*)(rot + 64), (unsigned*)(rot + 65), rot + 66};
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_svd_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, R, ldr, n, Gm,
                     Uout ? Uacc : (double*)nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int G = (n + 1) / 2;
  if (G > num_cu) G = num_cu;
  if (G < 1) G = 1;
  double tol = (double)(n > 1 ? n : 1) * 2.220446049250313e-16;
  double* Uarg = Uout ? Uacc : nullptr;
  void* args[] = {&Gm, &Uarg, &n, &max_sweeps, &tol, &rot, &sweeps_out_dev, &bar};
  e = hipLaunchCooperativeKernel((const void*)k_jacobi_coop, dim3(G), dim3(SVD_NT), args, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_svd_norms, dim3(n), dim3(256), 0, s, Gm, n, norms);
  hipLaunchKernelGGL(k_svd_sort_write, dim3(n), dim3(256), 0, s, Gm, Uarg, n, norms, sigma, V, ldv, Uout, ldu);
  return hipGetLastError();
}

hipError_t fs_launch_svd(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv, void* work,
                         int num_cu, int max_sweeps, int* sweeps_out_dev, hipStream_t s) {
  return fs_launch_svd_full(R, ldr, n, sigma, V, ldv, nullptr, 0, work, num_cu, max_sweeps, sweeps_out_dev, s);
}
