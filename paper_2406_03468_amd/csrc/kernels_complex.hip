// Complex least squares through its realification.
//
// The Prony problems of Section 5.2 (Appendix B) are complex: A in C^{m x n}, b in C^m.  The map
//   A -> A_R = [Re A, -Im A; Im A, Re A]  (2m x 2n),   x -> [Re x; Im x],   b -> [Re b; Im b]
// is an isometry of the residual (||A x - b|| = ||A_R x_R - b_R||) and A_R has the singular
// values of A, each twice, so the real solvers run unchanged on (A_R, b_R).  Inputs are complex128
// column-major arrays with interleaved (re, im) doubles; A_R is written column-major with
// leading dimension 2m.  Pure data movement: one read of A, two writes of its size.
#include "common.hpp"
#include "internal.hpp"

namespace {

typedef double fs_c2d __attribute__((ext_vector_type(2)));

constexpr int RZ_NT = 256;

// one work-group per (column, tile of RZ_NT complex rows): blockIdx.x = j * ntile + tile
__global__ __launch_bounds__(RZ_NT) void k_realify_A(int64_t m, int n, int ntile, const double* __restrict__ A,
                                                     int64_t lda, double* __restrict__ Ar) {
  const int j = (int)(blockIdx.x / (unsigned)ntile);
  const int64_t i = (int64_t)(blockIdx.x % (unsigned)ntile) * RZ_NT + threadIdx.x;
  if (i >= m || j >= n) return;
  const fs_c2d a = *reinterpret_cast<const fs_c2d*>(A + 2 * ((int64_t)j * lda + i));
  const int64_t ld = 2 * m;
  double* c0 = Ar + (int64_t)j * ld;        // column j:      [Re a; Im a]
  double* c1 = Ar + (int64_t)(n + j) * ld;  // column n + j:  [-Im a; Re a]
  c0[i] = a.x;
  c0[m + i] = a.y;
  c1[i] = -a.y;
  c1[m + i] = a.x;
}

__global__ __launch_bounds__(RZ_NT) void k_realify_b(int64_t m, const double* __restrict__ b, double* __restrict__ br) {
  const int64_t i = (int64_t)blockIdx.x * RZ_NT + threadIdx.x;
  if (i >= m) return;
  const fs_c2d v = *reinterpret_cast<const fs_c2d*>(b + 2 * i);
  br[i] = v.x;
  br[m + i] = v.y;
}

__global__ __launch_bounds__(RZ_NT) void k_complexify_x(int n, const double* __restrict__ xr, double* __restrict__ x) {
  const int j = blockIdx.x * RZ_NT + threadIdx.x;
  if (j >= n) return;
  *reinterpret_cast<fs_c2d*>(x + 2 * (int64_t)j) = fs_c2d{xr[j], xr[n + j]};
}

}  // namespace

hipError_t fs_launch_realify(int64_t m, int n, const double* A, int64_t lda, const double* b, double* Ar, double* br,
                             hipStream_t s) {
  const int64_t ntile = (m + RZ_NT - 1) / RZ_NT;
  if (ntile * n > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_realify_A, dim3((unsigned)(ntile * n)), dim3(RZ_NT), 0, s, m, n, (int)ntile, A, lda, Ar);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_realify_b, dim3((unsigned)((m + RZ_NT - 1) / RZ_NT)), dim3(RZ_NT), 0, s, m, b, br);
  return hipGetLastError();
}

hipError_t fs_launch_complexify_x(int n, const double* xr, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_complexify_x, dim3((unsigned)((n + RZ_NT - 1) / RZ_NT)), dim3(RZ_NT), 0, s, n, xr, x);
  return hipGetLastError();
}
