// Explicit inverse X = R^{-1} of an upper-triangular R (n x n, ldr), for refinement steps that apply
// P = R^{-1} many times with the same R: each application then is one dense product with X (a pass
// over n^2 doubles that stay in cache) instead of a chain of dependent substitution blocks.
//
// The inverse is formed by blocks of 64 with the recursive 2 x 2 block form of a triangular inverse:
//   [R11 R12; 0 R22]^{-1} = [X11, -X11 R12 X22; 0, X22],  X11 = R11^{-1},  X22 = R22^{-1}.
// The diagonal 64 x 64 blocks are inverted by substitution on the identity.  Then, for
// block sizes s = 64, 128, 256, ..., the upper-right block X12 of every 2s x 2s diagonal block is
// formed from blocks the earlier levels finished: T12 = R12 X22, then X12 = -X11 T12.  Every entry of
// an upper-right tile belongs to exactly one level (the highest bit in which its row and column block
// indices differ), so the levels write disjoint tiles.  X is written whole (ld n, zeros below the
// diagonal); T is an n x n scratch whose tiles at the X12 positions hold the level's T12.
#include "common.hpp"
#include "internal.hpp"

namespace {

constexpr int TI_B = 64;
constexpr int TI_NT = 256;
constexpr int TI_KC = 64;  // inner-dimension chunk of the level products

// One work-group per diagonal block J: X_JJ = R_JJ^{-1} by right-looking substitution on the identity,
// all 64 columns at once: for i = 63 .. 0, row i of X is t_i / r_ii, then rows k < i of the
// right-hand sides take t_k -= r_ki x_i (a rank-1 update).  Thread (g, c) = (tid / 64, tid % 64) holds
// rows g, g + 4, ..., g + 60 of column c in registers.  Then block column J is written from row j0
// down (the diagonal block, zeros below it).
__global__ __launch_bounds__(TI_NT) void k_tri_inv_diag(const double* __restrict__ R, int64_t ldr, int n,
                                                        double* __restrict__ X) {
  __shared__ double rb[TI_B][TI_B + 1];  // rb[r][c] = R[j0 + r][j0 + c] (upper triangle; 1 on a padded diagonal)
  __shared__ double xrow[2][TI_B];
  const int j0 = (int)blockIdx.x * TI_B, tid = threadIdx.x;
  const int nb = min(TI_B, n - j0);
  {  // all 16 loads of a thread in flight before the LDS stores
    double v[TI_B * TI_B / TI_NT];
#pragma unroll
    for (int u = 0; u < TI_B * TI_B / TI_NT; ++u) {
      const int q = tid + TI_NT * u, r = q & (TI_B - 1), c = q / TI_B;
      v[u] = (r < nb && c < nb && r <= c) ? R[(int64_t)(j0 + c) * ldr + j0 + r] : ((r == c && r >= nb) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < TI_B * TI_B / TI_NT; ++u) {
      const int q = tid + TI_NT * u;
      rb[q & (TI_B - 1)][q / TI_B] = v[u];
    }
  }
  const int g = tid >> 6, c = tid & (TI_B - 1);
  double t[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) t[u] = (g + 4 * u == c) ? 1.0 : 0.0;
  __syncthreads();
#pragma unroll
  for (int i = TI_B - 1; i >= 0; --i) {
    const int gi = i & 3, ui = i >> 2;
    if (g == gi) {
      const double xv = t[ui] / rb[i][i];
      t[ui] = xv;
      xrow[i & 1][c] = xv;
    }
    __syncthreads();
    const double xi = xrow[i & 1][c];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (4 * u + 3 < i || (4 * u < i && g + 4 * u < i)) t[u] = fma(-rb[g + 4 * u][i], xi, t[u]);
    }
  }
  const int rows = n - j0;  // rows j0 .. n-1 of the block's columns
  if (c < nb) {
    double* col = X + (int64_t)(j0 + c) * n + j0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (g + 4 * u < nb) col[g + 4 * u] = t[u];
    for (int r = TI_B + g; r < rows; r += 4) col[r] = 0.0;
  }
}

// Level s of the recursion.  Pair p: rows [a, a + s), columns [a + s, a + s + s2), a = 2 p s,
// s2 = min(s, n - a - s).  mode 0: T12 = R12 X22 (inner dimension s2; X22 is upper triangular, so
// output column j takes k <= j only); mode 1: X12 = -X11 T12 (inner dimension s; X11 upper
// triangular, so output row i takes k >= i only).  64 x 64 output tiles (blockIdx.x: row tile,
// blockIdx.y: column tile, blockIdx.z: pair), 256 threads with 4 x 4 outputs each, the inner
// dimension in chunks of 64 staged in LDS.
__global__ __launch_bounds__(TI_NT) void k_tri_inv_level(const double* __restrict__ R, int64_t ldr, int n, int s,
                                                         int mode, double* __restrict__ X, double* __restrict__ T) {
  const int a = 2 * (int)blockIdx.z * s;
  if (a + s >= n) return;
  const int s2 = min(s, n - a - s);
  const int i0 = (int)blockIdx.x * TI_B, j0 = (int)blockIdx.y * TI_B;
  if (i0 >= s || j0 >= s2) return;
  const double* A;
  const double* B;
  int64_t lda;
  int K, kbeg, kend;
  double* C;
  double alpha;
  if (mode == 0) {
    A = R + (int64_t)(a + s) * ldr + a;  // R12: s x s2
    lda = ldr;
    B = X + (int64_t)(a + s) * n + (a + s);  // X22: s2 x s2
    K = s2;
    kbeg = 0;
    kend = min(K, j0 + TI_B);
    C = T + (int64_t)(a + s) * n + a;
    alpha = 1.0;
  } else {
    A = X + (int64_t)a * n + a;  // X11: s x s
    lda = n;
    B = T + (int64_t)(a + s) * n + a;  // T12: s x s2
    K = s;
    kbeg = i0;
    kend = K;
    C = X + (int64_t)(a + s) * n + a;
    alpha = -1.0;
  }
  const int64_t ldb = n, ldc = n;
  __shared__ double As[TI_KC][TI_B + 1];  // As[k][r] = A[i0 + r][k0 + k]
  __shared__ double Bs[TI_B][TI_KC + 1];  // Bs[c][k] = B[k0 + k][j0 + c]
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  // both 64 x 64 chunks of the next inner-dimension step are loaded (into registers) while the
  // current one is multiplied out of LDS.  A rows i0 + r < s always (s is a multiple of 64); B
  // columns j0 + c < s2.
  double av[16], bv[16];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = tid & (TI_B - 1), k = (tid >> 6) + 4 * u;
      av[u] = (k0 + k < kend) ? A[(int64_t)(k0 + k) * lda + i0 + r] : 0.0;
      const int kb = tid & (TI_KC - 1), cb = (tid >> 6) + 4 * u;
      bv[u] = (k0 + kb < kend && j0 + cb < s2) ? B[(int64_t)(j0 + cb) * ldb + k0 + kb] : 0.0;
    }
  };
  load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += TI_KC) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      As[(tid >> 6) + 4 * u][tid & (TI_B - 1)] = av[u];
      Bs[(tid >> 6) + 4 * u][tid & (TI_KC - 1)] = bv[u];
    }
    __syncthreads();
    if (k0 + TI_KC < kend) load(k0 + TI_KC);
#pragma unroll 8
    for (int k = 0; k < TI_KC; ++k) {
      double a4[4], b4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = As[k][tr + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b4[v] = Bs[tc + 16 * v][k];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a4[u], b4[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int c = j0 + tc + 16 * v;
    if (c >= s2) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) C[(int64_t)c * ldc + i0 + tr + 16 * u] = alpha * acc[u][v];
  }
}

}  // namespace

hipError_t fs_launch_tri_inv(const double* R, int64_t ldr, int n, double* X, double* T, hipStream_t s) {
  if (n < 1 || ldr < n || !R || !X || !T) return hipErrorInvalidValue;
  const int nb = (n + TI_B - 1) / TI_B;
  hipLaunchKernelGGL(k_tri_inv_diag, dim3((unsigned)nb), dim3(TI_NT), 0, s, R, ldr, n, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int lv = TI_B; lv < n; lv *= 2) {
    const unsigned tiles = (unsigned)(lv / TI_B);
    const unsigned pairs = (unsigned)((n + 2 * lv - 1) / (2 * lv));
    for (int mode = 0; mode < 2; ++mode) {
      hipLaunchKernelGGL(k_tri_inv_level, dim3(tiles, tiles, pairs), dim3(TI_NT), 0, s, R, ldr, n, lv, mode, X, T);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}
