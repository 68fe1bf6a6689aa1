// Sparse sign embedding: index stream generation and the sketch S [A b].
//
// Paper, Section 4.2 ("Choice of embedding"): S = zeta^{-1/2} [s_1 ... s_m], each column s_j with
// zeta nonzeros +-1 at uniformly random distinct positions in [0, d).  The generator is this
// library's own counter-based stream on Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11):
//   key = (seed mod 2^32, seed >> 32)
//   positions of column j: the words of Philox((j mod 2^32, j >> 32, t, 0)), t = 0, 1, ..., in
//     order; word w gives floor(w d / 2^32) unless (w d) mod 2^32 < 2^32 mod d (Lemire's unbiased
//     multiply-shift) or the value was already accepted for this column; after 64 blocks the
//     remaining positions are the smallest unused ones;
//   signs: bit k (k-th accepted position) of Philox((j mod 2^32, j >> 32, k / 128, 1)), word
//     (k mod 128) / 32, bit k mod 32; a set bit means -1.
// Each entry is stored as (position << 1) | sign_bit in 16 bits (d < 32768) or 32 bits.
//
// Sketch apply: one work-group per (panel of columns, chunk of sketch rows).  The panel of
// columns of Y lives in LDS (one fp64 column at d = 12000 is 96 KB); the work-group streams its
// columns of A top to bottom (coalesced, contiguous) together with the index stream and adds
// +-a_ij into the LDS copy of Y with fp64 LDS atomics.  The column norms of A (column scaling,
// Alg 4's first statement) are accumulated in the same read, and the write-out applies
// zeta^{-1/2} / ||a_j||.
#include "common.hpp"
#include "internal.hpp"

namespace {

constexpr int T_MAX_BLOCKS = 64;
constexpr int ZETA_MAX = 64;

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

template <typename IDX>
__global__ __launch_bounds__(256) void k_sketch_indices(int64_t col0, int64_t ncols, int d, int zeta, uint32_t k0,
                                                        uint32_t k1, IDX* __restrict__ out) {
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= ncols) return;
  const uint64_t j = (uint64_t)(col0 + jj);
  const uint32_t jlo = (uint32_t)j, jhi = (uint32_t)(j >> 32);
  const uint32_t thresh = (uint32_t)((((uint64_t)1) << 32) % (uint64_t)d);
  uint32_t pos[ZETA_MAX];
  int cnt = 0;
  for (int t = 0; t < T_MAX_BLOCKS && cnt < zeta; ++t) {
    const U4 w = philox4x32_10(U4{jlo, jhi, (uint32_t)t, 0u}, k0, k1);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (cnt >= zeta) break;
      const uint64_t prod = (uint64_t)ws[q] * (uint64_t)d;
      if ((uint32_t)prod < thresh) continue;
      const uint32_t cand = (uint32_t)(prod >> 32);
      bool dup = false;
      for (int i = 0; i < cnt; ++i) dup |= (pos[i] == cand);
      if (!dup) pos[cnt++] = cand;
    }
  }
  for (uint32_t v = 0; cnt < zeta; ++v) {  // completion rule (practically unreachable)
    bool dup = false;
    for (int i = 0; i < cnt; ++i) dup |= (pos[i] == v);
    if (!dup) pos[cnt++] = v;
  }
  for (int blk = 0; blk * 128 < zeta; ++blk) {
    const U4 w = philox4x32_10(U4{jlo, jhi, (uint32_t)blk, 1u}, k0, k1);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    for (int k = blk * 128; k < zeta && k < blk * 128 + 128; ++k) {
      const int kk = k - blk * 128;
      const uint32_t bit = (ws[kk >> 5] >> (kk & 31)) & 1u;
      out[jj * zeta + k] = (IDX)((pos[k] << 1) | bit);
    }
  }
}

// One work-group per (column panel, sketch-row chunk).  Columns c < n come from A, columns
// n <= c < ncols from B (ldb).  PW is the compile-time panel width (columns held in LDS at once);
// np <= PW columns are active.  Each thread walks RU rows per step with all their loads issued
// before the LDS atomics (memory-level parallelism), and, for panels of up to 4 columns (2 with
// 32-bit entries), the next step's loads before the current step's atomics; for zeta = 8 with 16-bit entries the eight
// entries of a row come in one 16-byte load.  TA is the element type of A (double, or float for the
// mixed-precision form's FP32 copy); R32 rounds double inputs to FP32 first (the mixed form without
// a resident copy).  The LDS accumulator is FP64 in every form: on gfx950 an FP32 LDS atomic add
// measured 7x slower than an FP64 one (1e6 x 8 scatters into one 12000-entry column: 10.0 ms
// against 1.36 ms), so FP32 sums would make the sketch slower, not faster.
template <typename IDX, int NT, int PW, bool Z8, typename TA, bool R32>
__global__ __launch_bounds__(NT) void k_sketch_apply(const TA* __restrict__ A, int64_t lda, int64_t m, int n,
                                                     const double* __restrict__ B, int64_t ldb,
                                                     const IDX* __restrict__ idx, int d, int zeta, int chunk,
                                                     int ncols, double* __restrict__ Y, int64_t ldy,
                                                     double* __restrict__ colnorm2, int scale_by_norm,
                                                     int write_bnorm) {
  static_assert(!Z8 || sizeof(IDX) == 2, "the 16-byte index load packs eight 16-bit entries");
  constexpr int RU = PW >= 16 ? 1 : (PW >= 8 ? 2 : 4);  // rows in flight per thread (register budget)
  extern __shared__ __align__(16) unsigned char ysh_raw[];
  double* ysh = reinterpret_cast<double*>(ysh_raw);  // [PW][chunk]
  __shared__ double sred[NT / 64];
  const int npanels = (ncols + PW - 1) / PW;
  const int pnl = blockIdx.x % npanels;
  const int chk = blockIdx.x / npanels;
  const int c0 = pnl * PW;
  const int np = min(PW, ncols - c0);
  const int h0 = chk * chunk;
  const int hc = min(chunk, d - h0);
  const int tid = threadIdx.x;

  for (int i = tid; i < PW * chunk; i += NT) ysh[i] = 0.0;
  __syncthreads();

  const TA* colA[PW];
  const double* colB[PW];
  double ss[PW];
  int bad = 0;  // a NaN or Inf entry in one of the panel's columns (marked as a NaN norm below)
#pragma unroll
  for (int p = 0; p < PW; ++p) {
    const int col = c0 + p;
    colA[p] = (p < np && col < n) ? A + (int64_t)col * lda : nullptr;
    colB[p] = (p < np && col >= n) ? B + (int64_t)(col - n) * ldb : nullptr;
    ss[p] = 0.0;
  }
  auto scatter = [&](uint32_t ev, const double (&a)[PW]) {
    const int pos = (int)(ev >> 1) - h0;
    if (pos >= 0 && pos < hc) {
      const bool neg = (ev & 1u) != 0;
#pragma unroll
      for (int p = 0; p < PW; ++p)
        if (p < np) atomicAdd(&ysh[p * chunk + pos], neg ? -a[p] : a[p]);
    }
  };

  // RU rows per thread and step; with two register buffers the loads of the next step are issued
  // before the atomics of the current one, so that HBM reads and LDS atomics of a wave overlap.
  auto load_rows = [&](double (&a)[RU][PW], uint4 (&e8)[RU], int64_t i0) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      const bool ok = i < m;
#pragma unroll
      for (int p = 0; p < PW; ++p)
        a[u][p] = (ok && p < np) ? (colA[p] ? (R32 ? (double)(float)colA[p][i] : (double)colA[p][i]) : colB[p][i])
                                 : 0.0;
      if (Z8) e8[u] = ok ? *reinterpret_cast<const uint4*>(idx + i * 8) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto process_rows = [&](const double (&a)[RU][PW], const uint4 (&e8)[RU], int64_t i0) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = i0 + (int64_t)u * NT;
      if (i >= m) break;
#pragma unroll
      for (int p = 0; p < PW; ++p) {
        ss[p] = fma(a[u][p], a[u][p], ss[p]);
        bad |= (int)(!isfinite(a[u][p])) << p;
      }
      if (Z8) {
        const uint32_t w4[4] = {e8[u].x, e8[u].y, e8[u].z, e8[u].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          scatter(w4[q] & 0xFFFFu, a[u]);
          scatter(w4[q] >> 16, a[u]);
        }
      } else {
        const IDX* e = idx + i * zeta;
        for (int k = 0; k < zeta; ++k) scatter((uint32_t)e[k], a[u]);
      }
    }
  };
  const int64_t S = (int64_t)NT * RU;
  if constexpr (PW * sizeof(IDX) <= 8) {  // (wider panels have no registers for a second buffer)
    double a0[RU][PW], a1[RU][PW];
    uint4 e0[RU], e1[RU];
    load_rows(a0, e0, tid);
    for (int64_t i0 = tid; i0 < m; i0 += 2 * S) {
      load_rows(a1, e1, i0 + S);
      process_rows(a0, e0, i0);
      if (i0 + S >= m) break;
      load_rows(a0, e0, i0 + 2 * S);
      process_rows(a1, e1, i0 + S);
    }
  } else {
    for (int64_t i0 = tid; i0 < m; i0 += S) {
      double a[RU][PW];
      uint4 e8[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        const bool ok = i < m;
#pragma unroll
        for (int p = 0; p < PW; ++p)
          a[u][p] = (ok && p < np) ? (colA[p] ? (R32 ? (double)(float)colA[p][i] : (double)colA[p][i]) : colB[p][i])
                                   : 0.0;
        if (Z8) e8[u] = ok ? *reinterpret_cast<const uint4*>(idx + i * 8) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        if (i >= m) break;
#pragma unroll
        for (int p = 0; p < PW; ++p) {
          ss[p] = fma(a[u][p], a[u][p], ss[p]);
          bad |= (int)(!isfinite(a[u][p])) << p;
        }
        if (Z8) {
          const uint32_t w4[4] = {e8[u].x, e8[u].y, e8[u].z, e8[u].w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            scatter(w4[q] & 0xFFFFu, a[u]);
            scatter(w4[q] >> 16, a[u]);
          }
        } else {
          const IDX* e = idx + i * zeta;
          for (int k = 0; k < zeta; ++k) scatter((uint32_t)e[k], a[u]);
        }
      }
    }
  }
  __syncthreads();

  const double inv_sqrt_zeta = 1.0 / sqrt((double)zeta);
  for (int p = 0; p < PW; ++p) {
    if (p >= np) continue;  // np is uniform across the work-group
    const int col = c0 + p;
    const double nrm2 = block_sum<NT>(ss[p], sred);
    // non-finite data gives a NaN norm; finite data whose squares overflow gives +Inf
    const bool nonfinite = block_sum<NT>((double)((bad >> p) & 1), sred) > 0.0;
    double f = inv_sqrt_zeta;
    if (chk == 0 && tid == 0 && (col < n || write_bnorm)) colnorm2[col] = nonfinite ? NAN : nrm2;
    if (col < n) {
      if (scale_by_norm && nrm2 > 0.0) f = inv_sqrt_zeta / sqrt(nrm2);
    }
    for (int h = tid; h < hc; h += NT) Y[(int64_t)col * ldy + h0 + h] = ysh[p * chunk + h] * f;
  }
}

template <typename IDX, int PW, typename TA, bool R32>
void launch_apply_pw(const TA* A, int64_t lda, int64_t m, int n, const double* B, int64_t ldb, const void* idx, int d,
                     int zeta, int chunk, int ncols, double* Y, int64_t ldy, double* colnorm2, int sbn, int wbn,
                     int nchunks, hipStream_t s) {
  constexpr int NT = 1024;
  const int npanels = (ncols + PW - 1) / PW;
  const size_t shmem = (size_t)PW * chunk * sizeof(double);
  const dim3 grid((unsigned)(npanels * nchunks));
  if constexpr (sizeof(IDX) == 2) {
    if (zeta == 8) {
      (void)hipFuncSetAttribute((const void*)k_sketch_apply<IDX, NT, PW, true, TA, R32>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      hipLaunchKernelGGL((k_sketch_apply<IDX, NT, PW, true, TA, R32>), grid, dim3(NT), shmem, s, A, lda, m, n, B,
                         ldb, (const IDX*)idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn);
      return;
    }
  }
  (void)hipFuncSetAttribute((const void*)k_sketch_apply<IDX, NT, PW, false, TA, R32>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  hipLaunchKernelGGL((k_sketch_apply<IDX, NT, PW, false, TA, R32>), grid, dim3(NT), shmem, s, A, lda, m, n, B, ldb,
                     (const IDX*)idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn);
}

template <typename IDX, typename TA, bool R32>
void launch_apply(const TA* A, int64_t lda, int64_t m, int n, const double* B, int64_t ldb, const void* idx, int d,
                  int zeta, int pw, int chunk, int ncols, double* Y, int64_t ldy, double* colnorm2, int sbn, int wbn,
                  int nchunks, hipStream_t s) {
  switch (pw) {
    case 16: launch_apply_pw<IDX, 16, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn, nchunks, s); break;
    case 8: launch_apply_pw<IDX, 8, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn, nchunks, s); break;
    case 4: launch_apply_pw<IDX, 4, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn, nchunks, s); break;
    case 2: launch_apply_pw<IDX, 2, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn, nchunks, s); break;
    default: launch_apply_pw<IDX, 1, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, chunk, ncols, Y, ldy, colnorm2, sbn, wbn, nchunks, s); break;
  }
}

template <typename TA, bool R32>
hipError_t sketch_apply_t(const TA* A, int64_t lda, int64_t m, int n, const double* B, int64_t ldb, int nb,
                          const void* idx, bool idx16, int d, int zeta, double* Y, int64_t ldy, double* colnorm2,
                          bool scale_by_norm, bool write_bnorm, int lds_bytes, hipStream_t s) {
  const int ncols = n + (B ? nb : 0);
  const int lds_elems = lds_bytes / (int)sizeof(double);
  const int chunk = d < lds_elems ? d : lds_elems;
  int fit = lds_elems / d;  // columns of Y that fit in LDS at once
  int pw = 1;
  while (pw * 2 <= fit && pw * 2 <= 16 && pw < ncols) pw *= 2;
  const int nchunks = (d + chunk - 1) / chunk;
  if (idx16)
    launch_apply<uint16_t, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, pw, chunk, ncols, Y, ldy, colnorm2,
                                     scale_by_norm ? 1 : 0, write_bnorm ? 1 : 0, nchunks, s);
  else
    launch_apply<uint32_t, TA, R32>(A, lda, m, n, B, ldb, idx, d, zeta, pw, chunk, ncols, Y, ldy, colnorm2,
                                     scale_by_norm ? 1 : 0, write_bnorm ? 1 : 0, nchunks, s);
  return hipGetLastError();
}

__global__ void k_to_fp32(const double* __restrict__ A, int64_t lda, int64_t m, int n, float* __restrict__ A32,
                          int64_t lda32) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  for (int64_t r = q; r < m; r += (int64_t)gridDim.x * blockDim.x) A32[(int64_t)c * lda32 + r] = (float)A[(int64_t)c * lda + r];
}

}  // namespace

hipError_t fs_launch_sketch_indices(int64_t m, int d, int zeta, uint64_t seed, int64_t col0, int64_t ncols, void* idx,
                                    bool idx16, hipStream_t s) {
  (void)m;
  if (zeta < 1 || zeta > ZETA_MAX || zeta > d) return hipErrorInvalidValue;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int64_t nb = (ncols + 255) / 256;
  if (idx16)
    hipLaunchKernelGGL(k_sketch_indices<uint16_t>, dim3((unsigned)nb), dim3(256), 0, s, col0, ncols, d, zeta, k0, k1,
                       (uint16_t*)idx);
  else
    hipLaunchKernelGGL(k_sketch_indices<uint32_t>, dim3((unsigned)nb), dim3(256), 0, s, col0, ncols, d, zeta, k0, k1,
                       (uint32_t*)idx);
  return hipGetLastError();
}

hipError_t fs_launch_sketch_apply(const double* A, int64_t lda, int64_t m, int n, const double* B, int64_t ldb,
                                  int nb, const void* idx, bool idx16, int d, int zeta, double* Y, int64_t ldy,
                                  double* colnorm2, bool scale_by_norm, bool write_bnorm, int lds_bytes,
                                  hipStream_t s) {
  return sketch_apply_t<double, false>(A, lda, m, n, B, ldb, nb, idx, idx16, d, zeta, Y, ldy, colnorm2,
                                       scale_by_norm, write_bnorm, lds_bytes, s);
}

hipError_t fs_launch_sketch_apply_fp32(const double* A, int64_t lda, const float* A32, int64_t lda32, int64_t m,
                                       int n, const double* B, int64_t ldb, int nb, const void* idx, bool idx16,
                                       int d, int zeta, double* Y, int64_t ldy, double* colnorm2,
                                       bool scale_by_norm, bool write_bnorm, int lds_bytes, hipStream_t s) {
  if (A32)
    return sketch_apply_t<float, false>(A32, lda32, m, n, B, ldb, nb, idx, idx16, d, zeta, Y, ldy, colnorm2,
                                        scale_by_norm, write_bnorm, lds_bytes, s);
  return sketch_apply_t<double, true>(A, lda, m, n, B, ldb, nb, idx, idx16, d, zeta, Y, ldy, colnorm2,
                                      scale_by_norm, write_bnorm, lds_bytes, s);
}

hipError_t fs_launch_to_fp32(const double* A, int64_t lda, int64_t m, int n, float* A32, int64_t lda32, hipStream_t s) {
  if (n < 1 || m < 1) return hipSuccess;
  const int64_t bx = (m + 255) / 256;
  const unsigned gx = (unsigned)(bx < 1024 ? bx : 1024);
  hipLaunchKernelGGL(k_to_fp32, dim3(gx, (unsigned)n), dim3(256), 0, s, A, lda, m, n, A32, lda32);
  return hipGetLastError();
}
