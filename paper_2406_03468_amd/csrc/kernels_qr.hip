// Householder QR of the sketch Y = S [A b] (d x k, column-major, d >= k).
//
// The paper factors the sketch with Householder QR (eq:sketch_qr; Lemma 6.3 assumes Householder).
// This is a blocked right-looking Householder QR run as ONE cooperative kernel:
//   * work-group g owns a contiguous block of rows of Y for the whole factorization;
//   * a panel of NB columns is factored column by column with a single grid-wide reduction per
//     column: each work-group reduces x^T [panel columns] over its rows (x = the current column
//     below the diagonal) and the owner of the diagonal row publishes that row; from these
//     every work-group derives ||x||, the reflector H = I - tau v v^T with v = x + sign(x_0)||x|| e_1,
//     v^T y = x^T y + sign(x_0)||x|| y_0 for every other panel column, and the next column of the
//     compact-WY factor T (LAPACK's forward column-wise recurrence) -- redundantly, in the same
//     fixed order, so all copies agree bit for bit;
//   * the trailing columns are updated as Y <- Y - V T^T (V^T Y): V^T Y is summed over row blocks
//     (per-work-group partials, then a column-distributed fixed-order reduction), then each
//     work-group updates its own rows; both products run on the FP64 matrix cores
//     (v_mfma_f64_16x16x4f64).
// Y is only ever touched by the work-group owning the rows; the partials exchanged between
// work-groups go through coherent stores/loads, so the grid barriers need no cache flushes.
// R is left in the upper triangle of Y[0:k, 0:k] with a non-negative diagonal (rows of R whose
// reflector produced a negative diagonal are negated, which changes Q's columns, not Q R).
#include "common.hpp"
#include "internal.hpp"

namespace {

constexpr int NB = 32;        // panel width (divides 64)
constexpr int QR_NT = 512;    // threads per work-group (two waves per SIMD: one work-group per CU by LDS)
constexpr int RBMAX = 256;    // max rows owned by one work-group
constexpr int LOG2NB = 5;
constexpr int NRG = QR_NT / NB;   // row groups
constexpr int LOG2NRG = 4;
static_assert(NRG == 1 << LOG2NRG && NRG <= 64, "a row group's lanes lie in one wave");
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(QR_NT) void k_qr_coop(double* __restrict__ Y, int64_t ldy, int d, int k, int RB,
                                                   double* __restrict__ part,   // [2][G][NB] partial dots, then [2][NB] row j
                                                   double* __restrict__ wpart,  // [k][G][NB]
                                                   double* __restrict__ wred,   // [NB][k]
                                                   GridBarrier bar) {
  unsigned bgen = 0;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int rs = g * RB;
  const int re = (rs + RB < d) ? rs + RB : d;
  const int nr = (re > rs) ? re - rs : 0;

  __shared__ double pan[RBMAX][NB + 1];
  __shared__ double vm[RBMAX][NB + 1];  // the panel's V, zeros written out (rows past nr stay zero)
  __shared__ double T[NB][NB + 1];
  __shared__ double sred[QR_NT / 64][NB];
  __shared__ double sdots[NB], srow[NB], sw[NB], svtv[NB], srdiag[NB];
  __shared__ double sW[NRG][NB + 1];
  __shared__ double swt[NB];
  __shared__ signed char sneg[RBMAX];

  for (int r = tid; r < RBMAX; r += QR_NT) sneg[r] = 0;
  for (int i = tid; i < RBMAX * (NB + 1); i += QR_NT) (&vm[0][0])[i] = 0.0;
  // coherent views of the exchange buffers (bulk SC1 loads/stores)
  const auto rpart = co_rsrc(part, sizeof(double) * (size_t)2 * G * 2 * NB);
  const auto rwpart = co_rsrc(wpart, sizeof(double) * (size_t)G * NB * k);
  const auto rwred = co_rsrc(wred, sizeof(double) * (size_t)NB * k);

  const int c = tid % NB;
  const int rg = tid / NB;
  // MFMA lane roles (v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
  // holds D[4i + l/16][l%16], i = 0..3)
  const int wid = tid >> 6, lj = tid & 15, lk = (tid & 63) >> 4;

  for (int k0 = 0; k0 < k; k0 += NB) {
    const int nbp = (k - k0 < NB) ? k - k0 : NB;
    const int k1 = k0 + nbp;
    for (int q = tid; q < nr * nbp; q += QR_NT) {
      const int r = q % nr, cc = q / nr;
      pan[r][cc] = Y[(int64_t)(k0 + cc) * ldy + rs + r];
    }
    __syncthreads();

    for (int jj = 0; jj < nbp; ++jj) {
      const int j = k0 + jj;
      const int par = j & 1;
      const int rstart = (j > rs) ? j - rs : 0;
      // (1) partial x^T P over own rows i >= j, and the owner's copy of row j.
      double s = 0.0;
      if (c < nbp)
        for (int r = rstart + rg; r < nr; r += NRG) s = fma(pan[r][jj], pan[r][c], s);
      s = wave_sum_high<LOG2NB>(s);
      if ((tid & 63) < NB) sred[tid >> 6][c] = s;
      __syncthreads();
      // partial dots [par][G][NB]; row j (one owner) in its own slot [par][NB] after them
      const size_t prow = (size_t)2 * G * NB;
      if (tid < NB) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < QR_NT / 64; ++w) t += sred[w][tid];
        st_cob(rpart, 8 * (((size_t)par * G + g) * NB + tid), t);
        if (j >= rs && j < re) st_cob(rpart, 8 * (prow + (size_t)par * NB + tid), (tid < nbp) ? pan[j - rs][tid] : 0.0);
      }
      grid_barrier_co(bar, (unsigned)G, bgen);
      // (2) every work-group reduces all partial dots in the same order: entry e = tid % NB, eight
      //     groups of work-groups per entry (independent loads in flight), then a fixed-order sum;
      //     the owner's row j is read directly.
      {
        const int e = tid % NB, grp = tid / NB;
        // batches of 16 independent loads in flight (offsets past G read 0 through the range check)
        double t = 0.0;
        for (int g0 = grp; g0 < G; g0 += 16 * NRG) {
          double vals[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int gg = g0 + q * NRG;
            vals[q] = ld_cob(rpart, gg < G ? 8 * (((size_t)par * G + gg) * NB + e) : (size_t)0xFFFFFFF0u);
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) t += vals[q];
        }
        sW[grp][e] = t;
        const double rowv = (tid < NB) ? ld_cob(rpart, 8 * (prow + (size_t)par * NB + tid)) : 0.0;
        __syncthreads();
        if (tid < NB) {
          double t2 = 0.0;
#pragma unroll
          for (int q = 0; q < NRG; ++q) t2 += sW[q][tid];
          sdots[tid] = t2;
          srow[tid] = rowv;
        }
      }
      __syncthreads();
      // (3) reflector scalars.
      const double alpha = sqrt(sdots[jj]);
      const double x0 = srow[jj];
      const double sg = (x0 >= 0.0) ? 1.0 : -1.0;
      const double vhead = x0 + sg * alpha;
      const double tau = (alpha > 0.0) ? 1.0 / (alpha * (alpha + fabs(x0))) : 0.0;  // 2 / (v^T v)
      if (tid < nbp) {
        const double vty = sdots[tid] + sg * alpha * srow[tid];
        sw[tid] = (tid > jj) ? tau * vty : 0.0;
        svtv[tid] = (tid < jj) ? vty : 0.0;
      }
      if (tid == 0) srdiag[jj] = -sg * alpha;
      __syncthreads();
      {  // column jj of T: entry i < jj is -tau T[i][i:jj] svtv[i:jj], summed by the NRG lanes of row i
        const int i = tid / NRG, l = tid % NRG;
        double t = 0.0;
        if (i < jj)
          for (int c2 = i + l; c2 < jj; c2 += NRG) t = fma(T[i][c2], svtv[c2], t);
        t = wave_sum_low<LOG2NRG>(t);
        if (l == 0 && i <= jj) T[i][jj] = (i == jj) ? tau : -tau * t;
      }
      // (4) apply the reflector to the rest of the panel (own rows i >= j).
      if (c > jj && c < nbp) {
        const double wc = sw[c];
        for (int r = rstart + rg; r < nr; r += NRG) {
          const double v = (rs + r == j) ? vhead : pan[r][jj];
          pan[r][c] = fma(-v, wc, pan[r][c]);
        }
      }
      __syncthreads();
      if (tid == 0 && j >= rs && j < re) {
        pan[j - rs][jj] = vhead;
        sneg[j - rs] = (sg > 0.0) ? 1 : 0;  // R_jj = -sg * alpha < 0 when sg > 0
      }
      __syncthreads();
    }
    // write the panel rows back (V below the diagonal, v heads on the diagonal for now)
    for (int q = tid; q < nr * nbp; q += QR_NT) {
      const int r = q % nr, cc = q / nr;
      Y[(int64_t)(k0 + cc) * ldy + rs + r] = pan[r][cc];
    }

    if (k1 < k) {
      const int ntr = k - k1;
      const int r_lo = (k0 > rs) ? k0 - rs : 0;
      // V of the panel with its zeros written out (V[r][q] is nonzero only for q <= rs + r - k0 and
      // q < nbp), so the trailing-update loops below carry no per-element selects
      for (int i = tid; i < nr * NB; i += QR_NT) {
        const int r = i / NB, q = i % NB;
        vm[r][q] = (q <= rs + r - k0 && q < nbp) ? pan[r][q] : 0.0;
      }
      __syncthreads();
      // (T1) partial W_g = V_own^T Y_own[:, k1:k] on the matrix cores, as its transpose
      //      Y_own[:, k1:k]^T V_own: one 16 x 16 tile (16 trailing columns, 16 entries q) per wave at
      //      a time, rows in chunks of 64 where the k-slot l/16 of step s takes row 16 (l/16) + s
      //      (each lane reads 16 consecutive rows of its column); rows below r_lo or past nr carry
      //      zero V.  Partials are stored column by column, [cc][g][q], so that each column's G x NB
      //      partials are contiguous for the reduction.
      const int nct = (ntr + 15) / 16;
      const int c_lo = (r_lo / 64) * 64;
      for (int t = wid; t < 2 * nct; t += QR_NT / 64) {
        const int qt = (t & 1) * 16, ct = (t >> 1) * 16, cc = ct + lj;
        const bool cin = cc < ntr;
        const double* ycol = Y + (int64_t)(k1 + (cin ? cc : 0)) * ldy + rs;
        v4d acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};  // two chains (even, odd steps)
        for (int c0 = c_lo; c0 < nr; c0 += 64) {
          double bv[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int row = c0 + 16 * lk + u;
            bv[u] = (cin && row < nr) ? ycol[row] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 16; u += 2) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[u], vm[c0 + 16 * lk + u][qt + lj], acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[u + 1], vm[c0 + 16 * lk + u + 1][qt + lj], acc2, 0, 0, 0);
          }
        }
        acc += acc2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cs = ct + 4 * i + lk;
          if (cs < ntr) st_cob(rwpart, 8 * (((size_t)cs * G + g) * NB + qt + lj), acc[i]);
        }
      }
      grid_barrier_co(bar, (unsigned)G, bgen);
      // (T2) W = sum_g W_g (fixed order), W' = T^T W, for a slice of columns per work-group: thread
      //      (c, rg) sums every NRG-th work-group's partial of entry c, then the NRG sums are added.
      for (int cc = g; cc < ntr; cc += G) {
        double wsum = 0.0;
        if (c < nbp) {
          for (int g0 = rg; g0 < G; g0 += 8 * NRG) {
            double vals[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int gg = g0 + q * NRG;
              vals[q] = ld_cob(rwpart, gg < G ? 8 * (((size_t)cc * G + gg) * NB + c) : (size_t)0xFFFFFFF0u);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) wsum += vals[q];
          }
        }
        sW[rg][c] = wsum;
        __syncthreads();
        if (tid < NB) {
          double w = 0.0;
#pragma unroll
          for (int q = 0; q < NRG; ++q) w += sW[q][tid];
          swt[tid] = w;
        }
        __syncthreads();
        if (tid < nbp) {
          double wp = 0.0;
          for (int c2 = 0; c2 <= tid; ++c2) wp = fma(T[c2][tid], swt[c2], wp);
          st_cob(rwred, 8 * ((size_t)tid * k + cc), wp);
        }
        __syncthreads();
      }
      grid_barrier_co(bar, (unsigned)G, bgen);
      // (T3) own rows: Y[:, k1:k] -= V W' on the matrix cores, as (W'^T V^T)^T: per wave a tile of
      //      16 trailing columns (W' loaded once) against every 16-row tile from r_lo; each of the
      //      four results is 16 consecutive rows of one column across 16 lanes.
      for (int t = wid; t < nct; t += QR_NT / 64) {
        const int ct = t * 16;
        double av[NB / 4];
#pragma unroll
        for (int u = 0; u < NB / 4; ++u) {
          const int q = 4 * u + lk, cc = ct + lj;
          av[u] = (q < nbp && cc < ntr) ? ld_cob(rwred, 8 * ((size_t)q * k + cc)) : 0.0;
        }
        // two row tiles at a time: their Y loads are in flight during the products
        for (int rt = (r_lo / 16) * 16; rt < nr; rt += 32) {
          double yv[2][4];
          bool ok[2][4];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = rt + 16 * h + lj, cc = ct + 4 * i + lk;
              ok[h][i] = row >= r_lo && row < nr && cc < ntr;
              yv[h][i] = ok[h][i] ? Y[(int64_t)(k1 + cc) * ldy + rs + row] : 0.0;
            }
          const int r2 = (rt + 16 + lj < RBMAX) ? rt + 16 + lj : RBMAX - 1;  // past nr: unused
          v4d acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int u = 0; u < NB / 4; ++u) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], vm[rt + lj][4 * u + lk], acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], vm[r2][4 * u + lk], acc2, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int cc = ct + 4 * i + lk;
            if (ok[0][i]) Y[(int64_t)(k1 + cc) * ldy + rs + rt + lj] = yv[0][i] - acc[i];
            if (ok[1][i]) Y[(int64_t)(k1 + cc) * ldy + rs + rt + 16 + lj] = yv[1][i] - acc2[i];
          }
        }
      }
    }
    // diagonal of R for this panel's rows owned here (after every thread's write-back of the panel:
    // without a trailing update, nothing else orders the two stores to the diagonal)
    __syncthreads();
    for (int jj = tid; jj < nbp; jj += QR_NT) {
      const int j = k0 + jj;
      if (j >= rs && j < re) Y[(int64_t)j * ldy + j] = srdiag[jj];
    }
    __syncthreads();
  }
  // non-negative diagonal: negate rows of R with a negative diagonal (own rows j < k)
  for (int r = 0; r < nr; ++r) {
    const int j = rs + r;
    if (j >= k) break;
    if (sneg[r])
      for (int cc = j + tid; cc < k; cc += QR_NT) Y[(int64_t)cc * ldy + j] = -Y[(int64_t)cc * ldy + j];
  }
}

void qr_grid(int d, int num_cu, int* G, int* RB) {
  int g = (d + 63) / 64;
  if (g > num_cu) g = num_cu;
  if (g < 1) g = 1;
  int rb = (d + g - 1) / g;
  *G = g;
  *RB = rb;
}

}  // namespace

int* fs_qr_err_word(void* work, int d, int k, int num_cu) {
  int G, RB;
  qr_grid(d, num_cu, &G, &RB);
  double* part = (double*)work;
  double* wred = part + (size_t)2 * G * 2 * NB + (size_t)G * NB * k;
  unsigned* words = (unsigned*)(wred + (size_t)NB * k);
  return (int*)(words + FS_BAR_WORDS - 1);
}

int fs_qr_grid_size(int d, int num_cu) {
  int G, RB;
  qr_grid(d, num_cu, &G, &RB);
  return G;
}

size_t fs_qr_work_bytes(int d, int k, int num_cu) {
  int G, RB;
  qr_grid(d, num_cu, &G, &RB);
  return sizeof(double) * ((size_t)2 * G * 2 * NB + (size_t)G * NB * k + (size_t)NB * k) +
         sizeof(unsigned) * FS_BAR_WORDS + 512;
}

hipError_t fs_launch_qr(double* Y, int64_t ldy, int d, int k, void* work, int num_cu, hipStream_t s) {
  int G, RB;
  qr_grid(d, num_cu, &G, &RB);
  if (RB > RBMAX) return hipErrorInvalidValue;
  double* part = (double*)work;
  double* wpart = part + (size_t)2 * G * 2 * NB;
  double* wred = wpart + (size_t)G * NB * k;
  unsigned* words = (unsigned*)(wred + (size_t)NB * k);
  GridBarrier bar{words, nullptr, (int*)(words + FS_BAR_WORDS - 1)};
  hipLaunchKernelGGL(k_barrier_reset, dim3(1), dim3(256), 0, s, words, FS_BAR_WORDS);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&Y, &ldy, &d, &k, &RB, &part, &wpart, &wred, &bar};
  return fs_launch_resident((const void*)k_qr_coop, dim3(G), dim3(QR_NT), args, 0, s);
}
