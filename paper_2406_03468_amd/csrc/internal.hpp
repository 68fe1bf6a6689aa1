// Internal interfaces between the host orchestration and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// ---------------------------------------------------------------- fused passes over A
struct PassArgs {
  const double* A;       // m x n column-major
  int64_t lda;
  int64_t m;
  int n;
  const double* zs;      // n, pre-scaled vector (D^{-1} z)
  const double* b;       // m, residual mode when non-null
  double* partial;       // [G][n] work-group partials
  double* partial_r2;    // [G]
  const int* stop;       // device stop flag (may be null)
  double* rout = nullptr;  // m, residual mode only: receives r = b - A zs (may be null)
};
// One problem of a batched pass (fs_launch_pass_batched): its operands, the slice of the grid that
// works on it (G work-groups from wg0) and where its reduced result goes.
struct BatchPass {
  const double* A;
  int64_t lda;
  int64_t m;
  int n;
  const double* zs;      // n, pre-scaled vector
  const double* b;       // m (residual passes)
  double* partial;       // [G][n]
  double* partial_r2;    // [G]
  const int* stop;       // the problem's stop flag
  int wg0, G;
  double* out;           // n: out_scale .* (A^T w)
  const double* out_scale;
  double* r2_out;        // ||w||^2 (residual passes)
};

struct PassConfig {
  int H;  // tile rows (0 = unfused fallback)
  int G;  // work-groups
};
PassConfig fs_pass_config(int64_t m, int n, int num_cu);
// out = out_scale .* (A^T w), w = A zs (normal) or b - A zs (residual, r2_out = ||w||^2).
hipError_t fs_launch_pass(const PassArgs& a, const PassConfig& cfg, double* out, const double* out_scale,
                          double* r2_out, double* w_scratch, hipStream_t s);
// Passes of many problems in two launches per (H, L, vec) group: list (device) holds `count` problems
// that all use tile height H and L column slots per lane (L = ceil(n / (512 / (H / 2)))), their
// work-group slices consecutive from 0 to total_wgs; vec: every A 16-byte aligned with even lda (16-byte
// loads), else 8-byte loads.  resid: residual passes (b used, r2_out written).  max_n: the largest n of
// the list (grid of the reduction).
hipError_t fs_launch_pass_batched(const BatchPass* list, int count, int H, int L, bool vec, bool resid,
                                  int total_wgs, int max_n, hipStream_t s);
// Only the fused kernel (per-work-group partials, no final reduction); fused configurations only.
hipError_t fs_launch_pass_kernel_only(const PassArgs& a, const PassConfig& cfg, hipStream_t s);

// ---------------------------------------------------------------- sparse sign sketch
// Index stream: per source row j, zeta entries (position << 1 | sign_bit), 16- or 32-bit.
hipError_t fs_launch_sketch_indices(int64_t m, int d, int zeta, uint64_t seed, int64_t col0, int64_t ncols,
                                    void* idx, bool idx16, hipStream_t s);
// Y[:, j] = (1/sqrt(zeta)) * colscale_j * S M[:, j] for the n columns of A and the nb columns of B
// (ldb; none when B is null); colnorm2[j] = ||M[:, j]||^2 is produced in the same read (columns of
// B only if write_bnorm).  If scale_by_norm, column j < n of Y is divided by ||A[:, j]|| (zero
// columns: by 1).
hipError_t fs_launch_sketch_apply(const double* A, int64_t lda, int64_t m, int n, const double* B, int64_t ldb,
                                  int nb, const void* idx, bool idx16, int d, int zeta, double* Y, int64_t ldy,
                                  double* colnorm2, bool scale_by_norm, bool write_bnorm, int lds_bytes,
                                  hipStream_t s);
// The same with FP32 accumulation in LDS (mixed-precision form), reading A32 (FP32 copy, lda32) if
// non-null, else A converted on the fly.  Y and the column norms are FP64.
hipError_t fs_launch_sketch_apply_fp32(const double* A, int64_t lda, const float* A32, int64_t lda32, int64_t m,
                                       int n, const double* B, int64_t ldb, int nb, const void* idx, bool idx16,
                                       int d, int zeta, double* Y, int64_t ldy, double* colnorm2,
                                       bool scale_by_norm, bool write_bnorm, int lds_bytes, hipStream_t s);
// A32 = fl32(A) (column-major, lda32 >= m).
hipError_t fs_launch_to_fp32(const double* A, int64_t lda, int64_t m, int n, float* A32, int64_t lda32, hipStream_t s);
// Realification of a complex least-squares problem (complex128 interleaved, column-major):
// Ar = [Re A, -Im A; Im A, Re A] (2m x 2n, ld 2m), br = [Re b; Im b]; and x = xr[0:n] + i xr[n:2n].
hipError_t fs_launch_realify(int64_t m, int n, const double* A, int64_t lda, const double* b, double* Ar, double* br,
                             hipStream_t s);
hipError_t fs_launch_complexify_x(int n, const double* xr, double* x, hipStream_t s);

// ---------------------------------------------------------------- QR of the sketch
// In-place Householder QR of the d x k matrix Y (ldy), d >= k.  On exit the upper triangle of
// Y[0:k, 0:k] holds R with a non-negative diagonal; the reflectors are not kept.
// work: device scratch of fs_qr_work_bytes(d, k) bytes.
size_t fs_qr_work_bytes(int d, int k, int num_cu);
hipError_t fs_launch_qr(double* Y, int64_t ldy, int d, int k, void* work, int num_cu, hipStream_t s);

// ---------------------------------------------------------------- triangular solves with R (n x n, ldr)
// x = R^{-1} y (upper, back substitution) or x = R^{-T} y (forward substitution); in place on x.
hipError_t fs_launch_trsv(const double* R, int64_t ldr, int n, bool transpose, const double* y, double* x,
                          const double* yscale, const double* xscale, const int* stop, hipStream_t s);
// Triangular solves across work-groups (one per 64-row block, dependency flags); ws holds
// fs_trsv_flow_bytes(n) bytes, cleared once by fs_trsv_flow_reset before the first launch on it.
size_t fs_trsv_flow_bytes(int n);
hipError_t fs_trsv_flow_reset(int n, void* ws, hipStream_t s);
int* fs_trsv_flow_err_word(int n, void* ws);
hipError_t fs_launch_trsv_flow(const double* R, int64_t ldr, int n, bool transpose, const double* y, double* x,
                               const double* yscale, const double* xscale, const int* stop, void* ws, hipStream_t s);
// X = R^{-1} (n x n, ld n, zeros below the diagonal) by blocks of 64 (the recursive 2 x 2 block form);
// T: n x n doubles of scratch.
hipError_t fs_launch_tri_inv(const double* R, int64_t ldr, int n, double* X, double* T, hipStream_t s);
// nrhs independent solves (one work-group each): Xb[:, r] = R^{-1} Yb[:, r] (or R^{-T}).
hipError_t fs_launch_trsv_batched(const double* R, int64_t ldr, int n, bool transpose, const double* Yb, int64_t ldy,
                                  double* Xb, int64_t ldx, int nrhs, hipStream_t s);

// ---------------------------------------------------------------- SVD of R (one-sided Jacobi)
size_t fs_svd_work_bytes(int n);
// Also returns U_R (left singular vectors of R) when Uout is non-null.
hipError_t fs_launch_svd_full(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                              double* Uout, int64_t ldu, void* work, int num_cu, int max_sweeps,
                              int* sweeps_out_dev, hipStream_t s);
// The same; the block-Jacobi sweeps stop early once *abort_flag (device, may be null) is set by another
// stream (the results are then not used).
hipError_t fs_launch_svd_abortable(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                                   double* Uout, int64_t ldu, void* work, int num_cu, int max_sweeps,
                                   int* sweeps_out_dev, const int* abort_flag, hipStream_t s);
hipError_t fs_launch_svd(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                         void* work, int num_cu, int max_sweeps, int* sweeps_out_dev, hipStream_t s);

// ---------------------------------------------------------------- multi-RHS passes (k <= 64)
struct MultiPassArgs {
  const double* A;     // m x n column-major
  int64_t lda;
  int64_t m;
  int n;
  int k;               // right-hand sides (<= 64); kp = 16 * ceil(k / 16)
  const double* Zs;    // n x kp row-major, pre-scaled (D^{-1} Z), zero columns beyond k
  const double* B;     // m x k column-major (ldb): residual mode when non-null
  int64_t ldb;
  double* W;           // m x kp row-major scratch
  double* Vpart;       // [nchunk][n][kp] scratch
  double* r2part;      // [ceil(m/256)][kp] scratch
  int64_t rc;          // rows per gather chunk
  const double* scale; // n (may be null): V rows scaled by it
  double* V;           // n x kp row-major output
  double* r2;          // kp output (residual mode): ||b_j - A z_j||^2
  const int* stop;     // device stop flag (may be null)
};
int fs_multi_blocks(int k);
size_t fs_multi_work_doubles(int64_t m, int n, int k, int64_t* rc_out);
hipError_t fs_launch_multi_pass(const MultiPassArgs& a, hipStream_t s);

// Work-groups of the cooperative grids (for reservations when several streams share the GPU).
int fs_qr_grid_size(int d, int num_cu);
int fs_svd_grid_size(int n, int num_cu, bool with_u);
// Device address of the barrier-timeout flag of the last QR / SVD launch on this workspace
// (nonzero: a grid barrier gave up waiting; the results are not valid).
int* fs_qr_err_word(void* work, int d, int k, int num_cu);
int* fs_svd_err_word(void* work, int n);
