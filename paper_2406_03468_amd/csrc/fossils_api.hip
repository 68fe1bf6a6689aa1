// Host orchestration behind the C ABI declared in include/fossils.h.
//
// One solve (adaptive stopping) runs on the context's stream:
//   sketch index stream -> Y = S [A D^{-1} b] and ||a_j||^2 (one read of A)
//   -> Householder QR of Y (cooperative kernel) -> SVD of R (cooperative Jacobi)
//   -> x_0 = R^{-1} t -> for i in {0,1}: residual pass, c = P^T g (P = V Sigma^{-1} or R^{-1}), inner iterations
//      (z = P dy, v = A^T A z in one read of A, u = P^T v, heavy-ball or CG update),
//      x += P dy -> x = D^{-1} x.
// The inner loop's scalars and stop flag live in device memory (DevState); kernels of an inner
// iteration return at once when the flag is set, and the host reads the flag once per kw_every
// iterations.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fossils.h"
#include "common.hpp"
#include "context.hpp"
#include "internal.hpp"
#include "state.hpp"

hipError_t fs_launch_svd_full(const double* R, int64_t ldr, int n, double* sigma, double* V, int64_t ldv,
                              double* Uout, int64_t ldu, void* work, int num_cu, int max_sweeps, int* sweeps_out_dev,
                              hipStream_t s);

static thread_local std::string g_last_detail;

void fs_set_last_hip_error(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_detail = buf;
}

namespace {
constexpr double U_ROUND = FS_U_ROUND;
fs_status grow(DevBuf& b, size_t bytes) { return fs_grow(b, bytes); }
void free_buf(DevBuf& b) { fs_free_buf(b); }
bool idx16_ok(int d) { return fs_idx16_ok(d); }
fs_status validate_problem(int64_t m, int32_t n, const void* A, int64_t lda, const void* b, const void* x) {
  return fs_validate_problem(m, n, A, lda, b, x);
}
fs_status validate_options(int64_t m, int32_t n, const fs_options& o) { return fs_validate_options(m, n, o); }
}  // namespace

hipError_t fs_wait(fs_context_s* ctx, hipStream_t s) {
  if (!ctx->coop_budget) return hipStreamSynchronize(s);
  hipError_t e = hipSuccess;
  if (!ctx->ev_wait && (e = hipEventCreateWithFlags(&ctx->ev_wait, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventRecord(ctx->ev_wait, s)) != hipSuccess) return e;
  // short waits: polls that only yield the core; longer ones: 20 us sleeps between polls
  for (int polls = 0; (e = hipEventQuery(ctx->ev_wait)) == hipErrorNotReady; ++polls) {
    if (polls < 64) std::this_thread::yield();
    else std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  return e;
}

fs_status fs_grow(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return FS_OK;
  if (b.fixed) return FS_ERR_TOO_LARGE;  // a fixed slice is never reallocated
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    fs_set_last_hip_error(e, "hipMalloc", __FILE__, __LINE__);
    (void)hipGetLastError();
    return FS_ERR_NOMEM;
  }
  b.bytes = bytes;
  return FS_OK;
}

void fs_free_buf(DevBuf& b) {
  if (b.p && !b.fixed) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  b.fixed = false;
}

std::vector<DevBuf*> fs_workspace_buffers(Workspace& w) {
  return {&w.idx, &w.Y,       &w.colnorm2, &w.dinv,  &w.qrwork, &w.svdwork, &w.sigma, &w.V,    &w.UR,
          &w.partial, &w.pr2, &w.wscratch, &w.gemvpart, &w.vecs, &w.state, &w.mwork, &w.mvecs, &w.mstate,
          &w.lsqr, &w.hist, &w.cplx, &w.trsv, &w.batch};
}

size_t fs_workspace_bytes(Workspace& w) {
  size_t t = 0;
  for (DevBuf* b : fs_workspace_buffers(w)) t += b->bytes;
  return t;
}

void fs_workspace_free(Workspace& w) {
  for (DevBuf* b : fs_workspace_buffers(w)) fs_free_buf(*b);
}

fs_status fs_validate_problem(int64_t m, int32_t n, const void* A, int64_t lda, const void* b, const void* x) {
  if (!A || !b || !x) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < n || lda < m) return FS_ERR_SHAPE;
  return FS_OK;
}

fs_status fs_validate_options(int64_t m, int32_t n, const fs_options& o) {
  if (o.d < n || o.zeta < 1 || o.zeta > o.d || o.zeta > 64) return FS_ERR_SHAPE;
  if (o.kw_every < 1 || o.max_inner < 1 || o.steps < 1 || o.steps > 2) return FS_ERR_INVALID_ARG;
  if (!(o.gamma >= 0) || !(o.rho >= 0) || !(o.tau_factor > 0) || !(o.eta_factor > 0)) return FS_ERR_INVALID_ARG;
  if (o.precond != FS_PRECOND_QR && o.precond != FS_PRECOND_SVD) return FS_ERR_INVALID_ARG;
  if (o.precision != FS_FP64 && o.precision != FS_MIXED) return FS_ERR_INVALID_ARG;
  if (o.fixed_q < -1) return FS_ERR_INVALID_ARG;
  if (n > 15000) return FS_ERR_TOO_LARGE;       // TRSV keeps x in LDS
  if ((int64_t)o.d > 65536) return FS_ERR_TOO_LARGE;  // QR row blocks
  if (o.max_sweeps < 1) return FS_ERR_INVALID_ARG;
  if (o.graph_sweeps != 0 && o.graph_sweeps != 1) return FS_ERR_INVALID_ARG;
  if (o.overlap_pass_groups < 0) return FS_ERR_INVALID_ARG;
  if (o.init != FS_INIT_SKETCH && o.init != FS_INIT_ZERO) return FS_ERR_INVALID_ARG;
  if (o.overlap_svd != 0 && o.overlap_svd != 1) return FS_ERR_INVALID_ARG;
  (void)m;
  return FS_OK;
}

// History of the solve beside the SVD of R: the first step's iterates and ||Delta||^2 per iteration,
// then the second step's KW checkpoints recorded before Sigma and V exist (dy, g and V^T g per
// checkpoint, and four scalars each); then R^{-1} (n x n, the steps' P while the SVD runs) and the
// scratch its blocked formation uses (n x n).
static int fs_kw_slots(const fs_options& o) { return o.max_inner / o.kw_every + 2; }
size_t fs_hist_bytes(int n, const fs_options& o) {
  const size_t N = (size_t)n, C = (size_t)fs_kw_slots(o);
  return 8 * ((size_t)o.max_inner * N + (size_t)o.max_inner + 8 + 3 * C * N + 4 * C + 2 * N * N);
}

// Upper bound of the workspace one single-right-hand-side solve (FOSSILS, SPIR, LSQR; FP64 or mixed)
// grows to on a GPU with num_cu compute units: every buffer solve() sizes, at its largest.
size_t fs_solve_footprint_cu(int64_t m, int32_t n, const fs_options& o, int num_cu) {
  if (n < 1 || m < n || o.d < n || o.zeta < 1) return 0;
  const size_t d = (size_t)o.d, k = (size_t)n + 1, N = (size_t)n;
  size_t b = (size_t)m * o.zeta * (fs_idx16_ok(o.d) ? 2 : 4);  // index stream
  b += 8 * d * k;                                                // sketch Y
  b += fs_qr_work_bytes(o.d, (int)k, num_cu) + fs_svd_work_bytes(n);
  b += 8 * (2 * N * N + 4 * N + N * ((N + 63) / 64 + 1) + 22 * N);  // V, U_R, vectors
  const size_t gmax = std::max<size_t>(2 * (size_t)num_cu, 512);    // fused-pass partials (tuned: up to 2 per CU)
  b += 8 * (gmax * N + gmax + 64) + sizeof(DevState) + 64;
  b += 8 * (size_t)m;   // the unfused pass's row scratch (a leading dimension too large for 32-bit offsets)
  b += 16 * (size_t)m;  // the LSQR form's two m-vectors (counted for every method)
  if (o.overlap_svd) b += fs_hist_bytes(n, o);  // first-step history and deferred KW checkpoints
  b += fs_trsv_flow_bytes(n);
  return b;
}

size_t fs_carve_workspace(Workspace& w, unsigned char* base, int64_t m, int32_t n, const fs_options& o, int num_cu) {
  const size_t d = (size_t)o.d, k = (size_t)n + 1, N = (size_t)n;
  const size_t gmax = std::max<size_t>(2 * (size_t)num_cu, 512);
  size_t off = 0;
  auto slice = [&](DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (base) {
      b.p = base + off;
      b.bytes = bytes;
      b.fixed = true;
    }
    off += (bytes + 255) / 256 * 256;
  };
  // every buffer solve() sizes for FOSSILS in the serial order, at the size it asks for
  slice(w.idx, (size_t)m * o.zeta * (fs_idx16_ok(o.d) ? 2 : 4));
  slice(w.Y, 8 * d * k);
  slice(w.colnorm2, 8 * (N + 1));
  slice(w.dinv, 8 * N);
  slice(w.qrwork, fs_qr_work_bytes(o.d, (int)k, num_cu));
  slice(w.svdwork, fs_svd_work_bytes(n));
  slice(w.sigma, 8 * N);
  slice(w.V, 8 * N * N);
  slice(w.UR, 8 * N * N);
  slice(w.gemvpart, 8 * N * ((N + 63) / 64 + 1));
  slice(w.vecs, 8 * 22 * N);
  slice(w.state, sizeof(DevState) + 64);
  slice(w.partial, 8 * gmax * N);
  slice(w.pr2, 8 * gmax + 64);
  slice(w.wscratch, 8 * (size_t)m);
  slice(w.trsv, fs_trsv_flow_bytes(n));
  return off;
}

extern "C" {

const char* fs_status_string(fs_status s) {
  switch (s) {
    case FS_OK: return "FS_OK";
    case FS_WARN_RANK_DEFICIENT: return "FS_WARN_RANK_DEFICIENT";
    case FS_WARN_NOT_CONVERGED: return "FS_WARN_NOT_CONVERGED";
    case FS_ERR_INVALID_ARG: return "FS_ERR_INVALID_ARG";
    case FS_ERR_SHAPE: return "FS_ERR_SHAPE";
    case FS_ERR_NOMEM: return "FS_ERR_NOMEM";
    case FS_ERR_DEVICE: return "FS_ERR_DEVICE";
    case FS_ERR_NONFINITE: return "FS_ERR_NONFINITE";
    case FS_ERR_TOO_LARGE: return "FS_ERR_TOO_LARGE";
    case FS_ERR_UNKNOWN_TICKET: return "FS_ERR_UNKNOWN_TICKET";
    case FS_ERR_UNSUPPORTED: return "FS_ERR_UNSUPPORTED";
    default: break;
  }
  return "FS_UNKNOWN_STATUS";
}

const char* fs_last_error_detail(void) { return g_last_detail.c_str(); }

fs_status fs_options_default(int64_t m, int32_t n, fs_options* o) {
  if (!o) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < n) return FS_ERR_SHAPE;
  memset(o, 0, sizeof(*o));
  int64_t d = 12 * (int64_t)n;
  o->d = (int32_t)d;
  o->zeta = 8;
  if (o->zeta > o->d) o->zeta = o->d;
  o->seed = 12345;
  o->eta = 0.0;
  o->eta_factor = 1.0;
  o->gamma = 10.0;
  o->rho = 0.4;
  o->kw_every = 5;
  o->max_inner = 100;
  o->tau_factor = 30.0;
  o->column_scaling = 1;
  o->precond = FS_PRECOND_SVD;  // Alg 4: P = V Sigma^{-1} (two GEMVs per iteration instead of two TRSVs)
  o->fixed_q = 0;
  o->steps = 2;
  o->precision = FS_FP64;
  o->max_sweeps = 40;
  o->init = FS_INIT_SKETCH;
  o->overlap_svd = 1;
  o->graph_sweeps = 0;  // measured no faster than kernel-by-kernel launches (the host enqueues ahead)
  o->overlap_pass_groups = 0;
  return FS_OK;
}

fs_status fs_context_create(int device, void* hip_stream, fs_context* out) {
  if (!out) return FS_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  FS_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return FS_ERR_INVALID_ARG;
  FS_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FS_HIP(hipGetDeviceProperties(&prop, device));
  fs_context c = new fs_context_s();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->num_cu = prop.multiProcessorCount;
  c->lds_bytes = (int)std::min<size_t>(prop.sharedMemPerBlock, (size_t)160 * 1024);
  if (c->lds_bytes > 128 * 1024) c->lds_bytes = 128 * 1024 + 16 * 1024;  // leave room for static LDS
  hipError_t e = hipHostMalloc((void**)&c->st_host, sizeof(DevState), hipHostMallocDefault);
  if (e != hipSuccess) {
    fs_set_last_hip_error(e, "hipHostMalloc", __FILE__, __LINE__);
    delete c;
    return FS_ERR_NOMEM;
  }
  for (auto& ev : c->ev) (void)hipEventCreate(&ev);
  *out = c;
  return FS_OK;
}

fs_status fs_context_destroy(fs_context c) {
  if (!c) return FS_ERR_INVALID_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  fs_workspace_free(c->ws);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) {
    (void)hipStreamSynchronize(c->aux_stream);
    (void)hipStreamDestroy(c->aux_stream);
  }
  if (c->ev_aux) (void)hipEventDestroy(c->ev_aux);
  if (c->ev_wait) (void)hipEventDestroy(c->ev_wait);
  fs_batch_helpers_destroy(c);
  for (auto& ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->st_host) (void)hipHostFree(c->st_host);
  delete c;
  return FS_OK;
}

// ---------------------------------------------------------------- sketch handle
fs_status sketch_create(fs_context ctx, int64_t m, int32_t d, int32_t zeta, uint64_t seed, fs_sketch* out) {
  if (!ctx || !out) return FS_ERR_INVALID_ARG;
  *out = nullptr;
  if (m < 1 || d < 1 || zeta < 1 || zeta > d || zeta > 64) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  fs_sketch sk = new fs_sketch_s();
  sk->ctx = ctx;
  sk->m = m;
  sk->d = d;
  sk->zeta = zeta;
  sk->seed = seed;
  sk->idx16 = idx16_ok(d);
  const size_t bytes = (size_t)m * zeta * (sk->idx16 ? 2 : 4);
  hipError_t e = hipMalloc(&sk->idx, bytes);
  if (e != hipSuccess) {
    fs_set_last_hip_error(e, "hipMalloc", __FILE__, __LINE__);
    delete sk;
    return FS_ERR_NOMEM;
  }
  e = fs_launch_sketch_indices(m, d, zeta, seed, 0, m, sk->idx, sk->idx16, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    fs_set_last_hip_error(e, "sketch index generation", __FILE__, __LINE__);
    (void)hipFree(sk->idx);
    delete sk;
    return FS_ERR_DEVICE;
  }
  *out = sk;
  return FS_OK;
}

fs_status sketch_destroy(fs_sketch sk) {
  if (!sk) return FS_ERR_INVALID_ARG;
  (void)hipSetDevice(sk->ctx->device);
  (void)hipStreamSynchronize(sk->ctx->stream);
  if (sk->idx) (void)hipFree(sk->idx);
  delete sk;
  return FS_OK;
}

fs_status sketch_indices(fs_sketch sk, int64_t col0, int64_t ncols, int32_t* rows_host, int8_t* signs_host) {
  if (!sk || !rows_host || !signs_host) return FS_ERR_INVALID_ARG;
  if (col0 < 0 || ncols < 0 || col0 + ncols > sk->m) return FS_ERR_SHAPE;
  if (ncols == 0) return FS_OK;
  FS_HIP(hipSetDevice(sk->ctx->device));
  const size_t esz = sk->idx16 ? 2 : 4;
  std::vector<uint8_t> buf((size_t)ncols * sk->zeta * esz);
  FS_HIP(hipMemcpyAsync(buf.data(), (const uint8_t*)sk->idx + (size_t)col0 * sk->zeta * esz, buf.size(),
                        hipMemcpyDeviceToHost, sk->ctx->stream));
  FS_HIP(hipStreamSynchronize(sk->ctx->stream));
  const size_t cnt = (size_t)ncols * sk->zeta;
  for (size_t i = 0; i < cnt; ++i) {
    uint32_t e = sk->idx16 ? ((const uint16_t*)buf.data())[i] : ((const uint32_t*)buf.data())[i];
    rows_host[i] = (int32_t)(e >> 1);
    signs_host[i] = (e & 1u) ? -1 : 1;
  }
  return FS_OK;
}

fs_status sketch_apply(fs_sketch sk, int32_t n, const double* A, int64_t lda, const double* b, double* Y,
                       int64_t ldy, double* colnorm2, int32_t scale_columns) {
  if (!sk || !A || !Y) return FS_ERR_INVALID_ARG;
  if (n < 1 || lda < sk->m || ldy < sk->d) return FS_ERR_SHAPE;
  fs_context ctx = sk->ctx;
  FS_HIP(hipSetDevice(ctx->device));
  double* cn = colnorm2;
  if (!cn) {
    FS_TRY(grow(ctx->ws.colnorm2, sizeof(double) * (n + 1)));
    cn = (double*)ctx->ws.colnorm2.p;
  }
  FS_K(fs_launch_sketch_apply(A, lda, sk->m, n, b, sk->m, 1, sk->idx, sk->idx16, sk->d, sk->zeta, Y, ldy, cn,
                              scale_columns != 0, false, ctx->lds_bytes, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return FS_OK;
}

// ---------------------------------------------------------------- step-level calls
fs_status fs_sketch_qr(fs_context ctx, int32_t d, int32_t k, double* Y, int64_t ldy) {
  if (!ctx || !Y) return FS_ERR_INVALID_ARG;
  if (k < 1 || d < k || ldy < d) return FS_ERR_SHAPE;
  if (d > 65536) return FS_ERR_TOO_LARGE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_TRY(grow(ctx->ws.qrwork, fs_qr_work_bytes(d, k, ctx->num_cu)));
  FS_K(fs_launch_qr(Y, ldy, d, k, ctx->ws.qrwork.p, ctx->num_cu, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return FS_OK;
}

fs_status fs_svd_triangular(fs_context ctx, int32_t n, const double* R, int64_t ldr, double* sigma, double* V,
                            int64_t ldv, int32_t* sweeps_host) {
  if (!ctx || !R || !sigma || !V) return FS_ERR_INVALID_ARG;
  if (n < 1 || ldr < n || ldv < n) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_TRY(grow(ctx->ws.svdwork, fs_svd_work_bytes(n)));
  FS_TRY(grow(ctx->ws.state, sizeof(DevState) + 64));
  int* sw = (int*)((char*)ctx->ws.state.p + sizeof(DevState));
  FS_K(fs_launch_svd(R, ldr, n, sigma, V, ldv, ctx->ws.svdwork.p, ctx->num_cu, 40, sw, ctx->stream));
  int swh = 0;
  FS_HIP(hipMemcpyAsync(&swh, sw, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  if (sweeps_host) *sweeps_host = swh;
  return FS_OK;
}

// Tile heights the fused pass is built for at this n: L = ceil(n H / 1024) column slots per lane
// must lie in the instantiated range of that height.
static bool pass_tile_ok(int H, int n) {
  const int64_t L = ((int64_t)n * H + 1023) / 1024;
  switch (H) {
    case 64: return L >= 1 && L <= 4;
    case 32: return L >= 1 && L <= 32;  // (residual passes above 8 slots run with 16 rows)
    case 16: return L >= 1 && L <= 16;
    case 8:
    case 4: return L >= 5 && L <= 16;
    default: return false;
  }
}
static int m_bucket(int64_t m) {
  int b = 0;
  while ((int64_t(2) << b) <= m) ++b;
  return b;  // floor(log2 m)
}
static bool pass_groups_ok(int G, int num_cu) { return G >= 8 && G % 8 == 0 && G <= 2 * num_cu; }

static PassConfig pass_config(fs_context ctx, int64_t m, int32_t n, int64_t lda) {
  PassConfig cfg = fs_pass_config(m, n, ctx->num_cu);
  if (ctx->pass_force) {
    cfg = PassConfig{ctx->pass_force_H, ctx->pass_force_G};
  } else if (!ctx->pass_tuned.empty()) {
    const auto it = ctx->pass_tuned.find({n, m_bucket(m)});
    if (it != ctx->pass_tuned.end()) cfg = PassConfig{it->second.first, it->second.second};
  }
  // a cap on the fused pass's work-groups (multiples of 8 keep its XCD banding)
  if (cfg.H && ctx->pass_group_cap > 0 && cfg.G > ctx->pass_group_cap)
    cfg.G = std::max(8, ctx->pass_group_cap / 8 * 8);
  // 32-bit lane offsets inside a column slot (see the fused-pass kernel), for the tile height of the
  // residual pass too (16 rows where the normal pass takes 32 above 256 columns)
  if (cfg.H) {
    const int hres = (cfg.H == 32 && n > 256) ? 16 : cfg.H;
    const int64_t cpr = 512 / (hres / 2);
    if ((cpr * lda + cfg.H) * 8 >= (int64_t(1) << 32)) cfg = PassConfig{0, 512};
  }
  return cfg;
}

static fs_status ensure_pass_ws(fs_context ctx, int64_t m, int32_t n, int64_t lda) {
  const PassConfig cfg = pass_config(ctx, m, n, lda);
  FS_TRY(grow(ctx->ws.partial, sizeof(double) * (size_t)cfg.G * n));
  FS_TRY(grow(ctx->ws.pr2, sizeof(double) * (size_t)cfg.G + 64));
  if (!cfg.H) FS_TRY(grow(ctx->ws.wscratch, sizeof(double) * (size_t)m));
  return FS_OK;
}

// Enqueue one fused pass; the workspace must already be sized (ensure_pass_ws), so no buffer
// is reallocated while earlier work on the stream may still use it.
static fs_status run_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* zs,
                          const double* b, double* out, const double* out_scale, double* r2_dev, const int* stop,
                          double* rout = nullptr) {
  const PassConfig cfg = pass_config(ctx, m, n, lda);
  if (ctx->ws.partial.bytes < sizeof(double) * (size_t)cfg.G * n) return FS_ERR_INVALID_ARG;
  PassArgs a{A, lda, m, n, zs, b, (double*)ctx->ws.partial.p, (double*)ctx->ws.pr2.p, stop, rout};
  FS_K(fs_launch_pass(a, cfg, out, out_scale, r2_dev, (double*)ctx->ws.wscratch.p, ctx->stream));
  return FS_OK;
}

fs_status fs_normal_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z,
                         double* v) {
  if (!ctx || !A || !z || !v) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < 1 || lda < m) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  FS_TRY(ensure_pass_ws(ctx, m, n, lda));
  FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return FS_OK;
}

fs_status fs_residual_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                           const double* x, double* g, double* rnorm2_host) {
  if (!ctx || !A || !b || !x || !g) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < 1 || lda < m) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  FS_TRY(grow(ctx->ws.state, sizeof(DevState) + 64));
  FS_TRY(ensure_pass_ws(ctx, m, n, lda));
  double* r2 = (double*)((char*)ctx->ws.state.p + sizeof(DevState) + 8);
  FS_TRY(run_pass(ctx, m, n, A, lda, x, b, g, nullptr, r2, nullptr));
  double r2h = 0;
  FS_HIP(hipMemcpyAsync(&r2h, r2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  if (rnorm2_host) *rnorm2_host = r2h;
  return FS_OK;
}

fs_status fs_time_normal_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z,
                              double* v, int32_t repeats, double* ms_per_pass_host, double* ms_kernel_host) {
  if (!ctx || !A || !z || !v || !ms_per_pass_host) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < 1 || lda < m || repeats < 1) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  FS_TRY(ensure_pass_ws(ctx, m, n, lda));
  FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));  // warm-up
  hipEvent_t* ev = ctx->ev;
  FS_HIP(hipEventRecord(ev[0], ctx->stream));
  for (int r = 0; r < repeats; ++r) FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));
  FS_HIP(hipEventRecord(ev[1], ctx->stream));
  // the fused kernel alone: same launches without the partial-sum reduction
  const PassConfig cfg = pass_config(ctx, m, n, lda);
  PassArgs a{A, lda, m, n, z, nullptr, (double*)ctx->ws.partial.p, (double*)ctx->ws.pr2.p, nullptr};
  FS_HIP(hipEventRecord(ev[2], ctx->stream));
  for (int r = 0; r < repeats; ++r) FS_K(fs_launch_pass_kernel_only(a, cfg, ctx->stream));
  FS_HIP(hipEventRecord(ev[3], ctx->stream));
  FS_HIP(hipEventSynchronize(ev[3]));
  float t01 = 0, t23 = 0;
  FS_HIP(hipEventElapsedTime(&t01, ev[0], ev[1]));
  FS_HIP(hipEventElapsedTime(&t23, ev[2], ev[3]));
  *ms_per_pass_host = (double)t01 / repeats;
  if (ms_kernel_host) *ms_kernel_host = (double)t23 / repeats;
  return FS_OK;
}

fs_status fs_tune_pass(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* z, double* v,
                       int32_t repeats, int32_t* H_out, int32_t* G_out, double* ms_out) {
  if (!ctx || !A || !z || !v) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < 1 || lda < m || repeats < 1) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  struct ForceReset {  // the override ends on every exit path
    fs_context c;
    ~ForceReset() { c->pass_force = false; }
  } force_reset{ctx};
  const int nc = ctx->num_cu;
  const int gs[4] = {std::max(8, nc / 2 / 8 * 8), std::max(8, nc * 3 / 4 / 8 * 8), std::max(8, nc / 8 * 8),
                     std::max(8, 2 * nc / 8 * 8)};
  double best = INFINITY;
  int bH = 0, bG = 0;
  hipEvent_t* ev = ctx->ev;
  for (int H : {64, 32, 16, 8, 4}) {
    if (!pass_tile_ok(H, n)) continue;
    for (int G : gs) {
      if (!pass_groups_ok(G, nc)) continue;
      ctx->pass_force = true;
      ctx->pass_force_H = H;
      ctx->pass_force_G = G;
      if (pass_config(ctx, m, n, lda).H != H) continue;  // (lda too large for the fused pass)
      FS_TRY(ensure_pass_ws(ctx, m, n, lda));
      FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));  // warm-up
      FS_HIP(hipEventRecord(ev[0], ctx->stream));
      for (int r = 0; r < repeats; ++r) FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));
      FS_HIP(hipEventRecord(ev[1], ctx->stream));
      FS_HIP(hipEventSynchronize(ev[1]));
      float t = 0;
      FS_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
      const double ms = (double)t / repeats;
      if (ms < best) {
        best = ms;
        bH = H;
        bG = G;
      }
    }
  }
  ctx->pass_force = false;
  if (bH == 0) return FS_ERR_SHAPE;  // no fused configuration at this shape
  ctx->pass_tuned[{n, m_bucket(m)}] = {bH, bG};
  FS_TRY(ensure_pass_ws(ctx, m, n, lda));
  FS_TRY(run_pass(ctx, m, n, A, lda, z, nullptr, v, nullptr, nullptr, nullptr));  // v from the kept one
  FS_HIP(hipStreamSynchronize(ctx->stream));
  if (H_out) *H_out = bH;
  if (G_out) *G_out = bG;
  if (ms_out) *ms_out = best;
  return FS_OK;
}

fs_status fs_set_pass_tuning(fs_context ctx, int64_t m, int32_t n, int32_t H, int32_t G) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  if (n < 1 || m < 1) return FS_ERR_SHAPE;
  if (!pass_tile_ok(H, n) || !pass_groups_ok(G, ctx->num_cu)) return FS_ERR_INVALID_ARG;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));  // (the workspace is sized per call; nothing in flight)
  ctx->pass_tuned[{n, m_bucket(m)}] = {H, G};
  return FS_OK;
}

fs_status fs_clear_pass_tuning(fs_context ctx) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  ctx->pass_tuned.clear();
  return FS_OK;
}

size_t fs_solve_footprint(int64_t m, int32_t n, const fs_options* opts) {
  fs_options o;
  if (opts) o = *opts;
  else if (fs_options_default(m, n, &o) != FS_OK) return 0;
  return fs_solve_footprint_cu(m, n, o, 256);
}

fs_status fs_context_workspace(fs_context ctx, size_t* bytes) {
  if (!ctx || !bytes) return FS_ERR_INVALID_ARG;
  *bytes = fs_workspace_bytes(ctx->ws);
  return FS_OK;
}

fs_status fs_context_trim(fs_context ctx) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->aux_stream) FS_HIP(hipStreamSynchronize(ctx->aux_stream));
  fs_workspace_free(ctx->ws);
  return FS_OK;
}

fs_status fs_trsv(fs_context ctx, int32_t n, const double* R, int64_t ldr, int32_t transpose, const double* y,
                  double* x) {
  if (!ctx || !R || !y || !x) return FS_ERR_INVALID_ARG;
  if (n < 1 || ldr < n) return FS_ERR_SHAPE;
  if (n > 15000) return FS_ERR_TOO_LARGE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  FS_TRY(grow(ctx->ws.trsv, fs_trsv_flow_bytes(n)));
  FS_K(fs_trsv_flow_reset(n, ctx->ws.trsv.p, ctx->stream));
  FS_K(fs_launch_trsv_flow(R, ldr, n, transpose != 0, y, x, nullptr, nullptr, nullptr, ctx->ws.trsv.p, ctx->stream));
  int err = 0;
  FS_HIP(hipMemcpyAsync(&err, fs_trsv_flow_err_word(n, ctx->ws.trsv.p), sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  if (err) {
    fs_set_last_hip_error(hipErrorLaunchTimeOut, "triangular solve gave up waiting for a block", __FILE__, __LINE__);
    return FS_ERR_DEVICE;
  }
  return FS_OK;
}

fs_status fs_triangular_inverse(fs_context ctx, int32_t n, const double* R, int64_t ldr, double* X) {
  if (!ctx || !R || !X) return FS_ERR_INVALID_ARG;
  if (n < 1 || ldr < n) return FS_ERR_SHAPE;
  if (n > 15000) return FS_ERR_TOO_LARGE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  FS_TRY(grow(ctx->ws.UR, sizeof(double) * (size_t)n * n));  // scratch of the block products
  FS_K(fs_launch_tri_inv(R, ldr, n, X, (double*)ctx->ws.UR.p, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return FS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- the solver
namespace {

enum Method { M_FOSSILS = 0, M_SPIR = 1, M_SPIR_LSQR = 2 };

struct Vecs {
  double *x, *x0, *c, *dy, *dy_old, *zs, *v, *u, *g, *xh, *w, *res, *p, *t, *tmp, *z;
};

// Captures `len` calls of iteration(j) (j = 0 .. len-1) on stream s into a graph and replays it up to
// `reps` times, polling after each replay (poll sets `stopped`).  Capture is thread-local, so other
// threads' HIP calls (the server's other slots) are unaffected; a failure inside the capture ends it
// before returning.  The captured work is kernels only (no memset nodes).
// The capture runs on the context's private capture stream (the caller's stream may be the null
// stream, which cannot be captured): while capturing, `s` (the solve's launch stream, captured by
// reference in the iteration) and ctx->stream point at it; the graph is then launched on the
// caller's stream.
template <typename Iter, typename Poll>
static fs_status sweep_graph_run(fs_context ctx, hipStream_t& s, int len, int reps, Iter&& iteration, Poll&& poll,
                                 bool& stopped) {
  if (!ctx->cap_stream) FS_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  const hipStream_t launch = s;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  FS_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  s = ctx->cap_stream;
  ctx->stream = ctx->cap_stream;
  fs_status st = FS_OK;
  for (int j = 0; j < len && st == FS_OK; ++j) st = iteration(j);
  s = launch;
  ctx->stream = launch;
  const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
  if (st != FS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  FS_HIP(ec);
  const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  FS_HIP(ei);
  for (int r = 0; r < reps && !stopped && st == FS_OK; ++r) {
    const hipError_t el = hipGraphLaunch(ge, launch);
    if (el != hipSuccess) {
      fs_set_last_hip_error(el, "hipGraphLaunch", __FILE__, __LINE__);
      st = FS_ERR_DEVICE;
      break;
    }
    st = poll();
  }
  (void)hipGraphExecDestroy(ge);
  return st;
}

fs_status solve(fs_context ctx, Method method, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                double* x_out, const fs_options* opts_in, fs_info* info, const float* A32 = nullptr,
                int64_t lda32 = 0) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  FS_TRY(validate_problem(m, n, A, lda, b, x_out));
  fs_options o;
  if (opts_in) o = *opts_in;
  else FS_TRY(fs_options_default(m, n, &o));
  FS_TRY(validate_options(m, n, o));
  FS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  FS_HIP(fs_wait(ctx, s));  // workspace may be reallocated below
  if (ctx->aux_stream) FS_HIP(fs_wait(ctx, ctx->aux_stream));
  Workspace& W = ctx->ws;
  const int d = o.d, zeta = o.zeta, k = n + 1;
  // The SVD of R beside the first refinement step (see fs_options.overlap_svd).
  // (only while the SVD leaves at least half of the compute units to the passes: an SVD grid that
  // holds nearly all of them would leave the step's passes a few units, slower than the serial order)
  // (the mixed form too: a kept FP32 sketch whose SVD then reports u32 condest too large restarts
  // the solve from an FP64 sketch, see the join below)
  const bool defer_fp64 = o.overlap_svd && o.precond == FS_PRECOND_SVD && o.fixed_q == 0 &&
                          (method == M_FOSSILS || method == M_SPIR) &&
                          2 * fs_svd_grid_size(n, ctx->num_cu, false) <= ctx->num_cu;
  bool defer = defer_fp64;
  const bool i16 = idx16_ok(d);

  // ---- workspace
  FS_TRY(grow(W.idx, (size_t)m * zeta * (i16 ? 2 : 4)));
  FS_TRY(grow(W.Y, sizeof(double) * (size_t)d * k));
  FS_TRY(grow(W.colnorm2, sizeof(double) * (size_t)(n + 1)));
  FS_TRY(grow(W.dinv, sizeof(double) * (size_t)n));
  FS_TRY(grow(W.qrwork, fs_qr_work_bytes(d, k, ctx->num_cu)));
  FS_TRY(grow(W.svdwork, fs_svd_work_bytes(n)));
  FS_TRY(grow(W.sigma, sizeof(double) * (size_t)n));
  FS_TRY(grow(W.V, sizeof(double) * (size_t)n * n));
  FS_TRY(grow(W.UR, sizeof(double) * (size_t)n * n));
  FS_TRY(grow(W.gemvpart, sizeof(double) * (size_t)n * ((n + 63) / 64 + 1)));
  const int NV = 22;  // 16 vectors of the iteration, 6 of the spectral bounds
  FS_TRY(grow(W.vecs, sizeof(double) * (size_t)NV * n));
  FS_TRY(grow(W.state, sizeof(DevState) + 64));
  FS_TRY(grow(W.trsv, fs_trsv_flow_bytes(n)));
  FS_TRY(ensure_pass_ws(ctx, m, n, lda));
  if (defer_fp64) {  // (also for a mixed solve, which may fall back to an FP64 sketch and overlap)
    FS_TRY(grow(W.hist, fs_hist_bytes(n, o)));
    if (!ctx->aux_stream) FS_HIP(hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking));
    if (!ctx->ev_aux) FS_HIP(hipEventCreateWithFlags(&ctx->ev_aux, hipEventDisableTiming));
  }
  double* hist_dy = defer_fp64 ? (double*)W.hist.p : nullptr;
  double* hist_dn = defer_fp64 ? hist_dy + (size_t)o.max_inner * n : nullptr;
  const int kw_slots = fs_kw_slots(o);
  double* kw_dy = defer_fp64 ? hist_dn + o.max_inner + 8 : nullptr;  // deferred KW checkpoints
  double* kw_g = defer_fp64 ? kw_dy + (size_t)kw_slots * n : nullptr;
  double* kw_w = defer_fp64 ? kw_g + (size_t)kw_slots * n : nullptr;
  double* kw_s = defer_fp64 ? kw_w + (size_t)kw_slots * n : nullptr;
  double* rinv = defer_fp64 ? kw_s + 4 * (size_t)kw_slots : nullptr;  // R^{-1} (ld n)
  double* rinv_scratch = defer_fp64 ? rinv + (size_t)n * n : nullptr;
  bool rinv_ok = false;  // rinv holds R^{-1} of the current R
  const bool lsqr = (method == M_SPIR_LSQR);
  if (lsqr) FS_TRY(grow(W.lsqr, sizeof(double) * 2 * (size_t)m));
  double* rbuf = lsqr ? (double*)W.lsqr.p : nullptr;  // r of the last LSQR pass (m)
  double* ubar = lsqr ? rbuf + m : nullptr;          // alpha u (m)
  double* vb = (double*)W.vecs.p;
  Vecs v{vb, vb + n, vb + 2 * n, vb + 3 * n, vb + 4 * n, vb + 5 * n, vb + 6 * n, vb + 7 * n,
         vb + 8 * n, vb + 9 * n, vb + 10 * n, vb + 11 * n, vb + 12 * n, vb + 13 * n, vb + 14 * n, vb + 15 * n};
  DevState* st = (DevState*)W.state.p;
  int* svd_sweeps_dev = (int*)((char*)W.state.p + sizeof(DevState));
  const int* stop = &st->stop;
  double* Y = (double*)W.Y.p;
  double* cn2 = (double*)W.colnorm2.p;
  double* dinv = (double*)W.dinv.p;
  double* sigma = (double*)W.sigma.p;
  double* V = (double*)W.V.p;
  double* gpart = (double*)W.gemvpart.p;
  double* UR = (double*)W.UR.p;
  const double* R = Y;  // upper triangle of Y[0:n, 0:n], ld = d
  const int64_t ldr = d;
  const double* tvec = Y + (int64_t)n * d;  // t = (Q^T S b)[0:n]

  // ---- host copy of the initial state
  const double eta = ((o.eta > 0) ? o.eta : sqrt((double)n / d)) * o.eta_factor;
  const double beta0 = eta * eta;                            // eq:optimal-coeffs
  FS_K(fs_vec_state_init(st, (1.0 - beta0) * (1.0 - beta0), beta0, o.max_inner, s));
  FS_K(fs_trsv_flow_reset(n, W.trsv.p, s));

  hipEvent_t* ev = ctx->ev;
  FS_HIP(hipEventRecord(ev[0], s));
  FS_K(fs_launch_sketch_indices(m, d, zeta, o.seed, 0, m, W.idx.p, i16, s));
  std::vector<double> cnh(n + 1);
  int svd_sweeps = 0;
  // Sketch (Alg 1 first statement; Alg 4 column scaling in the same read of A), QR of the sketch,
  // SVD of R (Alg 4: Sigma, V for normest, condest, truncation and the KW estimate), then a read-back
  // of the statistics.  fp32: the mixed-precision form's sketch (FP32 accumulation, from A32 if given).
  bool early_fallback = false;
  auto factor = [&](bool fp32, bool defer_svd) -> fs_status {
    if (fp32)
      FS_K(fs_launch_sketch_apply_fp32(A, lda, A32, lda32, m, n, b, m, 1, W.idx.p, i16, d, zeta, Y, d, cn2,
                                       o.column_scaling != 0, true, ctx->lds_bytes, s));
    else
      FS_K(fs_launch_sketch_apply(A, lda, m, n, b, m, 1, W.idx.p, i16, d, zeta, Y, d, cn2, o.column_scaling != 0,
                                  true, ctx->lds_bytes, s));
    FS_K(fs_vec_scaling(n, cn2, o.column_scaling != 0, dinv, st, s));
    FS_HIP(hipEventRecord(ev[1], s));
    // grid-synchronizing kernels: work-groups reserved against other slots of a server, the QR's and
    // the (smaller, longer-running) SVD's one after the other
    {
      CoopSection coop(ctx, fs_qr_grid_size(d, ctx->num_cu));
      FS_K(fs_launch_qr(Y, d, d, k, W.qrwork.p, ctx->num_cu, s));
      FS_HIP(hipEventRecord(ev[2], s));
    }
    // with the SVD beside the refinement: R^{-1} for the spectral bounds, x_0 and the steps that run
    // before Sigma and V exist
    rinv_ok = false;
    if (defer_svd && rinv) {
      FS_K(fs_launch_tri_inv(R, ldr, n, rinv, rinv_scratch, s));
      rinv_ok = true;
    }
    const double* rinv_b = rinv_ok ? rinv : nullptr;
    bool bounds_done = false;
    if (fp32) {
      // A lower bound of cond(R) (diag(R), then power and inverse iteration, about 0.5 ms at n = 1000)
      // decides before the SVD whether the FP32-copy sketch can be kept: a bound that already passes
      // u32 condest > 2 drops it at once (the SVD would only confirm); otherwise the SVD's condest
      // decides later.
      FS_K(fs_vec_diag_bounds(n, R, ldr, st, s));
      FS_K(fs_vec_spectral_bounds(n, R, ldr, rinv_b, 4, (double*)W.vecs.p + (size_t)16 * n, gpart, W.trsv.p, st,
                                  s));
      FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
      FS_HIP(fs_wait(ctx, s));
      bounds_done = true;
      if (!(ctx->st_host->condest * FS_MIXED_COND_FACTOR <= FS_MIXED_DISTORTION)) {
        early_fallback = true;
        return FS_OK;
      }
    }
    if (defer_svd) {
      // the SVD is launched by the caller on the second stream (after this event); until it fills in
      // normest and condest they hold lower bounds -- from diag(R), sharpened by a few steps of power
      // and inverse iteration on the main stream beside the SVD -- so the first step stops on its own
      // no earlier than the true rule would (its threshold is recomputed and the step cut back if the
      // SVD arrives first)
      FS_HIP(hipEventRecord(ctx->ev_aux, s));
      if (!bounds_done) {
        FS_K(fs_vec_diag_bounds(n, R, ldr, st, s));
        FS_K(fs_vec_spectral_bounds(n, R, ldr, rinv_b, 4, (double*)W.vecs.p + (size_t)16 * n, gpart, W.trsv.p, st,
                                  s));
      }
    } else {
      CoopSection coop(ctx, fs_svd_grid_size(n, ctx->num_cu, false));
      FS_K(fs_launch_svd_full(R, ldr, n, sigma, V, n, nullptr, n, W.svdwork.p, ctx->num_cu, o.max_sweeps,
                              svd_sweeps_dev, s));
      FS_K(fs_vec_sigma_stats(n, sigma, o.tau_factor, st, s));
      FS_HIP(hipEventRecord(ev[3], s));
    }
    FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(cnh.data(), cn2, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, s));
    int bar_err[2] = {0, 0};
    FS_HIP(hipMemcpyAsync(&bar_err[0], fs_qr_err_word(W.qrwork.p, d, k, ctx->num_cu), sizeof(int),
                          hipMemcpyDeviceToHost, s));
    if (!defer_svd) {
      FS_HIP(hipMemcpyAsync(&svd_sweeps, svd_sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s));
      FS_HIP(hipMemcpyAsync(&bar_err[1], fs_svd_err_word(W.svdwork.p, n), sizeof(int), hipMemcpyDeviceToHost, s));
    }
    FS_HIP(fs_wait(ctx, s));
    if (bar_err[0] || bar_err[1]) {
      fs_set_last_hip_error(hipErrorLaunchTimeOut, "grid barrier of the QR/SVD kernels gave up waiting", __FILE__,
                            __LINE__);
      return FS_ERR_DEVICE;
    }
    // the sketch marks a column holding NaN or Inf with a NaN norm; an infinite norm of finite data
    // means its squares overflow FP64 (entries beyond ~1e154): too large for the column scaling
    for (int j = 0; j <= n; ++j)
      if (std::isnan(cnh[j])) return FS_ERR_NONFINITE;
    for (int j = 0; j <= n; ++j)
      if (!std::isfinite(cnh[j])) return FS_ERR_TOO_LARGE;
    return FS_OK;
  };
  const bool mixed = (o.precision == FS_MIXED);
  int flags = 0;
  FS_TRY(factor(mixed, defer));
  if (mixed && (early_fallback || !(ctx->st_host->condest * FS_MIXED_COND_FACTOR <= FS_MIXED_DISTORTION))) {
    // The FP32 sketch perturbs S A by about u32 ||A||: as a preconditioner its R keeps A_s R^{-1}
    // well conditioned only while condest u32 is small (the hazard of Lemma 6.3 at single precision).
    // Otherwise (decided from diag(R) alone before the SVD, or from the SVD's condest) the sketch is
    // redone in FP64 (the FP64 correction of R) and the solve continues as an FP64 one, with the SVD
    // beside the first step when that applies.
    flags |= FS_FLAG_FP64_SKETCH;
    defer = defer_fp64;
    FS_TRY(factor(false, defer));
  }
  if (defer && cnh[n] == 0.0) {  // b = 0 ends the solve below: no overlap, the SVD runs here
    defer = false;
    CoopSection cs(ctx, fs_svd_grid_size(n, ctx->num_cu, false));
    FS_K(fs_launch_svd_full(R, ldr, n, sigma, V, n, nullptr, n, W.svdwork.p, ctx->num_cu, o.max_sweeps,
                            svd_sweeps_dev, s));
    FS_K(fs_vec_sigma_stats(n, sigma, o.tau_factor, st, s));
    FS_HIP(hipEventRecord(ev[3], s));
    FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(&svd_sweeps, svd_sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    FS_HIP(fs_wait(ctx, s));
  }
  // The deferred SVD: on the second stream after the QR, with its work-group reservation held
  // until that stream drains; the guard drains it on every exit path (the workspace is shared).
  std::unique_ptr<CoopSection> svd_coop;
  struct AuxDrain {
    fs_context c;
    hipStream_t a = nullptr;
    ~AuxDrain() {
      if (a && fs_wait(c, a) != hipSuccess) (void)hipStreamSynchronize(a);
    }
  } aux_drain{ctx};
  auto launch_aux_svd = [&]() -> fs_status {
    hipStream_t a = ctx->aux_stream;
    aux_drain.a = a;
    FS_HIP(hipStreamWaitEvent(a, ctx->ev_aux, 0));
    svd_coop = std::make_unique<CoopSection>(ctx, fs_svd_grid_size(n, ctx->num_cu, false), a);
    FS_K(fs_launch_svd_abortable(R, ldr, n, sigma, V, n, nullptr, n, W.svdwork.p, ctx->num_cu, o.max_sweeps,
                                 svd_sweeps_dev, &st->svd_abort, a));
    FS_K(fs_vec_sigma_stats(n, sigma, o.tau_factor, st, a));
    FS_HIP(hipEventRecord(ev[3], a));
    return FS_OK;
  };
  if (defer) FS_TRY(launch_aux_svd());
  const double b2 = cnh[n];
  DevState hs = *ctx->st_host;
  fs_info inf{};
  inf.normest = hs.normest;
  inf.condest = hs.condest;
  inf.rank = n;
  inf.svd_sweeps = svd_sweeps;
  if (b2 == 0.0) {  // b = 0: x = 0
    FS_HIP(hipMemsetAsync(x_out, 0, sizeof(double) * n, s));
    FS_HIP(fs_wait(ctx, s));
    if (info) *info = inf;
    return FS_OK;
  }
  bool use_svd = (o.precond == FS_PRECOND_SVD) && !defer;  // the deferred first step uses P = R^{-1}
  int rk = n;
  // Alg 4: numerically rank deficient -> truncated SVD preconditioner (needs the SVD's statistics)
  auto set_rank_deficient = [&]() -> fs_status {
    flags |= 1;
    rk = hs.rank_trunc > 0 ? hs.rank_trunc : 1;
    use_svd = true;
    // the truncated start x_0 = V_r Sigma_r^{-1} U_r^T t needs U_R: redo the SVD accumulating it
    // (rank-deficient problems only)
    CoopSection cs(ctx, fs_svd_grid_size(n, ctx->num_cu, true));
    FS_K(fs_launch_svd_full(R, ldr, n, sigma, V, n, UR, n, W.svdwork.p, ctx->num_cu, o.max_sweeps, svd_sweeps_dev, s));
    return FS_OK;
  };
  if (!defer && !(hs.condest <= 1.0 / (o.tau_factor * U_ROUND))) FS_TRY(set_rank_deficient());
  inf.rank = rk;
  int nr = use_svd ? rk : n;  // length of the preconditioned variables dy, c, ...

  // P y (into out, n) and P^T v (into out, nr); yscale/xscale fold D^{-1}.
  // Beside the SVD (and in a second step begun before it ends) P = R^{-1} is applied many times with
  // the same R: there it is a product with the explicit inverse, formed once after the QR.
  auto applyP = [&](const double* y, double* out, const double* oscale, const double* addv, const int* stp) -> fs_status {
    if (use_svd) {
      FS_K(fs_vec_gemv_v(V, n, n, nr, y, sigma, oscale, addv, out, gpart, stp, s));
    } else if (rinv_ok) {
      FS_K(fs_vec_gemv_v(rinv, n, n, n, y, nullptr, oscale, addv, out, gpart, stp, s));
    } else {
      FS_K(fs_launch_trsv_flow(R, ldr, n, false, y, out, nullptr, oscale, stp, W.trsv.p, s));
      if (addv) FS_K(fs_vec_add_norm(n, addv, out, out, nullptr, stp, s));
    }
    return FS_OK;
  };
  auto applyPT = [&](const double* vin, double* out, const int* stp) -> fs_status {
    if (use_svd) {
      FS_K(fs_vec_gemv_vt(V, n, n, nr, vin, sigma, out, stp, s));
    } else if (rinv_ok) {
      FS_K(fs_vec_gemv_vt(rinv, n, n, n, vin, nullptr, out, stp, s));
    } else {
      FS_K(fs_launch_trsv_flow(R, ldr, n, true, vin, out, nullptr, nullptr, stp, W.trsv.p, s));
    }
    return FS_OK;
  };

  // ---- x_0: sketch-and-solve (eq:sketch-and-solve-2.3; Alg 4 with the SVD factors)
  auto start_x0 = [&]() -> fs_status {
    if (flags & 1) {
      // truncated SVD start (Alg 4): x_0 = V_r Sigma_r^{-1} U_r^T t
      FS_K(fs_vec_gemv_vt(UR, n, n, nr, tvec, nullptr, v.tmp, nullptr, s));
      FS_K(fs_vec_gemv_v(V, n, n, nr, v.tmp, sigma, nullptr, nullptr, v.x, gpart, nullptr, s));
    } else if (rinv_ok) {  // full rank, beside the SVD: x_0 = R^{-1} t with the explicit inverse
      FS_K(fs_vec_gemv_v(rinv, n, n, n, tvec, nullptr, nullptr, nullptr, v.x, gpart, nullptr, s));
    } else {  // full rank: V Sigma^{-1} U_R^T t = R^{-1} t (eq:sketch-and-solve-2.3)
      FS_K(fs_launch_trsv_flow(R, ldr, n, false, tvec, v.x, nullptr, nullptr, nullptr, W.trsv.p, s));
    }
    if (o.init == FS_INIT_ZERO) FS_HIP(hipMemsetAsync(v.x, 0, sizeof(double) * n, s));  // (not captured)
    FS_K(fs_vec_mul(n, v.x, nullptr, v.x0, nullptr, s));
    return FS_OK;
  };
  FS_TRY(start_x0());

  // theta^2 and the first-step threshold need ||b||^2 and ||A_s||_F^2
  {
    // st->theta2 = fro2 / b2: computed on the host from the read-back fro2 (set by k_scaling)
    FS_K(fs_vec_set_double(&st->theta2, hs.fro2 / b2, s));
    FS_K(fs_vec_set_double(&st->b2, b2, s));
  }

  int iters[2] = {0, 0};
  bool conv_last = true;
  double cnorm[2] = {0, 0};
  int q_fixed = 0;
  if (o.fixed_q != 0) {
    if (o.fixed_q > 0) {
      q_fixed = o.fixed_q;
    } else {  // Theorem 7.1: alpha, beta from 1.01 eta; q_0 from condest
      const double e2 = 1.01 * eta;
      const double ku = hs.condest * U_ROUND;
      q_fixed = (ku >= 1.0) ? 11 : (int)ceil(std::max(1.0 + 2.0 * log(1.0 / ku) / log(1.0 / e2), 11.0));
      const double b1 = e2 * e2;                               // Thm 7.1 (D)
      FS_K(fs_vec_set_double(&st->alpha, (1.0 - b1) * (1.0 - b1), s));
      FS_K(fs_vec_set_double(&st->beta, b1, s));
    }
  }
  FS_HIP(hipEventRecord(ev[4], s));

  struct PassCapReset {  // the cap applies to this solve's overlapped step only, on every exit path
    fs_context c;
    ~PassCapReset() { c->pass_group_cap = 0; }
  } pass_cap_reset{ctx};
  // Join the SVD running beside the refinement: statistics and barrier status.  Returns 1 when the
  // solve restarts (a kept FP32 sketch fails its condest, or R is numerically rank deficient).
  auto join_svd = [&](int& restarted) -> fs_status {
    restarted = 0;
    FS_HIP(fs_wait(ctx, ctx->aux_stream));
    svd_coop.reset();
    int bar_err = 0;
    FS_HIP(hipMemcpyAsync(&bar_err, fs_svd_err_word(W.svdwork.p, n), sizeof(int), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(&svd_sweeps, svd_sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FS_HIP(fs_wait(ctx, s));
    if (bar_err) {
      fs_set_last_hip_error(hipErrorLaunchTimeOut, "grid barrier of the SVD kernel gave up waiting", __FILE__,
                            __LINE__);
      return FS_ERR_DEVICE;
    }
    hs.normest = ctx->st_host->normest;
    hs.condest = ctx->st_host->condest;
    hs.rank_trunc = ctx->st_host->rank_trunc;
    inf.normest = hs.normest;
    inf.condest = hs.condest;
    inf.svd_sweeps = svd_sweeps;
    defer = false;
    if (mixed && !(flags & FS_FLAG_FP64_SKETCH) && !(hs.condest * FS_MIXED_COND_FACTOR <= FS_MIXED_DISTORTION)) {
      // the FP32 sketch kept on diag(R)'s evidence fails on its SVD's condest: discard the
      // overlapped steps and restart from an FP64 sketch, its SVD again beside the first step
      flags |= FS_FLAG_FP64_SKETCH;
      FS_TRY(factor(false, true));
      FS_TRY(launch_aux_svd());
      defer = true;
      hs = *ctx->st_host;
      FS_K(fs_vec_set_double(&st->theta2, hs.fro2 / b2, s));  // ||A_s||_F of the FP64 column scaling
      use_svd = false;
      nr = n;
      FS_TRY(start_x0());
      restarted = 1;
      return FS_OK;
    }
    if (!(hs.condest <= 1.0 / (o.tau_factor * U_ROUND))) {
      // numerically rank deficient after all: start over in the serial order with the truncated
      // preconditioner (the overlapped steps are discarded)
      FS_TRY(set_rank_deficient());
      inf.rank = rk;
      nr = rk;
      FS_TRY(start_x0());
      restarted = 1;
    }
    return FS_OK;
  };
  bool early = false;  // the second step runs with P = R^{-1} while the SVD is still running
  bool svd_abandoned = false;  // that step met its rule through the bound ||R^{-T} g||: no SVD needed
  // The bound certifies the rule only where the substitution R^{-T} g is accurate to a few percent
  // (n u condest <= 0.1, condest from its lower bound) and, in the mixed form, once the sketch is FP64.
  const bool kw_bound_ok = !(mixed && !(flags & FS_FLAG_FP64_SKETCH)) && hs.condest * n * U_ROUND <= 0.1;
  for (int step = 0; step < o.steps; ++step) {
    const bool dstep = defer && step == 0;  // first step beside the SVD (P = R^{-1}, iterates recorded)
    bool thr_known = !dstep;
    // beside the SVD the passes take only the compute units its work-groups leave free (at least
    // half of them here): a pass with more work-groups than free units runs a second, partial wave
    int group_cap = 0;
    if (dstep || early) {
      const int free_cu = ctx->num_cu - fs_svd_grid_size(n, ctx->num_cu, false);
      group_cap = (o.overlap_pass_groups > 0) ? o.overlap_pass_groups : free_cu / 8 * 8;
    }
    ctx->pass_group_cap = group_cap;
    // residual pass at x (scaled coordinates): g = D^{-1} A^T (b - A D^{-1} x), r2
    FS_K(fs_vec_mul(n, v.x, dinv, v.zs, nullptr, s));
    FS_TRY(run_pass(ctx, m, n, A, lda, v.zs, b, v.g, dinv, &st->r2, nullptr, rbuf));
    if (step == 0) {
      FS_K(fs_vec_first_threshold(n, v.x0, o.gamma, o.rho, st, s));
      FS_HIP(hipEventRecord(ev[5], s));
    }
    FS_TRY(applyPT(v.g, v.c, nullptr));
    // FOSSILS: dy = dy_old = c.  SPIR: dy = 0, res = p = c.
    // LSQR: v = c / ||c||, w = v, dy = 0, ubar = alpha_1 u_1 = (alpha_1 / beta_1) r.
    if (method == M_FOSSILS) FS_K(fs_vec_step_init(nr, v.c, v.dy, v.dy_old, v.dy, false, st, s));
    else if (lsqr) {
      FS_K(fs_vec_lsqr_init(nr, v.c, v.p, v.res, v.dy, st, s));
      FS_K(fs_vec_lsqr_ubar(m, rbuf, ubar, 1.0, st, s));
    } else FS_K(fs_vec_step_init(nr, v.c, v.res, v.p, v.dy, true, st, s));
    const bool fixed = (method == M_FOSSILS && q_fixed > 0);
    const int cap = fixed ? q_fixed - 1 : o.max_inner;
    if (fixed) FS_K(fs_vec_set_int(&st->max_inner, cap, s));
    const bool first = (step == 0) && !fixed;
    bool stopped = false;
    bool kw_deferred = early && step == 1;  // KW checkpoints recorded until Sigma and V exist
    int kw_recorded = 0;
    // one inner iteration (every kernel returns at once after the device-side stop flag is set)
    auto iteration = [&](int j) -> fs_status {
      const double* dir = (method == M_FOSSILS) ? v.dy : v.p;
      FS_TRY(applyP(dir, v.zs, dinv, nullptr, stop));                   // z' = D^{-1} P dir
      if (lsqr) {
        // r = alpha u - A_s P v (stored), h = P^T A_s^T r, beta^2 = ||r||^2: one residual pass
        FS_TRY(run_pass(ctx, m, n, A, lda, v.zs, ubar, v.v, dinv, &st->r2, stop, rbuf));
        FS_TRY(applyPT(v.v, v.u, stop));
        FS_K(fs_vec_lsqr_step(nr, v.u, v.p, v.res, v.dy, st, first, s));
        FS_K(fs_vec_lsqr_ubar(m, rbuf, ubar, -1.0, st, s));
      } else {
        FS_TRY(run_pass(ctx, m, n, A, lda, v.zs, nullptr, v.v, dinv, nullptr, stop));  // v = D^{-1} A^T A z'
        FS_TRY(applyPT(v.v, v.u, stop));                                 // u = P^T v
        if (method == M_FOSSILS) FS_K(fs_vec_polyak(nr, v.c, v.u, v.dy, v.dy_old, st, first, s));
        else FS_K(fs_vec_cg(nr, v.p, v.u, v.res, v.dy, st, first, s));
        if (dstep) FS_K(fs_vec_record_iter(j, nr, v.dy, hist_dy, hist_dn, st, s));
      }
      const bool kw_now = (!fixed) && (step == 1) && (j % o.kw_every == 0);
      if (kw_now) {  // second-step rule (Alg 4): sketched KW at x_hat = x + P dy
        FS_TRY(applyP(v.dy, v.xh, nullptr, v.x, stop));
        FS_K(fs_vec_add_norm(n, v.xh, nullptr, v.xh, &st->x2, stop, s));
        FS_K(fs_vec_mul(n, v.xh, dinv, v.zs, stop, s));
        FS_TRY(run_pass(ctx, m, n, A, lda, v.zs, b, v.g, dinv, &st->r2, stop));
        if (kw_deferred) {
          if (kw_recorded < kw_slots) {
            FS_K(fs_vec_kw_record(kw_recorded, j, n, v.dy, v.g, kw_dy, kw_g, kw_s, st, s));
            ++kw_recorded;
          }
          // the rule through ||R^{-T} g|| >= the sketched KW estimate: when even the bound meets it,
          // the step stops here without Sigma and V (the first checkpoint where it holds; the exact
          // rule might have stopped at an earlier one)
          if (kw_bound_ok) {
            FS_TRY(applyPT(v.g, v.w, stop));  // R^{-T} g
            FS_K(fs_vec_kw_upper(n, v.w, 1.25, st, s));
          }
        } else {
          FS_K(fs_vec_gemv_vt(V, n, n, n, v.g, nullptr, v.w, stop, s));
          FS_K(fs_vec_kw(n, v.w, sigma, st, s));
        }
      }
      return FS_OK;
    };
    auto poll_stop = [&]() -> fs_status {
      FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
      FS_HIP(fs_wait(ctx, s));
      if (ctx->st_host->stop) stopped = true;
      return FS_OK;
    };
    // the SVD's statistics have arrived: the real first-step threshold, then the cut back to the
    // first recorded iteration that meets it
    auto apply_threshold = [&]() -> fs_status {
      FS_HIP(hipStreamWaitEvent(s, ev[3], 0));
      FS_K(fs_vec_first_threshold(n, v.x0, o.gamma, o.rho, st, s));
      FS_K(fs_vec_rollback(nr, hist_dy, hist_dn, v.dy, st, s));
      thr_known = true;
      return FS_OK;
    };
    // the second step beside the SVD: once Sigma and V exist, the recorded KW checkpoints are
    // evaluated in order (the step may end at one of them) and later checks are evaluated at once
    int restarted = 0;
    auto finish_deferred = [&]() -> fs_status {
      FS_TRY(join_svd(restarted));
      if (restarted) return FS_OK;
      ctx->pass_group_cap = 0;  // the whole GPU for the rest of the step
      for (int c = 0; c < kw_recorded; ++c)
        FS_K(fs_vec_gemv_vt(V, n, n, n, kw_g + (size_t)c * n, nullptr, kw_w + (size_t)c * n, nullptr, s));
      FS_K(fs_vec_kw_replay(n, kw_recorded, kw_w, sigma, kw_dy, kw_s, v.dy, st, s));
      kw_deferred = false;
      return FS_OK;
    };
    const int sweep = o.kw_every;
    if (dstep) {
      for (int j = 0; j < cap && !stopped; ++j) {
        FS_TRY(iteration(j));
        const bool poll = ((j + 1) % sweep) == 0 || j == cap - 1;
        if (poll) {
          if (!thr_known && hipEventQuery(ev[3]) == hipSuccess) FS_TRY(apply_threshold());
          FS_TRY(poll_stop());
          // a kept FP32 sketch whose SVD reports u32 condest too large: this step will be discarded
          // (the join restarts from an FP64 sketch), so it stops here
          if (thr_known && mixed && !(flags & FS_FLAG_FP64_SKETCH) &&
              !(ctx->st_host->condest * FS_MIXED_COND_FACTOR <= FS_MIXED_DISTORTION))
            stopped = true;
        }
      }
      // The step stopped on the diag(R) lower bounds before the SVD finished: the threshold it used
      // is at most the true one (the step ran at least as long as the first-step rule asks), and the
      // second step starts now with P = R^{-1}.  Otherwise the cut back to the true rule.
      // (only where substitution with R is accurate to a few percent, n u condest <= 0.1 with condest
      // from its lower bound: for a worse conditioned R the second step's KW estimate, taken at
      // x + R^{-1} dy, does not reach the rule's floor, and that step waits for P = V Sigma^{-1})
      early = !thr_known && o.steps == 2 && !fixed && !o.graph_sweeps && ctx->st_host->converged != 0 &&
              ctx->st_host->condest * n * U_ROUND <= 0.1;
      if (!thr_known && !early) FS_TRY(apply_threshold());
      if (early) flags |= FS_FLAG_EARLY_SECOND_STEP;
      else flags &= ~FS_FLAG_EARLY_SECOND_STEP;
    } else if (o.graph_sweeps && !fixed && !kw_deferred && cap % sweep == 0) {
      // kw_every iterations (the KW check, when due, is the first of them) captured once as a graph
      // and replayed; the host polls the stop flag after each replay, as the launch-by-launch loop does
      FS_TRY(sweep_graph_run(ctx, s, sweep, cap / sweep, iteration, poll_stop, stopped));
    } else {
      for (int j = 0; j < cap && !stopped; ++j) {
        FS_TRY(iteration(j));
        const bool poll = ((j + 1) % sweep) == 0 || j == cap - 1;
        if (poll && !fixed) {
          FS_TRY(poll_stop());
          if (kw_deferred && ctx->st_host->svd_abort) {
            kw_deferred = false;  // stopped on the bound; the SVD winds down unused
            svd_abandoned = true;
          } else if (kw_deferred && (stopped || hipEventQuery(ev[3]) == hipSuccess)) {
            FS_TRY(finish_deferred());
            if (restarted) break;
            FS_TRY(poll_stop());
          }
        }
      }
      if (kw_deferred && !restarted) {  // (the loop ended at the cap)
        FS_TRY(poll_stop());
        if (ctx->st_host->svd_abort) svd_abandoned = true;
        else FS_TRY(finish_deferred());
      }
    }
    if (restarted) {
      early = false;
      iters[0] = 0;
      step = -1;
      continue;
    }
    // x <- x + P dy
    FS_TRY(applyP(v.dy, v.z, nullptr, v.x, nullptr));
    FS_K(fs_vec_mul(n, v.z, nullptr, v.x, nullptr, s));
    FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FS_HIP(hipEventRecord(ev[6 + (step > 0 ? 1 : 0)], s));
    FS_HIP(fs_wait(ctx, s));
    iters[step] = ctx->st_host->iters;
    cnorm[step] = sqrt(ctx->st_host->cnorm2);
    conv_last = ctx->st_host->converged != 0 || fixed;
    if (fixed) FS_K(fs_vec_set_int(&st->max_inner, o.max_inner, s));  // restore the cap
    if (dstep && !early) {
      // join the SVD: statistics, barrier status; then the second step with P = V Sigma^{-1}
      FS_TRY(join_svd(restarted));
      if (restarted) {
        iters[0] = 0;
        step = -1;
        continue;
      }
      use_svd = true;  // P = V Sigma^{-1} for the second step (full rank: nr = n)
    }
  }
  if (svd_abandoned) {
    // the SVD stops at its next sweep boundary; normest and condest stay the lower bounds
    FS_HIP(fs_wait(ctx, ctx->aux_stream));
    svd_coop.reset();
    FS_HIP(hipMemcpyAsync(&svd_sweeps, svd_sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    inf.svd_sweeps = svd_sweeps;
    flags |= FS_FLAG_SVD_ABANDONED;
  }
  // x_out = D^{-1} x
  FS_K(fs_vec_mul(n, v.x, dinv, x_out, nullptr, s));
  FS_HIP(hipMemcpyAsync(ctx->st_host, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  int trsv_err = 0;
  FS_HIP(hipMemcpyAsync(&trsv_err, fs_trsv_flow_err_word(n, W.trsv.p), sizeof(int), hipMemcpyDeviceToHost, s));
  FS_HIP(fs_wait(ctx, s));
  if (trsv_err) {
    fs_set_last_hip_error(hipErrorLaunchTimeOut, "triangular solve gave up waiting for a block", __FILE__, __LINE__);
    return FS_ERR_DEVICE;
  }
  if (o.steps == 2 && o.fixed_q == 0 && !conv_last) flags |= 2;
  inf.iters[0] = iters[0];
  inf.iters[1] = iters[1];
  inf.flags = flags;
  inf.be_sk = ctx->st_host->be_sk;
  inf.kw_evals = ctx->st_host->kw_evals;
  inf.cnorm[0] = cnorm[0];
  inf.cnorm[1] = cnorm[1];
  auto el = [&](int a, int bb) -> double {
    float t = 0;
    return (hipEventElapsedTime(&t, ev[a], ev[bb]) == hipSuccess) ? (double)t : -1.0;
  };
  inf.phase_ms[0] = el(0, 1);
  inf.phase_ms[1] = el(1, 2);
  inf.phase_ms[2] = el(2, 3);
  inf.phase_ms[3] = el(4, 5);
  inf.phase_ms[4] = el(5, 6);
  inf.phase_ms[5] = (o.steps > 1) ? el(6, 7) : 0.0;
  if (info) *info = inf;
  if (flags & 1) return FS_WARN_RANK_DEFICIENT;
  if (flags & 2) return FS_WARN_NOT_CONVERGED;
  return FS_OK;
}

}  // namespace

extern "C" {

fs_status fossils_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                        double* x, const fs_options* opts, fs_info* info) {
  return solve(ctx, M_FOSSILS, m, n, A, lda, b, x, opts, info);
}

fs_status spir_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b, double* x,
                     const fs_options* opts, fs_info* info) {
  return solve(ctx, M_SPIR, m, n, A, lda, b, x, opts, info);
}

}  // extern "C"

fs_status fs_fossils_solve_fixed(fs_context ctx, unsigned char* base, size_t cap, int64_t m, int32_t n,
                                 const double* A, int64_t lda, const double* b, double* x, const fs_options& o,
                                 fs_info* info) {
  if (!ctx || !base) return FS_ERR_INVALID_ARG;
  if (o.overlap_svd != 0 || o.graph_sweeps != 0) return FS_ERR_INVALID_ARG;
  FS_TRY(validate_problem(m, n, A, lda, b, x));
  FS_TRY(validate_options(m, n, o));
  if (fs_carve_workspace(ctx->ws, nullptr, m, n, o, ctx->num_cu) > cap) return FS_ERR_TOO_LARGE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  // the context's own buffers are set aside for this call and put back on every exit path
  struct Swap {
    fs_context c;
    Workspace saved;
    ~Swap() { c->ws = saved; }
  } swap{ctx, ctx->ws};
  ctx->ws = Workspace{};
  (void)fs_carve_workspace(ctx->ws, base, m, n, o, ctx->num_cu);
  return solve(ctx, M_FOSSILS, m, n, A, lda, b, x, &o, info);
}

extern "C" {

fs_status spir_lsqr_solve(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                          double* x, const fs_options* opts, fs_info* info) {
  return solve(ctx, M_SPIR_LSQR, m, n, A, lda, b, x, opts, info);
}

// Complex least squares (the Prony problems of Section 5.2): the real solver on the realification
// (2m x 2n, same residual norms, each singular value twice), its solution mapped back.
static fs_status solve_complex(fs_context ctx, Method method, int64_t m, int32_t n, const double* A, int64_t lda,
                               const double* b, double* x, const fs_options* opts, fs_info* info) {
  if (!ctx || !A || !b || !x) return FS_ERR_INVALID_ARG;
  if (((uintptr_t)A | (uintptr_t)b | (uintptr_t)x) & 15) return FS_ERR_INVALID_ARG;  // complex128 alignment
  if (n < 1 || m < n || lda < m || n > (1 << 29)) return FS_ERR_SHAPE;
  const int64_t M2 = 2 * m;
  const int32_t N2 = 2 * n;
  fs_options o;
  if (opts) o = *opts;
  else FS_TRY(fs_options_default(M2, N2, &o));
  FS_TRY(validate_options(M2, N2, o));
  FS_HIP(hipSetDevice(ctx->device));
  FS_HIP(hipStreamSynchronize(ctx->stream));  // the realification buffer may be reallocated
  Workspace& W = ctx->ws;
  FS_TRY(grow(W.cplx, sizeof(double) * ((size_t)M2 * N2 + M2 + N2)));
  double* Ar = (double*)W.cplx.p;
  double* br = Ar + (size_t)M2 * N2;
  double* xr = br + M2;
  FS_K(fs_launch_realify(m, n, A, lda, b, Ar, br, ctx->stream));
  const fs_status st = solve(ctx, method, M2, N2, Ar, M2, br, xr, &o, info);
  if (st < 0) return st;
  FS_K(fs_launch_complexify_x(n, xr, x, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return st;
}

fs_status fossils_solve_complex(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                                double* x, const fs_options* opts, fs_info* info) {
  return solve_complex(ctx, M_FOSSILS, m, n, A, lda, b, x, opts, info);
}

fs_status spir_solve_complex(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                             double* x, const fs_options* opts, fs_info* info) {
  return solve_complex(ctx, M_SPIR, m, n, A, lda, b, x, opts, info);
}

fs_status fossils_solve_mixed(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const float* A32,
                              int64_t lda32, const double* b, double* x, const fs_options* opts, fs_info* info) {
  if (A32 && lda32 < m) return FS_ERR_SHAPE;
  fs_options o;
  if (opts) o = *opts;
  else FS_TRY(fs_options_default(m, n, &o));
  o.precision = FS_MIXED;
  return solve(ctx, M_FOSSILS, m, n, A, lda, b, x, &o, info, A32, lda32);
}

fs_status fs_to_fp32(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, float* A32, int64_t lda32) {
  if (!ctx || !A || !A32) return FS_ERR_INVALID_ARG;
  if (m < 1 || n < 1 || lda < m || lda32 < m) return FS_ERR_SHAPE;
  FS_HIP(hipSetDevice(ctx->device));
  FS_K(fs_launch_to_fp32(A, lda, m, n, A32, lda32, ctx->stream));
  FS_HIP(hipStreamSynchronize(ctx->stream));
  return FS_OK;
}

}  // extern "C"
