// Internal: the context, workspace and host-side helpers shared by the orchestration files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <condition_variable>
#include <map>
#include <mutex>

#include "../../include/fossils.h"
#include "common.hpp"
#include "state.hpp"

constexpr double FS_U_ROUND = 2.220446049250313e-16;
// Mixed precision: the sketch of the FP32 copy is accepted while u32 condest <= 2 (condest <= ~3.4e7).
constexpr double FS_MIXED_COND_FACTOR = 5.9604644775390625e-08;
constexpr double FS_MIXED_DISTORTION = 2.0;
// Size of the device array behind fossils_solve_noalloc (per GPU, for the life of the process).
constexpr size_t FS_NOALLOC_SCRATCH_BYTES = size_t(256) << 20;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool fixed = false;  // a slice of caller-provided memory: never reallocated or freed by the library
};

struct Workspace {
  DevBuf idx, Y, colnorm2, dinv, qrwork, svdwork, sigma, V, UR, partial, pr2, wscratch, gemvpart, vecs, state;
  DevBuf mwork, mvecs, mstate;  // multi-RHS solves
  DevBuf lsqr;                  // LSQR form of SPIR: the residual r and ubar = alpha u (2 m-vectors)
  DevBuf hist;                  // first step beside the SVD: iterates and ||Delta||^2 per iteration
  DevBuf cplx;                  // complex problems: the realified A (2m x 2n), b and x
  DevBuf trsv;                  // triangular solves across work-groups: published x and block flags
  DevBuf batch;                 // fossils_solve_batched: per-problem factors, vectors and work-lists
};

struct fs_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  int pass_group_cap = 0;  // > 0: at most this many work-groups per fused pass (the first step beside the SVD)
  int lds_bytes = 0;
  Workspace ws;
  DevState* st_host = nullptr;  // pinned copy for read-back
  hipEvent_t ev[8] = {};
  // Set by a server whose slots share the GPU (see CoopBudget).
  struct CoopBudget* coop_budget = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture (created on first use)
  hipStream_t aux_stream = nullptr;  // second stream: the SVD of R beside the first refinement step
  hipEvent_t ev_aux = nullptr;       // (both created on first use)
  hipEvent_t ev_wait = nullptr;      // host waits of a server slot (fs_wait; created on first use)
  // Fused-pass configurations picked by fs_tune_pass (or loaded with fs_set_pass_tuning), keyed
  // by (n, floor(log2 m)); used by every pass of that shape instead of the built-in rule.
  std::map<std::pair<int, int>, std::pair<int, int>> pass_tuned;  // -> (H, G)
  bool pass_force = false;     // while tuning: every pass uses pass_force_cfg
  int pass_force_H = 0, pass_force_G = 0;
  struct BatchHelpers* batch = nullptr;  // fossils_solve_batched: setup contexts (created on first use)
};

// Cooperative kernels (QR, SVD) need every work-group of their grid resident at once.  Slots of a
// server reserve their grid's work-groups (at most one per CU for these kernels: their LDS use
// leaves room for one) from a budget of num_cu before launching, and give them back once the
// stream has drained; grids that fit together run concurrently, and two grids can never hold parts
// of the GPU while waiting for each other.  Other kernels need no reservation: they finish on
// their own and free their CUs.
struct CoopBudget {
  std::mutex mu;
  std::condition_variable cv;
  int total = 0, avail = 0;
};

// Waits for the work enqueued on s.  A context with a budget is a server slot, one of several host threads
// that share the host's cores: it polls an event with short sleeps, so that a waiting slot does not hold a
// core another slot needs to launch its work.  A lone solve synchronizes the stream (lowest latency).
hipError_t fs_wait(fs_context_s* ctx, hipStream_t s);

// Holds a reservation of `need` work-groups (if the context has a budget) until the stream drains.
struct CoopSection {
  fs_context_s* ctx;
  hipStream_t strm;
  int need = 0;
  CoopSection(fs_context_s* c, int need_wgs, hipStream_t on = nullptr) : ctx(c), strm(on ? on : c->stream) {
    CoopBudget* b = c->coop_budget;
    if (!b) return;
    need = std::max(1, std::min(need_wgs, b->total));
    std::unique_lock<std::mutex> lk(b->mu);
    b->cv.wait(lk, [&] { return b->avail >= need; });
    b->avail -= need;
  }
  ~CoopSection() {
    if (!need) return;
    if (fs_wait(ctx, strm) != hipSuccess) (void)hipStreamSynchronize(strm);
    CoopBudget* b = ctx->coop_budget;
    {
      std::lock_guard<std::mutex> lk(b->mu);
      b->avail += need;
    }
    b->cv.notify_all();
  }
};

struct fs_sketch_s {
  fs_context ctx = nullptr;
  int64_t m = 0;
  int d = 0, zeta = 0;
  uint64_t seed = 0;
  bool idx16 = true;
  void* idx = nullptr;
};

// Grow-only device buffer (the caller synchronizes the stream before growing).
fs_status fs_grow(DevBuf& b, size_t bytes);
void fs_free_buf(DevBuf& b);
size_t fs_workspace_bytes(Workspace& w);  // device bytes the workspace holds
void fs_workspace_free(Workspace& w);     // frees every buffer (nothing in flight may use them)
size_t fs_solve_footprint_cu(int64_t m, int32_t n, const fs_options& o, int num_cu);
// Bytes of the fixed workspace a FOSSILS solve in the serial order (overlap_svd 0, graph_sweeps 0)
// needs; with base != nullptr, also points the buffers of w at consecutive 256-byte aligned slices
// of [base, base + the returned size) (marked fixed).
size_t fs_carve_workspace(Workspace& w, unsigned char* base, int64_t m, int32_t n, const fs_options& o, int num_cu);
// fossils_solve on a workspace of fixed slices (fs_carve_workspace) of caller-provided device memory:
// nothing is allocated; opts must have overlap_svd = 0 and graph_sweeps = 0.
fs_status fs_fossils_solve_fixed(fs_context ctx, unsigned char* base, size_t cap, int64_t m, int32_t n,
                                 const double* A, int64_t lda, const double* b, double* x, const fs_options& opts,
                                 fs_info* info);
// Destroys the setup contexts of fossils_solve_batched (if any).
void fs_batch_helpers_destroy(fs_context_s* c);
fs_status fs_validate_problem(int64_t m, int32_t n, const void* A, int64_t lda, const void* b, const void* x);
fs_status fs_validate_options(int64_t m, int32_t n, const fs_options& o);
inline bool fs_idx16_ok(int d) { return d <= 32767; }

#define FS_TRY(expr)                 \
  do {                               \
    fs_status s_ = (expr);           \
    if (s_ != FS_OK) return s_;      \
  } while (0)

#define FS_K(expr)                                                   \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) {                                          \
      fs_set_last_hip_error(e_, #expr, __FILE__, __LINE__);          \
      return FS_ERR_DEVICE;                                          \
    }                                                                \
  } while (0)
