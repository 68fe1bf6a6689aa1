// Internal: the context, workspace and host-side helpers shared by the orchestration files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/fossils.h"
#include "common.hpp"
#include "state.hpp"

constexpr double FS_U_ROUND = 2.220446049250313e-16;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Workspace {
  DevBuf idx, Y, colnorm2, dinv, qrwork, svdwork, sigma, V, UR, partial, pr2, wscratch, gemvpart, vecs, state;
  DevBuf mwork, mvecs, mstate;  // multi-RHS solves
};

struct fs_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  int lds_bytes = 0;
  Workspace ws;
  DevState* st_host = nullptr;  // pinned copy for read-back
  hipEvent_t ev[8] = {};
  // Set by a server whose slots share the GPU: cooperative kernels (QR, SVD) of different
  // contexts must not run concurrently (each grid has to be fully resident).
  std::mutex* coop_lock = nullptr;
};

// Holds the cooperative-kernel lock of ctx (if any) until the context's stream has drained.
struct CoopSection {
  fs_context_s* ctx;
  std::unique_lock<std::mutex> lk;
  explicit CoopSection(fs_context_s* c) : ctx(c) {
    if (c->coop_lock) lk = std::unique_lock<std::mutex>(*c->coop_lock);
  }
  ~CoopSection() {
    if (lk.owns_lock()) (void)hipStreamSynchronize(ctx->stream);
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
